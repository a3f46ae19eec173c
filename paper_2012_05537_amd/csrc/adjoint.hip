// Reverse-mode kernels (placeholder until the adjoint is built).
#include "sllbm_internal.h"
