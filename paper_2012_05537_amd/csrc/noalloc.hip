// Allocation-free totals: sllbm_totals_noalloc.
//
// For callers that cannot allocate device memory (work under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  The
// operation is that of sllbm_totals (Clenshaw-Curtis integrals of the Eq. (7)
// moments over an equal-cell periodic mesh) on a caller state, with the
// result left on the device.  Its scratch, the per-block reduction partials
// and the 1-D node weights, lives in one file-scope device array; the host
// takes that array's device address once per device (hipGetSymbolAddress,
// with the device current) and passes it to the same kernels sllbm_totals
// launches, so both give the same bits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "sllbm_internal.h"

namespace sllbm {

namespace {

constexpr int NA_BLOCKS = 1024;                              // reduction blocks, as in sllbm_totals
constexpr int64_t PARTIAL_DOUBLES = NA_BLOCKS * 8;
constexpr int64_t SCRATCH_DOUBLES = 32768;                   // 256 KB per device
constexpr int64_t MAX_AXIS_NODES = SCRATCH_DOUBLES - PARTIAL_DOUBLES;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

// Device address of this device's copy of the scratch array (the array's
// name is only a host-side stand-in).  The caller has made dev current.
hipError_t scratch_on(int dev, double **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

struct LocalWeights {
    double w[3][MAXP];   // weight of local point l of a cell along each axis (shared faces summed)
    int N[3];
    int p;
};

// nodew = [x nodes][y nodes][z nodes], the separable node weights of sllbm_totals
__global__ void __launch_bounds__(256) k_fill_node_weights(LocalWeights lw, double *__restrict__ nodew)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = lw.N[0] + lw.N[1] + lw.N[2];
    if (n >= total) return;
    const int a = n < lw.N[0] ? 0 : (n < lw.N[0] + lw.N[1] ? 1 : 2);
    const int g = n - (a > 0 ? lw.N[0] : 0) - (a > 1 ? lw.N[1] : 0);
    nodew[n] = lw.w[a][g % lw.p];
}

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceScope()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

}  // namespace sllbm

using namespace sllbm;

extern "C" int sllbm_totals_noalloc(const sllbm_config *cfg, const void *state, double *out, void *stream)
{
    if (!cfg) return set_global_error(SLLBM_EINVAL, "cfg is NULL");
    if (cfg->velocity_set != SLLBM_D3Q45 && cfg->velocity_set != SLLBM_D2Q19)
        return set_global_error(SLLBM_EINVAL, "velocity_set must be SLLBM_D3Q45 or SLLBM_D2Q19");
    const bool d2 = cfg->velocity_set == SLLBM_D2Q19;
    const int p = cfg->order;
    if (p < 1 || p > MAXP) return set_global_error(SLLBM_EINVAL, "order must be in 1..6");
    if (cfg->precision != SLLBM_FP64 && cfg->precision != SLLBM_FP32_MIXED)
        return set_global_error(SLLBM_EINVAL, "unknown precision");
    if (d2 && cfg->n_el[2] != 1) return set_global_error(SLLBM_EINVAL, "n_el[2] must be 1 for SLLBM_D2Q19");
    int64_t Na[3];
    for (int a = 0; a < 3; ++a) {
        if (cfg->n_el[a] < 1) return set_global_error(SLLBM_EINVAL, "n_el must be >= 1");
        if (a < (d2 ? 2 : 3) && (!(cfg->length[a] > 0.0) || !std::isfinite(cfg->length[a])))
            return set_global_error(SLLBM_EINVAL, "length must be positive");
        Na[a] = (d2 && a == 2) ? 1 : static_cast<int64_t>(cfg->n_el[a]) * p;
    }
    if (Na[0] + Na[1] + Na[2] > MAX_AXIS_NODES)
        return set_global_error(SLLBM_EINVAL, "grid exceeds the static scratch: N_x + N_y + N_z must be <= 24576");
    const int64_t nodes = Na[0] * Na[1] * Na[2];
    if (nodes >= (int64_t(1) << 31)) return set_global_error(SLLBM_EINVAL, "grid too large");
    if (!state || !out) return set_global_error(SLLBM_EINVAL, "NULL state or out");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return set_global_error(SLLBM_EDEVICE, "no HIP device available");
    if (cfg->device < 0 || cfg->device >= ndev || cfg->device >= MAX_DEVICES)
        return set_global_error(SLLBM_EINVAL, "device ordinal out of range");

    DeviceScope scope(cfg->device);
    double *scr = nullptr;
    hipError_t e = scratch_on(cfg->device, &scr);
    if (e != hipSuccess) return set_global_error(SLLBM_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    double *partials = scr, *nodew = scr + PARTIAL_DOUBLES;

    LocalWeights lw{};
    double cc[MAXP + 1];
    clenshaw_curtis(p, cc);
    for (int a = 0; a < 3; ++a) {
        const double h = cfg->length[a] / cfg->n_el[a];
        for (int l = 0; l < p; ++l) lw.w[a][l] = (d2 && a == 2) ? 1.0 : 0.5 * h * (l == 0 ? cc[0] + cc[p] : cc[l]);
        lw.N[a] = static_cast<int>(Na[a]);
    }
    lw.p = p;
    Geometry g{};
    g.p = p;
    for (int a = 0; a < 3; ++a) {
        g.nel[a] = cfg->n_el[a];
        g.N[a] = static_cast<int>(Na[a]);
    }
    g.nodes = nodes;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int total = static_cast<int>(Na[0] + Na[1] + Na[2]);
    hipLaunchKernelGGL(k_fill_node_weights, dim3((total + 255) / 256), dim3(256), 0, st, lw, nodew);
    if ((e = hipGetLastError()) != hipSuccess)
        return set_global_error(SLLBM_EDEVICE, std::string("node weights: ") + hipGetErrorString(e));
    const CollisionParams cp{};
    if (d2)
        e = cfg->precision == SLLBM_FP64
                ? Launch2D<double>::totals(g, static_cast<const double *>(state), nodew, partials, NA_BLOCKS, out, st)
                : Launch2D<float>::totals(g, static_cast<const float *>(state), nodew, partials, NA_BLOCKS, out, st);
    else
        e = cfg->precision == SLLBM_FP64
                ? Launch<double>::totals(g, cp, static_cast<const double *>(state), nodew, nullptr, partials,
                                         NA_BLOCKS, out, st)
                : Launch<float>::totals(g, cp, static_cast<const float *>(state), nodew, nullptr, partials, NA_BLOCKS,
                                        out, st);
    if (e != hipSuccess) return set_global_error(SLLBM_EDEVICE, std::string("totals: ") + hipGetErrorString(e));
    return SLLBM_OK;
}
