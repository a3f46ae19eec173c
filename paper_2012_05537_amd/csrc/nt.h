// Non-temporal global accesses for the step kernels on grids whose state
// exceeds the Infinity Cache.  The collision reads and writes every value
// once, and the streaming writes every output once: at such sizes caching
// those lines only evicts lines that a later read could use (measured at
// 128^3 and 256^3 nodes: the collision 5-6 % and the streaming 1-3 % faster).
// When the state fits in the cache the plain forms are faster, because the
// next kernel of the step reads its input from there.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sllbm {

constexpr int64_t INFINITY_CACHE_BYTES = int64_t(256) << 20;   // MI355X

inline bool use_nontemporal(int64_t state_bytes) { return state_bytes > INFINITY_CACHE_BYTES; }

template <bool NT, typename T>
__device__ __forceinline__ T load_hint(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void store_hint(T *p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

}  // namespace sllbm
