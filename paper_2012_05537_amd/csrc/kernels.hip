// HIP kernels (gfx950) of the SLLBM library besides the streaming
// (stream.hip) and the reverse mode (adjoint.hip): the collision of a whole
// state, equilibrium initialisation, FP64 moments and deterministic totals.
#include <hip/hip_runtime.h>

#include <cmath>

#include "collision.h"
#include "nt.h"
#include "sllbm_internal.h"
#include "velset.h"
#include "xcd.h"

namespace sllbm {

// Collision of a whole state (Eq. (5) right-hand side with App. D), two
// lanes per node (f on the even lane, g on the odd one), the values in
// registers: D3Q45 in FP64, D2Q19 in FP32, and the cases that k_collide_lds
// below does not take (N not a multiple of 16 / sizeof(S), an input not
// 16-byte aligned).  in and out may be the same buffer (each lane reads its
// values first).  NTH: non-temporal loads and stores (states larger than
// the Infinity Cache).
template <typename S, class L, bool NTH>
__global__ void __launch_bounds__(256) k_collide(int64_t N, CollisionParams cp, const S *in, S *out)
{
    constexpr int NQ = L::Q;
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t n = t >> 1;
    const int pop = static_cast<int>(t & 1);
    if (n >= N) return;                    // both lanes of a pair leave together
    const int64_t o = static_cast<int64_t>(pop) * NQ * N + n;
    const S *p = in + o;
    S v[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) v[i] = load_hint<NTH>(&p[static_cast<int64_t>(i) * N]);
    // derive the store addresses afresh: otherwise the 45 load addresses stay
    // live through the collision (90 registers)
    S *d = out + o;
    if constexpr (sizeof(S) == 4) {
        // FP32 storage: store every value as the relaxation forms it; the
        // D3Q45 collision is latency-bound here (two waves per SIMD), and
        // stores spread over it measured 7 % faster at 256^3 nodes (no gain
        // in FP64)
        asm volatile("" : "+v"(d));
        collide_half_s<L, S>(v, pop != 0, cp,
                             [d, N](int i, S x) { store_hint<NTH>(&d[static_cast<int64_t>(i) * N], x); });
    } else {
        collide_half<L, S>(v, pop != 0, cp);
        asm volatile("" : "+v"(d));
#pragma unroll
        for (int i = 0; i < NQ; ++i) store_hint<NTH>(&d[static_cast<int64_t>(i) * N], v[i]);
    }
}

// DMA copy of 16 bytes per lane from g into LDS at l + 16 * lane (l is
// wave-uniform).  AUX is the copy's cache-policy operand (2: non-temporal,
// 0: the default policy).  A device function of its own: the 16-byte form
// exists on gfx950 only, and the host pass drops the launch stub of a
// kernel whose body names it.
template <int AUX, typename T>
__device__ __forceinline__ void dma16(const T *g, T *l)
{
    __builtin_amdgcn_global_load_lds(g, l, 16, 0, AUX);
}

// The collision with its values staged in LDS; used for D3Q45 in FP32
// storage and D2Q19 in FP64, for N a multiple of 16 / sizeof(S) and a
// 16-byte aligned input.  A block collides NB = 512 / sizeof(S) consecutive
// nodes (128 in FP32, 64 in FP64; blocks in XCD order) with NB / 32 waves.
// Their 2Q rows of NB values (row r = pop * Q + i, 512 contiguous bytes of
// plane r) are copied from memory into LDS by DMA, 16 bytes per lane, so
// one instruction moves two rows (1 KB) and no register holds them; every
// value is then read from LDS for the moments and again for the relaxation.
// Lane l of wave w holds node w * 32 + (l & 31) of the block and population
// l >> 5 (partner lane l ^ 32).  For D3Q45 in FP32: 136 VGPRs and 45 KB of
// LDS per block (3 waves per SIMD), where the register form needs 224 VGPRs
// (2 waves) and reads 128-byte segments per plane and half-wave.
// in may equal out: every copy has landed before the barrier, and a block
// writes only its own nodes.  NTH: non-temporal copies and stores.
template <typename S, class L, bool NTH>
__global__ void __launch_bounds__(1024 / sizeof(S), 3) k_collide_lds(int64_t N, CollisionParams cp, const S *in,
                                                                     S *out)
{
    constexpr int NQ = L::Q, ROWS = 2 * NQ, NB = 512 / sizeof(S), NW = NB / 32, VL = 16 / sizeof(S);
    __shared__ S tile[ROWS][NB];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nb = static_cast<int64_t>(xcd_linear(blockIdx.x, gridDim.x)) * NB;
    {
        // instruction m of the block copies rows 2m (lanes 0-31) and 2m + 1
        // (lanes 32-63), VL nodes per lane; a lane's nodes are all below N or
        // all beyond it (N % VL == 0)
        const int64_t col = nb + VL * (lane & 31);
        if (col < N) {
            const S *src = in + static_cast<int64_t>(lane >> 5) * N + col;
            for (int m = w; m < ROWS / 2; m += NW)
                dma16<NTH ? 2 : 0>(src + static_cast<int64_t>(2 * m) * N, &tile[2 * m][0]);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);               // this wave's copies have landed
    __syncthreads();                             // and every other wave's
    const int pop = lane >> 5;
    const int c = w * 32 + (lane & 31);
    const int64_t n = nb + c;
    if (n >= N) return;                          // both lanes of a pair leave together
    const S *sl = &tile[pop * NQ][c];
    S *d = out + static_cast<int64_t>(pop) * NQ * N + n;
    asm volatile("" : "+v"(d));
    collide_core<L, S, 32>([&](int i) { return sl[i * NB]; }, [] { asm volatile("" ::: "memory"); }, pop != 0, cp,
                           [d, N](int i, S x) { store_hint<NTH>(&d[static_cast<int64_t>(i) * N], x); });
}

// The same collision with each lane pair taking nodes n, n + G, ... (G lane
// pairs in the grid): the next node's values are loaded while the current
// node collides.  The D2Q19 FP64 collision where k_collide_lds does not
// apply; there (216 VGPRs, 2 waves/SIMD) it hides the load latency better
// than one node per pair at 4 waves/SIMD
// (a launch of that form has only two rounds of waves at 512^2 nodes); with
// 45 velocities the second set of registers does not fit.  in may equal out:
// node n + G belongs to this lane pair only.
template <typename S, class L>
__global__ void __launch_bounds__(256) k_collide_pf(int64_t N, CollisionParams cp, const S *in, S *out)
{
    constexpr int NQ = L::Q;
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t pairs = static_cast<int64_t>(gridDim.x) * blockDim.x / 2;
    int64_t n = t >> 1;
    const int pop = static_cast<int>(t & 1);
    if (n >= N) return;                    // both lanes of a pair leave together
    const int64_t po = static_cast<int64_t>(pop) * NQ * N;
    S v[NQ], nx[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) v[i] = in[po + static_cast<int64_t>(i) * N + n];
    while (true) {
        const int64_t n2 = n + pairs;
        const bool more = n2 < N;          // equal on both lanes of a pair
        if (more) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) nx[i] = in[po + static_cast<int64_t>(i) * N + n2];
        }
        collide_half<L, S>(v, pop != 0, cp);
        S *d = out + po + n;
        asm volatile("" : "+v"(d));
#pragma unroll
        for (int i = 0; i < NQ; ++i) d[static_cast<int64_t>(i) * N] = v[i];
        if (!more) break;
#pragma unroll
        for (int i = 0; i < NQ; ++i) v[i] = nx[i];
        n = n2;
    }
}

// u: [D][N] (the lattice's dimension)
template <typename S, class L>
__global__ void __launch_bounds__(256) k_init_equilibrium(int64_t N, CollisionParams cp,
                                                          const double *__restrict__ rho,
                                                          const double *__restrict__ u,
                                                          const double *__restrict__ T, S *__restrict__ state)
{
    for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double r = rho[n], ux = u[n], uy = u[N + n], uz = L::D == 3 ? u[2 * N + n] : 0.0, Tn = T[n];
        const double u2 = ux * ux + uy * uy + uz * uz;
        const double th = Tn - 1.0;
        const double betaT = cp.beta * Tn;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const double c = L::T.xi[i][0] * ux + L::T.xi[i][1] * uy + L::T.xi[i][2] * uz;
            const EqShell e = eq_shell<L::D>(u2, th, L::T.x2[i]);
            const double br = fma(c, fma(c, fma(c, fma(c, 1.0 / 24.0, 1.0 / 6.0), e.a2), e.a1), e.a0);
            const double feq = L::T.w[i] * r * br;
            state[static_cast<int64_t>(i) * N + n] = static_cast<S>(feq);
            state[static_cast<int64_t>(L::Q + i) * N + n] = static_cast<S>(betaT * feq);
        }
    }
}

// rho, j, 2 rho E of node n (Eq. (7)), in double (jz = 0 in two dimensions)
template <typename S, class L>
__device__ __forceinline__ void node_sums(const S *__restrict__ state, int64_t N, int64_t n, double &rho,
                                          double &jx, double &jy, double &jz, double &twoE)
{
    rho = jx = jy = jz = twoE = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double fi = static_cast<double>(state[static_cast<int64_t>(i) * N + n]);
        rho += fi;
        jx = fma(fi, L::T.xi[i][0], jx);
        jy = fma(fi, L::T.xi[i][1], jy);
        if constexpr (L::D == 3) jz = fma(fi, L::T.xi[i][2], jz);
        twoE = fma(fi, L::T.x2[i], twoE) + static_cast<double>(state[static_cast<int64_t>(L::Q + i) * N + n]);
    }
}

// u: [D][N]
template <typename S, class L>
__global__ void __launch_bounds__(256) k_moments(int64_t N, CollisionParams cp, const S *__restrict__ state,
                                                 double *__restrict__ rho, double *__restrict__ u,
                                                 double *__restrict__ T)
{
    for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double r, jx, jy, jz, twoE;
        node_sums<S, L>(state, N, n, r, jx, jy, jz, twoE);
        const double ux = jx / r, uy = jy / r, uz = jz / r;
        if (rho) rho[n] = r;
        if (u) {
            u[n] = ux;
            u[N + n] = uy;
            if constexpr (L::D == 3) u[2 * N + n] = uz;
        }
        if (T) T[n] = (twoE / r - (ux * ux + uy * uy + uz * uz)) / (2.0 * cp.Cv);
    }
}

// Block-level sum of NV doubles per thread, in a fixed order (deterministic).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *red)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * blockDim.x + tid] = v[k];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int k = 0; k < NV; ++k) red[k * blockDim.x + tid] += red[k * blockDim.x + tid + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = red[k * blockDim.x];
}

// Stage 1 of the totals: per-block weighted sums of rho, rho u, rho E.
template <typename S, class L>
__global__ void __launch_bounds__(256) k_totals_partial(Geometry geo, const S *__restrict__ state,
                                                        const double *__restrict__ nodew,
                                                        const double *__restrict__ full_w,
                                                        double *__restrict__ partials)
{
    __shared__ double red[5 * 256];
    const int64_t N = geo.nodes;
    double acc[5] = {0, 0, 0, 0, 0};
    const double *wx = nodew, *wy = nodew + geo.N[0], *wz = wy + geo.N[1];
    for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int gx = static_cast<int>(n % geo.N[0]);
        const int64_t r = n / geo.N[0];
        const int gy = static_cast<int>(r % geo.N[1]);
        const int gz = static_cast<int>(r / geo.N[1]);
        const double W = full_w ? full_w[n] : wx[gx] * wy[gy] * wz[gz];
        double rho, jx, jy, jz, twoE;
        node_sums<S, L>(state, N, n, rho, jx, jy, jz, twoE);
        acc[0] = fma(W, rho, acc[0]);
        acc[1] = fma(W, jx, acc[1]);
        acc[2] = fma(W, jy, acc[2]);
        acc[3] = fma(W, jz, acc[3]);
        acc[4] = fma(W, 0.5 * twoE, acc[4]);
    }
    block_sum<5>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = acc[k];
    }
}

// Stage 2: one block of 256 threads adds the per-block partials: thread t
// sums blocks t, t + 256, ... in order, then a fixed tree (deterministic).
template <int NV>
__global__ void __launch_bounds__(256) k_reduce_partials(const double *__restrict__ partials, int nblocks,
                                                         double *__restrict__ out, int accumulate)
{
    __shared__ double red[NV * 256];
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += partials[b * NV + k];
    block_sum<NV>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = accumulate ? out[k] + acc[k] : acc[k];
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static int node_grid(int64_t N)
{
    int64_t b = (N + 255) / 256;
    return static_cast<int>(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

template <typename S, class L>
static hipError_t collide_lat(const Geometry &g, const CollisionParams &cp, const S *in, S *out, hipStream_t st)
{
    if constexpr ((L::Q == 45 && sizeof(S) == 4) || (L::Q == Q2D && sizeof(S) == 8)) {
        // LDS-staged form, measured against the register forms: D3Q45 FP32
        // at 256^3 nodes 3.02 -> 2.29 ms, D2Q19 FP64 at 512^2 nodes 34 ->
        // 28 us (no faster for D2Q19 in FP32, slower for D3Q45 in FP64 at
        // 128^3 and 256^3 nodes); its 16-byte copies need aligned rows
        constexpr int NB = 512 / sizeof(S), VL = 16 / sizeof(S);
        if (g.nodes % VL == 0 && reinterpret_cast<uintptr_t>(in) % 16 == 0) {
            const int64_t b = (g.nodes + NB - 1) / NB;
            if (use_nontemporal(2 * L::Q * g.nodes * static_cast<int64_t>(sizeof(S))))
                hipLaunchKernelGGL((k_collide_lds<S, L, true>), dim3(static_cast<unsigned>(b)), dim3(2 * NB), 0, st,
                                   g.nodes, cp, in, out);
            else
                hipLaunchKernelGGL((k_collide_lds<S, L, false>), dim3(static_cast<unsigned>(b)), dim3(2 * NB), 0,
                                   st, g.nodes, cp, in, out);
            return hipGetLastError();
        }
    }
    if constexpr (L::Q == Q2D && sizeof(S) == 8) {
        // otherwise two nodes per lane pair (measured 12 % faster at 512^2
        // nodes than one; in FP32 the one-node form is faster)
        const int64_t blocks = (g.nodes + 255) / 256;
        hipLaunchKernelGGL((k_collide_pf<S, L>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, g.nodes, cp,
                           in, out);
        return hipGetLastError();
    }
    const int64_t blocks = (2 * g.nodes + 255) / 256;
    if (use_nontemporal(2 * L::Q * g.nodes * static_cast<int64_t>(sizeof(S))))
        hipLaunchKernelGGL((k_collide<S, L, true>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, g.nodes, cp,
                           in, out);
    else
        hipLaunchKernelGGL((k_collide<S, L, false>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, g.nodes,
                           cp, in, out);
    return hipGetLastError();
}

template <typename S, class L>
static hipError_t init_lat(const Geometry &g, const CollisionParams &cp, const double *rho, const double *u,
                           const double *T, S *state, hipStream_t st)
{
    hipLaunchKernelGGL((k_init_equilibrium<S, L>), dim3(node_grid(g.nodes)), dim3(256), 0, st, g.nodes, cp, rho, u,
                       T, state);
    return hipGetLastError();
}

template <typename S, class L>
static hipError_t moments_lat(const Geometry &g, const CollisionParams &cp, const S *state, double *rho, double *u,
                              double *T, hipStream_t st)
{
    hipLaunchKernelGGL((k_moments<S, L>), dim3(node_grid(g.nodes)), dim3(256), 0, st, g.nodes, cp, state, rho, u,
                       T);
    return hipGetLastError();
}

template <typename S, class L>
static hipError_t totals_lat(const Geometry &g, const S *state, const double *nodew, const double *full_w,
                             double *partials, int nblocks, double *out5, hipStream_t st)
{
    hipLaunchKernelGGL((k_totals_partial<S, L>), dim3(nblocks), dim3(256), 0, st, g, state, nodew, full_w, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reduce_partials<5>), dim3(1), dim3(256), 0, st, partials, nblocks, out5, 0);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::collide_only(const Geometry &g, const CollisionParams &cp, S *state, hipStream_t st)
{
    return collide_into(g, cp, state, state, st);
}

template <typename S>
hipError_t Launch<S>::collide_into(const Geometry &g, const CollisionParams &cp, const S *in, S *out, hipStream_t st)
{
    return collide_lat<S, D3Q45>(g, cp, in, out, st);
}

template <typename S>
hipError_t Launch<S>::init_equilibrium(const Geometry &g, const CollisionParams &cp, const double *rho,
                                       const double *u, const double *T, S *state, hipStream_t st)
{
    return init_lat<S, D3Q45>(g, cp, rho, u, T, state, st);
}

template <typename S>
hipError_t Launch<S>::moments(const Geometry &g, const CollisionParams &cp, const S *state, double *rho,
                              double *u, double *T, hipStream_t st)
{
    return moments_lat<S, D3Q45>(g, cp, state, rho, u, T, st);
}

template <typename S>
hipError_t Launch<S>::totals(const Geometry &g, const CollisionParams &, const S *state, const double *nodew,
                             const double *full_w, double *partials, int nblocks, double *out5, hipStream_t st)
{
    return totals_lat<S, D3Q45>(g, state, nodew, full_w, partials, nblocks, out5, st);
}

template <typename S>
hipError_t Launch2D<S>::collide_into(const Geometry &g, const CollisionParams &cp, const S *in, S *out,
                                     hipStream_t st)
{
    return collide_lat<S, D2Q19>(g, cp, in, out, st);
}

template <typename S>
hipError_t Launch2D<S>::init_equilibrium(const Geometry &g, const CollisionParams &cp, const double *rho,
                                         const double *u, const double *T, S *state, hipStream_t st)
{
    return init_lat<S, D2Q19>(g, cp, rho, u, T, state, st);
}

template <typename S>
hipError_t Launch2D<S>::moments(const Geometry &g, const CollisionParams &cp, const S *state, double *rho,
                                double *u, double *T, hipStream_t st)
{
    return moments_lat<S, D2Q19>(g, cp, state, rho, u, T, st);
}

template <typename S>
hipError_t Launch2D<S>::totals(const Geometry &g, const S *state, const double *nodew, double *partials,
                               int nblocks, double *out5, hipStream_t st)
{
    return totals_lat<S, D2Q19>(g, state, nodew, nullptr, partials, nblocks, out5, st);
}

template struct Launch<double>;
template struct Launch<float>;
template struct Launch2D<double>;
template struct Launch2D<float>;

}  // namespace sllbm
