// HIP kernels (gfx950) of the SLLBM library besides the forward streaming
// (stream.hip) and the reverse mode (adjoint.hip): the table-driven streaming
// used for the transposed operator S^T (any tap count), the collision of a
// whole state, equilibrium initialisation, FP64 moments and deterministic
// totals.
//
// Table-driven streaming.  Psi_i = Iz (x) Iy (x) Ix is applied by sum
// factorisation: a thread block owns a tile of whole cells, stages the
// tile's departure window of f_i and g_i in LDS (coalesced loads, x
// fastest), interpolates along z, then y, then x, and keeps the result of
// its node in registers; every axis row is a list of (offset, weight) taps.
#include <hip/hip_runtime.h>

#include <cmath>

#include "collision.h"
#include "sllbm_internal.h"
#include "velset.h"

namespace sllbm {

__device__ __forceinline__ int pmod(int x, int n)
{
    int r = x % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------
// Sum-factorised streaming of one velocity for one tile
// ---------------------------------------------------------------------------

struct TileInfo {
    int X0[3];    // first node of the tile per axis
    int TN[3];    // nodes of the tile per axis (whole cells)
    int nE[3];    // cells of the tile per axis
    int lx, ly, lz;
    bool valid;
};

__device__ __forceinline__ TileInfo tile_info(const Geometry &geo)
{
    TileInfo t;
    int b = blockIdx.x;
    int tc[3];
    tc[0] = b % geo.ntile[0];
    b /= geo.ntile[0];
    tc[1] = b % geo.ntile[1];
    tc[2] = b / geo.ntile[1];
    const int p = geo.p;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int e0 = tc[a] * geo.TE[a];
        t.nE[a] = min(geo.TE[a], geo.nel[a] - e0);
        t.X0[a] = e0 * p;
        t.TN[a] = t.nE[a] * p;
    }
    const int FTx = geo.TE[0] * p, FTy = geo.TE[1] * p;
    const int tid = threadIdx.x;
    t.lx = tid % FTx;
    t.ly = (tid / FTx) % FTy;
    t.lz = tid / (FTx * FTy);
    t.valid = t.lx < t.TN[0] && t.ly < t.TN[1] && t.lz < t.TN[2];
    return t;
}

template <typename S>
struct StreamSmem {
    S *sF, *sG, *bF, *bG, *cF, *cG;
};

template <typename S>
__device__ __forceinline__ StreamSmem<S> carve_smem(const Geometry &geo, const StreamTables &tab)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    S *base = reinterpret_cast<S *>(smem_raw);
    const int FTy = geo.TE[1] * geo.p, FTz = geo.TE[2] * geo.p;
    const int ns = tab.wmax[0] * tab.wmax[1] * tab.wmax[2];
    const int nb = tab.wmax[0] * tab.wmax[1] * FTz;
    const int nc = tab.wmax[0] * FTy * FTz;
    StreamSmem<S> s;
    s.sF = base;
    s.sG = s.sF + ns;
    s.bF = s.sG + ns;
    s.bG = s.bF + nb;
    s.cF = s.bG + nb;
    s.cG = s.cF + nc;
    return s;
}

// Streams velocity i of the two populations stored at fin / gin (each [N])
// through the 1-D tables; the result for the thread's node is returned in
// fo / go.  All threads of the block must call it (it synchronises).
template <typename S>
__device__ __forceinline__ void stream_velocity(int i, const Geometry &geo, const StreamTables &tab,
                                                const TileInfo &t, const StreamSmem<S> &sm,
                                                const S *__restrict__ fin, const S *__restrict__ gin,
                                                S &fo, S &go)
{
    const int p = geo.p, K = tab.K;
    const S *__restrict__ wt = static_cast<const S *>(tab.wt);
    int lo[3], W[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = tab.lo[i * 3 + a];
        W[a] = (t.nE[a] - 1) * p + tab.span[i * 3 + a];
    }
    const int ox = t.X0[0] + lo[0], oy = t.X0[1] + lo[1], oz = t.X0[2] + lo[2];
    const int nthr = blockDim.x;

    // 1. departure window of the tile -> LDS (x fastest, coalesced)
    const int nw = W[0] * W[1] * W[2];
    for (int w = threadIdx.x; w < nw; w += nthr) {
        const int wx = w % W[0];
        const int r = w / W[0];
        const int wy = r % W[1];
        const int wz = r / W[1];
        const int gx = pmod(ox + wx, geo.N[0]);
        const int gy = pmod(oy + wy, geo.N[1]);
        const int gz = pmod(oz + wz, geo.N[2]);
        const int64_t n = (static_cast<int64_t>(gz) * geo.N[1] + gy) * geo.N[0] + gx;
        sm.sF[w] = fin[n];
        sm.sG[w] = gin[n];
    }
    __syncthreads();

    // 2. z-pass: (wx, wy, tz)
    {
        const int32_t *offz = tab.off + ((i * 3 + 2) * p) * K;
        const S *wz = wt + ((i * 3 + 2) * p) * K;
        const int nb = W[0] * W[1] * t.TN[2];
        for (int o = threadIdx.x; o < nb; o += nthr) {
            const int wx = o % W[0];
            const int r = o / W[0];
            const int wy = r % W[1];
            const int tz = r / W[1];
            const int l = tz % p;
            const int e0 = tz - l - lo[2];
            S af = 0, ag = 0;
            for (int k = 0; k < K; ++k) {
                const int sz = e0 + offz[l * K + k];
                const S c = wz[l * K + k];
                const int idx = (sz * W[1] + wy) * W[0] + wx;
                af = fma(c, sm.sF[idx], af);
                ag = fma(c, sm.sG[idx], ag);
            }
            sm.bF[o] = af;
            sm.bG[o] = ag;
        }
    }
    __syncthreads();

    // 3. y-pass: (wx, ty, tz)
    {
        const int32_t *offy = tab.off + ((i * 3 + 1) * p) * K;
        const S *wy_ = wt + ((i * 3 + 1) * p) * K;
        const int nc = W[0] * t.TN[1] * t.TN[2];
        for (int o = threadIdx.x; o < nc; o += nthr) {
            const int wx = o % W[0];
            const int r = o / W[0];
            const int ty = r % t.TN[1];
            const int tz = r / t.TN[1];
            const int l = ty % p;
            const int e0 = ty - l - lo[1];
            S af = 0, ag = 0;
            for (int k = 0; k < K; ++k) {
                const int sy = e0 + offy[l * K + k];
                const S c = wy_[l * K + k];
                const int idx = (tz * W[1] + sy) * W[0] + wx;
                af = fma(c, sm.bF[idx], af);
                ag = fma(c, sm.bG[idx], ag);
            }
            sm.cF[o] = af;
            sm.cG[o] = ag;
        }
    }
    __syncthreads();

    // 4. x-pass: the thread's own node
    if (t.valid) {
        const int32_t *offx = tab.off + ((i * 3 + 0) * p) * K;
        const S *wx_ = wt + ((i * 3 + 0) * p) * K;
        const int l = t.lx % p;
        const int e0 = t.lx - l - lo[0];
        const int row = (t.lz * t.TN[1] + t.ly) * W[0];
        S af = 0, ag = 0;
        for (int k = 0; k < K; ++k) {
            const int sx = e0 + offx[l * K + k];
            const S c = wx_[l * K + k];
            af = fma(c, sm.cF[row + sx], af);
            ag = fma(c, sm.cG[row + sx], ag);
        }
        fo = af;
        go = ag;
    }
    // The next call's writes are separated from this call's LDS reads by at
    // least one barrier each (window -> z-pass, b -> y-pass, c -> x-pass).
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

template <typename S>
__global__ void __launch_bounds__(256) k_stream_tab(Geometry geo, StreamTables tab, const S *__restrict__ in,
                                                    S *__restrict__ out)
{
    const TileInfo t = tile_info(geo);
    const StreamSmem<S> sm = carve_smem<S>(geo, tab);
    const int64_t N = geo.nodes;
    S fv[Q], gv[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        stream_velocity<S>(i, geo, tab, t, sm, in + static_cast<int64_t>(i) * N,
                           in + static_cast<int64_t>(Q + i) * N, fv[i], gv[i]);
    }
    if (!t.valid) return;
    const int64_t node =
        (static_cast<int64_t>(t.X0[2] + t.lz) * geo.N[1] + (t.X0[1] + t.ly)) * geo.N[0] + t.X0[0] + t.lx;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        out[static_cast<int64_t>(i) * N + node] = fv[i];
        out[static_cast<int64_t>(Q + i) * N + node] = gv[i];
    }
}

// Collision of a whole state (Eq. (5) right-hand side with App. D), two
// lanes per node (f on the even lane, g on the odd one).  in and out may be
// the same buffer (each lane reads its 45 values first).
template <typename S>
__global__ void __launch_bounds__(256) k_collide(int64_t N, CollisionParams cp, const S *in, S *out)
{
    const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t n = t >> 1;
    const int pop = static_cast<int>(t & 1);
    if (n >= N) return;                    // both lanes of a pair leave together
    const int64_t o = static_cast<int64_t>(pop) * Q * N + n;
    const S *p = in + o;
    S v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = p[static_cast<int64_t>(i) * N];
    collide_half<S>(v, pop != 0, cp);
    // derive the store addresses afresh: otherwise the 45 load addresses stay
    // live through the collision (90 registers)
    S *d = out + o;
    asm volatile("" : "+v"(d));
#pragma unroll
    for (int i = 0; i < Q; ++i) d[static_cast<int64_t>(i) * N] = v[i];
}

template <typename S>
__global__ void __launch_bounds__(256) k_init_equilibrium(int64_t N, CollisionParams cp,
                                                          const double *__restrict__ rho,
                                                          const double *__restrict__ u,
                                                          const double *__restrict__ T, S *__restrict__ state)
{
    for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double r = rho[n], ux = u[n], uy = u[N + n], uz = u[2 * N + n], Tn = T[n];
        const double u2 = ux * ux + uy * uy + uz * uz;
        const double th = Tn - 1.0;
        const double betaT = cp.beta * Tn;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double c = vs::T.xi[i][0] * ux + vs::T.xi[i][1] * uy + vs::T.xi[i][2] * uz;
            const EqShell e = eq_shell(u2, th, vs::T.x2[i]);
            const double br = fma(c, fma(c, fma(c, fma(c, 1.0 / 24.0, 1.0 / 6.0), e.a2), e.a1), e.a0);
            const double feq = vs::T.w[i] * r * br;
            state[static_cast<int64_t>(i) * N + n] = static_cast<S>(feq);
            state[static_cast<int64_t>(Q + i) * N + n] = static_cast<S>(betaT * feq);
        }
    }
}

// rho, j, 2 rho E of node n (Eq. (7)), in double
template <typename S>
__device__ __forceinline__ void node_sums(const S *__restrict__ state, int64_t N, int64_t n, double &rho,
                                          double &jx, double &jy, double &jz, double &twoE)
{
    rho = jx = jy = jz = twoE = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double fi = static_cast<double>(state[static_cast<int64_t>(i) * N + n]);
        rho += fi;
        jx = fma(fi, vs::T.xi[i][0], jx);
        jy = fma(fi, vs::T.xi[i][1], jy);
        jz = fma(fi, vs::T.xi[i][2], jz);
        twoE = fma(fi, vs::T.x2[i], twoE) + static_cast<double>(state[static_cast<int64_t>(Q + i) * N + n]);
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_moments(int64_t N, CollisionParams cp, const S *__restrict__ state,
                                                 double *__restrict__ rho, double *__restrict__ u,
                                                 double *__restrict__ T)
{
    for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double r, jx, jy, jz, twoE;
        node_sums(state, N, n, r, jx, jy, jz, twoE);
        const double ux = jx / r, uy = jy / r, uz = jz / r;
        if (rho) rho[n] = r;
        if (u) {
            u[n] = ux;
            u[N + n] = uy;
            u[2 * N + n] = uz;
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
template <typename S>
__global__ void __launch_bounds__(256) k_totals_partial(Geometry geo, const S *__restrict__ state,
                                                        const double *__restrict__ nodew,
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
        const double W = wx[gx] * wy[gy] * wz[gz];
        double rho, jx, jy, jz, twoE;
        node_sums(state, N, n, rho, jx, jy, jz, twoE);
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

int tile_nodes(const Geometry &g) { return g.TE[0] * g.TE[1] * g.TE[2] * g.p * g.p * g.p; }

int blocks_for(const Geometry &g) { return g.ntile[0] * g.ntile[1] * g.ntile[2]; }

size_t stream_smem_bytes(const Geometry &g, const StreamTables &t, size_t elem)
{
    const size_t FTy = g.TE[1] * g.p, FTz = g.TE[2] * g.p;
    const size_t ns = static_cast<size_t>(t.wmax[0]) * t.wmax[1] * t.wmax[2];
    const size_t nb = static_cast<size_t>(t.wmax[0]) * t.wmax[1] * FTz;
    const size_t nc = static_cast<size_t>(t.wmax[0]) * FTy * FTz;
    return 2 * (ns + nb + nc) * elem;
}

static int node_grid(int64_t N)
{
    int64_t b = (N + 255) / 256;
    return static_cast<int>(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

static int stream_block(const Geometry &g)
{
    return ((tile_nodes(g) + 63) / 64) * 64;
}

template <typename Kern>
static hipError_t allow_smem(Kern kern, size_t smem)
{
    if (smem <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(smem));
}

template <typename S>
hipError_t Launch<S>::stream_only(const Geometry &g, const StreamTables &t, const S *in, S *out,
                                  hipStream_t st)
{
    const size_t smem = stream_smem_bytes(g, t, sizeof(S));
    hipError_t e = allow_smem(k_stream_tab<S>, smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stream_tab<S>), dim3(blocks_for(g)), dim3(stream_block(g)), smem, st, g, t, in, out);
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
    const int64_t blocks = (2 * g.nodes + 255) / 256;
    hipLaunchKernelGGL((k_collide<S>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, g.nodes, cp, in, out);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::init_equilibrium(const Geometry &g, const CollisionParams &cp, const double *rho,
                                       const double *u, const double *T, S *state, hipStream_t st)
{
    hipLaunchKernelGGL((k_init_equilibrium<S>), dim3(node_grid(g.nodes)), dim3(256), 0, st, g.nodes, cp, rho, u,
                       T, state);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::moments(const Geometry &g, const CollisionParams &cp, const S *state, double *rho,
                              double *u, double *T, hipStream_t st)
{
    hipLaunchKernelGGL((k_moments<S>), dim3(node_grid(g.nodes)), dim3(256), 0, st, g.nodes, cp, state, rho, u,
                       T);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::totals(const Geometry &g, const CollisionParams &, const S *state, const double *nodew,
                             double *partials, int nblocks, double *out5, hipStream_t st)
{
    hipLaunchKernelGGL((k_totals_partial<S>), dim3(nblocks), dim3(256), 0, st, g, state, nodew, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reduce_partials<5>), dim3(1), dim3(256), 0, st, partials, nblocks, out5, 0);
    return hipGetLastError();
}

template struct Launch<double>;
template struct Launch<float>;

}  // namespace sllbm
