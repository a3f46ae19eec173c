// HIP kernels (gfx950) of the SLLBM hot path: semi-Lagrangian streaming
// (Eqs. (8)-(9)) fused with the local BGK + quasi-equilibrium collision
// (Eq. (5), App. A, B, D), plus FP64 moments, totals and the equilibrium
// initialisation.
//
// Streaming.  Psi_i = Iz (x) Iy (x) Ix is applied by sum factorisation.  A
// thread block owns a tile of whole cells; for every velocity it stages the
// tile's departure window of f_i and g_i in LDS (coalesced loads, x
// fastest), interpolates along z, then y, then x, and keeps the streamed
// value of its node in registers.  After all 45 velocities the node's 90
// pre-collision values are collided in registers and written once.
//
// Collision.  Moments, temperature, Sutherland viscosity, tau and tau_Pr are
// computed in double for both storage types.  The equilibrium uses the
// scalar form of the fourth-order Hermite series: with c = xi.u,
//   f_i^eq = w_i rho (A0 + c A1 + c^2 A2 + c^3/6 + c^4/24),
// where A0..A2 depend on |u|^2, T - 1 and |xi_i|^2 only (equal to the tensor
// contraction of Eq. (6) term by term).  The quasi-equilibrium term contracts
// the centred third moment of each population (10 unique components) with
// (w_i/3!) H^(3)_i; the centred third moment of the equilibrium is zero.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sllbm_internal.h"

namespace sllbm {

__constant__ double c_xi[Q][3];
__constant__ double c_w[Q];
__constant__ double c_x2[Q];
__constant__ double c_h3[Q][10];   // (w_i/6) * multiplicity * H3 component, unique (a<=b<=c) order

constexpr double SUTHERLAND_S = 0.40417;

int upload_velocity_constants(const VelocitySet &vs)
{
    double xi[Q][3], w[Q], x2[Q], h3[Q][10];
    static const int idx[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                                   {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
    static const double mult[10] = {1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
    for (int i = 0; i < Q; ++i) {
        const double *x = vs.xi[i];
        for (int k = 0; k < 3; ++k) xi[i][k] = x[k];
        w[i] = vs.w[i];
        x2[i] = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        for (int m = 0; m < 10; ++m) {
            int a = idx[m][0], b = idx[m][1], c = idx[m][2];
            double h = x[a] * x[b] * x[c] - ((b == c ? x[a] : 0.0) + (a == c ? x[b] : 0.0) + (a == b ? x[c] : 0.0));
            h3[i][m] = vs.w[i] / 6.0 * mult[m] * h;
        }
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_xi), xi, sizeof(xi)) != hipSuccess) return -1;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_w), w, sizeof(w)) != hipSuccess) return -1;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_x2), x2, sizeof(x2)) != hipSuccess) return -1;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_h3), h3, sizeof(h3)) != hipSuccess) return -1;
    return 0;
}

__device__ __forceinline__ int pmod(int x, int n)
{
    int r = x % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------
// Collision of one node, populations in registers (Eq. (5) + App. D)
// ---------------------------------------------------------------------------

struct NodeMacro {
    double rho, ux, uy, uz, T;
};

template <typename S>
__device__ __forceinline__ NodeMacro node_macro(const S (&f)[Q], const S (&g)[Q], double Cv)
{
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, K = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double fi = static_cast<double>(f[i]);
        rho += fi;
        jx = fma(fi, c_xi[i][0], jx);
        jy = fma(fi, c_xi[i][1], jy);
        jz = fma(fi, c_xi[i][2], jz);
        K = fma(fi, c_x2[i], K) + static_cast<double>(g[i]);
    }
    NodeMacro m;
    const double ir = 1.0 / rho;
    m.rho = rho;
    m.ux = jx * ir;
    m.uy = jy * ir;
    m.uz = jz * ir;
    const double u2 = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
    m.T = (K * ir - u2) / (2.0 * Cv);       // 2 rho E = rho |u|^2 + 2 C_v rho T
    return m;
}

__device__ __forceinline__ double viscosity(const CollisionParams &cp, double T)
{
    if (cp.law == SLLBM_CONSTANT) return cp.mu_inf;
    return cp.mu_inf * (1.0 + SUTHERLAND_S) * T * sqrt(T) / (T + SUTHERLAND_S);
}

// equilibrium bracket coefficients (D = 3), see file header
struct EqCoef {
    double a0, a1, a2;
};

__device__ __forceinline__ EqCoef eq_coef(double u2, double th, double x2)
{
    EqCoef e;
    e.a0 = 1.0 - 0.5 * u2 + 0.5 * th * (x2 - 3.0) + 0.125 * u2 * u2 - 0.25 * th * u2 * (x2 - 5.0) +
           0.125 * th * th * (x2 * x2 - 10.0 * x2 + 15.0);
    e.a1 = 1.0 - 0.5 * u2 + 0.5 * th * (x2 - 5.0);
    e.a2 = 0.5 - 0.25 * u2 + 0.25 * th * (x2 - 7.0);
    return e;
}

__device__ __forceinline__ double eq_bracket(const EqCoef &e, double c)
{
    return fma(c, fma(c, fma(c, fma(c, 1.0 / 24.0, 1.0 / 6.0), e.a2), e.a1), e.a0);
}

template <typename S>
__device__ __forceinline__ void collide_node(S (&f)[Q], S (&g)[Q], const CollisionParams &cp)
{
    const NodeMacro m = node_macro(f, g, cp.Cv);
    const double u2 = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
    const double P = m.rho * m.T;
    const double mu = viscosity(cp, m.T);
    const double tau = mu / (P * cp.dt) + 0.5;
    const double tau_pr = (tau - 0.5) * cp.inv_pr + 0.5;
    const double om = 1.0 / tau;
    const double kap = om - 1.0 / tau_pr;

    // centred third moments of f and g
    double qf[10], qg[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) qf[k] = qg[k] = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double dx = c_xi[i][0] - m.ux, dy = c_xi[i][1] - m.uy, dz = c_xi[i][2] - m.uz;
        const double dxx = dx * dx, dyy = dy * dy, dzz = dz * dz;
        const double mono[10] = {dxx * dx, dxx * dy, dxx * dz, dx * dyy, dx * dy * dz,
                                 dx * dzz, dyy * dy, dyy * dz, dy * dzz, dzz * dz};
        const double fi = static_cast<double>(f[i]), gi = static_cast<double>(g[i]);
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            qf[k] = fma(fi, mono[k], qf[k]);
            qg[k] = fma(gi, mono[k], qg[k]);
        }
    }

    const double th = m.T - 1.0;
    const double betaT = cp.beta * m.T;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double c = c_xi[i][0] * m.ux + c_xi[i][1] * m.uy + c_xi[i][2] * m.uz;
        const EqCoef e = eq_coef(u2, th, c_x2[i]);
        const double feq = c_w[i] * m.rho * eq_bracket(e, c);
        const double geq = betaT * feq;
        double fs = 0.0, gs = 0.0;
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            fs = fma(c_h3[i][k], qf[k], fs);
            gs = fma(c_h3[i][k], qg[k], gs);
        }
        const double fi = static_cast<double>(f[i]), gi = static_cast<double>(g[i]);
        f[i] = static_cast<S>(fi + om * (feq - fi) + kap * fs);
        g[i] = static_cast<S>(gi + om * (geq - gi) + kap * gs);
    }
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

template <typename S, bool COLLIDE>
__global__ void __launch_bounds__(256) k_stream_collide(Geometry geo, StreamTables tab, CollisionParams cp,
                                                        const S *__restrict__ in, S *__restrict__ out,
                                                        S *__restrict__ pre_out)
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
    if (pre_out != nullptr) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            pre_out[static_cast<int64_t>(i) * N + node] = fv[i];
            pre_out[static_cast<int64_t>(Q + i) * N + node] = gv[i];
        }
    }
    if constexpr (COLLIDE) collide_node<S>(fv, gv, cp);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        out[static_cast<int64_t>(i) * N + node] = fv[i];
        out[static_cast<int64_t>(Q + i) * N + node] = gv[i];
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_collide(int64_t N, CollisionParams cp, S *__restrict__ state)
{
    for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        S f[Q], g[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            f[i] = state[static_cast<int64_t>(i) * N + n];
            g[i] = state[static_cast<int64_t>(Q + i) * N + n];
        }
        collide_node<S>(f, g, cp);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            state[static_cast<int64_t>(i) * N + n] = f[i];
            state[static_cast<int64_t>(Q + i) * N + n] = g[i];
        }
    }
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
            const double c = c_xi[i][0] * ux + c_xi[i][1] * uy + c_xi[i][2] * uz;
            const double feq = c_w[i] * r * eq_bracket(eq_coef(u2, th, c_x2[i]), c);
            state[static_cast<int64_t>(i) * N + n] = static_cast<S>(feq);
            state[static_cast<int64_t>(Q + i) * N + n] = static_cast<S>(betaT * feq);
        }
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_moments(int64_t N, CollisionParams cp, const S *__restrict__ state,
                                                 double *__restrict__ rho, double *__restrict__ u,
                                                 double *__restrict__ T)
{
    for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        S f[Q], g[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            f[i] = state[static_cast<int64_t>(i) * N + n];
            g[i] = state[static_cast<int64_t>(Q + i) * N + n];
        }
        const NodeMacro m = node_macro(f, g, cp.Cv);
        if (rho) rho[n] = m.rho;
        if (u) {
            u[n] = m.ux;
            u[N + n] = m.uy;
            u[2 * N + n] = m.uz;
        }
        if (T) T[n] = m.T;
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
        double rho = 0, jx = 0, jy = 0, jz = 0, twoE = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double fi = static_cast<double>(state[static_cast<int64_t>(i) * N + n]);
            rho += fi;
            jx = fma(fi, c_xi[i][0], jx);
            jy = fma(fi, c_xi[i][1], jy);
            jz = fma(fi, c_xi[i][2], jz);
            twoE = fma(fi, c_x2[i], twoE) + static_cast<double>(state[static_cast<int64_t>(Q + i) * N + n]);
        }
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

// Stage 2: one block adds the per-block partials in block order.
template <int NV>
__global__ void k_reduce_partials(const double *__restrict__ partials, int nblocks, double *__restrict__ out,
                                  int accumulate)
{
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[b * NV + threadIdx.x];
        out[threadIdx.x] = accumulate ? out[threadIdx.x] + s : s;
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
hipError_t Launch<S>::stream_collide(const Geometry &g, const StreamTables &t, const CollisionParams &cp,
                                     const S *in, S *out, S *pre_out, hipStream_t st)
{
    const size_t smem = stream_smem_bytes(g, t, sizeof(S));
    hipError_t e = allow_smem(k_stream_collide<S, true>, smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stream_collide<S, true>), dim3(blocks_for(g)), dim3(stream_block(g)), smem, st, g, t,
                       cp, in, out, pre_out);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::stream_only(const Geometry &g, const StreamTables &t, const S *in, S *out,
                                  hipStream_t st)
{
    const size_t smem = stream_smem_bytes(g, t, sizeof(S));
    hipError_t e = allow_smem(k_stream_collide<S, false>, smem);
    if (e != hipSuccess) return e;
    CollisionParams cp{};
    hipLaunchKernelGGL((k_stream_collide<S, false>), dim3(blocks_for(g)), dim3(stream_block(g)), smem, st, g,
                       t, cp, in, out, static_cast<S *>(nullptr));
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::collide_only(const Geometry &g, const CollisionParams &cp, S *state, hipStream_t st)
{
    hipLaunchKernelGGL((k_collide<S>), dim3(node_grid(g.nodes)), dim3(256), 0, st, g.nodes, cp, state);
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
    hipLaunchKernelGGL((k_reduce_partials<5>), dim3(1), dim3(64), 0, st, partials, nblocks, out5, 0);
    return hipGetLastError();
}

template struct Launch<double>;
template struct Launch<float>;

}  // namespace sllbm
