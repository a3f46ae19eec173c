// Reverse mode of the SLLBM step (kernels and launchers).
//
// One step maps the pre-collision state X_n to X_{n+1} = S(C(X_n)), with C
// the node-local collision (Eq. (5) with App. D) and S the semi-Lagrangian
// streaming (Eq. (9)), which is linear.  Its vector-Jacobian product is
//   lambda_n = J_C(X_n)^T S^T lambda_{n+1}.
// S^T is the transposed streaming (stream.hip, stream_graded.hip); this file
// holds the collision VJP, the VJP of the equilibrium initialisation, and the
// flow functional used for gradients with its derivative.  All reverse arithmetic is in double; states are stored in the
// context's storage type.
//
// Collision VJP (per node, f on the even lane of a pair, g on the odd lane).
// With adjoints alpha_i of the post-collision values of the lane's population
// (alpha = a for f, b for g) and the forward quantities recomputed from X_n:
//   h'_i = h_i + omega (s h^eq_i - h_i) + kappa h*_i,  s = 1 (f), beta T (g),
//   omega = 1/tau, kappa = 1/tau - 1/tau_Pr,
// the reverse sweep accumulates, per lane, the scalars
//   sum alpha (s h^eq - h)            -> d omega
//   sum alpha h*                      -> d kappa
//   sum alpha s h^eq omega / rho      -> d rho
//   equilibrium terms in c = xi.u, |u|^2 and theta = T - 1 -> d u, d T
//   Abar_m = kappa sum_i alpha_i H3c_im  (adjoint of Qbar) -> d h, d u
// adds them over the pair, pushes them through tau(mu(T), P = rho T),
// T = (K/rho - |u|^2)/(2 C_v) and u = J/rho, and forms per velocity
//   lambda_f,k = (1 - omega) a_k + rho_bar + J_bar . xi_k + K_bar |xi_k|^2 + Abar_f : d_k^3
//   lambda_g,k = (1 - omega) b_k + K_bar + Abar_g : d_k^3,   d_k = xi_k - u.
// The node's contribution to dL/dmu_inf is mu_bar * (mu / mu_inf).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "collision.h"
#include "nt.h"
#include "sllbm_internal.h"
#include "velset.h"

namespace sllbm {

namespace {

template <int XM>
__device__ __forceinline__ double pair_sum(double v) { return v + __shfl_xor(v, XM); }

__device__ __forceinline__ double viscosity_factor(const CollisionParams &cp, double T, double &dfac_dT)
{
    if (cp.law == SLLBM_CONSTANT) {
        dfac_dT = 0.0;
        return 1.0;
    }
    // (1 + S) T^1.5 / (T + S)
    const double sq = sqrt(T);
    const double den = T + SUTHERLAND_S;
    const double fac = (1.0 + SUTHERLAND_S) * T * sq / den;
    dfac_dT = (1.0 + SUTHERLAND_S) * (1.5 * sq / den - T * sq / (den * den));
    return fac;
}

// bracket b(c) = a0 + a1 c + a2 c^2 + c^3/6 + c^4/24 and its derivatives in
// |u|^2 and theta; d a1/d|u|^2 = -1/2, d a2/d|u|^2 = -1/4, d a1/d theta =
// (x2 - 5)/2 and d a2/d theta = (x2 - 7)/4 are constants of the shell
struct Bracket {
    double a0, a1, a2;           // value coefficients
    double d0u;                  // d a0 / d |u|^2
    double d0t;                  // d a0 / d theta
};

__device__ __forceinline__ Bracket bracket(double u2, double th, double x2)
{
    Bracket b;
    const EqShell e = eq_shell<3>(u2, th, x2);
    b.a0 = e.a0;
    b.a1 = e.a1;
    b.a2 = e.a2;
    b.d0u = -0.5 + 0.25 * u2 - 0.25 * th * (x2 - 5.0);
    b.d0t = 0.5 * (x2 - 3.0) - 0.25 * u2 * (x2 - 5.0) + 0.25 * th * (x2 * x2 - 10.0 * x2 + 15.0);
    return b;
}

constexpr double D1U = -0.5, D2U = -0.25;
__host__ __device__ constexpr double d1t_of(double x2) { return 0.5 * (x2 - 5.0); }
__host__ __device__ constexpr double d2t_of(double x2) { return 0.25 * (x2 - 7.0); }

__device__ __forceinline__ double bval(const Bracket &b, double c)
{
    return fma(c, fma(c, fma(c, fma(c, 1.0 / 24.0, 1.0 / 6.0), b.a2), b.a1), b.a0);
}

__device__ __forceinline__ double bder(const Bracket &b, double c)    // d b / d c
{
    return fma(c, fma(c, fma(c, 1.0 / 6.0, 0.5), 2.0 * b.a2), b.a1);
}

}  // namespace

// ---------------------------------------------------------------------------
// Collision VJP: lam = J_C(X)^T mu, two lanes per node.  dmu_part[block]
// receives the block's sum of dL/dmu_inf.
// ---------------------------------------------------------------------------
// One lane of the collision VJP (its node's population is_g): X of the node
// from X + off (stride N), the lane's adjoint inputs alpha_i from AL(i), the
// partner lane l ^ XM; writes lambda of its population at lp (stride N) and
// returns the node's dL/dmu_inf (counted on the f lane).  Inactive lanes (a
// node past the end) compute on node 0 for their partner and write nothing.
template <typename S, bool NTH, int XM, class Alpha>
__device__ __forceinline__ double collide_vjp_lane(int64_t N, const CollisionParams &cp, const S *__restrict__ X,
                                                   int64_t off, bool is_g, bool active, Alpha &&AL, S *lp)
{
    // X enters only through its raw moments and sum alpha h, so it is dead
    // before the sweep
    RawMoments<D3Q45> rm;
    double dot_ah = 0.0;
    {
        double h[vs::Q];
#pragma unroll
        for (int i = 0; i < vs::Q; ++i) {
            h[i] = static_cast<double>(load_hint<NTH>(&X[off + static_cast<int64_t>(i) * N]));
        }
        rm = raw_moments<D3Q45>(h);
#pragma unroll
        for (int i = 0; i < vs::Q; ++i) dot_ah = fma(AL(i), h[i], dot_ah);
    }

    // ---- forward quantities (as in collide_half) ----
    const double ktr = rm.m2[0] + rm.m2[3] + rm.m2[5];
    const double p_m0 = __shfl_xor(rm.m0, XM);
    const double p_j0 = __shfl_xor(rm.m1[0], XM), p_j1 = __shfl_xor(rm.m1[1], XM), p_j2 = __shfl_xor(rm.m1[2], XM);
    const double p_tr = __shfl_xor(ktr, XM);
    const double rho = is_g ? p_m0 : rm.m0;
    const double J[3] = {is_g ? p_j0 : rm.m1[0], is_g ? p_j1 : rm.m1[1], is_g ? p_j2 : rm.m1[2]};
    const double ir = 1.0 / rho;
    const double u[3] = {J[0] * ir, J[1] * ir, J[2] * ir};
    const double K = is_g ? p_tr + rm.m0 : ktr + p_m0;
    const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double Cv = cp.Cv;
    const double T = (K * ir - u2) / (2.0 * Cv);
    double qb[10];
    centred_third<D3Q45>(rm, u, qb);
    const double P = rho * T;
    double dfac;
    const double fac = viscosity_factor(cp, T, dfac);
    const double mu_v = cp.mu_inf * fac;
    const double tau = mu_v / (P * cp.dt) + 0.5;
    const double tau_pr = (tau - 0.5) * cp.inv_pr + 0.5;
    const double om = 1.0 / tau;
    const double kap = 1.0 / tau - 1.0 / tau_pr;
    const double th = T - 1.0;
    const double eqs = is_g ? cp.beta * T : 1.0;

    // centred second moment of the own population (for the Qbar -> u term);
    // the raw moments are dead after this
    double C2[6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b)
            C2[sym2(a, b)] = rm.m2[sym2(a, b)] - u[a] * rm.m1[b] - u[b] * rm.m1[a] + rm.m0 * u[a] * u[b];

    Bracket br[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) br[s] = bracket(u2, th, vs::SHELL_X2[s]);

    // ---- reverse sweep over the velocities (own population) ----
    double s_ka = 0, s_heq = 0, s_eqT = 0, s_u2 = 0, s_th = 0;
    double ubar[3] = {0, 0, 0};
    double abar[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) abar[m] = 0.0;
    {   // rest velocity: c = 0, h* = 0
        const double w = vs::T.w[0];
        const double feq = w * rho * br[0].a0;
        const double heq = eqs * feq;
        s_heq = fma(AL(0), heq, s_heq);
        s_eqT = fma(AL(0), feq, s_eqT);
        s_u2 = fma(AL(0) * w * rho * eqs, br[0].d0u, s_u2);
        s_th = fma(AL(0) * w * rho * eqs, br[0].d0t, s_th);
    }
#pragma unroll
    for (int q = 0; q < 22; ++q) {
        const int i = vs::PAIRS.a[q], j = vs::PAIRS.b[q];
        const Bracket &b = br[vs::T.shell[i]];
        const double w = vs::T.w[i];
        const double c = fma_nz(vs::T.xi[i][2], u[2],
                                fma_nz(vs::T.xi[i][1], u[1], vs::T.xi[i][0] == 0.0 ? 0.0 : vs::T.xi[i][0] * u[0]));
        const double feq_i = w * rho * bval(b, c), feq_j = w * rho * bval(b, -c);
        const double heq_i = eqs * feq_i, heq_j = eqs * feq_j;
        double hs = 0.0;
#pragma unroll
        for (int m = 0; m < 10; ++m) hs = fma_nz(vs::H3.c[i][m], qb[m], hs);
        const double ai = AL(i), aj = AL(j);
        s_ka += (ai - aj) * hs;
        s_heq += ai * heq_i + aj * heq_j;
        s_eqT += ai * feq_i + aj * feq_j;
        const double wre = w * rho * eqs;
        const double gu = wre * (ai * bder(b, c) - aj * bder(b, -c));      // d/du through c
        ubar[0] = fma_nz(vs::T.xi[i][0], gu, ubar[0]);
        ubar[1] = fma_nz(vs::T.xi[i][1], gu, ubar[1]);
        ubar[2] = fma_nz(vs::T.xi[i][2], gu, ubar[2]);
        const double sp = ai + aj, sm = ai - aj;
        const double x2 = vs::SHELL_X2[vs::T.shell[i]];
        s_u2 += wre * (sp * (b.d0u + c * c * D2U) + sm * c * D1U);
        s_th += wre * (sp * (b.d0t + c * c * d2t_of(x2)) + sm * c * d1t_of(x2));
#pragma unroll
        for (int m = 0; m < 10; ++m) abar[m] = fma_nz(vs::H3.c[i][m], sm, abar[m]);
    }
#pragma unroll
    for (int m = 0; m < 10; ++m) abar[m] *= kap;

    // Qbar -> u: -sum_m abar_m (delta_ad C2_bc + delta_bd C2_ac + delta_cd C2_ab)
    double uq[3] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < 10; ++m) {
        const int a = vs::IDX3[m][0], b = vs::IDX3[m][1], c = vs::IDX3[m][2];
        uq[a] -= abar[m] * C2[sym2(b, c)];
        uq[b] -= abar[m] * C2[sym2(a, c)];
        uq[c] -= abar[m] * C2[sym2(a, b)];
    }

    // ---- pair totals (sum alpha (s h^eq - h) = s_heq - dot_ah) ----
    const double S_om = pair_sum<XM>(s_heq - dot_ah), S_ka = pair_sum<XM>(s_ka);
    const double S_heq = pair_sum<XM>(om * s_heq);
    const double S_eqT = pair_sum<XM>(is_g ? om * cp.beta * s_eqT : 0.0);
    const double S_u2 = pair_sum<XM>(om * s_u2), S_th = pair_sum<XM>(om * s_th);
    double U[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) U[a] = pair_sum<XM>(om * ubar[a] + uq[a]);

    // omega = 1/tau, kappa = 1/tau - 1/tau_pr
    const double om_bar = S_om + S_ka;
    const double ompr_bar = -S_ka;
    const double tau_bar = -om_bar / (tau * tau) - ompr_bar / (tau_pr * tau_pr) * cp.inv_pr;
    const double mu_bar = tau_bar / (P * cp.dt);
    const double P_bar = -tau_bar * mu_v / (P * P * cp.dt);
    double T_bar = mu_bar * cp.mu_inf * dfac + P_bar * rho + S_th + S_eqT;
    double rho_bar = P_bar * T + S_heq * ir;
    double ub[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) ub[a] = U[a] + 2.0 * u[a] * S_u2;
    // T = (K/rho - |u|^2) / (2 C_v)
    const double K_bar = T_bar / (2.0 * Cv * rho);
    rho_bar -= T_bar * K * ir * ir / (2.0 * Cv);
#pragma unroll
    for (int a = 0; a < 3; ++a) ub[a] -= T_bar * u[a] / Cv;
    // u = J / rho
    double J_bar[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) J_bar[a] = ub[a] * ir;
    rho_bar -= (ub[0] * u[0] + ub[1] * u[1] + ub[2] * u[2]) * ir;

    // ---- per-velocity outputs ----
    // Abar : (xi - u)^3 = T3 - T2 + T1 - T0 and Abar : (-xi - u)^3 = -(T3 + T2 + T1 + T0)
    // with T3 = Abar : xi xi xi, T2 = Bs : xi xi, T1 = Cv . xi, T0 = Abar : u u u,
    // where Bs and Cv collect Abar with one and two of its indices contracted with u
    if (active) {
        double Bs[6] = {0, 0, 0, 0, 0, 0}, Cu[3] = {0, 0, 0}, T0 = 0.0;
#pragma unroll
        for (int m = 0; m < 10; ++m) {
            const int a = vs::IDX3[m][0], b = vs::IDX3[m][1], c = vs::IDX3[m][2];
            Bs[sym2(b, c)] = fma(abar[m], u[a], Bs[sym2(b, c)]);
            Bs[sym2(a, c)] = fma(abar[m], u[b], Bs[sym2(a, c)]);
            Bs[sym2(a, b)] = fma(abar[m], u[c], Bs[sym2(a, b)]);
            Cu[a] = fma(abar[m], u[b] * u[c], Cu[a]);
            Cu[b] = fma(abar[m], u[a] * u[c], Cu[b]);
            Cu[c] = fma(abar[m], u[a] * u[b], Cu[c]);
            T0 = fma(abar[m], u[a] * u[b] * u[c], T0);
        }
        asm volatile("" : "+v"(lp));      // fresh store addresses (the load addresses are not kept live)
        const double one_m = 1.0 - om;
        const double base_f = rho_bar, x2g = is_g ? 0.0 : 1.0, kg = is_g ? K_bar : 0.0;
        {   // rest velocity: xi = 0
            double r = one_m * AL(0) - T0 + kg;
            if (!is_g) r += base_f;
            store_hint<NTH>(&lp[0], static_cast<S>(r));
        }
#pragma unroll
        for (int q = 0; q < 22; ++q) {
            const int i = vs::PAIRS.a[q], j = vs::PAIRS.b[q];
            const double x = vs::T.xi[i][0], y = vs::T.xi[i][1], z = vs::T.xi[i][2];
            double T3 = 0.0;
#pragma unroll
            for (int m = 0; m < 10; ++m) T3 = fma_nz(vs::H3.mono[i][m], abar[m], T3);
            const double T2 = Bs[0] * (x * x) + Bs[1] * (x * y) + Bs[2] * (x * z) + Bs[3] * (y * y) +
                              Bs[4] * (y * z) + Bs[5] * (z * z);
            const double T1 = Cu[0] * x + Cu[1] * y + Cu[2] * z;
            const double jx = is_g ? 0.0 : J_bar[0] * x + J_bar[1] * y + J_bar[2] * z;
            const double common = kg + x2g * (base_f + K_bar * vs::T.x2[i]);
            const double ri = one_m * AL(i) + common + jx + (T3 - T2 + T1 - T0);
            const double rj = one_m * AL(j) + common - jx - (T3 + T2 + T1 + T0);
            store_hint<NTH>(&lp[static_cast<int64_t>(i) * N], static_cast<S>(ri));
            store_hint<NTH>(&lp[static_cast<int64_t>(j) * N], static_cast<S>(rj));
        }
    }

    // ---- dL/dmu_inf: mu = mu_inf * fac, counted once per node (f lane) ----
    return active && !is_g ? mu_bar * fac : 0.0;
}

// Grid-stride over lane pairs; the whole block runs the same number of
// iterations, so every shuffle partner is live.  mu and lam may be the same
// buffer: each lane reads its 45 values before writing them.
// NTH: non-temporal loads and stores (states larger than the Infinity Cache)
template <typename S, bool NTH>
__global__ void __launch_bounds__(256) k_collide_vjp(int64_t N, CollisionParams cp, const S *__restrict__ X,
                                                     const S *mu, S *lam, double *__restrict__ dmu_part)
{
    __shared__ double red[256];
    double dmu_acc = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t0 = blockIdx.x * static_cast<int64_t>(blockDim.x); t0 < 2 * N; t0 += stride) {
        const int64_t t = t0 + threadIdx.x;
        const int64_t n = t >> 1;
        const int pop = static_cast<int>(t & 1);
        const bool active = n < N;
        const int64_t off = static_cast<int64_t>(pop) * vs::Q * N + (active ? n : 0);
        double al[vs::Q];
#pragma unroll
        for (int i = 0; i < vs::Q; ++i) al[i] = static_cast<double>(load_hint<NTH>(&mu[off + static_cast<int64_t>(i) * N]));
        dmu_acc += collide_vjp_lane<S, NTH, 1>(N, cp, X, off, pop != 0, active, [&](int i) { return al[i]; },
                                               lam + off);
    }
    red[threadIdx.x] = dmu_acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) dmu_part[blockIdx.x] = red[0];
}

// DMA copy of 16 bytes per lane from g into LDS at l + 16 * lane (l is
// wave-uniform; AUX 2: non-temporal).  Untyped, in a device function of its
// own: the 16-byte form exists on gfx950 only.
template <int AUX>
__device__ __forceinline__ void dma16_adj(const void *g, void *l)
{
    __builtin_amdgcn_global_load_lds(g, l, 16, 0, AUX);
}

// The collision VJP in FP32 storage with the adjoint inputs alpha staged in
// LDS: per iteration a block takes 128 consecutive nodes, copies their 90
// rows of mu (row r = pop * 45 + i, 512 contiguous bytes) into LDS by 16-byte
// DMA copies, and each lane reads its alpha_i from there (lane l of wave w:
// node w * 32 + (l & 31), population l >> 5, partner l ^ 32).  256 VGPRs
// and 38 spilled at two waves per SIMD, against 330 registers and one wave
// for k_collide_vjp.  N % 4 == 0 and mu 16-byte aligned; mu and lam may be
// the same buffer (every copy of an iteration lands before its writes, and
// the next iteration's copies wait for all its reads).
template <bool NTH>
__global__ void __launch_bounds__(256, 2) k_collide_vjp_lds(int64_t N, CollisionParams cp,
                                                            const float *__restrict__ X, const float *mu, float *lam,
                                                            double *__restrict__ dmu_part)
{
    constexpr int NB = 128, ROWS = 2 * vs::Q;
    __shared__ float tile[ROWS][NB];
    __shared__ double red[256];
    double dmu_acc = 0.0;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pop = lane >> 5;
    const int c = w * 32 + (lane & 31);
    for (int64_t nb = static_cast<int64_t>(blockIdx.x) * NB; nb < N; nb += static_cast<int64_t>(gridDim.x) * NB) {
        __syncthreads();                         // the previous nodes' reads of the tile are done
        const int64_t col = nb + 4 * (lane & 31);
        if (col < N) {
            const float *src = mu + static_cast<int64_t>(lane >> 5) * N + col;
            for (int m = w; m < ROWS / 2; m += 4)
                dma16_adj<NTH ? 2 : 0>(src + static_cast<int64_t>(2 * m) * N, &tile[2 * m][0]);
        }
        __builtin_amdgcn_s_waitcnt(0);           // this wave's copies have landed
        __syncthreads();                         // and every other wave's
        const int64_t n = nb + c;
        const bool active = n < N;
        const int64_t off = static_cast<int64_t>(pop) * vs::Q * N + (active ? n : 0);
        const float *sl = &tile[pop * vs::Q][c];
        dmu_acc += collide_vjp_lane<float, NTH, 32>(N, cp, X, off, pop != 0, active,
                                                    [&](int i) { return static_cast<double>(sl[i * NB]); }, lam + off);
    }
    red[threadIdx.x] = dmu_acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) dmu_part[blockIdx.x] = red[0];
}

// Fixed-order sum of n block partials by one block of 256 threads; the
// result is added to *acc (add != 0) or stored there.  Deterministic.
__global__ void __launch_bounds__(256) k_accumulate(const double *__restrict__ part, int n, double *__restrict__ acc,
                                                    int add)
{
    __shared__ double red[256];
    // eight interleaved running sums per thread (eight loads in flight), combined in a fixed order
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int b = threadIdx.x;
    for (; b + 7 * 256 < n; b += 8 * 256) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] += part[b + k * 256];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (b + k * 256 < n) a[k] += part[b + k * 256];
    const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *acc = add ? *acc + red[0] : red[0];
}

// ---------------------------------------------------------------------------
// VJP of the equilibrium initialisation: fields -> (f^eq, g^eq)
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) k_init_vjp(int64_t N, CollisionParams cp, const double *__restrict__ rho,
                                                  const double *__restrict__ u, const double *__restrict__ T,
                                                  const S *__restrict__ lam, double *__restrict__ drho,
                                                  double *__restrict__ du, double *__restrict__ dT)
{
    const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (n >= N) return;
    const double r = rho[n], uu[3] = {u[n], u[N + n], u[2 * N + n]}, Tn = T[n];
    const double u2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
    const double th = Tn - 1.0;
    const double bT = cp.beta * Tn;
    double gr = 0, gu[3] = {0, 0, 0}, gu2 = 0, gt = 0;
#pragma unroll
    for (int i = 0; i < vs::Q; ++i) {
        const double a = static_cast<double>(lam[static_cast<int64_t>(i) * N + n]);
        const double b = static_cast<double>(lam[static_cast<int64_t>(vs::Q + i) * N + n]);
        const Bracket br = bracket(u2, th, vs::T.x2[i]);
        const double c = vs::T.xi[i][0] * uu[0] + vs::T.xi[i][1] * uu[1] + vs::T.xi[i][2] * uu[2];
        const double w = vs::T.w[i];
        const double e = a + bT * b;                       // adjoint of f^eq_i (through f and g)
        const double bv = bval(br, c);
        gr += e * w * bv;
        const double gc = e * w * r * bder(br, c);
        gu[0] = fma(gc, vs::T.xi[i][0], gu[0]);
        gu[1] = fma(gc, vs::T.xi[i][1], gu[1]);
        gu[2] = fma(gc, vs::T.xi[i][2], gu[2]);
        const double x2 = vs::T.x2[i];
        gu2 += e * w * r * (br.d0u + c * D1U + c * c * D2U);
        gt += e * w * r * (br.d0t + c * d1t_of(x2) + c * c * d2t_of(x2)) + b * cp.beta * w * r * bv;
    }
    if (drho) drho[n] = gr;
    if (du) {
        du[n] = gu[0] + 2.0 * uu[0] * gu2;
        du[N + n] = gu[1] + 2.0 * uu[1] * gu2;
        du[2 * N + n] = gu[2] + 2.0 * uu[2] * gu2;
    }
    if (dT) dT[n] = gt;
}

// ---------------------------------------------------------------------------
// VJP of the moments (Eq. (7) with 2 rho E = rho |u|^2 + 2 C_v rho T): given
// adjoints of rho, u, T at every node, lam = d(rho, u, T)/d(state)^T (...).
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) k_moments_vjp(int64_t N, CollisionParams cp, const S *__restrict__ st,
                                                     const double *__restrict__ drho, const double *__restrict__ du,
                                                     const double *__restrict__ dT, S *__restrict__ lam)
{
    const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (n >= N) return;
    double r = 0, j[3] = {0, 0, 0}, K = 0;
#pragma unroll
    for (int i = 0; i < vs::Q; ++i) {
        const double f = static_cast<double>(st[static_cast<int64_t>(i) * N + n]);
        const double g = static_cast<double>(st[static_cast<int64_t>(vs::Q + i) * N + n]);
        r += f;
        j[0] = fma(f, vs::T.xi[i][0], j[0]);
        j[1] = fma(f, vs::T.xi[i][1], j[1]);
        j[2] = fma(f, vs::T.xi[i][2], j[2]);
        K += fma(f, vs::T.x2[i], g);
    }
    const double ir = 1.0 / r;
    const double u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
    const double Tb = dT ? dT[n] : 0.0;
    double rb = drho ? drho[n] : 0.0;
    double ub[3] = {du ? du[n] : 0.0, du ? du[N + n] : 0.0, du ? du[2 * N + n] : 0.0};
    // T = (K/rho - |u|^2) / (2 C_v)
    const double Kb = Tb / (2.0 * cp.Cv * r);
    rb -= Tb * K * ir * ir / (2.0 * cp.Cv);
#pragma unroll
    for (int a = 0; a < 3; ++a) ub[a] -= Tb * u[a] / cp.Cv;
    // u = J / rho
    rb -= (ub[0] * u[0] + ub[1] * u[1] + ub[2] * u[2]) * ir;
    const double Jb[3] = {ub[0] * ir, ub[1] * ir, ub[2] * ir};
#pragma unroll
    for (int i = 0; i < vs::Q; ++i) {
        lam[static_cast<int64_t>(i) * N + n] = static_cast<S>(rb + Jb[0] * vs::T.xi[i][0] + Jb[1] * vs::T.xi[i][1] +
                                                              Jb[2] * vs::T.xi[i][2] + Kb * vs::T.x2[i]);
        lam[static_cast<int64_t>(vs::Q + i) * N + n] = static_cast<S>(Kb);
    }
}

// ---------------------------------------------------------------------------
// Flow functional L = sum over cells of the tensor Clenshaw-Curtis quadrature
// of (1/2) rho |u|^2 + (div u)^2, div u from each cell's own polynomial.
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) k_rho_u(int64_t N, const S *__restrict__ st, double *__restrict__ rho,
                                               double *__restrict__ u)
{
    const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (n >= N) return;
    double r = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < vs::Q; ++i) {
        const double f = static_cast<double>(st[static_cast<int64_t>(i) * N + n]);
        r += f;
        j[0] = fma(f, vs::T.xi[i][0], j[0]);
        j[1] = fma(f, vs::T.xi[i][1], j[1]);
        j[2] = fma(f, vs::T.xi[i][2], j[2]);
    }
    rho[n] = r;
    u[n] = j[0] / r;
    u[N + n] = j[1] / r;
    u[2 * N + n] = j[2] / r;
}

struct CellGeo {
    int N[3], nel[3], p;
    int64_t nodes;
    double h[3];                 // cell width per axis (equal cells)
    const double *hw;            // graded mesh: widths of the x, then y, then z cells (NULL: equal cells)
    const double *jac;           // distorted mesh: per cell point J^-1 (row-major) and |det J| (NULL: J = I)
    const double *full_w;        // distorted mesh: per-node quadrature weights (NULL: separable weights)
};

// width of cell e along axis a
__device__ __forceinline__ double cell_h(const CellGeo &g, int a, int e)
{
    if (!g.hw) return g.h[a];
    const int off = a == 0 ? 0 : (a == 1 ? g.nel[0] : g.nel[0] + g.nel[1]);
    return g.hw[off + e];
}

__device__ __forceinline__ int64_t node_of(const CellGeo &g, int gx, int gy, int gz)
{
    gx %= g.N[0];
    gy %= g.N[1];
    gz %= g.N[2];
    return (static_cast<int64_t>(gz) * g.N[1] + gy) * g.N[0] + gx;
}

// per cell point: partial loss; sdiv[c] = 2 W_c div_c (for the gradient)
__global__ void __launch_bounds__(256) k_loss_cells(CellGeo g, const double *__restrict__ dmat,
                                                    const double *__restrict__ ccw, const double *__restrict__ rho,
                                                    const double *__restrict__ u, double *__restrict__ sdiv,
                                                    double *__restrict__ part)
{
    __shared__ double red[256];
    const int p = g.p, p1 = p + 1;
    const int64_t ncp = static_cast<int64_t>(g.nel[0]) * g.nel[1] * g.nel[2] * p1 * p1 * p1;
    double acc = 0.0;
    for (int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; c < ncp;
         c += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int64_t r = c;
        const int kx = static_cast<int>(r % p1); r /= p1;
        const int ky = static_cast<int>(r % p1); r /= p1;
        const int kz = static_cast<int>(r % p1); r /= p1;
        const int ex = static_cast<int>(r % g.nel[0]); r /= g.nel[0];
        const int ey = static_cast<int>(r % g.nel[1]);
        const int ez = static_cast<int>(r / g.nel[1]);
        const int gx = ex * p + kx, gy = ey * p + ky, gz = ez * p + kz;
        const double hx = cell_h(g, 0, ex), hy = cell_h(g, 1, ey), hz = cell_h(g, 2, ez);
        double div = 0.0;
        double W = (0.5 * hx * ccw[kx]) * (0.5 * hy * ccw[ky]) * (0.5 * hz * ccw[kz]);
        if (!g.jac) {
            for (int m = 0; m <= p; ++m) {
                div += dmat[kx * p1 + m] * u[node_of(g, ex * p + m, gy, gz)] / hx;
                div += dmat[ky * p1 + m] * u[g.nodes + node_of(g, gx, ey * p + m, gz)] / hy;
                div += dmat[kz * p1 + m] * u[2 * g.nodes + node_of(g, gx, gy, ez * p + m)] / hz;
            }
        } else {
            // distorted cell: div u = sum_ab (d u_a / d r_b) (J^-1)_ba
            double gr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int m = 0; m <= p; ++m) {
                const int64_t nx = node_of(g, ex * p + m, gy, gz), ny = node_of(g, gx, ey * p + m, gz),
                              nz = node_of(g, gx, gy, ez * p + m);
                const double dx = dmat[kx * p1 + m] / hx, dy = dmat[ky * p1 + m] / hy, dz = dmat[kz * p1 + m] / hz;
                for (int a = 0; a < 3; ++a) {
                    gr[a][0] = fma(dx, u[a * g.nodes + nx], gr[a][0]);
                    gr[a][1] = fma(dy, u[a * g.nodes + ny], gr[a][1]);
                    gr[a][2] = fma(dz, u[a * g.nodes + nz], gr[a][2]);
                }
            }
            const double *Ji = g.jac + c * 10;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) div = fma(gr[a][b], Ji[b * 3 + a], div);
            W *= Ji[9];
        }
        const int64_t n = node_of(g, gx, gy, gz);
        const double ux = u[n], uy = u[g.nodes + n], uz = u[2 * g.nodes + n];
        acc += W * (0.5 * rho[n] * (ux * ux + uy * uy + uz * uz) + div * div);
        if (sdiv) sdiv[c] = 2.0 * W * div;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// TGV diagnostics (Sec. III C) per cell point: (1/2) rho |u|^2, mu(T) |curl u|^2
// and (4/3) mu(T) (div u)^2, derivatives from the cell's own polynomial,
// weighted by the tensor Clenshaw-Curtis rule; per-block partial sums.
__global__ void __launch_bounds__(256) k_diag_cells(CellGeo g, CollisionParams cp, const double *__restrict__ dmat,
                                                    const double *__restrict__ ccw, const double *__restrict__ rho,
                                                    const double *__restrict__ u, const double *__restrict__ T,
                                                    double *__restrict__ part)
{
    __shared__ double red[3][256];
    const int p = g.p, p1 = p + 1;
    const int64_t ncp = static_cast<int64_t>(g.nel[0]) * g.nel[1] * g.nel[2] * p1 * p1 * p1;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; c < ncp;
         c += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int64_t r = c;
        int k[3], e[3];
        k[0] = static_cast<int>(r % p1); r /= p1;
        k[1] = static_cast<int>(r % p1); r /= p1;
        k[2] = static_cast<int>(r % p1); r /= p1;
        e[0] = static_cast<int>(r % g.nel[0]); r /= g.nel[0];
        e[1] = static_cast<int>(r % g.nel[1]);
        e[2] = static_cast<int>(r / g.nel[1]);
        const int gx = e[0] * p + k[0], gy = e[1] * p + k[1], gz = e[2] * p + k[2];
        const double hx = cell_h(g, 0, e[0]), hy = cell_h(g, 1, e[1]), hz = cell_h(g, 2, e[2]);
        double grad[3][3];                       // grad[a][b] = d u_a / d x_b
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) grad[a][b] = 0.0;
        for (int m = 0; m <= p; ++m) {
            const int64_t nx = node_of(g, e[0] * p + m, gy, gz);
            const int64_t ny = node_of(g, gx, e[1] * p + m, gz);
            const int64_t nz = node_of(g, gx, gy, e[2] * p + m);
            const double dx = dmat[k[0] * p1 + m] / hx, dy = dmat[k[1] * p1 + m] / hy,
                         dz = dmat[k[2] * p1 + m] / hz;
            for (int a = 0; a < 3; ++a) {
                grad[a][0] = fma(dx, u[a * g.nodes + nx], grad[a][0]);
                grad[a][1] = fma(dy, u[a * g.nodes + ny], grad[a][1]);
                grad[a][2] = fma(dz, u[a * g.nodes + nz], grad[a][2]);
            }
        }
        double W = (0.5 * hx * ccw[k[0]]) * (0.5 * hy * ccw[k[1]]) * (0.5 * hz * ccw[k[2]]);
        if (g.jac) {
            // distorted cell: physical gradient (d u / d r) J^-1, weight times |det J|
            const double *Ji = g.jac + c * 10;
            double gp[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    gp[a][b] = grad[a][0] * Ji[b] + grad[a][1] * Ji[3 + b] + grad[a][2] * Ji[6 + b];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) grad[a][b] = gp[a][b];
            W *= Ji[9];
        }
        const int64_t n = node_of(g, gx, gy, gz);
        const double w0 = grad[2][1] - grad[1][2], w1 = grad[0][2] - grad[2][0], w2 = grad[1][0] - grad[0][1];
        const double div = grad[0][0] + grad[1][1] + grad[2][2];
        const double ux = u[n], uy = u[g.nodes + n], uz = u[2 * g.nodes + n];
        const double mu = viscosity_of(cp, T[n]);
        acc[0] = fma(W, 0.5 * rho[n] * (ux * ux + uy * uy + uz * uz), acc[0]);
        acc[1] = fma(W, mu * (w0 * w0 + w1 * w1 + w2 * w2), acc[1]);
        acc[2] = fma(W, (4.0 / 3.0) * mu * div * div, acc[2]);
    }
    for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) part[blockIdx.x * 3 + q] = red[q][0];
}

// Fixed-order sum of n partial triples by one block (deterministic).
__global__ void __launch_bounds__(256) k_sum3(const double *__restrict__ part, int n, double *__restrict__ out)
{
    __shared__ double red[3][256];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < n; b += 256)
        for (int q = 0; q < 3; ++q) acc[q] += part[b * 3 + q];
    for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) out[q] = red[q][0];
}

// dL/d(state) at every node: dL/drho and dL/du gathered from the cell points
// whose value or derivative stencil contains the node, then chained through
// rho = sum f and u = sum f xi / rho (g does not enter L).
template <typename S>
__global__ void __launch_bounds__(256) k_loss_grad(CellGeo g, const double *__restrict__ dmat,
                                                   const double *__restrict__ nodew, const double *__restrict__ rho,
                                                   const double *__restrict__ u, const double *__restrict__ sdiv,
                                                   S *__restrict__ lam)
{
    const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (n >= g.nodes) return;
    const int p = g.p, p1 = p + 1;
    const int gi[3] = {static_cast<int>(n % g.N[0]), static_cast<int>((n / g.N[0]) % g.N[1]),
                       static_cast<int>(n / (static_cast<int64_t>(g.N[0]) * g.N[1]))};
    const double W = g.full_w ? g.full_w[n] : nodew[gi[0]] * nodew[g.N[0] + gi[1]] * nodew[g.N[0] + g.N[1] + gi[2]];
    const double r = rho[n];
    const double uu[3] = {u[n], u[g.nodes + n], u[2 * g.nodes + n]};
    double du[3];
    // the cell (and local index) containing node index gi along an axis: own cell, and
    // for a cell end point also the previous cell with local index p
    int ce[3][2], ck[3][2], nopt[3];
    for (int a = 0; a < 3; ++a) {
        const int e = gi[a] / p, l = gi[a] % p;
        ce[a][0] = e;
        ck[a][0] = l;
        nopt[a] = 1;
        if (l == 0) {
            ce[a][1] = (e - 1 + g.nel[a]) % g.nel[a];
            ck[a][1] = p;
            nopt[a] = 2;
        }
    }
    // component a of u enters div u at the cell points whose derivative
    // stencil along axis d holds the node: on undistorted cells only d = a,
    // on distorted cells every d, with the factor (J^-1)_da of the point
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (!g.jac && d != a) continue;
            const int b = (d + 1) % 3, c = (d + 2) % 3;
            for (int od = 0; od < nopt[d]; ++od)           // cell along d and the node's index in it
                for (int ob = 0; ob < nopt[b]; ++ob)
                    for (int oc = 0; oc < nopt[c]; ++oc)
                        for (int kd = 0; kd <= p; ++kd) {    // cell point along d
                            int E[3], kk[3];
                            E[d] = ce[d][od];
                            kk[d] = kd;
                            E[b] = ce[b][ob];
                            kk[b] = ck[b][ob];
                            E[c] = ce[c][oc];
                            kk[c] = ck[c][oc];
                            const int64_t cp =
                                ((static_cast<int64_t>(E[2]) * g.nel[1] + E[1]) * g.nel[0] + E[0]) * (p1 * p1 * p1) +
                                (kk[2] * p1 + kk[1]) * p1 + kk[0];
                            double f = dmat[kd * p1 + ck[d][od]] / cell_h(g, d, E[d]);
                            if (g.jac) f *= g.jac[cp * 10 + d * 3 + a];
                            s += sdiv[cp] * f;
                        }
        }
        du[a] = r * uu[a] * W + s;
    }
    const double drho = 0.5 * (uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]) * W -
                        (du[0] * uu[0] + du[1] * uu[1] + du[2] * uu[2]) / r;
    const double dj[3] = {du[0] / r, du[1] / r, du[2] / r};
#pragma unroll
    for (int i = 0; i < vs::Q; ++i) {
        lam[static_cast<int64_t>(i) * g.nodes + n] =
            static_cast<S>(drho + dj[0] * vs::T.xi[i][0] + dj[1] * vs::T.xi[i][1] + dj[2] * vs::T.xi[i][2]);
        lam[static_cast<int64_t>(vs::Q + i) * g.nodes + n] = static_cast<S>(0);
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static CellGeo cell_geo(const Geometry &g, const double *hh, const double *hw, const double *jac = nullptr,
                        const double *full_w = nullptr)
{
    CellGeo c;
    for (int a = 0; a < 3; ++a) {
        c.N[a] = g.N[a];
        c.nel[a] = g.nel[a];
        c.h[a] = hh[a];
    }
    c.hw = hw;
    c.jac = jac;
    c.full_w = full_w;
    c.p = g.p;
    c.nodes = g.nodes;
    return c;
}

template <typename S>
hipError_t Launch<S>::loss(const Geometry &g, const S *state, const double *dmat, const double *ccw, const double *h,
                           const double *hw, const double *cjac, double *scratch_rho, double *scratch_u,
                           double *partials, int nblocks, double *out1, hipStream_t st)
{
    const unsigned nb = static_cast<unsigned>((g.nodes + 255) / 256);
    hipLaunchKernelGGL((k_rho_u<S>), dim3(nb), dim3(256), 0, st, g.nodes, state, scratch_rho, scratch_u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss_cells, dim3(nblocks), dim3(256), 0, st, cell_geo(g, h, hw, cjac), dmat, ccw,
                       scratch_rho, scratch_u, static_cast<double *>(nullptr), partials);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(256), 0, st, partials, nblocks, out1, 0);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::loss_grad(const Geometry &g, const S *state, const double *dmat, const double *ccw,
                                const double *nodew, const double *h, const double *hw, const double *cjac,
                                const double *full_w, double *scratch_rho, double *scratch_u, double *scratch_div,
                                double *partials, int nblocks, S *lam, hipStream_t st)
{
    const unsigned nb = static_cast<unsigned>((g.nodes + 255) / 256);
    hipLaunchKernelGGL((k_rho_u<S>), dim3(nb), dim3(256), 0, st, g.nodes, state, scratch_rho, scratch_u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const CellGeo cg = cell_geo(g, h, hw, cjac, full_w);
    hipLaunchKernelGGL(k_loss_cells, dim3(nblocks), dim3(256), 0, st, cg, dmat, ccw, scratch_rho, scratch_u,
                       scratch_div, partials);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_loss_grad<S>), dim3(nb), dim3(256), 0, st, cg, dmat, nodew, scratch_rho, scratch_u,
                       scratch_div, lam);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::diagnostics(const Geometry &g, const CollisionParams &cp, const S *state, const double *dmat,
                                  const double *ccw, const double *h, const double *hw, const double *cjac,
                                  double *scratch_rho, double *scratch_u, double *scratch_T, double *partials,
                                  int nblocks, double *out3, hipStream_t st)
{
    hipError_t e = moments(g, cp, state, scratch_rho, scratch_u, scratch_T, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_cells, dim3(nblocks), dim3(256), 0, st, cell_geo(g, h, hw, cjac), cp, dmat, ccw,
                       scratch_rho, scratch_u, scratch_T, partials);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum3, dim3(1), dim3(256), 0, st, partials, nblocks, out3);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::collide_vjp(const Geometry &g, const CollisionParams &cp, const S *state_n, S *lam,
                                  double *dmu_partials, int nblocks, double *dmu, hipStream_t st)
{
    // lam <- J_C(X_n)^T lam in place
    const bool nt = use_nontemporal(90 * g.nodes * static_cast<int64_t>(sizeof(S)));
    int blocks = 0;
    bool staged = false;
    if constexpr (sizeof(S) == 4) {
        // FP32: alpha staged in LDS (measured per adjoint step: 3-5 % faster
        // at 128^3 and 256^3 nodes, 8 % at 64^3; in FP64 the staged form
        // spills 81 registers and is 17-20 % slower)
        if (g.nodes % 4 == 0 && reinterpret_cast<uintptr_t>(lam) % 16 == 0) {
            staged = true;
            blocks = static_cast<int>(std::min<int64_t>((g.nodes + 127) / 128, nblocks));
            if (nt)
                hipLaunchKernelGGL((k_collide_vjp_lds<true>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                                   g.nodes, cp, state_n, lam, lam, dmu_partials);
            else
                hipLaunchKernelGGL((k_collide_vjp_lds<false>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                                   g.nodes, cp, state_n, lam, lam, dmu_partials);
        }
    }
    if (!staged) {
        blocks = static_cast<int>(std::min<int64_t>((2 * g.nodes + 255) / 256, nblocks));
        if (nt)
            hipLaunchKernelGGL((k_collide_vjp<S, true>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                               g.nodes, cp, state_n, lam, lam, dmu_partials);
        else
            hipLaunchKernelGGL((k_collide_vjp<S, false>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                               g.nodes, cp, state_n, lam, lam, dmu_partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dmu) {
        hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(256), 0, st, dmu_partials, blocks, dmu, 1);
        e = hipGetLastError();
    }
    return e;
}

template <typename S>
hipError_t Launch<S>::init_equilibrium_vjp(const Geometry &g, const CollisionParams &cp, const double *rho,
                                           const double *u, const double *T, const S *lam0, double *drho, double *du,
                                           double *dT, hipStream_t st)
{
    const unsigned nb = static_cast<unsigned>((g.nodes + 255) / 256);
    hipLaunchKernelGGL((k_init_vjp<S>), dim3(nb), dim3(256), 0, st, g.nodes, cp, rho, u, T, lam0, drho, du, dT);
    return hipGetLastError();
}

template <typename S>
hipError_t Launch<S>::moments_vjp(const Geometry &g, const CollisionParams &cp, const S *state, const double *drho,
                                  const double *du, const double *dT, S *lam, hipStream_t st)
{
    const unsigned nb = static_cast<unsigned>((g.nodes + 255) / 256);
    hipLaunchKernelGGL((k_moments_vjp<S>), dim3(nb), dim3(256), 0, st, g.nodes, cp, state, drho, du, dT, lam);
    return hipGetLastError();
}

template struct Launch<double>;
template struct Launch<float>;

}  // namespace sllbm
