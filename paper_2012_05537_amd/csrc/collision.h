// Node-local collision of the SLLBM (Eq. (5) with the quasi-equilibrium
// extension of App. D) for populations held in registers.
//
// Arithmetic layout (equal to the definitions term by term):
//  * Moments in double for both storage types (Eq. (7)); the set is centrally
//    symmetric, so each pair (xi, -xi) contributes s = h_i + h_-i to the even
//    moments and d = h_i - h_-i to the odd ones.
//  * T from 2 rho E = rho |u|^2 + 2 C_v rho T; P = rho T; Sutherland mu(T);
//    tau = mu/(P dt) + 1/2, tau_Pr = (tau - 1/2)/Pr + 1/2.
//  * Centred third moments Qbar[h] = sum h (xi-u)^3 from the raw moments
//    M0..M3 of h; Qbar[h^eq] = 0 identically, so Qbar^neq = Qbar[h].
//  * Equilibrium (Eq. (6), App. A/B) in scalar form: with c = xi.u,
//      f^eq = w rho (A0 + A1 c + A2 c^2 + c^3/6 + c^4/24),
//    A0..A2 depending on |u|^2, T - 1 and the shell radius |xi|^2 only, and
//    g^eq = (2 C_v - D) T f^eq.
//  * h* = (w/3!) Qbar : H^(3)(xi); odd in xi, so h*_-i = -h*_i.
//  * Relaxation h' = h + (h^eq - h)/tau + (1/tau - 1/tau_Pr) h*.
// In FP32-mixed storage (S = float) the moments, transport coefficients,
// equilibrium coefficients and Qbar are double; the per-velocity polynomial,
// the H^(3) contraction and the relaxation run in float.
#pragma once

#include <hip/hip_runtime.h>

#include "sllbm_internal.h"
#include "velset.h"

namespace sllbm {

constexpr double SUTHERLAND_S = 0.40417;

struct NodeState {
    double rho, ux, uy, uz, T;
};

__device__ __forceinline__ double viscosity_of(const CollisionParams &cp, double T)
{
    if (cp.law == SLLBM_CONSTANT) return cp.mu_inf;
    return cp.mu_inf * (1.0 + SUTHERLAND_S) * T * sqrt(T) / (T + SUTHERLAND_S);
}

// Raw moments of one population array over the pairs (d = odd part, s = even part).
struct RawMoments {
    double m0, m1[3], m2[6], m3[10];
};

template <typename S>
__device__ __forceinline__ RawMoments raw_moments(const S (&h)[vs::Q])
{
    RawMoments r;
    r.m0 = static_cast<double>(h[0]);
#pragma unroll
    for (int k = 0; k < 3; ++k) r.m1[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) r.m2[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 10; ++k) r.m3[k] = 0.0;
#pragma unroll
    for (int q = 0; q < 22; ++q) {
        const int i = vs::PAIRS.a[q], j = vs::PAIRS.b[q];
        const double hi = static_cast<double>(h[i]), hj = static_cast<double>(h[j]);
        const double s = hi + hj, d = hi - hj;
        const double x = vs::T.xi[i][0], y = vs::T.xi[i][1], z = vs::T.xi[i][2];
        r.m0 += s;
        r.m1[0] = fma(d, x, r.m1[0]);
        r.m1[1] = fma(d, y, r.m1[1]);
        r.m1[2] = fma(d, z, r.m1[2]);
        r.m2[0] = fma(s, x * x, r.m2[0]);
        r.m2[1] = fma(s, x * y, r.m2[1]);
        r.m2[2] = fma(s, x * z, r.m2[2]);
        r.m2[3] = fma(s, y * y, r.m2[3]);
        r.m2[4] = fma(s, y * z, r.m2[4]);
        r.m2[5] = fma(s, z * z, r.m2[5]);
#pragma unroll
        for (int m = 0; m < 10; ++m) r.m3[m] = fma(d, vs::H3.mono[i][m], r.m3[m]);
    }
    return r;
}

// index of (a, b) in the 6 unique components xx xy xz yy yz zz
__host__ __device__ constexpr int sym2(int a, int b)
{
    return (a > b) ? sym2(b, a) : (a == 0 ? b : (a == 1 ? 2 + b : 5));
}

// Qbar_abc = M3 - sym3(u M2) + sym3(u u M1) - M0 u u u
__device__ __forceinline__ void centred_third(const RawMoments &r, const double (&u)[3], double (&qb)[10])
{
#pragma unroll
    for (int m = 0; m < 10; ++m) {
        const int a = vs::IDX3[m][0], b = vs::IDX3[m][1], c = vs::IDX3[m][2];
        qb[m] = r.m3[m] - (u[a] * r.m2[sym2(b, c)] + u[b] * r.m2[sym2(a, c)] + u[c] * r.m2[sym2(a, b)]) +
                (u[a] * u[b] * r.m1[c] + u[a] * u[c] * r.m1[b] + u[b] * u[c] * r.m1[a]) - r.m0 * u[a] * u[b] * u[c];
    }
}

struct EqShell {
    double a0, a1, a2;
};

__device__ __forceinline__ EqShell eq_shell(double u2, double th, double x2)
{
    EqShell e;
    e.a0 = 1.0 - 0.5 * u2 + 0.5 * th * (x2 - 3.0) + 0.125 * u2 * u2 - 0.25 * th * u2 * (x2 - 5.0) +
           0.125 * th * th * (x2 * x2 - 10.0 * x2 + 15.0);
    e.a1 = 1.0 - 0.5 * u2 + 0.5 * th * (x2 - 5.0);
    e.a2 = 0.5 - 0.25 * u2 + 0.25 * th * (x2 - 7.0);
    return e;
}

constexpr double SHELL_X2[4] = {0.0, 3.0, 15.0, 9.0};

template <typename S>
__device__ __forceinline__ NodeState node_state(const RawMoments &rf, double G0, double Cv)
{
    NodeState n;
    n.rho = rf.m0;
    const double ir = 1.0 / n.rho;
    n.ux = rf.m1[0] * ir;
    n.uy = rf.m1[1] * ir;
    n.uz = rf.m1[2] * ir;
    const double u2 = n.ux * n.ux + n.uy * n.uy + n.uz * n.uz;
    const double K = rf.m2[0] + rf.m2[3] + rf.m2[5] + G0;      // 2 rho E
    n.T = (K * ir - u2) / (2.0 * Cv);
    return n;
}

template <typename S>
__device__ __forceinline__ void collide_regs(S (&f)[vs::Q], S (&g)[vs::Q], const CollisionParams &cp)
{
    using R = S;   // per-velocity arithmetic type
    // f moments and Qbar[f]
    RawMoments rm = raw_moments(f);
    double G0 = static_cast<double>(g[0]);
#pragma unroll
    for (int q = 0; q < 22; ++q) G0 += static_cast<double>(g[vs::PAIRS.a[q]]) + static_cast<double>(g[vs::PAIRS.b[q]]);
    const NodeState n = node_state<S>(rm, G0, cp.Cv);
    const double u[3] = {n.ux, n.uy, n.uz};
    double qf[10];
    centred_third(rm, u, qf);
    // g moments and Qbar[g]
    rm = raw_moments(g);
    double qg[10];
    centred_third(rm, u, qg);

    const double u2 = n.ux * n.ux + n.uy * n.uy + n.uz * n.uz;
    const double P = n.rho * n.T;
    const double tau = viscosity_of(cp, n.T) / (P * cp.dt) + 0.5;
    const double tau_pr = (tau - 0.5) * cp.inv_pr + 0.5;
    const R om = static_cast<R>(1.0 / tau);
    const R kap = static_cast<R>(1.0 / tau - 1.0 / tau_pr);
    const double th = n.T - 1.0;
    const R betaT = static_cast<R>(cp.beta * n.T);

    R A0[4], A1[4], A2[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const EqShell e = eq_shell(u2, th, SHELL_X2[s]);
        A0[s] = static_cast<R>(e.a0 * n.rho);
        A1[s] = static_cast<R>(e.a1 * n.rho);
        A2[s] = static_cast<R>(e.a2 * n.rho);
    }
    const R rho6 = static_cast<R>(n.rho / 6.0), rho24 = static_cast<R>(n.rho / 24.0);
    R qfr[10], qgr[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) {
        qfr[m] = static_cast<R>(qf[m]);
        qgr[m] = static_cast<R>(qg[m]);
    }
    const R ux = static_cast<R>(n.ux), uy = static_cast<R>(n.uy), uz = static_cast<R>(n.uz);

    // rest velocity: c = 0, h* = 0
    {
        const R feq = static_cast<R>(vs::T.w[0]) * A0[0];
        const R fi = f[0], gi = g[0];
        f[0] = fma(om, feq - fi, fi);
        g[0] = fma(om, betaT * feq - gi, gi);
    }
#pragma unroll
    for (int q = 0; q < 22; ++q) {
        const int i = vs::PAIRS.a[q], j = vs::PAIRS.b[q];
        const int s = vs::T.shell[i];
        const R w = static_cast<R>(vs::T.w[i]);
        const R c = static_cast<R>(vs::T.xi[i][0]) * ux + static_cast<R>(vs::T.xi[i][1]) * uy +
                    static_cast<R>(vs::T.xi[i][2]) * uz;
        const R c2 = c * c;
        const R even = fma(c2, fma(c2, rho24, A2[s]), A0[s]);
        const R odd = c * fma(c2, rho6, A1[s]);
        const R feq_i = w * (even + odd), feq_j = w * (even - odd);
        R fs = 0, gs = 0;
#pragma unroll
        for (int m = 0; m < 10; ++m) {
            fs = fma(static_cast<R>(vs::H3.c[i][m]), qfr[m], fs);
            gs = fma(static_cast<R>(vs::H3.c[i][m]), qgr[m], gs);
        }
        const R fi = f[i], fj = f[j], gi = g[i], gj = g[j];
        f[i] = fma(kap, fs, fma(om, feq_i - fi, fi));
        f[j] = fma(-kap, fs, fma(om, feq_j - fj, fj));
        g[i] = fma(kap, gs, fma(om, betaT * feq_i - gi, gi));
        g[j] = fma(-kap, gs, fma(om, betaT * feq_j - gj, gj));
    }
}

}  // namespace sllbm
