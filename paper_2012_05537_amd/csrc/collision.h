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
//    A0..A2 depending on |u|^2, T - 1, the shell radius |xi|^2 and the
//    dimension D only (the traces of the Hermite tensors), and
//    g^eq = (2 C_v - D) T f^eq.
// Every function is generic over the lattice L (D3Q45 or D2Q19 traits of
// velset.h); in two dimensions the z components are absent.
//  * h* = (w/3!) Qbar : H^(3)(xi); odd in xi, so h*_-i = -h*_i.
//  * Relaxation h' = h + (h^eq - h)/tau + (1/tau - 1/tau_Pr) h*.
// In FP32-mixed storage (S = float) the populations are read and written in
// float once per collision and every operation in between is double: on
// gfx950 an unpacked float FMA issues at the rate of a double one, and the
// per-velocity polynomial in float loses up to c^4/24 (about 50 at the
// outer shell and Mach 1.25) times its ulp to cancellation.
#pragma once

#include <hip/hip_runtime.h>

#include "sllbm_internal.h"
#include "velset.h"

namespace sllbm {

constexpr double SUTHERLAND_S = 0.40417;

// acc + c x for a coefficient c from the velocity-set tables.  After the loops
// over velocities are unrolled c is a compile-time constant, and the term is
// dropped where it is zero: an FMA with a literal zero is otherwise issued
// (x * 0 may be NaN or -0, so the compiler keeps it), 172 of them in the
// D3Q45 collision.  The result is the same except for the sign of a zero sum.
__device__ __forceinline__ double fma_nz(double c, double x, double acc)
{
    return c == 0.0 ? acc : fma(x, c, acc);
}

__device__ __forceinline__ double viscosity_of(const CollisionParams &cp, double T)
{
    if (cp.law == SLLBM_CONSTANT) return cp.mu_inf;
    return cp.mu_inf * (1.0 + SUTHERLAND_S) * T * sqrt(T) / (T + SUTHERLAND_S);
}

// Raw moments of one population array over the pairs (d = odd part, s =
// even part).  m2 in the 3-D component order xx xy xz yy yz zz (the z
// entries stay zero in two dimensions); m3 over the lattice's unique
// rank-3 components.
template <class L>
struct RawMoments {
    double m0, m1[3], m2[6], m3[L::NM3];
};

constexpr int IDX2[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};

template <class L, class Get>
__device__ __forceinline__ RawMoments<L> raw_moments_of(Get &&h)
{
    RawMoments<L> r;
    r.m0 = static_cast<double>(h(0));
#pragma unroll
    for (int k = 0; k < 3; ++k) r.m1[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) r.m2[k] = 0.0;
#pragma unroll
    for (int k = 0; k < L::NM3; ++k) r.m3[k] = 0.0;
#pragma unroll
    for (int q = 0; q < L::NPAIR; ++q) {
        const int i = L::PAIRS.a[q], j = L::PAIRS.b[q];
        const double hi = static_cast<double>(h(i)), hj = static_cast<double>(h(j));
        const double s = hi + hj, d = hi - hj;
        const double *x = L::T.xi[i];
        r.m0 += s;
#pragma unroll
        for (int a = 0; a < L::D; ++a) r.m1[a] = fma_nz(x[a], d, r.m1[a]);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (IDX2[k][1] < L::D) r.m2[k] = fma_nz(x[IDX2[k][0]] * x[IDX2[k][1]], s, r.m2[k]);
#pragma unroll
        for (int m = 0; m < L::NM3; ++m) r.m3[m] = fma_nz(L::H3.mono[i][m], d, r.m3[m]);
    }
    return r;
}

template <class L, typename S>
__device__ __forceinline__ RawMoments<L> raw_moments(const S (&h)[L::Q])
{
    return raw_moments_of<L>([&](int i) { return h[i]; });
}

// index of (a, b) in the 6 unique components xx xy xz yy yz zz
__host__ __device__ constexpr int sym2(int a, int b)
{
    return (a > b) ? sym2(b, a) : (a == 0 ? b : (a == 1 ? 2 + b : 5));
}

// Qbar_abc = M3 - sym3(u M2) + sym3(u u M1) - M0 u u u
template <class L>
__device__ __forceinline__ void centred_third(const RawMoments<L> &r, const double (&u)[3], double (&qb)[L::NM3])
{
#pragma unroll
    for (int m = 0; m < L::NM3; ++m) {
        const int a = L::IDX3[m][0], b = L::IDX3[m][1], c = L::IDX3[m][2];
        qb[m] = r.m3[m] - (u[a] * r.m2[sym2(b, c)] + u[b] * r.m2[sym2(a, c)] + u[c] * r.m2[sym2(a, b)]) +
                (u[a] * u[b] * r.m1[c] + u[a] * u[c] * r.m1[b] + u[b] * u[c] * r.m1[a]) - r.m0 * u[a] * u[b] * u[c];
    }
}

struct EqShell {
    double a0, a1, a2;
};

// Hermite series to fourth order contracted in the scalar invariants
// c = xi.u, |u|^2, |xi|^2 and theta = T - 1; the traces of H^(n) bring in
// D, D + 2 and D + 4 (for D = 3: x2 - 3, x2 - 5, x2 - 7, x2^2 - 10 x2 + 15).
template <int D>
__host__ __device__ __forceinline__ EqShell eq_shell(double u2, double th, double x2)
{
    constexpr double d0 = D, d2 = D + 2, d4 = D + 4;
    EqShell e;
    e.a0 = 1.0 - 0.5 * u2 + 0.5 * th * (x2 - d0) + 0.125 * u2 * u2 - 0.25 * th * u2 * (x2 - d2) +
           0.125 * th * th * (x2 * x2 - 2.0 * d2 * x2 + d0 * d2);
    e.a1 = 1.0 - 0.5 * u2 + 0.5 * th * (x2 - d2);
    e.a2 = 0.5 - 0.25 * u2 + 0.25 * th * (x2 - d4);
    return e;
}

// Collision of one node whose two populations are held by a lane pair,
// lanes l and l ^ XM: the lane with is_g = false holds f, its partner g.
// Each lane forms the raw moments of its own population; the pair exchanges
// rho, j, and the energy parts (tr M2[f] and M0[g]); each lane then builds
// Qbar of its own population and relaxes it (g^eq = (2 C_v - D) T f^eq).
// Both lanes of a pair must be active.
// get(i) returns the pre-collision value of velocity i (storage type S).  It
// is called twice per velocity, for the moments and for the relaxation, with
// fence() in between: a source in memory is then read again rather than held
// in registers through the collision.
// sink(i, value) receives every post-collision value as soon as it is formed.
template <class L, typename S, int XM = 1, class Get, class Fence, class Sink>
__device__ __forceinline__ void collide_core(Get &&get, Fence &&fence, bool is_g, const CollisionParams &cp,
                                             Sink &&sink)
{
    using R = double;   // arithmetic type of the per-velocity terms (storage S is read and written once)
    constexpr bool D3 = L::D == 3;
    const RawMoments<L> rm = raw_moments_of<L>(get);
    fence();
    const double ktr = D3 ? rm.m2[0] + rm.m2[3] + rm.m2[5] : rm.m2[0] + rm.m2[3];
    const double p_m0 = __shfl_xor(rm.m0, XM);
    const double p_j0 = __shfl_xor(rm.m1[0], XM);
    const double p_j1 = __shfl_xor(rm.m1[1], XM);
    const double p_j2 = D3 ? __shfl_xor(rm.m1[2], XM) : 0.0;
    const double p_tr = __shfl_xor(ktr, XM);
    const double rho = is_g ? p_m0 : rm.m0;
    const double ir = 1.0 / rho;
    const double u[3] = {(is_g ? p_j0 : rm.m1[0]) * ir, (is_g ? p_j1 : rm.m1[1]) * ir,
                         D3 ? (is_g ? p_j2 : rm.m1[2]) * ir : 0.0};
    const double K = is_g ? p_tr + rm.m0 : ktr + p_m0;          // 2 rho E
    const double u2 = D3 ? u[0] * u[0] + u[1] * u[1] + u[2] * u[2] : u[0] * u[0] + u[1] * u[1];
    const double T = (K * ir - u2) / (2.0 * cp.Cv);
    double qb[L::NM3];
    centred_third<L>(rm, u, qb);

    const double P = rho * T;
    const double tau = viscosity_of(cp, T) / (P * cp.dt) + 0.5;
    const double tau_pr = (tau - 0.5) * cp.inv_pr + 0.5;
    const R om = static_cast<R>(1.0 / tau);
    const R kap = static_cast<R>(1.0 / tau - 1.0 / tau_pr);
    const double th = T - 1.0;
    const R eqs = static_cast<R>(is_g ? cp.beta * T : 1.0);

    R A0[L::NSHELL], A1[L::NSHELL], A2[L::NSHELL];
#pragma unroll
    for (int s = 0; s < L::NSHELL; ++s) {
        const EqShell e = eq_shell<L::D>(u2, th, L::SHELL_X2[s]);
        A0[s] = static_cast<R>(e.a0 * rho);
        A1[s] = static_cast<R>(e.a1 * rho);
        A2[s] = static_cast<R>(e.a2 * rho);
    }
    const R rho6 = static_cast<R>(rho / 6.0), rho24 = static_cast<R>(rho / 24.0);
    R qr[L::NM3];
#pragma unroll
    for (int m = 0; m < L::NM3; ++m) qr[m] = static_cast<R>(qb[m]);
    const R ux = static_cast<R>(u[0]), uy = static_cast<R>(u[1]), uz = static_cast<R>(u[2]);
    {
        const R heq = eqs * static_cast<R>(L::T.w[0]) * A0[0];
        const R vi = get(0);
        sink(0, static_cast<S>(fma(om, heq - vi, vi)));
    }
#pragma unroll
    for (int q = 0; q < L::NPAIR; ++q) {
        const int i = L::PAIRS.a[q], j = L::PAIRS.b[q];
        const int s = L::T.shell[i];
        R c = fma_nz(L::T.xi[i][1], uy, L::T.xi[i][0] == 0.0 ? R(0) : static_cast<R>(L::T.xi[i][0]) * ux);
        if constexpr (D3) c = fma_nz(L::T.xi[i][2], uz, c);
        const R c2 = c * c;
        const R even = fma(c2, fma(c2, rho24, A2[s]), A0[s]);
        const R odd = c * fma(c2, rho6, A1[s]);
        const R we = eqs * static_cast<R>(L::T.w[i]);
        R hs = 0;
#pragma unroll
        for (int m = 0; m < L::NM3; ++m) hs = fma_nz(L::H3.c[i][m], qr[m], hs);
        const R vi = get(i), vj = get(j);
        sink(i, static_cast<S>(fma(kap, hs, fma(om, fma(we, even, we * odd) - vi, vi))));
        sink(j, static_cast<S>(fma(-kap, hs, fma(om, fma(we, even, -we * odd) - vj, vj))));
    }
}

// The same on values held in registers: sink(i, value) receives every
// post-collision value as soon as it is formed, and v holds them all on
// return as well.
template <class L, typename S, class Sink>
__device__ __forceinline__ void collide_half_s(S (&v)[L::Q], bool is_g, const CollisionParams &cp, Sink &&sink)
{
    collide_core<L, S>([&](int i) { return v[i]; }, [] {}, is_g, cp, [&](int i, S x) {
        v[i] = x;
        sink(i, x);
    });
}

template <class L, typename S>
__device__ __forceinline__ void collide_half(S (&v)[L::Q], bool is_g, const CollisionParams &cp)
{
    collide_half_s<L, S>(v, is_g, cp, [](int, S) {});
}

}  // namespace sllbm
