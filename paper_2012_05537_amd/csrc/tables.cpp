// Host-side tables of the SLLBM library: the D3Q45 velocity set, the GLC
// support points, Lagrange weights, Clenshaw-Curtis node weights, and the
// per-axis departure tables of the semi-Lagrangian streaming (Sec. II A).
//
// On a periodic mesh of equal cells the departure point of node g = e*p + l
// for velocity i lies, along axis a, at x_g - xi_ia dt; its cell is
// e + floor(t_l - xi_ia dt / h) and its local coordinate the fractional part,
// both independent of e.  The sparse matrix Psi_i of Eq. (9) is therefore the
// tensor product of three 1-D operators, each described by p rows of (p+1)
// taps; these rows are all that is stored.
#include <algorithm>
#include <cstdint>
#include <cmath>
#include <string>

#include "sllbm_internal.h"
#include "velset.h"

namespace sllbm {


// Degree-nine rules (Sec. II B), from the compile-time tables shared with
// the kernels (velset.h).
template <class L>
static void copy_lattice(VelocitySet &out)
{
    out = VelocitySet{};
    out.q = L::Q;
    out.dim = L::D;
    for (int i = 0; i < L::Q; ++i) {
        for (int k = 0; k < 3; ++k) out.xi[i][k] = L::T.xi[i][k];
        out.w[i] = L::T.w[i];
        out.opposite[i] = L::T.opp[i];
    }
}

bool build_velocity_set(VelocitySet &out, int set)
{
    if (set == SLLBM_D3Q45) copy_lattice<D3Q45>(out);
    else if (set == SLLBM_D2Q19) copy_lattice<D2Q19>(out);
    else return false;
    return true;
}

void glc_points(int p, double *t)
{
    for (int k = 0; k <= p; ++k) t[k] = 0.5 * (1.0 - std::cos(M_PI * k / p));
}

void lagrange_basis(int p, double s, double *ell)
{
    double t[MAXP + 1];
    glc_points(p, t);
    for (int k = 0; k <= p; ++k) {
        double num = 1.0, den = 1.0;
        for (int m = 0; m <= p; ++m) {
            if (m == k) continue;
            num *= s - t[m];
            den *= t[k] - t[m];
        }
        ell[k] = num / den;
    }
}

void lagrange_basis_deriv(int p, double s, double *dl)
{
    double t[MAXP + 1];
    glc_points(p, t);
    for (int k = 0; k <= p; ++k) {
        double den = 1.0;
        for (int m = 0; m <= p; ++m)
            if (m != k) den *= t[k] - t[m];
        // derivative of prod_{m != k} (s - t_m): sum over the dropped factor
        double sum = 0.0;
        for (int j = 0; j <= p; ++j) {
            if (j == k) continue;
            double prod = 1.0;
            for (int m = 0; m <= p; ++m)
                if (m != k && m != j) prod *= s - t[m];
            sum += prod;
        }
        dl[k] = sum / den;
    }
}

// Clenshaw-Curtis weights for the Chebyshev-Lobatto points on [-1, 1]:
// integrate the degree-p interpolant exactly, via the cosine series of 1.
void clenshaw_curtis(int p, double *w)
{
    for (int k = 0; k <= p; ++k) {
        double acc = 1.0;
        for (int j = 1; 2 * j <= p; ++j) {
            double c = (2 * j == p) ? 1.0 : 2.0;
            acc -= c * std::cos(2.0 * M_PI * j * k / p) / (4.0 * j * j - 1.0);
        }
        w[k] = ((k == 0 || k == p) ? 1.0 : 2.0) * acc / p;
    }
}

void build_cell_tables(const VelocitySet &vs, int p, const double h[3], double dt, std::vector<int32_t> &omin,
                       std::vector<int32_t> &lstar, std::vector<double> &w)
{
    double t[MAXP + 1];
    glc_points(p, t);
    const int nq = vs.q;
    omin.assign(nq * 3, 0);
    lstar.assign(nq * 3, p);
    w.assign(nq * 3 * p * (p + 1), 0.0);
    for (int i = 0; i < nq; ++i) {
        for (int a = 0; a < 3; ++a) {
            // node l of a cell departs to t_l - xi dt / h (cell units): cell
            // floor of that, local coordinate its fractional part (Eq. (9))
            const double shift = vs.xi[i][a] * dt / h[a];
            int cell[MAXP];
            for (int l = 0; l < p; ++l) {
                const double s = t[l] - shift;
                const double o = std::floor(s);
                cell[l] = static_cast<int>(o);
                lagrange_basis(p, s - o, &w[((i * 3 + a) * p + l) * (p + 1)]);
            }
            // t_l rises from 0 towards 1, so the departure cells are
            // non-decreasing and span at most two neighbours
            omin[i * 3 + a] = cell[0];
            for (int l = 0; l < p; ++l)
                if (cell[l] != cell[0] && lstar[i * 3 + a] == p) lstar[i * 3 + a] = l;
        }
    }
}

double axis_node_position(int p, int ne, double length, const std::vector<double> &faces, int g)
{
    const int e = g / p, l = g % p;
    if (faces.empty()) {
        const double h = length / ne;
        return e * h + h * 0.5 * (1.0 - std::cos(M_PI * l / p));
    }
    return faces[e] + (faces[e + 1] - faces[e]) * 0.5 * (1.0 - std::cos(M_PI * l / p));
}

void build_node_tables(const VelocitySet &vs, int p, int ne, double length, const std::vector<double> &faces,
                       int axis, double dt, std::vector<int32_t> &src, std::vector<double> &w)
{
    const int N = ne * p;
    src.assign(static_cast<size_t>(vs.q) * N, 0);
    w.assign(static_cast<size_t>(vs.q) * N * (p + 1), 0.0);
    for (int i = 0; i < vs.q; ++i) {
        const double shift = vs.xi[i][axis] * dt;
        for (int g = 0; g < N; ++g) {
            const double X = axis_node_position(p, ne, length, faces, g) - shift;   // departure point
            int64_t E;                                // departure cell, not wrapped (monotone in g)
            double t;                                 // local coordinate in [0, 1)
            if (faces.empty()) {
                const double sc = X / (length / ne);
                const double fl = std::floor(sc);
                E = static_cast<int64_t>(fl);
                t = sc - fl;
            } else {
                double k = std::floor(X / length);
                double Xw = X - k * length;
                if (Xw >= length) {                   // rounding of the wrap
                    Xw = 0.0;
                    k += 1.0;
                }
                int lo = 0, hi = ne;                  // faces[lo] <= Xw < faces[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) / 2;
                    if (faces[mid] <= Xw) lo = mid;
                    else hi = mid;
                }
                E = lo + static_cast<int64_t>(k) * ne;
                t = (Xw - faces[lo]) / (faces[lo + 1] - faces[lo]);
            }
            src[static_cast<size_t>(i) * N + g] = static_cast<int32_t>(E * p);
            lagrange_basis(p, t, &w[(static_cast<size_t>(i) * N + g) * (p + 1)]);
        }
    }
}

void build_transposed_node_tables(int N, int p, const std::vector<int32_t> &src, const std::vector<double> &w,
                                  int kt, std::vector<int32_t> &srcT, std::vector<double> &wT, int &band)
{
    srcT.assign(static_cast<size_t>(Q) * N, 0);
    wT.assign(static_cast<size_t>(Q) * N * std::max(kt, 1), 0.0);
    band = 1;
    std::vector<int64_t> lo(N), hi(N);
    for (int i = 0; i < Q; ++i) {
        const int32_t *s = &src[static_cast<size_t>(i) * N];
        int32_t *st = &srcT[static_cast<size_t>(i) * N];
        std::fill(lo.begin(), lo.end(), INT64_MAX);
        std::fill(hi.begin(), hi.end(), INT64_MIN);
        // forward output g reads input node s[g] + k; as an output of S^T,
        // input node m = (s[g] + k) mod N collects it from output g - jN
        // (the outputs repeat with period N, their inputs shifted by N)
        auto visit = [&](auto &&fn) {
            for (int g = 0; g < N; ++g)
                for (int k = 0; k <= p; ++k) {
                    const int64_t t = static_cast<int64_t>(s[g]) + k;
                    const int64_t m = ((t % N) + N) % N;
                    fn(static_cast<int>(m), g - (t - m), g, k);   // t - m = jN
                }
        };
        visit([&](int m, int64_t gu, int, int) {
            lo[m] = std::min(lo[m], gu);
            hi[m] = std::max(hi[m], gu);
        });
        // band starts: a node some output reads starts at its first reader; a
        // node none reads takes the start of the next read node (N later past
        // the wrap), so the starts stay non-decreasing
        int64_t next = 0;
        for (int m = 2 * N - 1; m >= 0; --m) {
            const int mm = m % N;
            if (hi[mm] >= lo[mm]) {
                next = lo[mm] + (m >= N ? N : 0);
                if (m < N) st[mm] = static_cast<int32_t>(lo[mm]);
            } else if (m < N) {
                st[mm] = static_cast<int32_t>(next);
            }
        }
        for (int m = 0; m < N; ++m)
            if (hi[m] >= lo[m]) band = std::max(band, static_cast<int>(hi[m] - lo[m] + 1));
        if (kt <= 0) continue;
        visit([&](int m, int64_t gu, int g, int k) {
            const int64_t slot = gu - st[m];
            if (slot >= 0 && slot < kt)
                wT[(static_cast<size_t>(i) * N + m) * kt + slot] = w[(static_cast<size_t>(i) * N + g) * (p + 1) + k];
        });
    }
}

}  // namespace sllbm
