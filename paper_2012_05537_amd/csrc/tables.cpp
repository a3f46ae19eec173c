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
#include <cmath>

#include "sllbm_internal.h"
#include "velset.h"

namespace sllbm {


// Degree-nine D3Q45 rule (Sec. II B), from the compile-time table shared with
// the kernels (velset.h).
void build_velocity_set(VelocitySet &out)
{
    for (int i = 0; i < Q; ++i) {
        for (int k = 0; k < 3; ++k) out.xi[i][k] = vs::T.xi[i][k];
        out.w[i] = vs::T.w[i];
        out.opposite[i] = vs::T.opp[i];
    }
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

void build_axis_tables(const VelocitySet &vs, int p, const double h[3], double dt, AxisTables &fwd,
                       AxisTables &adj)
{
    double t[MAXP + 1];
    glc_points(p, t);
    fwd.p = adj.p = p;
    fwd.K = p + 1;
    adj.K = 2 * p;
    fwd.off.assign(Q * 3 * p * fwd.K, 0);
    fwd.wt.assign(Q * 3 * p * fwd.K, 0.0);
    adj.off.assign(Q * 3 * p * adj.K, 0);
    adj.wt.assign(Q * 3 * p * adj.K, 0.0);
    fwd.lo.assign(Q * 3, 0);
    fwd.span.assign(Q * 3, 0);
    adj.lo.assign(Q * 3, 0);
    adj.span.assign(Q * 3, 0);

    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) {
            const double shift = vs.xi[i][a] * dt / h[a];   // displacement in cell widths
            int cell[MAXP];
            double W[MAXP][MAXP + 1];
            for (int l = 0; l < p; ++l) {
                double s = t[l] - shift;                      // departure point, cell units
                double o = std::floor(s);
                cell[l] = static_cast<int>(o);
                lagrange_basis(p, s - o, W[l]);
            }
            // forward rows: node l of cell e reads cell e + cell[l]
            const int base = (i * 3 + a) * p;
            int lo = 1 << 30, hi = -(1 << 30);
            for (int l = 0; l < p; ++l) {
                for (int k = 0; k <= p; ++k) {
                    int off = cell[l] * p + k;
                    fwd.off[(base + l) * fwd.K + k] = off;
                    fwd.wt[(base + l) * fwd.K + k] = W[l][k];
                    lo = std::min(lo, off);
                    hi = std::max(hi, off);
                }
            }
            fwd.lo[i * 3 + a] = lo;
            fwd.span[i * 3 + a] = hi - lo + 1;
            // transposed rows: source point m of cell E is read, with weight
            // W[l][m], by node l of cell E - cell[l]; the shared point m = 0 is
            // also point p of cell E-1, read by node l of cell E-1-cell[l].
            lo = 1 << 30;
            hi = -(1 << 30);
            for (int m = 0; m < p; ++m) {
                int n = 0;
                int *orow = &adj.off[(base + m) * adj.K];
                double *wrow = &adj.wt[(base + m) * adj.K];
                for (int l = 0; l < p; ++l, ++n) {
                    orow[n] = -cell[l] * p + l;
                    wrow[n] = W[l][m];
                }
                if (m == 0) {
                    for (int l = 0; l < p; ++l, ++n) {
                        orow[n] = -(1 + cell[l]) * p + l;
                        wrow[n] = W[l][p];
                    }
                }
                for (; n < adj.K; ++n) {          // padding taps: weight 0, in-window offset
                    orow[n] = orow[0];
                    wrow[n] = 0.0;
                }
                for (int k = 0; k < adj.K; ++k) {
                    lo = std::min(lo, orow[k]);
                    hi = std::max(hi, orow[k]);
                }
            }
            adj.lo[i * 3 + a] = lo;
            adj.span[i * 3 + a] = hi - lo + 1;
        }
    }
}

}  // namespace sllbm

namespace sllbm {

void build_cell_tables(const AxisTables &fwd, std::vector<int32_t> &omin, std::vector<int32_t> &lstar,
                        std::vector<double> &w)
{
    const int p = fwd.p, K = fwd.K;
    omin.assign(Q * 3, 0);
    lstar.assign(Q * 3, p);
    w.assign(Q * 3 * p * (p + 1), 0.0);
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < 3; ++a) {
            const int base = (i * 3 + a) * p;
            // departure cell of row l is off[l][0] / p; non-decreasing in l
            const int o0 = fwd.off[base * K] / p;
            omin[i * 3 + a] = o0;
            for (int l = 0; l < p; ++l) {
                const int o = fwd.off[(base + l) * K] / p - o0;
                if (o == 1 && lstar[i * 3 + a] == p) lstar[i * 3 + a] = l;
                for (int k = 0; k <= p; ++k) w[(base + l) * (p + 1) + k] = fwd.wt[(base + l) * K + k];
            }
        }
}

}  // namespace sllbm
