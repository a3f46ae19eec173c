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
#include <array>
#include <cmath>

#include "sllbm_internal.h"

namespace sllbm {

namespace {

using Vec3 = std::array<double, 3>;

// Sign variants of the cyclic permutations of (a, b, c), without duplicates.
std::vector<Vec3> signed_cycles(double a, double b, double c)
{
    std::vector<Vec3> out;
    const Vec3 rot[3] = {{a, b, c}, {b, c, a}, {c, a, b}};
    for (const Vec3 &r : rot) {
        for (int s = 0; s < 8; ++s) {
            Vec3 v{(s & 1) ? -r[0] : r[0], (s & 2) ? -r[1] : r[1], (s & 4) ? -r[2] : r[2]};
            bool seen = std::any_of(out.begin(), out.end(), [&](const Vec3 &u) {
                return std::fabs(u[0] - v[0]) + std::fabs(u[1] - v[1]) + std::fabs(u[2] - v[2]) < 1e-12;
            });
            if (!seen) out.push_back(v);
        }
    }
    return out;
}

void normalise_and_sort(std::vector<Vec3> &dirs)
{
    for (Vec3 &v : dirs) {
        double r = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (double &c : v) c /= r;
    }
    // lexicographic order, coordinates closer than 1e-9 count as equal
    std::sort(dirs.begin(), dirs.end(), [](const Vec3 &x, const Vec3 &y) {
        for (int k = 0; k < 3; ++k)
            if (std::fabs(x[k] - y[k]) > 1e-9) return x[k] < y[k];
        return false;
    });
}

}  // namespace

// Degree-nine D3Q45 rule (Sec. II B): the origin, an icosahedron at radius
// sqrt(3), the same icosahedron at radius sqrt(15), and its dual dodecahedron
// at radius 3, with weights 28/135, 25/432, 1/2160 and 1/216.
void build_velocity_set(VelocitySet &vs)
{
    const double phi = 0.5 * (1.0 + std::sqrt(5.0));
    std::vector<Vec3> ico = signed_cycles(0.0, 1.0, phi);
    std::vector<Vec3> dod = signed_cycles(1.0, 1.0, 1.0);
    std::vector<Vec3> dod2 = signed_cycles(0.0, phi, 1.0 / phi);
    dod.insert(dod.end(), dod2.begin(), dod2.end());
    normalise_and_sort(ico);
    normalise_and_sort(dod);
    struct Shell { const std::vector<Vec3> *dirs; double radius, weight; };
    const Shell shells[3] = {{&ico, std::sqrt(3.0), 25.0 / 432.0},
                             {&ico, std::sqrt(15.0), 1.0 / 2160.0},
                             {&dod, 3.0, 1.0 / 216.0}};
    int q = 0;
    vs.xi[0][0] = vs.xi[0][1] = vs.xi[0][2] = 0.0;
    vs.w[q++] = 28.0 / 135.0;
    for (const Shell &s : shells) {
        for (const Vec3 &d : *s.dirs) {
            for (int k = 0; k < 3; ++k) vs.xi[q][k] = s.radius * d[k];
            vs.w[q++] = s.weight;
        }
    }
    for (int i = 0; i < Q; ++i) {
        vs.opposite[i] = -1;
        for (int j = 0; j < Q; ++j) {
            double d = std::fabs(vs.xi[i][0] + vs.xi[j][0]) + std::fabs(vs.xi[i][1] + vs.xi[j][1]) +
                       std::fabs(vs.xi[i][2] + vs.xi[j][2]);
            if (d < 1e-12) vs.opposite[i] = j;
        }
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
