/*
 * Plain CPU reference ("oracle") of the 3-D compressible semi-Lagrangian
 * lattice Boltzmann method (SLLBM) of Wilde, Kraemer, Reith & Foysi,
 * "High-order semi-Lagrangian kinetic scheme for compressible turbulence"
 * (arXiv:2012.05537).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Everything is done the slow, literal way, in FP64:
 *   - the equilibrium is the full tensor contraction over all 3^n components
 *     of the Hermite series (Sec. II A, Eq. (6); App. A moments; App. B
 *     Hermite tensors);
 *   - the quasi-equilibrium term builds the centred third moment of h and of
 *     h^eq and contracts their difference with all 27 components of H^(3)
 *     (App. D);
 *   - streaming traces every (node, velocity) pair back to x - xi*dt, finds
 *     the enclosing cell (floor() on equal cells, bisection over the cell
 *     faces on a graded mesh), and sums the (p+1)^3 tensor-product
 *     Lagrange basis values over that cell's support points (Eqs. (8)-(9)).
 *     No per-axis factorisation and no precomputed tables are used.
 *
 * The file is compiled twice: once with R = double (symbols oracle_*), and
 * once with -DORACLE_COMPLEX, R = double complex (symbols oracle_cs_*).  The
 * complex build is used for complex-step derivatives (Squire & Trapp 1998):
 * every state-dependent operation below is analytic, and the only floor() is
 * applied to the state-independent departure position.
 *
 * Readings of the paper taken here:
 *   c_s = 1, T0 = 1, theta = T (lattice units); D = 3; C_v = 1/(gamma-1).
 *   T from 2 rho E = rho |u|^2 + 2 C_v rho T (the energy of the equilibria).
 *   Sutherland numerator 1 + S with S = 0.40417, so that mu(T=1) = mu_inf.
 *   Quasi-equilibrium h* carries the 1/3! of the third Hermite term; each
 *   population uses its own centred third moment.
 *   Velocity set: the degree-9 icosahedral D3Q45 rule (origin, two
 *   icosahedra of radii sqrt(3) and sqrt(15), one dodecahedron of radius 3).
 *   GLC support points t_k = (1 - cos(pi k / p))/2 per cell, unique periodic
 *   nodes (n_el * p per axis).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_COMPLEX
#include <complex.h>
typedef double complex R;
#define RSQRT(x) csqrt(x)
#define FN(name) oracle_cs_##name
#else
typedef double R;
#define RSQRT(x) sqrt(x)
#define FN(name) oracle_##name
#endif

#define Q 45
#define DIM 3

typedef struct {
    int n_el[3];           /* cells per axis (periodic) */
    int p;                 /* interpolation order (GLC points per cell edge - 1) */
    double length[3];      /* domain edge lengths */
    double dt;             /* time step */
    double gamma;          /* heat capacity ratio */
    double prandtl;        /* target Prandtl number of the quasi-equilibrium term */
    double mu_inf;         /* dynamic viscosity at T = 1 */
    double mu_inf_im;      /* imaginary part of mu_inf (complex build only) */
    int viscosity_law;     /* 0 = Sutherland, 1 = constant mu = mu_inf */
    const double *faces[3];/* graded mesh: n_el[a] + 1 cell-face coordinates per axis,
                              faces[a][0] = 0, faces[a][n_el] = length[a]; NULL = equal cells */
    const double *disp;    /* distorted mesh: node displacements [3][N] (periodic) added to the
                              equal-cell GLC positions; NULL = undistorted */
} oracle_cfg;

/* ------------------------------------------------------------------------- */
/* Velocity set (Sec. II B: degree-nine D3Q45 cubature with icosahedral      */
/* symmetry).  Built from the orbit directions and closed-form weights.      */
/* ------------------------------------------------------------------------- */

static int lex_less(const double *a, const double *b)
{
    for (int k = 0; k < 3; ++k) {
        if (fabs(a[k] - b[k]) > 1e-9) return a[k] < b[k];
    }
    return 0;
}

static void sort_dirs(double (*v)[3], int n)
{
    for (int i = 1; i < n; ++i) {           /* insertion sort, lexicographic */
        double t[3] = {v[i][0], v[i][1], v[i][2]};
        int j = i - 1;
        while (j >= 0 && lex_less(t, v[j])) {
            v[j + 1][0] = v[j][0]; v[j + 1][1] = v[j][1]; v[j + 1][2] = v[j][2];
            --j;
        }
        v[j + 1][0] = t[0]; v[j + 1][1] = t[1]; v[j + 1][2] = t[2];
    }
}

/* all sign variants of the three cyclic permutations of (a, b, c), deduplicated */
static int cyclic_signed(double a, double b, double c, double (*out)[3], int n)
{
    double base[3][3] = {{a, b, c}, {b, c, a}, {c, a, b}};
    for (int r = 0; r < 3; ++r) {
        for (int s = 0; s < 8; ++s) {
            double v[3];
            for (int k = 0; k < 3; ++k) v[k] = ((s >> k) & 1) ? -base[r][k] : base[r][k];
            int dup = 0;
            for (int m = 0; m < n; ++m) {
                if (fabs(out[m][0] - v[0]) < 1e-12 && fabs(out[m][1] - v[1]) < 1e-12 &&
                    fabs(out[m][2] - v[2]) < 1e-12) { dup = 1; break; }
            }
            if (!dup) { out[n][0] = v[0]; out[n][1] = v[1]; out[n][2] = v[2]; ++n; }
        }
    }
    return n;
}

int oracle_velocity_set(double *xi, double *w)
{
    const double phi = 0.5 * (1.0 + sqrt(5.0));
    double ico[12][3], dod[20][3];
    int ni = cyclic_signed(0.0, 1.0, phi, ico, 0);
    int nd = cyclic_signed(1.0, 1.0, 1.0, dod, 0);
    nd = cyclic_signed(0.0, phi, 1.0 / phi, dod, nd);
    if (ni != 12 || nd != 20) return -1;
    for (int m = 0; m < 12; ++m) {
        double r = sqrt(ico[m][0] * ico[m][0] + ico[m][1] * ico[m][1] + ico[m][2] * ico[m][2]);
        for (int k = 0; k < 3; ++k) ico[m][k] /= r;
    }
    for (int m = 0; m < 20; ++m) {
        double r = sqrt(dod[m][0] * dod[m][0] + dod[m][1] * dod[m][1] + dod[m][2] * dod[m][2]);
        for (int k = 0; k < 3; ++k) dod[m][k] /= r;
    }
    sort_dirs(ico, 12);
    sort_dirs(dod, 20);
    int q = 0;
    xi[0] = xi[1] = xi[2] = 0.0; w[q++] = 28.0 / 135.0;
    for (int m = 0; m < 12; ++m, ++q) {
        for (int k = 0; k < 3; ++k) xi[3 * q + k] = sqrt(3.0) * ico[m][k];
        w[q] = 25.0 / 432.0;
    }
    for (int m = 0; m < 12; ++m, ++q) {
        for (int k = 0; k < 3; ++k) xi[3 * q + k] = sqrt(15.0) * ico[m][k];
        w[q] = 1.0 / 2160.0;
    }
    for (int m = 0; m < 20; ++m, ++q) {
        for (int k = 0; k < 3; ++k) xi[3 * q + k] = 3.0 * dod[m][k];
        w[q] = 1.0 / 216.0;
    }
    return q;
}

/* ------------------------------------------------------------------------- */
/* Support points, Lagrange basis, Clenshaw-Curtis node weights (Sec. II A,  */
/* Eq. (8): cell-oriented interpolation on Gauss-Lobatto-Chebyshev points).  */
/* ------------------------------------------------------------------------- */

void oracle_glc_nodes(int p, double *t)
{
    for (int k = 0; k <= p; ++k) t[k] = 0.5 * (1.0 - cos(M_PI * (double)k / (double)p));
}

/* l_k(s) = prod_{m != k} (s - t_m) / (t_k - t_m) */
void oracle_lagrange(int p, double s, double *ell)
{
    double t[16];
    oracle_glc_nodes(p, t);
    for (int k = 0; k <= p; ++k) {
        double v = 1.0;
        for (int m = 0; m <= p; ++m) {
            if (m != k) v *= (s - t[m]) / (t[k] - t[m]);
        }
        ell[k] = v;
    }
}

/* d l_k / ds at s */
void oracle_lagrange_deriv(int p, double s, double *dell)
{
    double t[16];
    oracle_glc_nodes(p, t);
    for (int k = 0; k <= p; ++k) {
        double sum = 0.0;
        for (int j = 0; j <= p; ++j) {
            if (j == k) continue;
            double v = 1.0 / (t[k] - t[j]);
            for (int m = 0; m <= p; ++m) {
                if (m != k && m != j) v *= (s - t[m]) / (t[k] - t[m]);
            }
            sum += v;
        }
        dell[k] = sum;
    }
}

/* Clenshaw-Curtis weights of the Chebyshev extrema on [-1, 1] (sum = 2). */
void oracle_cc_weights(int p, double *wcc)
{
    for (int k = 0; k <= p; ++k) {
        double s = 0.0;
        for (int j = 1; j <= p / 2; ++j) {
            double b = (2 * j == p) ? 1.0 : 2.0;
            s += b / (4.0 * j * j - 1.0) * cos(2.0 * M_PI * j * k / p);
        }
        double c = (k == 0 || k == p) ? 1.0 : 2.0;
        wcc[k] = c / p * (1.0 - s);
    }
}

/* position of unique node g (= e*p + l) along an axis of equal cells */
static double node_pos(int g, int p, double h)
{
    int e = g / p, l = g % p;
    return e * h + h * 0.5 * (1.0 - cos(M_PI * (double)l / (double)p));
}

/* Graded meshes (cells of unequal width along an axis, still periodic and
 * axis-aligned): the GLC points of cell e are mapped onto [F_e, F_{e+1}]. */
static double face_of(const oracle_cfg *c, int a, int e)
{
    return c->faces[a] ? c->faces[a][e] : e * (c->length[a] / c->n_el[a]);
}

/* width of cell e along axis a (L / n_el on equal cells) */
static double cell_width(const oracle_cfg *c, int a, int e)
{
    return c->faces[a] ? c->faces[a][e + 1] - c->faces[a][e] : c->length[a] / c->n_el[a];
}

static double axis_node_pos(const oracle_cfg *c, int a, int g)
{
    int p = c->p;
    if (!c->faces[a]) return node_pos(g, p, c->length[a] / c->n_el[a]);
    int e = g / p, l = g % p;
    double F0 = face_of(c, a, e), F1 = face_of(c, a, e + 1);
    return F0 + (F1 - F0) * 0.5 * (1.0 - cos(M_PI * (double)l / (double)p));
}

/* Departure cell of node g along axis a for the displacement -shift: first
 * source node index base = E*p and local coordinate t in [0,1).  Equal
 * cells: floor(X/h).  Graded cells: X wrapped into [0, L), then the cell
 * whose faces enclose it (bisection over the faces). */
static void departure_cell(const oracle_cfg *c, int a, int g, double shift, int *base, double *t)
{
    int p = c->p, ne = c->n_el[a];
    if (!c->faces[a]) {
        double h = c->length[a] / ne;
        double X = node_pos(g, p, h) - shift;
        double s = X / h;
        double E = floor(s);
        long Ei = (long)E % ne;
        if (Ei < 0) Ei += ne;
        *base = (int)(Ei * p);
        *t = s - E;
        return;
    }
    double L = c->length[a];
    double X = axis_node_pos(c, a, g) - shift;
    X -= L * floor(X / L);
    if (X >= L) X = 0.0;                      /* rounding of the wrap */
    int lo = 0, hi = ne;                       /* faces[lo] <= X < faces[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (c->faces[a][mid] <= X) lo = mid; else hi = mid;
    }
    double F0 = c->faces[a][lo], F1 = c->faces[a][lo + 1];
    *base = lo * p;
    *t = (X - F0) / (F1 - F0);
}

void oracle_node_coords(const oracle_cfg *c, double *x, double *y, double *z)
{
    double *out[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        int n = c->n_el[a] * c->p;
        for (int g = 0; g < n; ++g) out[a][g] = axis_node_pos(c, a, g);
    }
}

/* ------------------------------------------------------------------------- */
/* Distorted meshes.  Node g of the equal-cell grid moves by the periodic    */
/* displacement d(g); every cell becomes the image of its reference cube     */
/* under the degree-p interpolant of its nodes' positions (isoparametric).   */
/* Since the GLC positions interpolate the identity, the cell map is         */
/* r -> r + D(r), D the cell-wise tensor interpolant of d.  Populations are  */
/* interpolated in reference coordinates, so the departure point            */
/* x_node + d_node - xi dt is located by solving r + D(r) = x_d (Newton, the */
/* cell re-chosen from r at every iteration; periodic in r).                 */
/* ------------------------------------------------------------------------- */

/* D and I + dD/dr at local coordinates t of cell e (wrapped cell indices) */
static void disp_cell(const oracle_cfg *c, const int *e, const double *t, double *D, double J[3][3])
{
    int p = c->p;
    int N[3];
    double h[3], ell[3][16], dl[3][16];
    for (int a = 0; a < 3; ++a) {
        N[a] = c->n_el[a] * p;
        h[a] = c->length[a] / c->n_el[a];
        oracle_lagrange(p, t[a], ell[a]);
        oracle_lagrange_deriv(p, t[a], dl[a]);
    }
    long Nl = (long)N[0] * N[1] * N[2];
    for (int a = 0; a < 3; ++a) {
        D[a] = 0.0;
        for (int b = 0; b < 3; ++b) J[a][b] = (a == b) ? 1.0 : 0.0;
    }
    if (!c->disp) return;                     /* undistorted: D = 0, J = I */
    for (int kz = 0; kz <= p; ++kz)
        for (int ky = 0; ky <= p; ++ky)
            for (int kx = 0; kx <= p; ++kx) {
                long node = ((long)((e[2] * p + kz) % N[2]) * N[1] + (e[1] * p + ky) % N[1]) * N[0]
                          + (e[0] * p + kx) % N[0];
                double v = ell[0][kx] * ell[1][ky] * ell[2][kz];
                double gx = dl[0][kx] * ell[1][ky] * ell[2][kz] / h[0];
                double gy = ell[0][kx] * dl[1][ky] * ell[2][kz] / h[1];
                double gz = ell[0][kx] * ell[1][ky] * dl[2][kz] / h[2];
                for (int a = 0; a < 3; ++a) {
                    double d = c->disp[(long)a * Nl + node];
                    D[a] += v * d;
                    J[a][0] += gx * d;
                    J[a][1] += gy * d;
                    J[a][2] += gz * d;
                }
            }
}

/* the same at reference point r (unwrapped): the cell is floor(r/h) */
static void disp_field(const oracle_cfg *c, const double *r, double *D, double J[3][3])
{
    int e[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double h = c->length[a] / c->n_el[a];
        double s = r[a] / h;
        double E = floor(s);
        t[a] = s - E;
        long Ei = (long)E % c->n_el[a];
        if (Ei < 0) Ei += c->n_el[a];
        e[a] = (int)Ei;
    }
    disp_cell(c, e, t, D, J);
}

static double det3(double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* reference point of the departure of node (gx, gy, gz) for displacement
 * -shift: cell base node per axis (wrapped) and local coordinates */
static void mapped_departure(const oracle_cfg *c, int gx, int gy, int gz, const double *shift, int *base,
                             double *t)
{
    int p = c->p;
    int N[3] = {c->n_el[0] * p, c->n_el[1] * p, c->n_el[2] * p};
    long Nl = (long)N[0] * N[1] * N[2];
    long n = ((long)gz * N[1] + gy) * N[0] + gx;
    int gi[3] = {gx, gy, gz};
    double xd[3], r[3];
    for (int a = 0; a < 3; ++a) {
        double r0 = node_pos(gi[a], p, c->length[a] / c->n_el[a]);
        xd[a] = r0 + c->disp[(long)a * Nl + n] - shift[a];
        r[a] = r0 - shift[a];                         /* start: the undistorted departure */
    }
    for (int it = 0; it < 100; ++it) {
        double D[3], J[3][3], F[3];
        disp_field(c, r, D, J);
        for (int a = 0; a < 3; ++a) F[a] = r[a] + D[a] - xd[a];
        /* r -= J^-1 F by Cramer's rule */
        double dt = det3(J), dr[3];
        for (int k = 0; k < 3; ++k) {
            double M[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) M[a][b] = (b == k) ? F[a] : J[a][b];
            dr[k] = det3(M) / dt;
        }
        double sz = 0.0;
        for (int a = 0; a < 3; ++a) {
            r[a] -= dr[a];
            sz += fabs(dr[a]) / (c->length[a] / c->n_el[a]);
        }
        if (sz < 1e-15) break;
    }
    for (int a = 0; a < 3; ++a) {
        double h = c->length[a] / c->n_el[a];
        double s = r[a] / h;
        double E = floor(s);
        long Ei = (long)E % c->n_el[a];
        if (Ei < 0) Ei += c->n_el[a];
        base[a] = (int)(Ei * p);
        t[a] = s - E;
    }
}

/* J = I + dD/dr of cell e at its support point k3, its inverse and |det J|
 * (J = I, |det J| = 1 on undistorted meshes). */
static void cell_point_jacobian(const oracle_cfg *c, const int *e, const int *k3, double Ji[3][3], double *adet)
{
    double tg[16], t[3], D[3], J[3][3];
    oracle_glc_nodes(c->p, tg);
    for (int a = 0; a < 3; ++a) t[a] = tg[k3[a]];
    disp_cell(c, e, t, D, J);
    double dt = det3(J);
    /* inverse by cofactors: Ji[a][b] = cof(J)[b][a] / det J */
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / dt;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / dt;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / dt;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / dt;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / dt;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / dt;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / dt;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / dt;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / dt;
    *adet = fabs(dt);
}

/* Domain integral weights of a distorted mesh: per node, the sum over the
 * cells that hold it of the tensor Clenshaw-Curtis weight of its local point
 * times |det(I + dD/dr)| of that cell there.  w: [N]. */
void oracle_mapped_node_weights(const oracle_cfg *c, double *w)
{
    int p = c->p;
    int N[3] = {c->n_el[0] * p, c->n_el[1] * p, c->n_el[2] * p};
    long Nl = (long)N[0] * N[1] * N[2];
    double wcc[16], tg[16];
    oracle_cc_weights(p, wcc);
    oracle_glc_nodes(p, tg);
    for (long n = 0; n < Nl; ++n) w[n] = 0.0;
    double h[3] = {c->length[0] / c->n_el[0], c->length[1] / c->n_el[1], c->length[2] / c->n_el[2]};
    for (int ez = 0; ez < c->n_el[2]; ++ez)
        for (int ey = 0; ey < c->n_el[1]; ++ey)
            for (int ex = 0; ex < c->n_el[0]; ++ex)
                for (int kz = 0; kz <= p; ++kz)
                    for (int ky = 0; ky <= p; ++ky)
                        for (int kx = 0; kx <= p; ++kx) {
                            /* the derivative of this cell's map at its point */
                            double t[3] = {tg[kx], tg[ky], tg[kz]};
                            int e[3] = {ex, ey, ez};
                            double D[3], J[3][3];
                            disp_cell(c, e, t, D, J);
                            double W = 0.125 * h[0] * h[1] * h[2] * wcc[kx] * wcc[ky] * wcc[kz];
                            long node = ((long)((ez * p + kz) % N[2]) * N[1] + (ey * p + ky) % N[1]) * N[0]
                                      + (ex * p + kx) % N[0];
                            w[node] += W * fabs(det3(J));
                        }
}

/* ------------------------------------------------------------------------- */
/* Hermite tensors (App. B) and equilibrium moments (App. A).                */
/* Full tensors of rank n, stored flat over 3^n components.                  */
/* ------------------------------------------------------------------------- */

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* H^(n)(xi) for n = 0..4 at one abscissa (c_s = 1). */
static void hermite_tensors(const double *x, double *H1, double *H2, double *H3, double *H4)
{
    for (int a = 0; a < 3; ++a) {
        H1[a] = x[a];
        for (int b = 0; b < 3; ++b) {
            H2[3 * a + b] = x[a] * x[b] - kd(a, b);
            for (int c = 0; c < 3; ++c) {
                H3[9 * a + 3 * b + c] = x[a] * x[b] * x[c]
                    - (x[a] * kd(b, c) + x[b] * kd(a, c) + x[c] * kd(a, b));
                for (int d = 0; d < 3; ++d) {
                    double Tsum = x[a] * x[b] * kd(c, d) + x[a] * x[c] * kd(b, d) + x[a] * x[d] * kd(b, c)
                                + x[b] * x[c] * kd(a, d) + x[b] * x[d] * kd(a, c) + x[c] * x[d] * kd(a, b);
                    double dd = kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c);
                    H4[27 * a + 9 * b + 3 * c + d] = x[a] * x[b] * x[c] * x[d] - Tsum + dd;
                }
            }
        }
    }
}

/* a^(n)_eq for n = 0..4 (App. A, T0 = 1, theta - 1 = T - 1). */
static void eq_moments(R rho, const R *u, R T, R *a0, R *a1, R *a2, R *a3, R *a4)
{
    R th = T - 1.0;
    *a0 = rho;
    for (int a = 0; a < 3; ++a) {
        a1[a] = rho * u[a];
        for (int b = 0; b < 3; ++b) {
            a2[3 * a + b] = rho * (u[a] * u[b] + th * kd(a, b));
            for (int c = 0; c < 3; ++c) {
                a3[9 * a + 3 * b + c] = rho * (u[a] * u[b] * u[c]
                    + th * (kd(a, b) * u[c] + kd(a, c) * u[b] + kd(b, c) * u[a]));
                for (int d = 0; d < 3; ++d) {
                    R dd = kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c);
                    R du = kd(a, b) * u[c] * u[d] + kd(a, c) * u[b] * u[d] + kd(a, d) * u[b] * u[c]
                         + kd(b, c) * u[a] * u[d] + kd(b, d) * u[a] * u[c] + kd(c, d) * u[a] * u[b];
                    a4[27 * a + 9 * b + 3 * c + d] = rho * (u[a] * u[b] * u[c] * u[d] + th * (dd * th + du));
                }
            }
        }
    }
}

/* f_i^eq = w_i sum_{n<=4} (1/n!) a^(n)_eq : H^(n)_i   (Eq. (6)), all 3^n terms. */
void FN(equilibrium)(R rho, const R *u, R T, R *feq)
{
    double xi[3 * Q], w[Q];
    oracle_velocity_set(xi, w);
    R a0, a1[3], a2[9], a3[27], a4[81];
    eq_moments(rho, u, T, &a0, a1, a2, a3, a4);
    for (int i = 0; i < Q; ++i) {
        double H1[3], H2[9], H3[27], H4[81];
        hermite_tensors(&xi[3 * i], H1, H2, H3, H4);
        R s0 = a0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
        for (int m = 0; m < 3; ++m) s1 += a1[m] * H1[m];
        for (int m = 0; m < 9; ++m) s2 += a2[m] * H2[m];
        for (int m = 0; m < 27; ++m) s3 += a3[m] * H3[m];
        for (int m = 0; m < 81; ++m) s4 += a4[m] * H4[m];
        feq[i] = w[i] * (s0 + s1 + s2 / 2.0 + s3 / 6.0 + s4 / 24.0);
    }
}

/* ------------------------------------------------------------------------- */
/* Collision (Eq. (5) with the quasi-equilibrium extension of App. D).       */
/* f, g: the 45 populations of one node.                                     */
/* ------------------------------------------------------------------------- */

static R mu_of_T(const oracle_cfg *c, R T)
{
    R mu_inf = c->mu_inf;
#ifdef ORACLE_COMPLEX
    mu_inf += c->mu_inf_im * I;
#endif
    if (c->viscosity_law == 1) return mu_inf;
    const double S = 0.40417;                       /* Sutherland law, Sec. III C */
    return mu_inf * (1.0 + S) * T * RSQRT(T) / (T + S);
}

/* Density, velocity, temperature from Eq. (7) (T0 = 1, R = 1). */
static void node_macro(const oracle_cfg *c, const double *xi, const R *f, const R *g,
                       R *rho, R *u, R *T)
{
    double Cv = 1.0 / (c->gamma - 1.0);
    R r = 0, j[3] = {0, 0, 0}, twoE = 0;
    for (int i = 0; i < Q; ++i) {
        const double *x = &xi[3 * i];
        double x2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        r += f[i];
        for (int a = 0; a < 3; ++a) j[a] += f[i] * x[a];
        twoE += f[i] * x2 + g[i];
    }
    R uu = 0;
    for (int a = 0; a < 3; ++a) { u[a] = j[a] / r; uu += u[a] * u[a]; }
    *rho = r;
    *T = (twoE / r - uu) / (2.0 * Cv);
}

/* centred third moment  Q_abc = sum_i h_i (xi_i - u)_a (xi_i - u)_b (xi_i - u)_c */
static void centred_third(const double *xi, const R *h, const R *u, R *Qt)
{
    for (int m = 0; m < 27; ++m) Qt[m] = 0;
    for (int i = 0; i < Q; ++i) {
        R d[3];
        for (int a = 0; a < 3; ++a) d[a] = xi[3 * i + a] - u[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int cc = 0; cc < 3; ++cc) Qt[9 * a + 3 * b + cc] += h[i] * d[a] * d[b] * d[cc];
    }
}

void FN(collide_node)(const oracle_cfg *c, const R *f, const R *g, R *fo, R *go)
{
    double xi[3 * Q], w[Q];
    oracle_velocity_set(xi, w);
    double Cv = 1.0 / (c->gamma - 1.0);
    R rho, u[3], T;
    node_macro(c, xi, f, g, &rho, u, &T);
    R P = rho * T;                                         /* P = rho T */
    R mu = mu_of_T(c, T);
    R tau = mu / (P * c->dt) + 0.5;                        /* tau = mu/(P c_s dt) + 1/2 */
    R tau_pr = (tau - 0.5) / c->prandtl + 0.5;             /* App. D */

    R feq[Q], geq[Q];
    FN(equilibrium)(rho, u, T, feq);
    for (int i = 0; i < Q; ++i) geq[i] = (2.0 * Cv - DIM) * T * feq[i];

    R Qf[27], Qfeq[27], Qg[27], Qgeq[27];
    centred_third(xi, f, u, Qf);
    centred_third(xi, feq, u, Qfeq);
    centred_third(xi, g, u, Qg);
    centred_third(xi, geq, u, Qgeq);

    for (int i = 0; i < Q; ++i) {
        double H1[3], H2[9], H3[27], H4[81];
        hermite_tensors(&xi[3 * i], H1, H2, H3, H4);
        R fs = 0, gs = 0;
        for (int m = 0; m < 27; ++m) {
            fs += (Qf[m] - Qfeq[m]) * H3[m];
            gs += (Qg[m] - Qgeq[m]) * H3[m];
        }
        fs *= w[i] / 6.0;
        gs *= w[i] / 6.0;
        fo[i] = f[i] - (f[i] - feq[i]) / tau + (1.0 / tau - 1.0 / tau_pr) * fs;
        go[i] = g[i] - (g[i] - geq[i]) / tau + (1.0 / tau - 1.0 / tau_pr) * gs;
    }
}

/* ------------------------------------------------------------------------- */
/* Whole-grid operations.  Populations are stored [45][N] with the node      */
/* index (gz * Ny + gy) * Nx + gx (x fastest).                               */
/* ------------------------------------------------------------------------- */

static long n_nodes(const oracle_cfg *c)
{
    return (long)c->n_el[0] * c->p * (long)c->n_el[1] * c->p * (long)c->n_el[2] * c->p;
}

long oracle_num_nodes(const oracle_cfg *c) { return n_nodes(c); }

void FN(init_equilibrium)(const oracle_cfg *c, const R *rho, const R *u, const R *T, R *f, R *g)
{
    long N = n_nodes(c);
    double Cv = 1.0 / (c->gamma - 1.0);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        R uu[3] = {u[n], u[N + n], u[2 * N + n]};
        R feq[Q];
        FN(equilibrium)(rho[n], uu, T[n], feq);
        for (int i = 0; i < Q; ++i) {
            f[(long)i * N + n] = feq[i];
            g[(long)i * N + n] = (2.0 * Cv - DIM) * T[n] * feq[i];
        }
    }
}

void FN(collide)(const oracle_cfg *c, R *f, R *g)
{
    long N = n_nodes(c);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        R fn[Q], gn[Q], fo[Q], go[Q];
        for (int i = 0; i < Q; ++i) { fn[i] = f[(long)i * N + n]; gn[i] = g[(long)i * N + n]; }
        FN(collide_node)(c, fn, gn, fo, go);
        for (int i = 0; i < Q; ++i) { f[(long)i * N + n] = fo[i]; g[(long)i * N + n] = go[i]; }
    }
}

/* Value of population i at the departure point of node (gx, gy, gz):
 * enclosing cell per axis, then the (p+1)^3 tensor Lagrange sum over it. */
static void departure_value(const oracle_cfg *c, const double *xi, int i, int gx, int gy, int gz,
                            const R *f, const R *g, R *fv, R *gv)
{
    int p = c->p;
    int N[3], base[3];
    double ell[3][16];
    int gidx[3] = {gx, gy, gz};
    for (int a = 0; a < 3; ++a) {
        N[a] = c->n_el[a] * p;
        double t;                                                    /* local coordinate in [0,1) */
        departure_cell(c, a, gidx[a], xi[3 * i + a] * c->dt, &base[a], &t);
        oracle_lagrange(p, t, ell[a]);
    }
    long Nl = (long)N[0] * N[1] * N[2];
    R sf = 0, sg = 0;
    for (int kz = 0; kz <= p; ++kz) {
        int zz = (base[2] + kz) % N[2];
        for (int ky = 0; ky <= p; ++ky) {
            int yy = (base[1] + ky) % N[1];
            for (int kx = 0; kx <= p; ++kx) {
                int xx = (base[0] + kx) % N[0];
                double psi = ell[0][kx] * ell[1][ky] * ell[2][kz];
                long src = (long)i * Nl + ((long)zz * N[1] + yy) * N[0] + xx;
                sf += psi * f[src];
                sg += psi * g[src];
            }
        }
    }
    *fv = sf;
    *gv = sg;
}

static void mapped_departure(const oracle_cfg *c, int gx, int gy, int gz, const double *shift, int *base,
                             double *t);

void FN(stream)(const oracle_cfg *c, const R *f, const R *g, R *fo, R *go)
{
    double xi[3 * Q], w[Q];
    oracle_velocity_set(xi, w);
    if (c->disp) {
        /* distorted mesh: departure cell and reference coordinates by Newton
         * on the cell maps, then the same (p+1)^3 tensor Lagrange sum */
        int p = c->p;
        int N[3] = {c->n_el[0] * p, c->n_el[1] * p, c->n_el[2] * p};
        long Nl = (long)N[0] * N[1] * N[2];
#pragma omp parallel for collapse(2) schedule(dynamic)
        for (int i = 0; i < Q; ++i) {
            for (long n = 0; n < Nl; ++n) {
                int gx = (int)(n % N[0]), gy = (int)((n / N[0]) % N[1]), gz = (int)(n / ((long)N[0] * N[1]));
                double sh[3] = {xi[3 * i] * c->dt, xi[3 * i + 1] * c->dt, xi[3 * i + 2] * c->dt};
                int base[3];
                double t[3], ell[3][16];
                mapped_departure(c, gx, gy, gz, sh, base, t);
                for (int a = 0; a < 3; ++a) oracle_lagrange(p, t[a], ell[a]);
                R sf = 0, sg = 0;
                for (int kz = 0; kz <= p; ++kz)
                    for (int ky = 0; ky <= p; ++ky)
                        for (int kx = 0; kx <= p; ++kx) {
                            long src = (long)i * Nl + ((long)((base[2] + kz) % N[2]) * N[1] + (base[1] + ky) % N[1])
                                     * N[0] + (base[0] + kx) % N[0];
                            double psi = ell[0][kx] * ell[1][ky] * ell[2][kz];
                            sf += psi * f[src];
                            sg += psi * g[src];
                        }
                fo[(long)i * Nl + n] = sf;
                go[(long)i * Nl + n] = sg;
            }
        }
        return;
    }
    int Nx = c->n_el[0] * c->p, Ny = c->n_el[1] * c->p, Nz = c->n_el[2] * c->p;
    long N = n_nodes(c);
#pragma omp parallel for collapse(2) schedule(static)
    for (int i = 0; i < Q; ++i) {
        for (int gz = 0; gz < Nz; ++gz) {
            for (int gy = 0; gy < Ny; ++gy) {
                for (int gx = 0; gx < Nx; ++gx) {
                    long n = ((long)gz * Ny + gy) * Nx + gx;
                    departure_value(c, xi, i, gx, gy, gz, f, g, &fo[(long)i * N + n], &go[(long)i * N + n]);
                }
            }
        }
    }
}

/* n time steps of Eq. (5): collide, then stream (state = pre-collision populations). */
int FN(step)(const oracle_cfg *c, R *f, R *g, int nsteps)
{
    long N = n_nodes(c);
    R *tf = (R *)malloc(sizeof(R) * Q * N);
    R *tg = (R *)malloc(sizeof(R) * Q * N);
    if (!tf || !tg) { free(tf); free(tg); return -1; }
    for (int s = 0; s < nsteps; ++s) {
        FN(collide)(c, f, g);
        FN(stream)(c, f, g, tf, tg);
        memcpy(f, tf, sizeof(R) * Q * N);
        memcpy(g, tg, sizeof(R) * Q * N);
    }
    free(tf);
    free(tg);
    return 0;
}

/* One step evaluated only at the listed nodes: out[45] f then out[45] g per
 * sample.  Every source point of every departure stencil is collided from
 * the full pre-collision state, exactly as the whole-grid step would. */
void FN(step_at_nodes)(const oracle_cfg *c, const R *f, const R *g, int nsamp, const long *nodes,
                       R *fo, R *go)
{
    double xi[3 * Q], w[Q];
    oracle_velocity_set(xi, w);
    int p = c->p;
    int N[3] = {c->n_el[0] * p, c->n_el[1] * p, c->n_el[2] * p};
    long Nl = (long)N[0] * N[1] * N[2];
#pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < nsamp; ++s) {
        long n = nodes[s];
        int gidx[3] = {(int)(n % N[0]), (int)((n / N[0]) % N[1]), (int)(n / ((long)N[0] * N[1]))};
        for (int i = 0; i < Q; ++i) {
            int base[3];
            double ell[3][16];
            for (int a = 0; a < 3; ++a) {
                double t;
                departure_cell(c, a, gidx[a], xi[3 * i + a] * c->dt, &base[a], &t);
                oracle_lagrange(p, t, ell[a]);
            }
            R sf = 0, sg = 0;
            for (int kz = 0; kz <= p; ++kz)
                for (int ky = 0; ky <= p; ++ky)
                    for (int kx = 0; kx <= p; ++kx) {
                        long src = ((long)((base[2] + kz) % N[2]) * N[1] + (base[1] + ky) % N[1]) * N[0]
                                 + (base[0] + kx) % N[0];
                        R fn[Q], gn[Q], fc[Q], gc[Q];
                        for (int j = 0; j < Q; ++j) { fn[j] = f[(long)j * Nl + src]; gn[j] = g[(long)j * Nl + src]; }
                        FN(collide_node)(c, fn, gn, fc, gc);
                        double psi = ell[0][kx] * ell[1][ky] * ell[2][kz];
                        sf += psi * fc[i];
                        sg += psi * gc[i];
                    }
            fo[(long)s * Q + i] = sf;
            go[(long)s * Q + i] = sg;
        }
    }
}

/* Streaming only (Eq. (9)), evaluated at the listed nodes of an equal-cell
 * or graded mesh: the whole-grid stream restricted to those nodes, the same
 * direct (p+1)^3 gather per node and velocity.  out[45] f then out[45] g per
 * sample. */
void FN(stream_at_nodes)(const oracle_cfg *c, const R *f, const R *g, int nsamp, const long *nodes,
                         R *fo, R *go)
{
    double xi[3 * Q], w[Q];
    oracle_velocity_set(xi, w);
    int N[3] = {c->n_el[0] * c->p, c->n_el[1] * c->p, c->n_el[2] * c->p};
#pragma omp parallel for schedule(static)
    for (int s = 0; s < nsamp; ++s) {
        long n = nodes[s];
        int gx = (int)(n % N[0]), gy = (int)((n / N[0]) % N[1]), gz = (int)(n / ((long)N[0] * N[1]));
        for (int i = 0; i < Q; ++i)
            departure_value(c, xi, i, gx, gy, gz, f, g, &fo[(long)s * Q + i], &go[(long)s * Q + i]);
    }
}

/* rho, u (stored [3][N]) and T at every node, Eq. (7). */
void FN(moments)(const oracle_cfg *c, const R *f, const R *g, R *rho, R *u, R *T)
{
    double xi[3 * Q], w[Q];
    oracle_velocity_set(xi, w);
    long N = n_nodes(c);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        R fn[Q], gn[Q], uu[3];
        for (int i = 0; i < Q; ++i) { fn[i] = f[(long)i * N + n]; gn[i] = g[(long)i * N + n]; }
        node_macro(c, xi, fn, gn, &rho[n], uu, &T[n]);
        for (int a = 0; a < 3; ++a) u[(long)a * N + n] = uu[a];
    }
}

/* Quadrature weight of unique node g along axis a: Clenshaw-Curtis weight of
 * its local point, mapped to its cell; cell end points are shared by two
 * cells (the previous one, periodically), so their weights add. */
static double node_weight(const oracle_cfg *c, int a, int g)
{
    double wcc[16];
    int p = c->p, ne = c->n_el[a];
    oracle_cc_weights(p, wcc);
    int e = g / p, l = g % p;
    double h = face_of(c, a, e + 1) - face_of(c, a, e);
    if (l != 0) return 0.5 * h * wcc[l];
    int ep = (e + ne - 1) % ne;
    double hp = face_of(c, a, ep + 1) - face_of(c, a, ep);
    return 0.5 * (h * wcc[0] + hp * wcc[p]);
}

/* Domain integrals of rho, rho u (3) and rho E (Eq. (7)), summed in node order. */
void FN(totals)(const oracle_cfg *c, const R *f, const R *g, R *out)
{
    double xi[3 * Q], w[Q];
    oracle_velocity_set(xi, w);
    int p = c->p;
    int Nx = c->n_el[0] * p, Ny = c->n_el[1] * p, Nz = c->n_el[2] * p;
    long N = n_nodes(c);
    for (int k = 0; k < 5; ++k) out[k] = 0;
    double *mw = NULL;                       /* distorted mesh: per-node weights */
    if (c->disp) {
        mw = (double *)malloc(sizeof(double) * N);
        oracle_mapped_node_weights(c, mw);
    }
    for (int gz = 0; gz < Nz; ++gz)
        for (int gy = 0; gy < Ny; ++gy)
            for (int gx = 0; gx < Nx; ++gx) {
                long n = ((long)gz * Ny + gy) * Nx + gx;
                double W = mw ? mw[n] : node_weight(c, 0, gx) * node_weight(c, 1, gy) * node_weight(c, 2, gz);
                R r = 0, j[3] = {0, 0, 0}, twoE = 0;
                for (int i = 0; i < Q; ++i) {
                    R fi = f[(long)i * N + n];
                    const double *x = &xi[3 * i];
                    r += fi;
                    for (int a = 0; a < 3; ++a) j[a] += fi * x[a];
                    twoE += fi * (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) + g[(long)i * N + n];
                }
                out[0] += W * r;
                for (int a = 0; a < 3; ++a) out[1 + a] += W * j[a];
                out[4] += W * 0.5 * twoE;
            }
    free(mw);
}

/* Flow functional used for gradients:
 *   L = sum over cells of the tensor Clenshaw-Curtis quadrature of
 *       (1/2) rho |u|^2 + (div u)^2,
 * with div u from the derivative of each cell's own interpolation polynomial
 * (so it is discontinuous across cell faces, as in Sec. III C); on a graded
 * mesh each cell uses its own width; on a distorted mesh the derivatives are
 * taken in physical coordinates through the cell map (d u/d x = (d u/d r)
 * J^-1, J = I + dD/dr) and every quadrature weight carries |det J|. */
R FN(loss)(const oracle_cfg *c, const R *f, const R *g)
{
    int p = c->p;
    int N[3] = {c->n_el[0] * p, c->n_el[1] * p, c->n_el[2] * p};
    long Nl = (long)N[0] * N[1] * N[2];
    R *rho = (R *)malloc(sizeof(R) * Nl), *u = (R *)malloc(sizeof(R) * 3 * Nl), *T = (R *)malloc(sizeof(R) * Nl);
    FN(moments)(c, f, g, rho, u, T);
    double t[16], wcc[16], Dm[16][16];
    oracle_glc_nodes(p, t);
    oracle_cc_weights(p, wcc);
    for (int k = 0; k <= p; ++k) {
        double dl[16];
        oracle_lagrange_deriv(p, t[k], dl);
        for (int m = 0; m <= p; ++m) Dm[k][m] = dl[m];     /* d l_m / ds at s = t_k */
    }
    R L = 0;
    for (int ez = 0; ez < c->n_el[2]; ++ez)
        for (int ey = 0; ey < c->n_el[1]; ++ey)
            for (int ex = 0; ex < c->n_el[0]; ++ex) {
                double h[3] = {cell_width(c, 0, ex), cell_width(c, 1, ey), cell_width(c, 2, ez)};
                for (int kz = 0; kz <= p; ++kz)
                    for (int ky = 0; ky <= p; ++ky)
                        for (int kx = 0; kx <= p; ++kx) {
                            int k3[3] = {kx, ky, kz}, e3[3] = {ex, ey, ez};
                            long n = ((long)((ez * p + kz) % N[2]) * N[1] + (ey * p + ky) % N[1]) * N[0]
                                   + (ex * p + kx) % N[0];
                            /* reference gradient d u_a / d r_b inside this cell, then the
                             * physical one through the cell map: d u / d x = (d u / d r) J^-1 */
                            R gr[3][3];
                            for (int a = 0; a < 3; ++a)
                                for (int b = 0; b < 3; ++b) {
                                    R d = 0;
                                    for (int m = 0; m <= p; ++m) {
                                        int gg[3] = {e3[0] * p + k3[0], e3[1] * p + k3[1], e3[2] * p + k3[2]};
                                        gg[b] = e3[b] * p + m;
                                        long nm = ((long)(gg[2] % N[2]) * N[1] + gg[1] % N[1]) * N[0] + gg[0] % N[0];
                                        d += Dm[k3[b]][m] * u[(long)a * Nl + nm];
                                    }
                                    gr[a][b] = d / h[b];
                                }
                            double Ji[3][3], adet;
                            cell_point_jacobian(c, e3, k3, Ji, &adet);
                            R div = 0;
                            for (int a = 0; a < 3; ++a)
                                for (int b = 0; b < 3; ++b) div += gr[a][b] * Ji[b][a];
                            R ke = 0;
                            for (int a = 0; a < 3; ++a) ke += u[(long)a * Nl + n] * u[(long)a * Nl + n];
                            double W = (0.5 * h[0] * wcc[kx]) * (0.5 * h[1] * wcc[ky]) * (0.5 * h[2] * wcc[kz]) * adet;
                            L += W * (0.5 * rho[n] * ke + div * div);
                        }
            }
    free(rho); free(u); free(T);
    return L;
}

/* TGV diagnostics of Sec. III C, as domain integrals over the cells with the
 * tensor Clenshaw-Curtis rule of each cell's support points and derivatives
 * of each cell's own interpolation polynomial:
 *   out[0] = kinetic energy        int (1/2) rho |u|^2
 *   out[1] = solenoidal dissipation int mu(T) |curl u|^2
 *   out[2] = dilatational dissipation (4/3) int mu(T) (div u)^2
 * (the paper's 1/(rho_ref Re) prefactor is the mu_inf inside mu(T)); on a
 * graded mesh each cell uses its own width; on a distorted mesh derivatives
 * and weights go through the cell map as in FN(loss). */
void FN(diagnostics)(const oracle_cfg *c, const R *f, const R *g, R *out)
{
    int p = c->p;
    int N[3] = {c->n_el[0] * p, c->n_el[1] * p, c->n_el[2] * p};
    long Nl = (long)N[0] * N[1] * N[2];
    R *rho = (R *)malloc(sizeof(R) * Nl), *u = (R *)malloc(sizeof(R) * 3 * Nl), *T = (R *)malloc(sizeof(R) * Nl);
    FN(moments)(c, f, g, rho, u, T);
    double t[16], wcc[16], Dm[16][16];
    oracle_glc_nodes(p, t);
    oracle_cc_weights(p, wcc);
    for (int k = 0; k <= p; ++k) {
        double dl[16];
        oracle_lagrange_deriv(p, t[k], dl);
        for (int m = 0; m <= p; ++m) Dm[k][m] = dl[m];
    }
    R ek = 0, es = 0, ec = 0;
    for (int ez = 0; ez < c->n_el[2]; ++ez)
        for (int ey = 0; ey < c->n_el[1]; ++ey)
            for (int ex = 0; ex < c->n_el[0]; ++ex) {
                double h[3] = {cell_width(c, 0, ex), cell_width(c, 1, ey), cell_width(c, 2, ez)};
                for (int kz = 0; kz <= p; ++kz)
                    for (int ky = 0; ky <= p; ++ky)
                        for (int kx = 0; kx <= p; ++kx) {
                            int k3[3] = {kx, ky, kz}, e3[3] = {ex, ey, ez};
                            long n = ((long)((ez * p + kz) % N[2]) * N[1] + (ey * p + ky) % N[1]) * N[0]
                                   + (ex * p + kx) % N[0];
                            R gr[3][3];               /* gr[a][b] = d u_a / d r_b inside this cell */
                            for (int a = 0; a < 3; ++a)
                                for (int b = 0; b < 3; ++b) {
                                    R d = 0;
                                    for (int m = 0; m <= p; ++m) {
                                        int gg[3] = {e3[0] * p + k3[0], e3[1] * p + k3[1], e3[2] * p + k3[2]};
                                        gg[b] = e3[b] * p + m;
                                        long nm = ((long)(gg[2] % N[2]) * N[1] + gg[1] % N[1]) * N[0] + gg[0] % N[0];
                                        d += Dm[k3[b]][m] * u[(long)a * Nl + nm];
                                    }
                                    gr[a][b] = d / h[b];
                                }
                            double Ji[3][3], adet;    /* cell map: d u / d x = (d u / d r) J^-1 */
                            cell_point_jacobian(c, e3, k3, Ji, &adet);
                            R grad[3][3];             /* grad[a][b] = d u_a / d x_b */
                            for (int a = 0; a < 3; ++a)
                                for (int b = 0; b < 3; ++b)
                                    grad[a][b] = gr[a][0] * Ji[0][b] + gr[a][1] * Ji[1][b] + gr[a][2] * Ji[2][b];
                            R w0 = grad[2][1] - grad[1][2], w1 = grad[0][2] - grad[2][0], w2 = grad[1][0] - grad[0][1];
                            R div = grad[0][0] + grad[1][1] + grad[2][2];
                            R ke = 0;
                            for (int a = 0; a < 3; ++a) ke += u[(long)a * Nl + n] * u[(long)a * Nl + n];
                            R mu = mu_of_T(c, T[n]);
                            double W = (0.5 * h[0] * wcc[kx]) * (0.5 * h[1] * wcc[ky]) * (0.5 * h[2] * wcc[kz]) * adet;
                            ek += W * 0.5 * rho[n] * ke;
                            es += W * mu * (w0 * w0 + w1 * w1 + w2 * w2);
                            ec += W * (4.0 / 3.0) * mu * div * div;
                        }
            }
    out[0] = ek;
    out[1] = es;
    out[2] = ec;
    free(rho); free(u); free(T);
}

#ifdef ORACLE_COMPLEX
/* The loss is returned through a pointer in the complex build (ctypes cannot
 * return a C99 complex by value portably). */
void oracle_cs_loss_out(const oracle_cfg *c, const R *f, const R *g, R *out) { *out = oracle_cs_loss(c, f, g); }
#endif
