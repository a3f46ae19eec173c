/*
 * Plain CPU reference ("oracle") of the two-dimensional variant of the
 * compressible semi-Lagrangian lattice Boltzmann method of Wilde, Kraemer,
 * Reith & Foysi (arXiv:2012.05537): the D2Q19 velocity set of Sec. II B with
 * the collision of Eq. (5) / App. D and the streaming of Eqs. (8)-(9) on a
 * periodic mesh of equal square-ish cells (the Sod shock tube and 2-D
 * Riemann problems of Sec. III A and III B).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Everything is done the slow, literal way, in FP64:
 *   - the velocity set is solved from its moment conditions at start-up
 *     (the paper cites the 19-point degree-nine rule but does not list it);
 *   - the equilibrium is the full contraction over all 2^n components of the
 *     Hermite series up to n = 4 (Eq. (6), App. A and B with D = 2);
 *   - the quasi-equilibrium term contracts the difference of the centred
 *     third moments of h and h^eq with all 8 components of H^(3) (App. D);
 *   - streaming traces every (node, velocity) pair back to x - xi*dt, finds
 *     the enclosing cell with floor() and sums the (p+1)^2 tensor-product
 *     Lagrange basis values over that cell's support points.
 *
 * Readings of the paper taken here (beyond those of the 3-D oracle:
 * c_s = 1, T0 = 1, C_v = 1/(gamma - 1), Sutherland numerator 1 + S):
 *   D = 2, so g^eq = (2 C_v - 2) T f^eq and the Hermite traces run over two
 *   axes.
 *   Velocity set: the origin and three rings of six points with hexagonal
 *   symmetry, exact for every polynomial of degree <= 9 against the weight
 *   exp(-|xi|^2/2)/(2 pi).  Those conditions fix the rule up to a rotation by
 *   30 degrees; the rotation taken puts the largest speed on the x axis (the
 *   Sod figure of Sec. III A has the longest abscissa cross about seven cells
 *   of 1/2000 at dt = 0.001, which needs an x component of about 3.36).
 *   Velocities are ordered by speed, then lexicographically by (x, y).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q2 19

typedef struct {
    int n_el[2];          /* cells per axis */
    int p;                /* GLC order */
    double length[2];     /* domain edge lengths */
    double dt;
    double gamma;
    double prandtl;
    double mu_inf;
    int viscosity_law;    /* 0 Sutherland, 1 constant */
} oracle2d_cfg;

/* ------------------------------------------------------------------------- */
/* The D2Q19 rule.                                                           */
/*                                                                           */
/* A rule with the symmetry of the regular hexagon integrates every          */
/* polynomial exactly once it integrates the invariant ones: |x|^(2k) and    */
/* |x|^(2k) Re((x + iy)^6).  For the 2-D standard normal E|x|^(2k) = 2^k k!, */
/* and E[|x|^(2k) Re z^6] = 0.  With the origin (weight W0) and rings r of   */
/* six points at squared radius a_r and total weight W_r, Re z^6 = s_r a_r^3 */
/* on ring r, s_r = +1 for a ring with a point on the x axis and -1 for one  */
/* turned by 30 degrees.  The conditions up to degree nine:                  */
/*   sum W_r a_r^k = 2^k k!         (k = 1..4)                               */
/*   sum W_r s_r a_r^3 = 0,  sum W_r s_r a_r^4 = 0                           */
/* With one turned ring A and two rings B, C on the axes: the turned ring    */
/* carries half of the k = 3, 4 sums, W_A a_A^3 = 24, W_A a_A^4 = 192, so    */
/* a_A = 8.  B and C then form a two-point rule for the moments nu_k left    */
/* over (k = 1..4): a_B, a_C are the roots of a^2 - s a + t with             */
/* nu_{k+2} = s nu_{k+1} - t nu_k, and W_B, W_C follow from nu_1, nu_2.      */
/* ------------------------------------------------------------------------- */

static int lex_less2(const double *a, const double *b)
{
    for (int k = 0; k < 2; ++k) {
        if (fabs(a[k] - b[k]) > 1e-9) return a[k] < b[k];
    }
    return 0;
}

int oracle2d_velocity_set(double *xi, double *w)
{
    const double mom[5] = {1.0, 2.0, 8.0, 48.0, 384.0};      /* 2^k k! */
    const double aA = (mom[4] / 2.0) / (mom[3] / 2.0);       /* (W_A a^4) / (W_A a^3) */
    const double WA = (mom[3] / 2.0) / (aA * aA * aA);
    double nu[5];
    for (int k = 1; k <= 4; ++k) nu[k] = (k <= 2 ? mom[k] - WA * pow(aA, k) : mom[k] / 2.0);
    /* nu3 = s nu2 - t nu1, nu4 = s nu3 - t nu2 */
    double det = nu[2] * (-nu[2]) - (-nu[1]) * nu[3];
    double s = (nu[3] * (-nu[2]) - (-nu[1]) * nu[4]) / det;
    double t = (nu[2] * nu[4] - nu[3] * nu[3]) / det;
    double disc = sqrt(s * s - 4.0 * t);
    double aB = 0.5 * (s - disc), aC = 0.5 * (s + disc);
    /* W_B aB + W_C aC = nu1, W_B aB^2 + W_C aC^2 = nu2 */
    double WB = (nu[2] - aC * nu[1]) / (aB * (aB - aC));
    double WC = (nu[1] - WB * aB) / aC;
    double W0 = 1.0 - WA - WB - WC;
    if (!(W0 > 0 && WA > 0 && WB > 0 && WC > 0 && t > 0)) return -1;

    /* rings in order of speed: B (on the axes), A (turned), C (on the axes) */
    const double ra[3] = {aB, aA, aC}, rw[3] = {WB, WA, WC}, turn[3] = {0.0, M_PI / 6.0, 0.0};
    int q = 0;
    xi[0] = xi[1] = 0.0;
    w[q++] = W0;
    for (int r = 0; r < 3; ++r) {
        double ring[6][2];
        for (int m = 0; m < 6; ++m) {
            double phi = turn[r] + M_PI / 3.0 * m;
            ring[m][0] = sqrt(ra[r]) * cos(phi);
            ring[m][1] = sqrt(ra[r]) * sin(phi);
            /* exact zeros for the points on an axis */
            if (fabs(ring[m][0]) < 1e-14) ring[m][0] = 0.0;
            if (fabs(ring[m][1]) < 1e-14) ring[m][1] = 0.0;
        }
        for (int m = 1; m < 6; ++m) {                       /* insertion sort by (x, y) */
            double v[2] = {ring[m][0], ring[m][1]};
            int j = m - 1;
            while (j >= 0 && lex_less2(v, ring[j])) {
                ring[j + 1][0] = ring[j][0];
                ring[j + 1][1] = ring[j][1];
                --j;
            }
            ring[j + 1][0] = v[0];
            ring[j + 1][1] = v[1];
        }
        for (int m = 0; m < 6; ++m, ++q) {
            xi[2 * q] = ring[m][0];
            xi[2 * q + 1] = ring[m][1];
            w[q] = rw[r] / 6.0;
        }
    }
    return q;
}

/* ------------------------------------------------------------------------- */
/* Support points, Lagrange basis, Clenshaw-Curtis weights (Eq. (8)).        */
/* ------------------------------------------------------------------------- */

static void glc_nodes(int p, double *t)
{
    for (int k = 0; k <= p; ++k) t[k] = 0.5 * (1.0 - cos(M_PI * (double)k / (double)p));
}

static void lagrange(int p, double s, double *ell)
{
    double t[16];
    glc_nodes(p, t);
    for (int k = 0; k <= p; ++k) {
        double v = 1.0;
        for (int m = 0; m <= p; ++m)
            if (m != k) v *= (s - t[m]) / (t[k] - t[m]);
        ell[k] = v;
    }
}

/* Clenshaw-Curtis weights of the Chebyshev extrema on [-1, 1] (sum = 2). */
static void cc_weights(int p, double *wcc)
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

static double node_pos(int g, int p, double h)
{
    int e = g / p, l = g % p;
    return e * h + h * 0.5 * (1.0 - cos(M_PI * (double)l / (double)p));
}

void oracle2d_node_coords(const oracle2d_cfg *c, double *x, double *y)
{
    double *out[2] = {x, y};
    for (int a = 0; a < 2; ++a) {
        int n = c->n_el[a] * c->p;
        for (int g = 0; g < n; ++g) out[a][g] = node_pos(g, c->p, c->length[a] / c->n_el[a]);
    }
}

/* ------------------------------------------------------------------------- */
/* Hermite tensors (App. B) and equilibrium moments (App. A), D = 2.         */
/* ------------------------------------------------------------------------- */

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

static void hermite2(const double *x, double *H1, double *H2, double *H3, double *H4)
{
    for (int a = 0; a < 2; ++a) {
        H1[a] = x[a];
        for (int b = 0; b < 2; ++b) {
            H2[2 * a + b] = x[a] * x[b] - kd(a, b);
            for (int c = 0; c < 2; ++c) {
                H3[4 * a + 2 * b + c] = x[a] * x[b] * x[c] - (x[a] * kd(b, c) + x[b] * kd(a, c) + x[c] * kd(a, b));
                for (int d = 0; d < 2; ++d) {
                    double Tsum = x[a] * x[b] * kd(c, d) + x[a] * x[c] * kd(b, d) + x[a] * x[d] * kd(b, c)
                                + x[b] * x[c] * kd(a, d) + x[b] * x[d] * kd(a, c) + x[c] * x[d] * kd(a, b);
                    double dd = kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c);
                    H4[8 * a + 4 * b + 2 * c + d] = x[a] * x[b] * x[c] * x[d] - Tsum + dd;
                }
            }
        }
    }
}

/* f_i^eq = w_i sum_{n<=4} (1/n!) a^(n)_eq : H^(n)_i (Eq. (6)); the moments of
 * the Maxwellian at (rho, u, T) about T0 = 1, theta = T - 1 (App. A). */
void oracle2d_equilibrium(double rho, const double *u, double T, double *feq)
{
    double xi[2 * Q2], w[Q2];
    oracle2d_velocity_set(xi, w);
    double th = T - 1.0;
    double a1[2], a2[4], a3[8], a4[16];
    for (int a = 0; a < 2; ++a) {
        a1[a] = rho * u[a];
        for (int b = 0; b < 2; ++b) {
            a2[2 * a + b] = rho * (u[a] * u[b] + th * kd(a, b));
            for (int c = 0; c < 2; ++c) {
                a3[4 * a + 2 * b + c] = rho * (u[a] * u[b] * u[c]
                    + th * (kd(a, b) * u[c] + kd(a, c) * u[b] + kd(b, c) * u[a]));
                for (int d = 0; d < 2; ++d) {
                    double dd = kd(a, b) * kd(c, d) + kd(a, c) * kd(b, d) + kd(a, d) * kd(b, c);
                    double du = kd(a, b) * u[c] * u[d] + kd(a, c) * u[b] * u[d] + kd(a, d) * u[b] * u[c]
                              + kd(b, c) * u[a] * u[d] + kd(b, d) * u[a] * u[c] + kd(c, d) * u[a] * u[b];
                    a4[8 * a + 4 * b + 2 * c + d] = rho * (u[a] * u[b] * u[c] * u[d] + th * (dd * th + du));
                }
            }
        }
    }
    for (int i = 0; i < Q2; ++i) {
        double H1[2], H2[4], H3[8], H4[16];
        hermite2(&xi[2 * i], H1, H2, H3, H4);
        double s1 = 0, s2 = 0, s3 = 0, s4 = 0;
        for (int m = 0; m < 2; ++m) s1 += a1[m] * H1[m];
        for (int m = 0; m < 4; ++m) s2 += a2[m] * H2[m];
        for (int m = 0; m < 8; ++m) s3 += a3[m] * H3[m];
        for (int m = 0; m < 16; ++m) s4 += a4[m] * H4[m];
        feq[i] = w[i] * (rho + s1 + s2 / 2.0 + s3 / 6.0 + s4 / 24.0);
    }
}

/* ------------------------------------------------------------------------- */
/* Collision (Eq. (5) with App. D).                                          */
/* ------------------------------------------------------------------------- */

static double mu_of_T(const oracle2d_cfg *c, double T)
{
    if (c->viscosity_law == 1) return c->mu_inf;
    const double S = 0.40417;
    return c->mu_inf * (1.0 + S) * T * sqrt(T) / (T + S);
}

static void node_macro(const oracle2d_cfg *c, const double *xi, const double *f, const double *g,
                       double *rho, double *u, double *T)
{
    double Cv = 1.0 / (c->gamma - 1.0);
    double r = 0, j[2] = {0, 0}, twoE = 0;
    for (int i = 0; i < Q2; ++i) {
        const double *x = &xi[2 * i];
        r += f[i];
        j[0] += f[i] * x[0];
        j[1] += f[i] * x[1];
        twoE += f[i] * (x[0] * x[0] + x[1] * x[1]) + g[i];
    }
    u[0] = j[0] / r;
    u[1] = j[1] / r;
    *rho = r;
    *T = (twoE / r - u[0] * u[0] - u[1] * u[1]) / (2.0 * Cv);
}

static void centred_third2(const double *xi, const double *h, const double *u, double *Qt)
{
    for (int m = 0; m < 8; ++m) Qt[m] = 0;
    for (int i = 0; i < Q2; ++i) {
        double d[2] = {xi[2 * i] - u[0], xi[2 * i + 1] - u[1]};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int cc = 0; cc < 2; ++cc) Qt[4 * a + 2 * b + cc] += h[i] * d[a] * d[b] * d[cc];
    }
}

void oracle2d_collide_node(const oracle2d_cfg *c, const double *f, const double *g, double *fo, double *go)
{
    double xi[2 * Q2], w[Q2];
    oracle2d_velocity_set(xi, w);
    double Cv = 1.0 / (c->gamma - 1.0);
    double rho, u[2], T;
    node_macro(c, xi, f, g, &rho, u, &T);
    double P = rho * T;
    double tau = mu_of_T(c, T) / (P * c->dt) + 0.5;
    double tau_pr = (tau - 0.5) / c->prandtl + 0.5;
    double feq[Q2], geq[Q2];
    oracle2d_equilibrium(rho, u, T, feq);
    for (int i = 0; i < Q2; ++i) geq[i] = (2.0 * Cv - 2.0) * T * feq[i];
    double Qf[8], Qfe[8], Qg[8], Qge[8];
    centred_third2(xi, f, u, Qf);
    centred_third2(xi, feq, u, Qfe);
    centred_third2(xi, g, u, Qg);
    centred_third2(xi, geq, u, Qge);
    for (int i = 0; i < Q2; ++i) {
        double H1[2], H2[4], H3[8], H4[16];
        hermite2(&xi[2 * i], H1, H2, H3, H4);
        double fs = 0, gs = 0;
        for (int m = 0; m < 8; ++m) {
            fs += (Qf[m] - Qfe[m]) * H3[m];
            gs += (Qg[m] - Qge[m]) * H3[m];
        }
        fs *= w[i] / 6.0;
        gs *= w[i] / 6.0;
        fo[i] = f[i] - (f[i] - feq[i]) / tau + (1.0 / tau - 1.0 / tau_pr) * fs;
        go[i] = g[i] - (g[i] - geq[i]) / tau + (1.0 / tau - 1.0 / tau_pr) * gs;
    }
}

/* ------------------------------------------------------------------------- */
/* Whole-grid operations: populations [19][N], node index gy * Nx + gx.      */
/* ------------------------------------------------------------------------- */

long oracle2d_num_nodes(const oracle2d_cfg *c)
{
    return (long)c->n_el[0] * c->p * (long)c->n_el[1] * c->p;
}

void oracle2d_init_equilibrium(const oracle2d_cfg *c, const double *rho, const double *u, const double *T,
                               double *f, double *g)
{
    long N = oracle2d_num_nodes(c);
    double Cv = 1.0 / (c->gamma - 1.0);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double uu[2] = {u[n], u[N + n]};
        double feq[Q2];
        oracle2d_equilibrium(rho[n], uu, T[n], feq);
        for (int i = 0; i < Q2; ++i) {
            f[(long)i * N + n] = feq[i];
            g[(long)i * N + n] = (2.0 * Cv - 2.0) * T[n] * feq[i];
        }
    }
}

void oracle2d_collide(const oracle2d_cfg *c, double *f, double *g)
{
    long N = oracle2d_num_nodes(c);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double fn[Q2], gn[Q2], fo[Q2], go[Q2];
        for (int i = 0; i < Q2; ++i) { fn[i] = f[(long)i * N + n]; gn[i] = g[(long)i * N + n]; }
        oracle2d_collide_node(c, fn, gn, fo, go);
        for (int i = 0; i < Q2; ++i) { f[(long)i * N + n] = fo[i]; g[(long)i * N + n] = go[i]; }
    }
}

/* departure cell of node g along an axis of equal cells for the shift
 * xi*dt: first source node (wrapped) and local coordinate in [0, 1) */
static void departure_cell(int g, int p, int ne, double h, double shift, int *base, double *t)
{
    double s = (node_pos(g, p, h) - shift) / h;
    double E = floor(s);
    long Ei = (long)E % ne;
    if (Ei < 0) Ei += ne;
    *base = (int)(Ei * p);
    *t = s - E;
}

void oracle2d_stream(const oracle2d_cfg *c, const double *f, const double *g, double *fo, double *go)
{
    double xi[2 * Q2], w[Q2];
    oracle2d_velocity_set(xi, w);
    int p = c->p;
    int Nx = c->n_el[0] * p, Ny = c->n_el[1] * p;
    long N = (long)Nx * Ny;
    double h[2] = {c->length[0] / c->n_el[0], c->length[1] / c->n_el[1]};
#pragma omp parallel for collapse(2) schedule(static)
    for (int i = 0; i < Q2; ++i) {
        for (int gy = 0; gy < Ny; ++gy) {
            for (int gx = 0; gx < Nx; ++gx) {
                int bx, by;
                double tx, ty, lx[16], ly[16];
                departure_cell(gx, p, c->n_el[0], h[0], xi[2 * i] * c->dt, &bx, &tx);
                departure_cell(gy, p, c->n_el[1], h[1], xi[2 * i + 1] * c->dt, &by, &ty);
                lagrange(p, tx, lx);
                lagrange(p, ty, ly);
                double sf = 0, sg = 0;
                for (int ky = 0; ky <= p; ++ky) {
                    int yy = (by + ky) % Ny;
                    for (int kx = 0; kx <= p; ++kx) {
                        int xx = (bx + kx) % Nx;
                        long src = (long)i * N + (long)yy * Nx + xx;
                        sf += lx[kx] * ly[ky] * f[src];
                        sg += lx[kx] * ly[ky] * g[src];
                    }
                }
                long n = (long)gy * Nx + gx;
                fo[(long)i * N + n] = sf;
                go[(long)i * N + n] = sg;
            }
        }
    }
}

/* n time steps of Eq. (5): collide, then stream. */
int oracle2d_step(const oracle2d_cfg *c, double *f, double *g, int nsteps)
{
    long N = oracle2d_num_nodes(c);
    double *tf = (double *)malloc(sizeof(double) * Q2 * N);
    double *tg = (double *)malloc(sizeof(double) * Q2 * N);
    if (!tf || !tg) { free(tf); free(tg); return -1; }
    for (int s = 0; s < nsteps; ++s) {
        oracle2d_collide(c, f, g);
        oracle2d_stream(c, f, g, tf, tg);
        memcpy(f, tf, sizeof(double) * Q2 * N);
        memcpy(g, tg, sizeof(double) * Q2 * N);
    }
    free(tf);
    free(tg);
    return 0;
}

/* rho, u ([2][N]) and T at every node, Eq. (7). */
void oracle2d_moments(const oracle2d_cfg *c, const double *f, const double *g, double *rho, double *u,
                      double *T)
{
    double xi[2 * Q2], w[Q2];
    oracle2d_velocity_set(xi, w);
    long N = oracle2d_num_nodes(c);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double fn[Q2], gn[Q2], uu[2];
        for (int i = 0; i < Q2; ++i) { fn[i] = f[(long)i * N + n]; gn[i] = g[(long)i * N + n]; }
        node_macro(c, xi, fn, gn, &rho[n], uu, &T[n]);
        u[n] = uu[0];
        u[N + n] = uu[1];
    }
}

/* weight of unique node g of an axis of equal cells: the Clenshaw-Curtis
 * weight of its local point, doubled at a shared cell end */
static double node_weight(int g, int p, double h)
{
    double wcc[16];
    cc_weights(p, wcc);
    int l = g % p;
    if (l != 0) return 0.5 * h * wcc[l];
    return 0.5 * h * (wcc[0] + wcc[p]);
}

/* Area integrals of rho, rho u_x, rho u_y and rho E, summed in node order. */
void oracle2d_totals(const oracle2d_cfg *c, const double *f, const double *g, double *out)
{
    double xi[2 * Q2], w[Q2];
    oracle2d_velocity_set(xi, w);
    int p = c->p;
    int Nx = c->n_el[0] * p, Ny = c->n_el[1] * p;
    long N = (long)Nx * Ny;
    double h[2] = {c->length[0] / c->n_el[0], c->length[1] / c->n_el[1]};
    for (int k = 0; k < 4; ++k) out[k] = 0;
    for (int gy = 0; gy < Ny; ++gy)
        for (int gx = 0; gx < Nx; ++gx) {
            long n = (long)gy * Nx + gx;
            double W = node_weight(gx, p, h[0]) * node_weight(gy, p, h[1]);
            double r = 0, jx = 0, jy = 0, twoE = 0;
            for (int i = 0; i < Q2; ++i) {
                double fi = f[(long)i * N + n];
                const double *x = &xi[2 * i];
                r += fi;
                jx += fi * x[0];
                jy += fi * x[1];
                twoE += fi * (x[0] * x[0] + x[1] * x[1]) + g[(long)i * N + n];
            }
            out[0] += W * r;
            out[1] += W * jx;
            out[2] += W * jy;
            out[3] += W * 0.5 * twoE;
        }
}
