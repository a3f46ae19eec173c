/* Host driver of the oracle for the AddressSanitizer / UndefinedBehaviorSanitizer
 * build (test infrastructure): includes the oracle source, so the real build
 * (R = double) and the complex-step build (-DORACLE_COMPLEX) are both
 * exercised, and calls every exported operation on small grids, including
 * ragged and one-cell axes, shifts of several cells, every order 1..6, graded
 * cells and a distorted mesh.  Exits non-zero if an output is not finite; the
 * sanitizers abort on any invalid access or undefined operation. */
#include "../../oracle/sllbm_oracle.c"

#include <stdio.h>

static double urand(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

static int finite_r(const R *a, long n)
{
    for (long k = 0; k < n; ++k) {
#ifdef ORACLE_COMPLEX
        if (!isfinite(creal(a[k])) || !isfinite(cimag(a[k]))) return 0;
#else
        if (!isfinite(a[k])) return 0;
#endif
    }
    return 1;
}

static int run_case(int nx, int ny, int nz, int p, double dt, int graded, int mapped, unsigned seed)
{
    oracle_cfg c;
    memset(&c, 0, sizeof c);
    c.n_el[0] = nx; c.n_el[1] = ny; c.n_el[2] = nz;
    c.p = p;
    for (int a = 0; a < 3; ++a) c.length[a] = 2.0 * M_PI;
    c.dt = dt;
    c.gamma = 1.4;
    c.prandtl = 0.71;
    c.mu_inf = 0.01;
    c.viscosity_law = (int)(seed & 1u);
    double *faces[3] = {NULL, NULL, NULL};
    if (graded) {
        for (int a = 0; a < 3; ++a) {
            faces[a] = malloc(sizeof(double) * (c.n_el[a] + 1));
            double tot = 0.0;
            faces[a][0] = 0.0;
            for (int e = 0; e < c.n_el[a]; ++e) faces[a][e + 1] = (tot += 1.0 + 0.4 * (urand(&seed) - 0.5));
            for (int e = 0; e <= c.n_el[a]; ++e) faces[a][e] *= c.length[a] / tot;
            faces[a][c.n_el[a]] = c.length[a];
            c.faces[a] = faces[a];
        }
    }
    const int Nx = nx * p, Ny = ny * p, Nz = nz * p;
    const long N = (long)Nx * Ny * Nz;
    double *x = malloc(sizeof(double) * Nx), *y = malloc(sizeof(double) * Ny), *z = malloc(sizeof(double) * Nz);
    oracle_node_coords(&c, x, y, z);
    double *disp = NULL;
    if (mapped) {
        disp = malloc(sizeof(double) * 3 * N);
        const double h = c.length[0] / nx;
        for (long n = 0; n < N; ++n) {
            const double X = x[n % Nx], Y = y[(n / Nx) % Ny], Z = z[n / ((long)Nx * Ny)];
            disp[n] = 0.1 * h * sin(Y + Z);
            disp[N + n] = 0.1 * h * sin(Z + X);
            disp[2 * N + n] = 0.1 * h * sin(X + Y);
        }
        c.disp = disp;
    }
    R *rho = malloc(sizeof(R) * N), *u = malloc(sizeof(R) * 3 * N), *T = malloc(sizeof(R) * N);
    for (long n = 0; n < N; ++n) {
        const double X = x[n % Nx], Y = y[(n / Nx) % Ny], Z = z[n / ((long)Nx * Ny)];
        rho[n] = 1.0 + 0.1 * sin(X) * cos(Y);
        u[n] = 0.3 * sin(X) * cos(Y) * cos(Z);
        u[N + n] = -0.3 * cos(X) * sin(Y) * cos(Z);
        u[2 * N + n] = 0.05 * sin(Z);
        T[n] = 1.0 + 0.05 * cos(X + Z);
    }
    R *f = malloc(sizeof(R) * Q * N), *g = malloc(sizeof(R) * Q * N);
    R *fo = malloc(sizeof(R) * Q * N), *go = malloc(sizeof(R) * Q * N);
    FN(init_equilibrium)(&c, rho, u, T, f, g);
    for (long k = 0; k < Q * N; ++k) {
        f[k] *= 1.0 + 0.01 * (urand(&seed) - 0.5);
        g[k] *= 1.0 + 0.01 * (urand(&seed) - 0.5);
    }
    int ok = 1;
    FN(collide)(&c, f, g);
    FN(stream)(&c, f, g, fo, go);
    ok &= finite_r(fo, Q * N) && finite_r(go, Q * N);
    if (FN(step)(&c, f, g, 1) != 0) return 0;
    ok &= finite_r(f, Q * N) && finite_r(g, Q * N);
    R tot[5], diag[3];
    FN(moments)(&c, f, g, rho, u, T);
    FN(totals)(&c, f, g, tot);
    ok &= finite_r(rho, N) && finite_r(u, 3 * N) && finite_r(T, N) && finite_r(tot, 5);
    if (!mapped) {
        long nodes[3] = {N - 1, N / 2, 0};
        R so[3 * Q], sg[3 * Q];
        FN(step_at_nodes)(&c, f, g, p <= 3 ? 3 : 1, nodes, so, sg);
        ok &= finite_r(so, (p <= 3 ? 3 : 1) * Q) && finite_r(sg, (p <= 3 ? 3 : 1) * Q);
        FN(stream_at_nodes)(&c, f, g, 3, nodes, so, sg);
        ok &= finite_r(so, 3 * Q) && finite_r(sg, 3 * Q);
        R L = FN(loss)(&c, f, g);
        ok &= finite_r(&L, 1);
        FN(diagnostics)(&c, f, g, diag);
        ok &= finite_r(diag, 3);
    } else {
        double *w = malloc(sizeof(double) * N);
        oracle_mapped_node_weights(&c, w);
        for (long n = 0; n < N; ++n) ok &= isfinite(w[n]) && w[n] > 0.0;
        free(w);
    }
    printf("case %dx%dx%d p=%d dt=%.2f graded=%d mapped=%d: %s\n", nx, ny, nz, p, dt, graded, mapped,
           ok ? "ok" : "NON-FINITE");
    free(rho); free(u); free(T); free(f); free(g); free(fo); free(go); free(x); free(y); free(z); free(disp);
    for (int a = 0; a < 3; ++a) free(faces[a]);
    return ok;
}

int main(void)
{
    setvbuf(stdout, NULL, _IONBF, 0);
    double xi[3 * Q], w[Q], t[16], ell[16], dl[16], wcc[16];
    if (oracle_velocity_set(xi, w) != Q) return 2;
    for (int p = 1; p <= 6; ++p) {
        oracle_glc_nodes(p, t);
        oracle_lagrange(p, 0.37, ell);
        oracle_lagrange_deriv(p, 0.61, dl);
        oracle_cc_weights(p, wcc);
    }
    int ok = 1;
    for (int p = 1; p <= 6; ++p) ok &= p <= 3 ? run_case(2, 1, 2, p, 0.3, 0, 0, 11u + p)
                                              : run_case(1, 1, 1, p, 0.3, 0, 0, 11u + p);
    ok &= run_case(3, 2, 1, 3, 2.5, 0, 0, 5u);      /* shifts of several cells, one-cell axis */
    ok &= run_case(3, 4, 2, 2, 0.6, 1, 0, 7u);      /* graded cells */
    ok &= run_case(3, 3, 3, 2, 0.2, 0, 1, 9u);      /* distorted cells */
    printf(ok ? "ALL OK\n" : "FAILED\n");
    return ok ? 0 : 1;
}
