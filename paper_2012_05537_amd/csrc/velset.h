// Compile-time D3Q45 velocity set (degree-nine cubature with icosahedral
// symmetry, Sec. II B): the origin, an icosahedron at radius sqrt(3), the
// same icosahedron at radius sqrt(15), and its dual dodecahedron at radius 3,
// with weights 28/135, 25/432, 1/2160 and 1/216.  Each shell is ordered
// lexicographically.  Being constexpr, every abscissa component, weight and
// Hermite coefficient folds into the kernels as an immediate.
#pragma once

namespace sllbm {
namespace vs {

constexpr int Q = 45;

// Newton iteration for sqrt, accurate to the last bit or one ulp
constexpr double csqrt(double a)
{
    double x = a > 1.0 ? a : 1.0;
    for (int k = 0; k < 200; ++k) {
        double nx = 0.5 * (x + a / x);
        if (nx == x) break;
        x = nx;
    }
    return x;
}

constexpr double cabs(double a) { return a < 0 ? -a : a; }

struct Dirs {
    double v[20][3];
    int n;
};

constexpr void add_signed_cycles(Dirs &d, double a, double b, double c)
{
    const double rot[3][3] = {{a, b, c}, {b, c, a}, {c, a, b}};
    for (int r = 0; r < 3; ++r) {
        for (int s = 0; s < 8; ++s) {
            double v[3] = {(s & 1) ? -rot[r][0] : rot[r][0], (s & 2) ? -rot[r][1] : rot[r][1],
                           (s & 4) ? -rot[r][2] : rot[r][2]};
            bool seen = false;
            for (int m = 0; m < d.n; ++m)
                if (cabs(d.v[m][0] - v[0]) + cabs(d.v[m][1] - v[1]) + cabs(d.v[m][2] - v[2]) < 1e-12) seen = true;
            if (!seen) {
                d.v[d.n][0] = v[0];
                d.v[d.n][1] = v[1];
                d.v[d.n][2] = v[2];
                ++d.n;
            }
        }
    }
}

constexpr bool lex_less(const double *x, const double *y)
{
    for (int k = 0; k < 3; ++k) {
        if (cabs(x[k] - y[k]) > 1e-9) return x[k] < y[k];
    }
    return false;
}

constexpr void normalise_sort(Dirs &d)
{
    for (int m = 0; m < d.n; ++m) {
        double r = csqrt(d.v[m][0] * d.v[m][0] + d.v[m][1] * d.v[m][1] + d.v[m][2] * d.v[m][2]);
        for (int k = 0; k < 3; ++k) d.v[m][k] /= r;
    }
    for (int i = 1; i < d.n; ++i) {
        double t[3] = {d.v[i][0], d.v[i][1], d.v[i][2]};
        int j = i - 1;
        while (j >= 0 && lex_less(t, d.v[j])) {
            for (int k = 0; k < 3; ++k) d.v[j + 1][k] = d.v[j][k];
            --j;
        }
        for (int k = 0; k < 3; ++k) d.v[j + 1][k] = t[k];
    }
}

struct Table {
    double xi[Q][3];
    double w[Q];
    double x2[Q];       // |xi|^2
    int shell[Q];       // 0 origin, 1 inner icosahedron, 2 outer icosahedron, 3 dodecahedron
    int opp[Q];         // index of -xi
};

constexpr Table make_table()
{
    Table t{};
    const double phi = 0.5 * (1.0 + csqrt(5.0));
    Dirs ico{};
    add_signed_cycles(ico, 0.0, 1.0, phi);
    Dirs dod{};
    add_signed_cycles(dod, 1.0, 1.0, 1.0);
    add_signed_cycles(dod, 0.0, phi, 1.0 / phi);
    normalise_sort(ico);
    normalise_sort(dod);
    const double radius[3] = {csqrt(3.0), csqrt(15.0), 3.0};
    const double weight[3] = {25.0 / 432.0, 1.0 / 2160.0, 1.0 / 216.0};
    int q = 0;
    t.xi[0][0] = t.xi[0][1] = t.xi[0][2] = 0.0;
    t.w[0] = 28.0 / 135.0;
    t.shell[0] = 0;
    ++q;
    for (int s = 0; s < 3; ++s) {
        const Dirs &d = (s < 2) ? ico : dod;
        for (int m = 0; m < d.n; ++m) {
            for (int k = 0; k < 3; ++k) t.xi[q][k] = radius[s] * d.v[m][k];
            t.w[q] = weight[s];
            t.shell[q] = s + 1;
            ++q;
        }
    }
    for (int i = 0; i < Q; ++i) {
        t.x2[i] = t.xi[i][0] * t.xi[i][0] + t.xi[i][1] * t.xi[i][1] + t.xi[i][2] * t.xi[i][2];
        t.opp[i] = i;
        for (int j = 0; j < Q; ++j) {
            if (cabs(t.xi[i][0] + t.xi[j][0]) + cabs(t.xi[i][1] + t.xi[j][1]) + cabs(t.xi[i][2] + t.xi[j][2]) < 1e-12)
                t.opp[i] = j;
        }
    }
    return t;
}

constexpr Table T = make_table();

// Velocity pairs (i, opp(i)) with i < opp(i): the 44 moving velocities.
struct Pairs {
    int a[22], b[22];
};

constexpr Pairs make_pairs()
{
    Pairs p{};
    int n = 0;
    for (int i = 1; i < Q; ++i) {
        if (T.opp[i] > i) {
            p.a[n] = i;
            p.b[n] = T.opp[i];
            ++n;
        }
    }
    return p;
}

constexpr Pairs PAIRS = make_pairs();

// Unique components (a <= b <= c) of a symmetric rank-3 tensor, their
// multiplicities, and the contraction coefficients
//   H3c[i][m] = (w_i / 3!) * mult_m * H^(3)_{abc}(xi_i)   (App. B, c_s = 1),
// so that (w_i/3!) Qbar : H^(3)_i = sum_m H3c[i][m] Qbar_m.
constexpr int IDX3[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                             {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
constexpr double MULT3[10] = {1, 3, 3, 3, 6, 3, 1, 3, 3, 1};

struct H3Table {
    double c[Q][10];
    double mono[Q][10];   // xi_a xi_b xi_c (unique order)
};

constexpr H3Table make_h3()
{
    H3Table h{};
    for (int i = 0; i < Q; ++i) {
        for (int m = 0; m < 10; ++m) {
            const int a = IDX3[m][0], b = IDX3[m][1], c = IDX3[m][2];
            const double *x = T.xi[i];
            const double hermite = x[a] * x[b] * x[c] -
                                   ((b == c ? x[a] : 0.0) + (a == c ? x[b] : 0.0) + (a == b ? x[c] : 0.0));
            h.c[i][m] = T.w[i] / 6.0 * MULT3[m] * hermite;
            h.mono[i][m] = x[a] * x[b] * x[c];
        }
    }
    return h;
}

constexpr H3Table H3 = make_h3();

}  // namespace vs
}  // namespace sllbm
