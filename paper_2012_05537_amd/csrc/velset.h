// Compile-time velocity sets (degree-nine cubature rules, Sec. II B).
//
// D3Q45: the origin, an icosahedron at radius sqrt(3), the same icosahedron
// at radius sqrt(15), and its dual dodecahedron at radius 3, with weights
// 28/135, 25/432, 1/2160 and 1/216.  Each shell is ordered
// lexicographically.
//
// D2Q19 (the two-dimensional set of Sec. II B, cited there without its
// values): the origin and three rings of six points with hexagonal
// symmetry.  Such a rule is exact to degree nine for the weight
// exp(-|xi|^2/2)/(2 pi) once it integrates |xi|^(2k) (k <= 4) and
// |xi|^(2k) Re((x + iy)^6) (k = 0, 1) exactly.  With the rings B and C on the
// axes and ring A turned by 30 degrees, the Re z^6 conditions split the
// k = 3, 4 moments (48, 384) in halves between A and B + C, so
// a_A = |xi_A|^2 = 8 with total weight 3/64; B and C are then the two-point
// rule of the remaining moments nu_k = sum W a^k (13/8, 5, 24, 192): a_B, a_C
// are the roots of a^2 - (96/7) a + 192/7, i.e. (48 -+ 8 sqrt(15))/7, and
// the origin keeps 31/96.  The turn of the rule is fixed by putting the
// largest speed on the x axis.  Rings in order of speed (B, A, C), each
// ordered lexicographically by (x, y).
//
// Being constexpr, every abscissa component, weight and Hermite coefficient
// folds into the kernels as an immediate.
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

template <int NQ>
struct Table {
    double xi[NQ][3];    // z component 0 in two dimensions
    double w[NQ];
    double x2[NQ];       // |xi|^2
    int shell[NQ];       // 0 origin, then shells in the order they are built
    int opp[NQ];         // index of -xi
};

template <int NQ>
constexpr void finish_table(Table<NQ> &t)
{
    for (int i = 0; i < NQ; ++i) {
        t.x2[i] = t.xi[i][0] * t.xi[i][0] + t.xi[i][1] * t.xi[i][1] + t.xi[i][2] * t.xi[i][2];
        t.opp[i] = i;
        for (int j = 0; j < NQ; ++j) {
            if (cabs(t.xi[i][0] + t.xi[j][0]) + cabs(t.xi[i][1] + t.xi[j][1]) + cabs(t.xi[i][2] + t.xi[j][2]) < 1e-12)
                t.opp[i] = j;
        }
    }
}

// shells: 1 inner icosahedron, 2 outer icosahedron, 3 dodecahedron
constexpr Table<Q> make_table()
{
    Table<Q> t{};
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
    finish_table(t);
    return t;
}

constexpr Table<Q> T = make_table();

// Velocity pairs (i, opp(i)) with i < opp(i): all moving velocities.
template <int NP>
struct Pairs {
    int a[NP], b[NP];
};

template <int NP, int NQ>
constexpr Pairs<NP> make_pairs(const Table<NQ> &t)
{
    Pairs<NP> p{};
    int n = 0;
    for (int i = 1; i < NQ; ++i) {
        if (t.opp[i] > i) {
            p.a[n] = i;
            p.b[n] = t.opp[i];
            ++n;
        }
    }
    return p;
}

constexpr Pairs<22> PAIRS = make_pairs<22>(T);

// Unique components (a <= b <= c) of a symmetric rank-3 tensor, their
// multiplicities, and the contraction coefficients
//   H3c[i][m] = (w_i / 3!) * mult_m * H^(3)_{abc}(xi_i)   (App. B, c_s = 1),
// so that (w_i/3!) Qbar : H^(3)_i = sum_m H3c[i][m] Qbar_m.
constexpr int IDX3[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                             {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
constexpr double MULT3[10] = {1, 3, 3, 3, 6, 3, 1, 3, 3, 1};

template <int NQ, int NM>
struct H3Table {
    double c[NQ][NM];
    double mono[NQ][NM];   // xi_a xi_b xi_c (unique order)
};

// idx/mult: the NM unique components of the dimension (the Kronecker deltas
// of H^(3) run over that dimension's axes only)
template <int NQ, int NM>
constexpr H3Table<NQ, NM> make_h3(const Table<NQ> &t, const int (&idx)[NM][3], const double (&mult)[NM])
{
    H3Table<NQ, NM> h{};
    for (int i = 0; i < NQ; ++i) {
        for (int m = 0; m < NM; ++m) {
            const int a = idx[m][0], b = idx[m][1], c = idx[m][2];
            const double *x = t.xi[i];
            const double hermite = x[a] * x[b] * x[c] -
                                   ((b == c ? x[a] : 0.0) + (a == c ? x[b] : 0.0) + (a == b ? x[c] : 0.0));
            h.c[i][m] = t.w[i] / 6.0 * mult[m] * hermite;
            h.mono[i][m] = x[a] * x[b] * x[c];
        }
    }
    return h;
}

constexpr H3Table<Q, 10> H3 = make_h3(T, IDX3, MULT3);
constexpr double SHELL_X2[4] = {0.0, 3.0, 15.0, 9.0};

}  // namespace vs

// D2Q19 (see the head of this file)
namespace vs2 {

using vs::finish_table;
using vs::H3Table;
using vs::make_h3;
using vs::make_pairs;
using vs::Pairs;
using vs::Table;

constexpr int Q = 19;

constexpr Table<Q> make_table()
{
    Table<Q> t{};
    const double s15 = vs::csqrt(15.0), h3 = 0.5 * vs::csqrt(3.0);
    const double aA = 8.0, aB = (48.0 - 8.0 * s15) / 7.0, aC = (48.0 + 8.0 * s15) / 7.0;
    const double nu1 = 2.0 - 3.0 / 64.0 * aA, nu2 = 8.0 - 3.0 / 64.0 * aA * aA;
    const double WB = (nu2 - aC * nu1) / (aB * (aB - aC)), WC = (nu1 - WB * aB) / aC;
    // unit directions of a ring on the axes and of the turned ring, each
    // already in lexicographic (x, y) order
    const double axis_dirs[6][2] = {{-1.0, 0.0}, {-0.5, -h3}, {-0.5, h3}, {0.5, -h3}, {0.5, h3}, {1.0, 0.0}};
    const double turn_dirs[6][2] = {{-h3, -0.5}, {-h3, 0.5}, {0.0, -1.0}, {0.0, 1.0}, {h3, -0.5}, {h3, 0.5}};
    const double radius2[3] = {aB, aA, aC}, weight[3] = {WB / 6.0, 3.0 / 64.0 / 6.0, WC / 6.0};
    t.w[0] = 31.0 / 96.0;
    int q = 1;
    for (int s = 0; s < 3; ++s) {
        const double r = vs::csqrt(radius2[s]);
        const double(&d)[6][2] = s == 1 ? turn_dirs : axis_dirs;
        for (int m = 0; m < 6; ++m, ++q) {
            t.xi[q][0] = r * d[m][0];
            t.xi[q][1] = r * d[m][1];
            t.xi[q][2] = 0.0;
            t.w[q] = weight[s];
            t.shell[q] = s + 1;
        }
    }
    finish_table(t);
    return t;
}

constexpr Table<Q> T = make_table();
constexpr Pairs<9> PAIRS = make_pairs<9>(T);
constexpr int IDX3[4][3] = {{0, 0, 0}, {0, 0, 1}, {0, 1, 1}, {1, 1, 1}};
constexpr double MULT3[4] = {1, 3, 3, 1};
constexpr H3Table<Q, 4> H3 = make_h3(T, IDX3, MULT3);
constexpr double SHELL_X2[4] = {0.0, T.x2[1], T.x2[7], T.x2[13]};

}  // namespace vs2

// Lattice traits read by the node-local kernels: Q velocities in D
// dimensions, NPAIR pairs (xi, -xi) after the rest velocity, NM3 unique
// components of a symmetric rank-3 tensor, NSHELL speeds.
struct D3Q45 {
    static constexpr int Q = vs::Q, D = 3, NPAIR = 22, NM3 = 10, NSHELL = 4;
    static constexpr const vs::Table<vs::Q> &T = vs::T;
    static constexpr const vs::Pairs<22> &PAIRS = vs::PAIRS;
    static constexpr const vs::H3Table<vs::Q, 10> &H3 = vs::H3;
    static constexpr const int (&IDX3)[10][3] = vs::IDX3;
    static constexpr const double (&SHELL_X2)[4] = vs::SHELL_X2;
};

struct D2Q19 {
    static constexpr int Q = vs2::Q, D = 2, NPAIR = 9, NM3 = 4, NSHELL = 4;
    static constexpr const vs::Table<vs2::Q> &T = vs2::T;
    static constexpr const vs::Pairs<9> &PAIRS = vs2::PAIRS;
    static constexpr const vs::H3Table<vs2::Q, 4> &H3 = vs2::H3;
    static constexpr const int (&IDX3)[4][3] = vs2::IDX3;
    static constexpr const double (&SHELL_X2)[4] = vs2::SHELL_X2;
};

}  // namespace sllbm
