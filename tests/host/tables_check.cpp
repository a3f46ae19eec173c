// Host-logic check of the graded-mesh tables (built on the CPU by the
// library): for 40 random graded or equal axes (p = 1..6, shifts up to
// several cells), the per-node forward rows and the transposed rows, each
// expanded to a dense N x N matrix, must be exact transposes of each other,
// and the transposed band starts must be non-decreasing.  Prints the largest
// entry difference and band width; exits non-zero on failure.
#include <cmath>
#include <cstdio>
#include <random>
#include "sllbm_internal.h"
using namespace sllbm;
int main()
{
    VelocitySet vs;
    build_velocity_set(vs);
    std::mt19937_64 rng(3);
    std::uniform_real_distribution<double> U(-1, 1);
    double worst = 0;
    int maxband = 0;
    for (int trial = 0; trial < 40; ++trial) {
        const int p = 1 + trial % 6, ne = 1 + (trial * 7) % 11;
        const double L = 2.0 + trial % 3;
        const double dt = 0.05 + 0.3 * (trial % 5);
        std::vector<double> faces;
        if (trial % 4 != 0) {
            faces.push_back(0);
            double sum = 0;
            std::vector<double> w(ne);
            for (auto &x : w) { x = 1 + 0.6 * U(rng); sum += x; }
            for (auto x : w) faces.push_back(faces.back() + x * L / sum);
            faces.back() = L;
        }
        const int N = ne * p;
        std::vector<int32_t> src, srcT;
        std::vector<double> w, wT;
        build_node_tables(vs, p, ne, L, faces, trial % 3, dt, src, w);
        int band = 0;
        build_transposed_node_tables(N, p, src, w, 0, srcT, wT, band);
        const int kt = band;
        build_transposed_node_tables(N, p, src, w, kt, srcT, wT, band);
        maxband = std::max(maxband, band);
        for (int i = 0; i < Q; ++i) {
            std::vector<double> Sm(N * N, 0.0), T(N * N, 0.0);
            for (int g = 0; g < N; ++g)
                for (int k = 0; k <= p; ++k) {
                    int m = ((src[i * N + g] + k) % N + N) % N;
                    Sm[g * N + m] += w[(i * N + g) * (p + 1) + k];
                }
            for (int m = 0; m < N; ++m) {
                if (m > 0 && srcT[i * N + m] < srcT[i * N + m - 1]) {
                    printf("non-monotone: trial %d p %d ne %d i %d m %d graded %d\n", trial, p, ne, i, m, (int)!faces.empty());
                    for (int q = 0; q < N; ++q) printf("%d ", src[i * N + q]);
                    printf("| ");
                    for (int q = 0; q < N; ++q) printf("%d ", srcT[i * N + q]);
                    printf("\n");
                    return 1;
                }
                for (int j = 0; j < kt; ++j) {
                    int g = ((srcT[i * N + m] + j) % N + N) % N;
                    T[m * N + g] += wT[(i * N + m) * kt + j];
                }
            }
            for (int g = 0; g < N; ++g)
                for (int m = 0; m < N; ++m) worst = std::max(worst, std::fabs(Sm[g * N + m] - T[m * N + g]));
        }
    }
    printf("max |S^T - T| = %.3e, largest band %d\n", worst, maxband);
    return worst < 1e-14 ? 0 : 1;
}
