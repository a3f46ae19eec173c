// Host-logic driver for the distorted-mesh tables (built on the CPU by the
// library): reads "p nx ny nz Lx Ly Lz dt" and the 3N displacements from
// stdin, runs build_mapped_tables for the 45 velocities and writes the
// departure cells, local coordinates and node weights as text.  Exit status 1
// (with the reason) if the builder refuses the mesh.
#include <cstdio>
#include <string>
#include <vector>
#include "sllbm_internal.h"
using namespace sllbm;
int main()
{
    int p, ne[3];
    double L[3], dt;
    if (std::scanf("%d %d %d %d %lf %lf %lf %lf", &p, &ne[0], &ne[1], &ne[2], &L[0], &L[1], &L[2], &dt) != 8) return 2;
    const long N = static_cast<long>(ne[0]) * p * ne[1] * p * ne[2] * p;
    std::vector<double> d(3 * N);
    for (auto &x : d)
        if (std::scanf("%lf", &x) != 1) return 2;
    VelocitySet vs;
    build_velocity_set(vs);
    std::vector<int32_t> cell;
    std::vector<double> t, w;
    std::string why;
    if (!build_mapped_tables(vs, p, ne, L, d.data(), dt, cell, t, w, why)) {
        std::printf("refused %s\n", why.c_str());
        return 1;
    }
    for (auto c : cell) std::printf("%d\n", c);
    for (auto x : t) std::printf("%.17g\n", x);
    for (auto x : w) std::printf("%.17g\n", x);
    return 0;
}
