// Host-logic driver for the distorted-mesh tables (built on the CPU by the
// library): reads "p nx ny nz Lx Ly Lz dt max_nodes" and the 3N
// displacements from stdin, runs build_mapped_tables for the 45 velocities
// and build_mapped_windows for the streaming's node tiles (windows of at most
// max_nodes nodes), and writes the departure cells, local coordinates, node
// weights, then the largest window and the window table, as text.  Exit
// status 1 (with the reason) if the builder refuses the mesh.
#include <cstdio>
#include <string>
#include <vector>
#include "sllbm_internal.h"
using namespace sllbm;
int main()
{
    int p, ne[3];
    double L[3], dt;
    int max_nodes;
    if (std::scanf("%d %d %d %d %lf %lf %lf %lf %d", &p, &ne[0], &ne[1], &ne[2], &L[0], &L[1], &L[2], &dt,
                   &max_nodes) != 9)
        return 2;
    const long N = static_cast<long>(ne[0]) * p * ne[1] * p * ne[2] * p;
    std::vector<double> d(3 * N);
    for (auto &x : d)
        if (std::scanf("%lf", &x) != 1) return 2;
    VelocitySet vs;
    build_velocity_set(vs);
    std::vector<int32_t> cell;
    std::vector<double> t, w;
    std::string why;
    std::vector<double> cj;
    if (!build_mapped_tables(vs, p, ne, L, d.data(), dt, cell, t, w, cj, why)) {
        std::printf("refused %s\n", why.c_str());
        return 1;
    }
    for (auto c : cell) std::printf("%d\n", c);
    for (auto x : t) std::printf("%.17g\n", x);
    for (auto x : w) std::printf("%.17g\n", x);
    std::vector<int32_t> win;
    const int tile[3] = {MAPPED_TX, MAPPED_TY, MAPPED_TZ};
    std::printf("%d\n", build_mapped_windows(vs.q, p, ne, cell, tile, max_nodes, win));
    for (auto v : win) std::printf("%d\n", v);
    return 0;
}
