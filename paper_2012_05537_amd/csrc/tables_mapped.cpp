// Host-side tables of the SLLBM library for distorted meshes (Sec. II A with
// curved cells): departure cells and local coordinates of every velocity and
// node, node and cell-point weights with the cell maps' Jacobians, and the
// source windows of the staged streaming kernel.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "sllbm_internal.h"

namespace sllbm {

// ---------------------------------------------------------------------------
// Distorted meshes: the equal-cell GLC grid with periodic node displacements
// d ([3][N]); each cell is the degree-p tensor interpolant of its nodes'
// positions, i.e. the map r -> r + D(r) with D the cell-wise interpolant of d
// (the GLC positions interpolate the identity).  Populations are interpolated
// in reference coordinates, so each departure point x_g + d_g - xi dt is
// located by Newton's method on r + D(r) = x_d.
// ---------------------------------------------------------------------------
namespace {

struct MapGrid {
    int p, ne[3], N[3];
    double h[3];
    const double *d;   // [3][N]
    int64_t nodes;
};

// D and I + dD/dr at local coordinates t of cell e (cell indices wrapped)
void map_at(const MapGrid &m, const int e[3], const double t[3], double D[3], double J[3][3])
{
    const int p = m.p;
    double l[3][MAXP + 1], dl[3][MAXP + 1];
    for (int a = 0; a < 3; ++a) {
        lagrange_basis(p, t[a], l[a]);
        lagrange_basis_deriv(p, t[a], dl[a]);
    }
    for (int a = 0; a < 3; ++a) {
        D[a] = 0.0;
        for (int b = 0; b < 3; ++b) J[a][b] = a == b ? 1.0 : 0.0;
    }
    for (int kz = 0; kz <= p; ++kz) {
        const int64_t zz = (e[2] * p + kz) % m.N[2];
        for (int ky = 0; ky <= p; ++ky) {
            const int64_t yy = (e[1] * p + ky) % m.N[1];
            for (int kx = 0; kx <= p; ++kx) {
                const int64_t node = (zz * m.N[1] + yy) * m.N[0] + (e[0] * p + kx) % m.N[0];
                const double v = l[0][kx] * l[1][ky] * l[2][kz];
                const double g[3] = {dl[0][kx] * l[1][ky] * l[2][kz] / m.h[0], l[0][kx] * dl[1][ky] * l[2][kz] / m.h[1],
                                     l[0][kx] * l[1][ky] * dl[2][kz] / m.h[2]};
                for (int a = 0; a < 3; ++a) {
                    const double da = m.d[a * m.nodes + node];
                    D[a] += v * da;
                    for (int b = 0; b < 3; ++b) J[a][b] += g[b] * da;
                }
            }
        }
    }
}

double det3(const double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// cell (wrapped) and local coordinates of the unwrapped reference point r
void locate(const MapGrid &m, const double r[3], int e[3], double t[3])
{
    for (int a = 0; a < 3; ++a) {
        const double s = r[a] / m.h[a];
        const double E = std::floor(s);
        t[a] = s - E;
        int64_t Ei = static_cast<int64_t>(E) % m.ne[a];
        if (Ei < 0) Ei += m.ne[a];
        e[a] = static_cast<int>(Ei);
    }
}

}  // namespace

bool build_mapped_tables(const VelocitySet &vs, int p, const int ne[3], const double length[3], const double *d,
                         double dt, std::vector<int32_t> &cell, std::vector<double> &tloc, std::vector<double> &nodew,
                         std::vector<double> &cjac, std::string &why)
{
    MapGrid m{};
    m.p = p;
    m.d = d;
    for (int a = 0; a < 3; ++a) {
        m.ne[a] = ne[a];
        m.N[a] = ne[a] * p;
        m.h[a] = length[a] / ne[a];
    }
    m.nodes = static_cast<int64_t>(m.N[0]) * m.N[1] * m.N[2];
    const int64_t N = m.nodes;
    double tg[MAXP + 1], cc[MAXP + 1];
    glc_points(p, tg);
    clenshaw_curtis(p, cc);
    // node weights, with the check that every cell map keeps its orientation;
    // per cell point (cells x fastest, points x fastest within a cell) the
    // inverse of J = I + dD/dr (row-major) and |det J|
    nodew.assign(N, 0.0);
    cjac.clear();
    cjac.reserve(static_cast<size_t>(ne[0]) * ne[1] * ne[2] * (p + 1) * (p + 1) * (p + 1) * 10);
    for (int ez = 0; ez < ne[2]; ++ez)
        for (int ey = 0; ey < ne[1]; ++ey)
            for (int ex = 0; ex < ne[0]; ++ex)
                for (int kz = 0; kz <= p; ++kz)
                    for (int ky = 0; ky <= p; ++ky)
                        for (int kx = 0; kx <= p; ++kx) {
                            const int e[3] = {ex, ey, ez};
                            const double t[3] = {tg[kx], tg[ky], tg[kz]};
                            double D[3], J[3][3];
                            map_at(m, e, t, D, J);
                            const double dj = det3(J);
                            if (!(dj > 0.0)) {
                                why = "distorted mesh: a cell map folds over (det J <= 0)";
                                return false;
                            }
                            const int64_t node = ((static_cast<int64_t>(ez * p + kz) % m.N[2]) * m.N[1] +
                                                  (ey * p + ky) % m.N[1]) * m.N[0] + (ex * p + kx) % m.N[0];
                            nodew[node] += 0.125 * m.h[0] * m.h[1] * m.h[2] * cc[kx] * cc[ky] * cc[kz] * dj;
                            // inverse by cofactors: Ji[a][b] = cof(J)[b][a] / det J
                            const double Ji[9] = {(J[1][1] * J[2][2] - J[1][2] * J[2][1]) / dj,
                                                  (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / dj,
                                                  (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / dj,
                                                  (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / dj,
                                                  (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / dj,
                                                  (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / dj,
                                                  (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / dj,
                                                  (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / dj,
                                                  (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / dj};
                            cjac.insert(cjac.end(), Ji, Ji + 9);
                            cjac.push_back(dj);
                        }
    // departure search, per velocity and node; velocities are split over up to
    // 16 host threads, each writing the slices of its own velocities
    cell.assign(static_cast<size_t>(vs.q) * N, 0);
    tloc.assign(static_cast<size_t>(3) * vs.q * N, 0.0);
    std::atomic<bool> failed{false};
    auto search = [&](int i) {
        for (int64_t n = 0; n < N && !failed.load(std::memory_order_relaxed); ++n) {
            const int g[3] = {static_cast<int>(n % m.N[0]), static_cast<int>((n / m.N[0]) % m.N[1]),
                              static_cast<int>(n / (static_cast<int64_t>(m.N[0]) * m.N[1]))};
            double xd[3], r[3];
            for (int a = 0; a < 3; ++a) {
                const double r0 = (g[a] / p) * m.h[a] + m.h[a] * tg[g[a] % p];
                const double sh = vs.xi[i][a] * dt;
                xd[a] = r0 + d[a * N + n] - sh;
                r[a] = r0 - sh;                   // start at the undistorted departure point
            }
            // Newton until the update stalls at rounding level, then the
            // residual decides (in cell widths)
            auto residual = [&](double F[3], double J[3][3]) {
                int e[3];
                double t[3], D[3];
                locate(m, r, e, t);
                map_at(m, e, t, D, J);
                double res = 0.0;
                for (int a = 0; a < 3; ++a) {
                    F[a] = r[a] + D[a] - xd[a];
                    res = std::max(res, std::fabs(F[a]) / m.h[a]);
                }
                return res;
            };
            for (int it = 0; it < 60; ++it) {
                double F[3], J[3][3];
                residual(F, J);
                const double dj = det3(J);
                double step = 0.0;
                for (int k = 0; k < 3; ++k) {        // Cramer's rule for J dr = F
                    double M[3][3];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) M[a][b] = b == k ? F[a] : J[a][b];
                    const double drk = det3(M) / dj;
                    r[k] -= drk;
                    step += std::fabs(drk) / m.h[k];
                }
                if (step < 1e-15) break;
            }
            double F[3], J[3][3];
            if (!(residual(F, J) < 1e-12)) {
                failed = true;
                return;
            }
            int e[3];
            double t[3];
            locate(m, r, e, t);
            cell[static_cast<size_t>(i) * N + n] = (e[2] * ne[1] + e[1]) * ne[0] + e[0];
            for (int a = 0; a < 3; ++a) tloc[(static_cast<size_t>(a) * vs.q + i) * N + n] = t[a];
        }
    };
    const int nt = static_cast<int>(std::max(1u, std::min(std::thread::hardware_concurrency(), 16u)));
    std::vector<std::thread> pool;
    for (int k = 0; k < nt; ++k)
        pool.emplace_back([&, k]() {
            for (int i = k; i < vs.q; i += nt) search(i);
        });
    for (auto &th : pool) th.join();
    if (failed) {
        why = "distorted mesh: the departure search did not converge (displacement too strong)";
        return false;
    }
    return true;
}

int build_mapped_windows(int q, int p, const int ne[3], const std::vector<int32_t> &cell, const int tile[3],
                         int max_nodes, std::vector<int32_t> &win)
{
    const int N[3] = {ne[0] * p, ne[1] * p, ne[2] * p};
    const int64_t nodes = static_cast<int64_t>(N[0]) * N[1] * N[2];
    const int nt[3] = {(N[0] + tile[0] - 1) / tile[0], (N[1] + tile[1] - 1) / tile[1], (N[2] + tile[2] - 1) / tile[2]};
    const int64_t ntiles = static_cast<int64_t>(nt[0]) * nt[1] * nt[2];
    win.assign(static_cast<size_t>(q) * ntiles * 4, 0);
    int largest = 0;
    for (int i = 0; i < q; ++i)
        for (int64_t t = 0; t < ntiles; ++t) {
            const int tc[3] = {static_cast<int>(t % nt[0]), static_cast<int>((t / nt[0]) % nt[1]),
                               static_cast<int>(t / (static_cast<int64_t>(nt[0]) * nt[1]))};
            int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
            for (int z = tc[2] * tile[2]; z < std::min(N[2], (tc[2] + 1) * tile[2]); ++z)
                for (int y = tc[1] * tile[1]; y < std::min(N[1], (tc[1] + 1) * tile[1]); ++y)
                    for (int x = tc[0] * tile[0]; x < std::min(N[0], (tc[0] + 1) * tile[0]); ++x) {
                        const int64_t n = (static_cast<int64_t>(z) * N[1] + y) * N[0] + x;
                        const int c = cell[static_cast<size_t>(i) * nodes + n];
                        const int dep[3] = {c % ne[0], (c / ne[0]) % ne[1], c / (ne[0] * ne[1])};
                        const int own[3] = {x / p, y / p, z / p};
                        for (int a = 0; a < 3; ++a) {
                            // departure cell unwrapped next to the node's own cell
                            int d = (dep[a] - own[a]) % ne[a];
                            if (d < 0) d += ne[a];
                            if (2 * d >= ne[a]) d -= ne[a];
                            const int u = own[a] + d;
                            lo[a] = std::min(lo[a], u);
                            hi[a] = std::max(hi[a], u);
                        }
                    }
            int32_t *w = &win[(static_cast<size_t>(i) * ntiles + t) * 4];
            int wn[3];
            // a window spans at most every cell of an axis once, so that the
            // kernel wraps a window node with one subtraction of N
            bool fits = true;
            for (int a = 0; a < 3; ++a) {
                fits = fits && hi[a] - lo[a] + 1 <= ne[a];
                int o = lo[a] % ne[a];
                if (o < 0) o += ne[a];
                w[a] = o;                                         // origin cell (wrapped)
                wn[a] = (hi[a] - lo[a] + 1) * p + 1;             // window nodes along the axis
            }
            const int64_t total = static_cast<int64_t>(wn[0]) * wn[1] * wn[2];
            if (fits && total <= max_nodes && wn[0] < 1024 && wn[1] < 1024 && wn[2] < 1024) {
                w[3] = wn[0] | (wn[1] << 10) | (wn[2] << 20);
                largest = std::max(largest, static_cast<int>(total));
            } else {
                w[3] = 0;                                         // gather from global memory
            }
        }
    return largest;
}

void build_mapped_inverse(int q, int64_t nodes, int ncells, const std::vector<int32_t> &cell,
                          std::vector<int32_t> &order, std::vector<int32_t> &start)
{
    order.assign(static_cast<size_t>(q) * nodes, 0);
    start.assign(static_cast<size_t>(q) * (ncells + 1), 0);
    for (int i = 0; i < q; ++i) {
        const int32_t *ci = &cell[static_cast<size_t>(i) * nodes];
        int32_t *st = &start[static_cast<size_t>(i) * (ncells + 1)];
        for (int64_t n = 0; n < nodes; ++n) ++st[ci[n] + 1];
        for (int c = 0; c < ncells; ++c) st[c + 1] += st[c];
        std::vector<int32_t> next(st, st + ncells);
        int32_t *oi = &order[static_cast<size_t>(i) * nodes];
        for (int64_t n = 0; n < nodes; ++n) oi[next[ci[n]]++] = static_cast<int32_t>(n);
    }
}

int mapped_t_chunk(int q, int p, int64_t ncells, size_t elem)
{
    const int64_t k3 = static_cast<int64_t>(p + 1) * (p + 1) * (p + 1);
    const int64_t per_velocity = ncells * 2 * k3 * static_cast<int64_t>(elem);
    // a pass may hold one state's bytes (2 q p^3 values per cell), or 256 MB
    // on small grids, where fewer passes mean fewer launches
    const int64_t budget = std::max<int64_t>(ncells * 2 * q * p * p * p * static_cast<int64_t>(elem), int64_t(256) << 20);
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(q, budget / per_velocity)));
}

}  // namespace sllbm
