// Internal declarations shared by the host tables, the kernels and the C ABI
// of the SLLBM library.  Not part of the public interface (include/sllbm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sllbm.h"

namespace sllbm {

constexpr int Q = 45;        // discrete velocities (D3Q45)
constexpr int Q2D = 19;      // discrete velocities of the two-dimensional set (D2Q19)
constexpr int MAXP = 6;      // largest supported interpolation order
constexpr int NPAIR = 22;    // velocity pairs (xi, -xi); velocity 0 is the rest velocity

// ---------------------------------------------------------------------------
// Host tables (built once per context, Sec. II A: departure points are
// tracked once at the start of a run, and equal cells share one table).
// ---------------------------------------------------------------------------

struct VelocitySet {
    int q;                    // 45 (D3Q45) or 19 (D2Q19)
    int dim;
    double xi[Q][3];          // first q rows used; z = 0 in two dimensions
    double w[Q];
    int opposite[Q];          // index of -xi_i
};

// set: SLLBM_D3Q45 or SLLBM_D2Q19; false for another value
bool build_velocity_set(VelocitySet &vs, int set = SLLBM_D3Q45);
void glc_points(int p, double *t);                       // t_k = (1 - cos(pi k/p))/2
void lagrange_basis(int p, double s, double *ell);       // ell_k(s) on the GLC points
void lagrange_basis_deriv(int p, double s, double *dl);  // d ell_k / ds
void clenshaw_curtis(int p, double *w);                  // weights on [-1,1]
// Per velocity i and axis a, the departure cells of the p nodes of a cell
// (displacement -xi_ia dt) are omin and omin + 1, the latter from node lstar
// on (lstar = p if none), and node l interpolates its cell with the weights
// w[i][a][l][0..p] (layout [Q][3][p][p+1]).
void build_cell_tables(const VelocitySet &vs, int p, const double h[3], double dt, std::vector<int32_t> &omin,
                       std::vector<int32_t> &lstar, std::vector<double> &w);

// Graded meshes (periodic, axis-aligned cells of unequal width): faces holds
// the n_el + 1 cell-face coordinates of the axis (empty: equal cells of
// length / n_el).  Node g = e*p + l sits at faces[e] + width_e t_l.
double axis_node_position(int p, int ne, double length, const std::vector<double> &faces, int g);
// Per-node departure tables of one axis: node g of velocity i interpolates
// the p + 1 source nodes src[i][g] + k (not wrapped: src is non-decreasing
// in g; reduce modulo n_el * p to address memory) with the weights
// w[i][g][k] (layout [Q][N][p+1]).
void build_node_tables(const VelocitySet &vs, int p, int ne, double length, const std::vector<double> &faces,
                       int axis, double dt, std::vector<int32_t> &src, std::vector<double> &w);
// The transpose of those per-node rows (for S^T): input node m of velocity i
// collects w[i][g][k] from every output g with src[i][g] + k = m (mod N); its
// readers are consecutive, g = srcT[i][m] + j, j < band, with weight
// wT[i][m][j] (layout [Q][N][kt], zero-padded).  band (out) is the largest
// count of readers; kt <= 0 only computes band.
void build_transposed_node_tables(int N, int p, const std::vector<int32_t> &src, const std::vector<double> &w,
                                  int kt, std::vector<int32_t> &srcT, std::vector<double> &wT, int &band);

// Source windows of the distorted-mesh streaming (MAPPED_TILE node tiles, x
// fastest): per velocity and tile, the departure cells of the tile's nodes
// unwrapped next to each node's own cell span [lo, hi] per axis; win holds
// the origin cell lo (wrapped) per axis and the window size in nodes
// ((hi - lo + 1) p + 1 per axis) packed as nx | ny << 10 | nz << 20, or 0 if
// the window exceeds max_nodes (that block gathers from global memory).
// Returns the largest window (nodes) of the blocks that stage one.
int build_mapped_windows(int q, int p, const int ne[3], const std::vector<int32_t> &cell, const int tile[3],
                         int max_nodes, std::vector<int32_t> &win);

// Distorted meshes: node displacements d ([3][N], periodic) of the equal-cell
// grid, each cell the degree-p interpolant of its nodes' positions.  For every
// velocity i and node n: the departure point's cell (linear cell index,
// x fastest) in cell[i*N + n] and its local coordinates in
// tloc[(a*q + i)*N + n]; the quadrature weight of every node (|det J| of the
// cells that hold it) in nodew; cjac: per cell point (cells x fastest, points
// x fastest within a cell) the inverse of the cell map's Jacobian
// J = I + dD/dr (9 values, row-major) and |det J|, for derivatives and
// quadrature in physical coordinates.  false (with why) if a cell map folds
// over or a departure search does not converge.
bool build_mapped_tables(const VelocitySet &vs, int p, const int ne[3], const double length[3], const double *d,
                         double dt, std::vector<int32_t> &cell, std::vector<double> &tloc, std::vector<double> &nodew,
                         std::vector<double> &cjac, std::string &why);

// Inverse departure lists of a distorted mesh (for the transposed
// streaming): per velocity i the nodes grouped by departure cell, increasing
// node index within a cell (a stable counting sort); the nodes departing into
// cell c are order[i*N + k] for k in [start[i*(C+1) + c], start[i*(C+1) + c + 1]),
// C = ncells.
void build_mapped_inverse(int q, int64_t nodes, int ncells, const std::vector<int32_t> &cell,
                          std::vector<int32_t> &order, std::vector<int32_t> &start);

// Velocities per pass of the transposed distorted-mesh streaming: the partial
// sums of a pass (2 (p+1)^3 values of elem bytes per cell and velocity) take
// at most the bytes of one state, or 256 MB if that is more
int mapped_t_chunk(int q, int p, int64_t ncells, size_t elem);

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Device-side parameter blocks (passed by value to kernels)
// ---------------------------------------------------------------------------

// Records the message of a failed call that has no context (returned by
// sllbm_last_error(NULL)); returns code.
int set_global_error(int code, const std::string &msg);

struct Geometry {
    int N[3];        // nodes per axis
    int nel[3];      // cells per axis
    int p;           // order
    int64_t nodes;   // N[0]*N[1]*N[2]
};

// Per-cell departure tables of the forward streaming, for each velocity i and
// axis a: omin = smallest departure-cell offset of the p rows, lstar = first
// row that uses cell omin + 1 (p if none), w = the p x (p+1) Lagrange weights.
template <typename S>
struct CellTables {
    const int32_t *omin;    // [q][3]
    const int32_t *lstar;   // [q][3]
    const S *w;             // [q][3][p][p+1]
};

// Per-node departure tables of a graded mesh (build_node_tables), one set
// per axis, in the storage type; wxm / wym bound the source window of an x-y
// tile of the graded streaming kernel over all velocities and tiles.
template <typename S>
struct NodeTables {
    const int32_t *src[3];  // [Q][N_a] first input node of each output node (not wrapped, non-decreasing)
    const S *w[3];          // [Q][N_a][k] weights of the k consecutive input nodes
    int k;                  // taps per output node (a value graded_taps_supported returns)
    int wxm, wym;
};

// GLC points of a cell and 1 / prod_{m != k} (t_k - t_m): ell_k(t) =
// inv_den[k] * prod_{m != k} (t - t_m)
struct GlcBasis {
    double t[MAXP + 1];
    double inv_den[MAXP + 1];
};

// Node tiles of the distorted-mesh streaming: one block per (tile, velocity)
// stages the source window of its departure cells in LDS.
constexpr int MAPPED_TX = 8, MAPPED_TY = 8, MAPPED_TZ = 4;   // 256 nodes
constexpr int MAPPED_WINDOW_BYTES = 48 * 1024;                // LDS for the f and g windows of a block
constexpr int MAPPED_MIN_WAVES = 5;                           // waves per SIMD the kernel is compiled for

// Device tables of a distorted mesh (build_mapped_tables); the local
// coordinates are kept in the storage type (FP32 contexts: 16 bytes per
// velocity and node instead of 28)
struct MappedTables {
    const int32_t *cell;    // [Q][N] departure cell, x fastest
    const void *tloc;       // [3][Q][N] local coordinates in [0, 1), storage type
    GlcBasis basis;
    const int32_t *win;     // [Q][tiles][4] source window per (velocity, tile), or NULL
    int win_nodes;          // largest window (nodes per population) of the blocks that use LDS
    const int32_t *inv_order;   // [Q][N] nodes by departure cell (build_mapped_inverse)
    const int32_t *inv_start;   // [Q][C + 1]
    void *partial;              // [qchunk][C][2][(p+1)^3] partial sums of the transposed streaming
    int qchunk;                 // velocities per pass (mapped_t_chunk)
};

struct CollisionParams {
    double dt;
    double Cv;        // 1/(gamma - 1)
    double beta;      // 2 C_v - D
    double inv_pr;    // 1/Pr
    double mu_inf;
    int law;          // SLLBM_SUTHERLAND / SLLBM_CONSTANT
};

// ---------------------------------------------------------------------------
// Launchers (kernels.hip).  All return hipError_t of the launch.
// ---------------------------------------------------------------------------

template <typename S>
struct Launch {
    static hipError_t collide_only(const Geometry &g, const CollisionParams &cp, S *state, hipStream_t st);
    static hipError_t collide_into(const Geometry &g, const CollisionParams &cp, const S *in, S *out,
                                   hipStream_t st);
    static hipError_t init_equilibrium(const Geometry &g, const CollisionParams &cp, const double *rho,
                                       const double *u, const double *T, S *state, hipStream_t st);
    static hipError_t moments(const Geometry &g, const CollisionParams &cp, const S *state, double *rho,
                              double *u, double *T, hipStream_t st);
    // nodew: the separable 1-D node weights; full_w (or NULL): per-node weights
    // of a distorted mesh, used instead
    static hipError_t totals(const Geometry &g, const CollisionParams &cp, const S *state,
                             const double *nodew, const double *full_w, double *partials, int nblocks, double *out5,
                             hipStream_t st);
    // h: cell width per axis; hw: graded cell widths (x, then y, then z cells) or NULL;
    // cjac: distorted mesh, per cell point J^-1 (9, row-major) and |det J| of the
    // cell map (build_mapped_tables), or NULL; full_w: per-node weights of a
    // distorted mesh (NULL: the separable nodew)
    static hipError_t loss(const Geometry &g, const S *state, const double *dmat, const double *ccw,
                           const double *h, const double *hw, const double *cjac, double *scratch_rho,
                           double *scratch_u, double *partials, int nblocks, double *out1, hipStream_t st);
    static hipError_t loss_grad(const Geometry &g, const S *state, const double *dmat, const double *ccw,
                                const double *nodew, const double *h, const double *hw, const double *cjac,
                                const double *full_w, double *scratch_rho, double *scratch_u, double *scratch_div,
                                double *partials, int nblocks, S *lam, hipStream_t st);
    // kinetic energy, solenoidal and dilatational dissipation (device out3)
    static hipError_t diagnostics(const Geometry &g, const CollisionParams &cp, const S *state, const double *dmat,
                                  const double *ccw, const double *h, const double *hw, const double *cjac,
                                  double *scratch_rho, double *scratch_u, double *scratch_T, double *partials,
                                  int nblocks, double *out3, hipStream_t st);
    // lam <- J_C(X_n)^T lam in place; dL/dmu_inf added to *dmu if not NULL
    static hipError_t collide_vjp(const Geometry &g, const CollisionParams &cp, const S *state_n, S *lam,
                                  double *dmu_partials, int nblocks, double *dmu, hipStream_t st);
    static hipError_t moments_vjp(const Geometry &g, const CollisionParams &cp, const S *state, const double *drho,
                                  const double *du, const double *dT, S *lam, hipStream_t st);
    static hipError_t init_equilibrium_vjp(const Geometry &g, const CollisionParams &cp, const double *rho,
                                           const double *u, const double *T, const S *lam0, double *drho,
                                           double *du, double *dT, hipStream_t st);
};

// The same node-local operations on the two-dimensional D2Q19 lattice
// (N_z = 1; velocity fields u are [2][N]; totals as out5 with zero z momentum).
template <typename S>
struct Launch2D {
    static hipError_t collide_into(const Geometry &g, const CollisionParams &cp, const S *in, S *out,
                                   hipStream_t st);
    static hipError_t init_equilibrium(const Geometry &g, const CollisionParams &cp, const double *rho,
                                       const double *u, const double *T, S *state, hipStream_t st);
    static hipError_t moments(const Geometry &g, const CollisionParams &cp, const S *state, double *rho,
                              double *u, double *T, hipStream_t st);
    static hipError_t totals(const Geometry &g, const S *state, const double *nodew, double *partials, int nblocks,
                             double *out5, hipStream_t st);
};

// two-dimensional streaming (stream2d.hip): per (velocity, population)
// plane, x-strips marching along y
// Mode algebra of the gradient workload (modes.hip).
constexpr int MAX_MODES = 64;
struct ModeAmplitudes {
    double a[MAX_MODES];
};
// out[k] = base[k] + sum_j am.a[j] basis[j n + k], k < n
hipError_t launch_superpose(int64_t n, int m, const ModeAmplitudes &am, const double *base, const double *basis,
                            double *out, hipStream_t st);
// out8[j] = sum_k basis[(m0 + j) n + k] v[k] for j < mc <= 8 (deterministic;
// partials holds nblocks * 8 doubles)
hipError_t launch_project_chunk(int64_t n, int m0, int mc, const double *basis, const double *v, double *partials,
                                int nblocks, double *out8, hipStream_t st);

template <typename S>
hipError_t launch_stream_2d(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st);

// forward streaming, z-march per (velocity, population) plane and x-y tile (stream.hip)
template <typename S>
hipError_t launch_stream_z(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st);
// transposed streaming S^T, the same march gathering over source-cell groups
// with the forward cell tables (stream.hip); any number of cells per axis
template <typename S>
hipError_t launch_stream_zt(const Geometry &g, const CellTables<S> &t, const S *in, S *out, hipStream_t st);
// streaming on a distorted mesh (stream_mapped.hip)
template <typename S>
hipError_t launch_stream_mapped(const Geometry &g, const MappedTables &t, const S *in, S *out, hipStream_t st);
// its transpose S^T (partial sums per departure cell, then per node; fixed
// order, no atomics; t.inv_order, t.partial required)
template <typename S>
hipError_t launch_stream_mapped_t(const Geometry &g, const MappedTables &t, const S *in, S *out, hipStream_t st);
// streaming on a graded mesh (stream_graded.hip)
template <typename S>
hipError_t launch_stream_graded(const Geometry &g, const NodeTables<S> &t, const S *in, S *out, hipStream_t st);
size_t graded_smem_bytes(int taps, int wxm, int wym, size_t elem);
int graded_window(const int32_t *src, int N, int taps, int T);
int graded_taps_supported(int taps);      // smallest supported tap count >= taps, 0 if none
int graded_tile_x();
int graded_window_pad(size_t elem);      // window rows are padded to this many nodes (16-byte loads)
int graded_max_window();                 // largest tile window (elements) the graded kernel takes
int graded_tile_y();

}  // namespace sllbm
