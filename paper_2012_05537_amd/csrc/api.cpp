// C ABI of the SLLBM library (declared in include/sllbm.h): argument
// validation, device memory, the step loop (collision, then streaming) and
// dispatch to the storage-type-specific launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sllbm_internal.h"

using namespace sllbm;

namespace {

constexpr int RED_BLOCKS = 1024;   // blocks of the deterministic reductions
constexpr int ADJ_BLOCKS = 4096;   // largest grid of the collision VJP (grid-stride beyond)

std::string g_create_error;

}  // namespace

struct sllbm_ctx {
    sllbm_config cfg{};
    Geometry geo{};
    VelocitySet vs{};
    CollisionParams cp{};
    int32_t *d_omin = nullptr, *d_lstar = nullptr;
    void *d_cw = nullptr;         // cell-table weights, storage type
    hipStream_t stream = nullptr;
    size_t elem = 8;
    bool d2 = false;              // two-dimensional lattice (D2Q19, N_z = 1)
    // State buffers: buf[cur] holds the pre-collision state X_k; the other
    // buffer receives C(X_k) during a step.
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    bool has_state = false;
    double *d_nodew = nullptr;     // [Nx + Ny + Nz] 1-D node quadrature weights
    double *d_ccw = nullptr;       // [p+1] Clenshaw-Curtis weights of a cell, mapped to [0, 1] per unit h
    double *d_dmat = nullptr;      // [(p+1)^2] d ell_m / ds at t_k
    double *d_partials = nullptr;  // [RED_BLOCKS * 8]
    double *d_small = nullptr;     // [16] reduction results
    double *d_scr_rho = nullptr;   // [N]   loss scratch
    double *d_scr_u = nullptr;     // [3N]
    double *d_scr_div = nullptr;   // [cells * (p+1)^3]
    double *d_scr_T = nullptr;     // [N]   diagnostics scratch
    double *d_adj_part = nullptr;  // [ADJ_BLOCKS] dmu_inf partials of the collision VJP
    // kernel timing: event pairs per launch kind (0 collision, 1 streaming)
    bool timing = false;
    std::vector<hipEvent_t> ev[2];
    int nev[2] = {0, 0};
    double h[3] = {0, 0, 0};       // cell widths (host)
    // graded mesh (sllbm_set_mesh): cell faces per graded axis (empty: equal
    // cells), per-node departure tables on the device
    bool graded = false;
    std::vector<double> faces[3];
    // per direction (0: S, 1: S^T) and axis
    int32_t *d_gsrc[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    void *d_gw[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int gk[2] = {0, 0}, gwxm[2] = {0, 0}, gwym[2] = {0, 0};
    double *d_hw = nullptr;        // graded cell widths: x cells, then y, then z (loss, diagnostics)
    // distorted mesh (sllbm_set_displacement): departure cells and local
    // coordinates per velocity and node, per-node quadrature weights
    bool mapped = false;
    int32_t *d_mcell = nullptr;
    void *d_mt = nullptr;          // local coordinates, storage type
    double *d_mw = nullptr;
    double *d_cjac = nullptr;      // per cell point J^-1 and |det J| of the cell map (loss, diagnostics)
    int32_t *d_mwin = nullptr;     // per (velocity, node tile) source window of the streaming
    int mwin_nodes = 0;            // largest staged window (nodes per population)
    int32_t *d_minv = nullptr;     // nodes by departure cell per velocity (transposed streaming)
    int32_t *d_minv_start = nullptr;
    void *d_mpart = nullptr;       // partial sums of the transposed streaming, mqchunk velocities
    int mqchunk = 0;
    GlcBasis glc{};
    std::string err;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int fail(sllbm_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

}  // namespace

// message of a failed call without a context (sllbm_last_error(NULL))
int sllbm::set_global_error(int code, const std::string &msg)
{
    g_create_error = msg;
    return code;
}

namespace {

int hip_fail(sllbm_ctx *c, hipError_t e, const char *what)
{
    return fail(c, SLLBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
hipError_t dalloc(T **p, size_t bytes)
{
    return hipMalloc(reinterpret_cast<void **>(p), bytes);
}

void free_ctx(sllbm_ctx *c)
{
    for (int k = 0; k < 2; ++k)
        for (hipEvent_t e : c->ev[k]) (void)hipEventDestroy(e);
    for (int k = 0; k < 2; ++k) (void)hipFree(c->buf[k]);
    for (int d = 0; d < 2; ++d)
        for (int a = 0; a < 3; ++a) {
            (void)hipFree(c->d_gsrc[d][a]);
            (void)hipFree(c->d_gw[d][a]);
        }
    (void)hipFree(c->d_hw);
    (void)hipFree(c->d_mcell);
    (void)hipFree(c->d_mt);
    (void)hipFree(c->d_mw);
    (void)hipFree(c->d_cjac);
    (void)hipFree(c->d_mwin);
    (void)hipFree(c->d_minv);
    (void)hipFree(c->d_minv_start);
    (void)hipFree(c->d_mpart);
    (void)hipFree(c->d_omin);
    (void)hipFree(c->d_lstar);
    (void)hipFree(c->d_cw);
    (void)hipFree(c->d_nodew);
    (void)hipFree(c->d_ccw);
    (void)hipFree(c->d_dmat);
    (void)hipFree(c->d_partials);
    (void)hipFree(c->d_small);
    (void)hipFree(c->d_scr_rho);
    (void)hipFree(c->d_scr_u);
    (void)hipFree(c->d_scr_div);
    (void)hipFree(c->d_scr_T);
    (void)hipFree(c->d_adj_part);
}

// departure tables of the forward streaming, in the storage type; the
// transposed streaming uses the same tables
template <typename S>
int upload_tables(sllbm_ctx *c, const double h[3])
{
    std::vector<int32_t> omin, lstar;
    std::vector<double> fw;
    build_cell_tables(c->vs, c->geo.p, h, c->cfg.dt, omin, lstar, fw);
    std::vector<S> fws(fw.begin(), fw.end());
    hipError_t e;
    if ((e = dalloc(&c->d_omin, omin.size() * sizeof(int32_t))) != hipSuccess ||
        (e = dalloc(&c->d_lstar, lstar.size() * sizeof(int32_t))) != hipSuccess ||
        (e = dalloc(reinterpret_cast<S **>(&c->d_cw), fws.size() * sizeof(S))) != hipSuccess)
        return fail(c, SLLBM_ENOMEM, std::string("table allocation: ") + hipGetErrorString(e));
    if ((e = hipMemcpy(c->d_omin, omin.data(), omin.size() * sizeof(int32_t), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(c->d_lstar, lstar.data(), lstar.size() * sizeof(int32_t), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(c->d_cw, fws.data(), fws.size() * sizeof(S), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "table upload");
    return SLLBM_OK;
}

template <typename S>
CellTables<S> cell_tables(const sllbm_ctx *c)
{
    return CellTables<S>{c->d_omin, c->d_lstar, static_cast<const S *>(c->d_cw)};
}

template <typename S>
NodeTables<S> node_tables(const sllbm_ctx *c, int dir)
{
    NodeTables<S> t{};
    for (int a = 0; a < 3; ++a) {
        t.src[a] = c->d_gsrc[dir][a];
        t.w[a] = static_cast<const S *>(c->d_gw[dir][a]);
    }
    t.k = c->gk[dir];
    t.wxm = c->gwxm[dir];
    t.wym = c->gwym[dir];
    return t;
}

bool is_fp64(const sllbm_ctx *c) { return c->cfg.precision == SLLBM_FP64; }

// calls that exist for the three-dimensional lattice only (adjoint, loss,
// diagnostics, graded meshes)
int refuse_2d(sllbm_ctx *c, const char *what)
{
    return fail(c, SLLBM_EINVAL, std::string(what) + " is not available on the two-dimensional lattice (D2Q19)");
}

// calls defined for axis-aligned cells only (transposed streaming and what
// builds on it, derivatives of the flow fields)
// per cell point J^-1 and |det J| of a distorted mesh (NULL otherwise)
const double *mapped_jac(const sllbm_ctx *c) { return c->mapped ? c->d_cjac : nullptr; }

int refuse_mapped(sllbm_ctx *c, const char *what)
{
    return fail(c, SLLBM_EINVAL, std::string(what) + " is not available on a distorted mesh");
}

MappedTables mapped_tables(const sllbm_ctx *c)
{
    return MappedTables{c->d_mcell, c->d_mt,        c->glc,  c->d_mwin, c->mwin_nodes,
                        c->d_minv,  c->d_minv_start, c->d_mpart, c->mqchunk};
}

const double *graded_hw(const sllbm_ctx *c) { return c->graded ? c->d_hw : nullptr; }

void *other(sllbm_ctx *c) { return c->buf[1 - c->cur]; }

int check_launch(sllbm_ctx *c, hipError_t e, const char *what)
{
    return e == hipSuccess ? SLLBM_OK : hip_fail(c, e, what);
}

// Per-node departure tables of the three axes (graded mesh) in the storage
// type, for S and for S^T, their tile windows, and the quadrature weights of
// the nodes.
template <typename S>
int upload_graded(sllbm_ctx *c)
{
    const Geometry &g = c->geo;
    const int p = g.p;
    hipError_t e;
    std::vector<int32_t> src[2][3];
    std::vector<double> w[2][3];
    int band = 1;
    for (int a = 0; a < 3; ++a) {
        build_node_tables(c->vs, p, g.nel[a], c->cfg.length[a], c->faces[a], a, c->cfg.dt, src[0][a], w[0][a]);
        int b = 1;
        build_transposed_node_tables(g.N[a], p, src[0][a], w[0][a], 0, src[1][a], w[1][a], b);
        band = std::max(band, b);
    }
    c->gk[0] = p + 1;
    c->gk[1] = graded_taps_supported(band);
    if (c->gk[1] == 0)
        return fail(c, SLLBM_EINVAL, "graded mesh: an input node is read by " + std::to_string(band) +
                                         " output nodes of one axis (at most 24 for the transposed streaming); "
                                         "the grading is too strong");
    for (int a = 0; a < 3; ++a) {
        int b = 1;
        build_transposed_node_tables(g.N[a], p, src[0][a], w[0][a], c->gk[1], src[1][a], w[1][a], b);
    }
    for (int d = 0; d < 2; ++d) {
        int wmax[2] = {0, 0};
        for (int a = 0; a < 3; ++a) {
            if (a < 2) {
                const int T = a == 0 ? graded_tile_x() : graded_tile_y();
                for (int i = 0; i < Q; ++i)
                    wmax[a] = std::max(wmax[a], graded_window(&src[d][a][static_cast<size_t>(i) * g.N[a]], g.N[a],
                                                              c->gk[d], T));
            }
            std::vector<S> ws(w[d][a].begin(), w[d][a].end());
            (void)hipFree(c->d_gsrc[d][a]);
            (void)hipFree(c->d_gw[d][a]);
            c->d_gsrc[d][a] = nullptr;
            c->d_gw[d][a] = nullptr;
            if ((e = dalloc(&c->d_gsrc[d][a], src[d][a].size() * sizeof(int32_t))) != hipSuccess ||
                (e = dalloc(reinterpret_cast<S **>(&c->d_gw[d][a]), ws.size() * sizeof(S))) != hipSuccess)
                return fail(c, SLLBM_ENOMEM, std::string("graded table allocation: ") + hipGetErrorString(e));
            if ((e = hipMemcpy(c->d_gsrc[d][a], src[d][a].data(), src[d][a].size() * sizeof(int32_t),
                               hipMemcpyHostToDevice)) != hipSuccess ||
                (e = hipMemcpy(c->d_gw[d][a], ws.data(), ws.size() * sizeof(S), hipMemcpyHostToDevice)) !=
                    hipSuccess)
                return hip_fail(c, e, "graded table upload");
        }
        // room for the 16-byte-aligned start of a window row: up to V - 1
        // more nodes, rows a multiple of V nodes long
        const int V = graded_window_pad(sizeof(S));
        c->gwxm[d] = (wmax[0] + V - 1 + V - 1) / V * V;
        c->gwym[d] = wmax[1];
        const size_t smem = graded_smem_bytes(c->gk[d], c->gwxm[d], c->gwym[d], sizeof(S));
        if (c->gwxm[d] * c->gwym[d] > graded_max_window())
            return fail(c, SLLBM_EINVAL, "graded mesh: the source window of a tile has " +
                                             std::to_string(c->gwxm[d] * c->gwym[d]) + " nodes (more than " +
                                             std::to_string(graded_max_window()) + "); the grading is too strong");
        if (smem > 160 * 1024)
            return fail(c, SLLBM_EINVAL, "graded mesh: the source window of a tile needs " + std::to_string(smem) +
                                             " bytes of LDS (more than 160 KB); the grading is too strong");
    }
    // node quadrature weights: Clenshaw-Curtis weight of the local point
    // times half the cell width; a cell's first point also carries the last
    // weight of the previous cell (periodic)
    double cc[MAXP + 1];
    clenshaw_curtis(p, cc);
    std::vector<double> nodew;
    for (int a = 0; a < 3; ++a) {
        const int ne = g.nel[a];
        auto width = [&](int el) {
            return c->faces[a].empty() ? c->cfg.length[a] / ne : c->faces[a][el + 1] - c->faces[a][el];
        };
        for (int n = 0; n < g.N[a]; ++n) {
            const int el = n / p, l = n % p;
            nodew.push_back(l == 0 ? 0.5 * (width(el) * cc[0] + width((el + ne - 1) % ne) * cc[p])
                                   : 0.5 * width(el) * cc[l]);
        }
    }
    if ((e = hipMemcpy(c->d_nodew, nodew.data(), nodew.size() * sizeof(double), hipMemcpyHostToDevice)) !=
        hipSuccess)
        return hip_fail(c, e, "node weight upload");
    std::vector<double> hw;
    for (int a = 0; a < 3; ++a)
        for (int el = 0; el < g.nel[a]; ++el)
            hw.push_back(c->faces[a].empty() ? c->cfg.length[a] / g.nel[a] : c->faces[a][el + 1] - c->faces[a][el]);
    (void)hipFree(c->d_hw);
    c->d_hw = nullptr;
    if ((e = dalloc(&c->d_hw, hw.size() * sizeof(double))) != hipSuccess)
        return fail(c, SLLBM_ENOMEM, std::string("cell width allocation: ") + hipGetErrorString(e));
    if ((e = hipMemcpy(c->d_hw, hw.data(), hw.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "cell width upload");
    return SLLBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------

extern "C" {

int sllbm_velocity_set(double *xi, double *w)
{
    if (!xi || !w) return SLLBM_EINVAL;
    return sllbm_lattice(SLLBM_D3Q45, xi, w);
}

int sllbm_lattice(int32_t velocity_set, double *xi, double *w)
{
    if (!xi || !w) return -1;
    VelocitySet vs;
    if (!build_velocity_set(vs, velocity_set)) return -1;
    for (int i = 0; i < vs.q; ++i) {
        for (int k = 0; k < 3; ++k) xi[3 * i + k] = vs.xi[i][k];
        w[i] = vs.w[i];
    }
    return vs.q;
}

const char *sllbm_last_error(const sllbm_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int64_t sllbm_num_nodes(const sllbm_ctx *ctx) { return ctx ? ctx->geo.nodes : -1; }

int64_t sllbm_state_bytes(const sllbm_ctx *ctx)
{
    return ctx ? static_cast<int64_t>(2 * ctx->vs.q) * ctx->geo.nodes * static_cast<int64_t>(ctx->elem) : -1;
}

int sllbm_create(const sllbm_config *cfg, sllbm_ctx **out)
{
    if (!out) return fail(nullptr, SLLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(nullptr, SLLBM_EINVAL, "cfg is NULL");
    if (cfg->velocity_set != SLLBM_D3Q45 && cfg->velocity_set != SLLBM_D2Q19)
        return fail(nullptr, SLLBM_EINVAL, "velocity_set must be SLLBM_D3Q45 or SLLBM_D2Q19");
    const bool d2 = cfg->velocity_set == SLLBM_D2Q19;
    if (cfg->order < 1 || cfg->order > MAXP) return fail(nullptr, SLLBM_EINVAL, "order must be in 1..6");
    for (int a = 0; a < (d2 ? 2 : 3); ++a) {
        if (cfg->n_el[a] < 1) return fail(nullptr, SLLBM_EINVAL, "n_el must be >= 1");
        if (!(cfg->length[a] > 0.0) || !std::isfinite(cfg->length[a]))
            return fail(nullptr, SLLBM_EINVAL, "length must be positive");
    }
    if (d2 && cfg->n_el[2] != 1) return fail(nullptr, SLLBM_EINVAL, "n_el[2] must be 1 for SLLBM_D2Q19");
    const int64_t nz = d2 ? 1 : static_cast<int64_t>(cfg->n_el[2]) * cfg->order;
    const int64_t nodes = static_cast<int64_t>(cfg->n_el[0]) * cfg->order * cfg->n_el[1] * cfg->order * nz;
    if (static_cast<int64_t>(cfg->n_el[0]) * cfg->order > (1 << 20) ||
        static_cast<int64_t>(cfg->n_el[1]) * cfg->order > (1 << 20) ||
        static_cast<int64_t>(cfg->n_el[2]) * cfg->order > (1 << 20) || nodes >= (int64_t(1) << 31))
        return fail(nullptr, SLLBM_EINVAL, "grid too large");
    if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return fail(nullptr, SLLBM_EINVAL, "dt must be positive");
    if (!(cfg->gamma > 1.0)) return fail(nullptr, SLLBM_EINVAL, "gamma must exceed 1");
    if (!(cfg->prandtl > 0.0)) return fail(nullptr, SLLBM_EINVAL, "prandtl must be positive");
    if (!(cfg->mu_inf > 0.0) || !std::isfinite(cfg->mu_inf))
        return fail(nullptr, SLLBM_EINVAL, "mu_inf must be positive");
    if (cfg->viscosity_law != SLLBM_SUTHERLAND && cfg->viscosity_law != SLLBM_CONSTANT)
        return fail(nullptr, SLLBM_EINVAL, "unknown viscosity_law");
    if (cfg->precision != SLLBM_FP64 && cfg->precision != SLLBM_FP32_MIXED)
        return fail(nullptr, SLLBM_EINVAL, "unknown precision");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(nullptr, SLLBM_EDEVICE, "no HIP device available");
    if (cfg->device < 0 || cfg->device >= ndev) return fail(nullptr, SLLBM_EINVAL, "device ordinal out of range");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess)
        return fail(nullptr, SLLBM_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, SLLBM_EDEVICE, std::string("library is built for gfx950, device is ") + prop.gcnArchName);

    DeviceGuard guard(cfg->device);
    sllbm_ctx *c = new sllbm_ctx();
    c->cfg = *cfg;
    c->elem = cfg->precision == SLLBM_FP64 ? sizeof(double) : sizeof(float);
    c->d2 = d2;
    Geometry &g = c->geo;
    g.p = cfg->order;
    for (int a = 0; a < 3; ++a) {
        g.nel[a] = cfg->n_el[a];
        g.N[a] = cfg->n_el[a] * cfg->order;
    }
    if (d2) g.N[2] = 1;                       // one node across z
    g.nodes = nodes;
    c->cp.dt = cfg->dt;
    c->cp.Cv = 1.0 / (cfg->gamma - 1.0);
    c->cp.beta = 2.0 * c->cp.Cv - (d2 ? 2.0 : 3.0);   // g^eq = (2 C_v - D) T f^eq
    c->cp.inv_pr = 1.0 / cfg->prandtl;
    c->cp.mu_inf = cfg->mu_inf;
    c->cp.law = cfg->viscosity_law;

    build_velocity_set(c->vs, cfg->velocity_set);
    double h[3];
    for (int a = 0; a < 3; ++a) c->h[a] = h[a] = cfg->length[a] / cfg->n_el[a];
    if (d2) c->h[2] = h[2] = 1.0;             // no z axis: unit width (xi_z = 0)

    auto bail = [&](int rc) {
        g_create_error = c->err;
        free_ctx(c);
        delete c;
        return rc;
    };
    int rc = is_fp64(c) ? upload_tables<double>(c, h) : upload_tables<float>(c, h);
    if (rc != SLLBM_OK) return bail(rc);

    const size_t sb = static_cast<size_t>(sllbm_state_bytes(c));
    hipError_t e;
    if ((e = hipMalloc(&c->buf[0], sb)) != hipSuccess || (e = hipMalloc(&c->buf[1], sb)) != hipSuccess)
        return bail(fail(c, SLLBM_ENOMEM, "state allocation of " + std::to_string(sb) + " bytes failed"));

    // quadrature weights and derivative matrix
    const int p = g.p;
    double cc[MAXP + 1], t[MAXP + 1];
    clenshaw_curtis(p, cc);
    glc_points(p, t);
    std::vector<double> nodew;
    for (int a = 0; a < 3; ++a)
        for (int n = 0; n < g.N[a]; ++n) {
            const int l = n % p;
            nodew.push_back(d2 && a == 2 ? 1.0 : 0.5 * h[a] * (l == 0 ? cc[0] + cc[p] : cc[l]));
        }
    std::vector<double> dmat((p + 1) * (p + 1));
    for (int k = 0; k <= p; ++k) {
        double dl[MAXP + 1];
        lagrange_basis_deriv(p, t[k], dl);
        for (int m = 0; m <= p; ++m) dmat[k * (p + 1) + m] = dl[m];
    }
    const int64_t cells = static_cast<int64_t>(g.nel[0]) * g.nel[1] * g.nel[2];
    const int64_t cpts = cells * (p + 1) * (p + 1) * (p + 1);
    if ((e = dalloc(&c->d_nodew, nodew.size() * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_ccw, (p + 1) * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_dmat, dmat.size() * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_partials, RED_BLOCKS * 8 * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_small, 16 * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_scr_rho, nodes * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_scr_u, 3 * nodes * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_scr_div, cpts * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_scr_T, nodes * sizeof(double))) != hipSuccess ||
        (e = dalloc(&c->d_adj_part, ADJ_BLOCKS * sizeof(double))) != hipSuccess)
        return bail(fail(c, SLLBM_ENOMEM, std::string("allocation failed: ") + hipGetErrorString(e)));
    if ((e = hipMemcpy(c->d_nodew, nodew.data(), nodew.size() * sizeof(double), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(c->d_ccw, cc, (p + 1) * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_dmat, dmat.data(), dmat.size() * sizeof(double), hipMemcpyHostToDevice)) !=
            hipSuccess)
        return bail(hip_fail(c, e, "upload"));
    *out = c;
    return SLLBM_OK;
}

int sllbm_destroy(sllbm_ctx *ctx)
{
    if (!ctx) return SLLBM_OK;
    {
        DeviceGuard guard(ctx->cfg.device);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        else (void)hipDeviceSynchronize();
        free_ctx(ctx);
    }
    delete ctx;
    return SLLBM_OK;
}

int sllbm_set_stream(sllbm_ctx *ctx, void *hip_stream)
{
    if (!ctx) return SLLBM_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return SLLBM_OK;
}

int sllbm_node_coords(const sllbm_ctx *ctx, double *x, double *y, double *z)
{
    if (!ctx || !x || !y || !z) return SLLBM_EINVAL;
    double *out[3] = {x, y, z};
    const int p = ctx->geo.p;
    for (int a = 0; a < 3; ++a)
        for (int n = 0; n < ctx->geo.N[a]; ++n)
            out[a][n] = axis_node_position(p, ctx->cfg.n_el[a], ctx->cfg.length[a], ctx->faces[a], n);
    return SLLBM_OK;
}

int sllbm_set_mesh(sllbm_ctx *ctx, const double *widths_x, const double *widths_y, const double *widths_z)
{
    if (!ctx) return SLLBM_EINVAL;
    const double *wd[3] = {widths_x, widths_y, widths_z};
    if (ctx->d2) return refuse_2d(ctx, "sllbm_set_mesh");
    if (ctx->mapped) return refuse_mapped(ctx, "sllbm_set_mesh");
    if (!wd[0] && !wd[1] && !wd[2]) return fail(ctx, SLLBM_EINVAL, "set_mesh: no graded axis given");
    std::vector<double> faces[3];
    for (int a = 0; a < 3; ++a) {
        if (!wd[a]) continue;
        faces[a].assign(1, 0.0);
        for (int e = 0; e < ctx->cfg.n_el[a]; ++e) {
            if (!(wd[a][e] > 0.0) || !std::isfinite(wd[a][e]))
                return fail(ctx, SLLBM_EINVAL, "set_mesh: cell widths must be positive and finite");
            faces[a].push_back(faces[a].back() + wd[a][e]);
        }
    }
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "set_mesh");
    std::vector<double> old_faces[3];
    double old_length[3];
    const bool was_graded = ctx->graded;
    for (int a = 0; a < 3; ++a) {
        old_faces[a] = ctx->faces[a];
        old_length[a] = ctx->cfg.length[a];
        if (faces[a].empty()) continue;
        ctx->cfg.length[a] = faces[a].back();
        ctx->faces[a] = faces[a];
    }
    auto upload = [&]() { return is_fp64(ctx) ? upload_graded<double>(ctx) : upload_graded<float>(ctx); };
    const int rc = upload();
    if (rc == SLLBM_OK) {
        ctx->graded = true;
        return SLLBM_OK;
    }
    // keep the previous mesh (its tables are rebuilt if it was graded)
    const std::string msg = ctx->err;
    for (int a = 0; a < 3; ++a) {
        ctx->faces[a] = old_faces[a];
        ctx->cfg.length[a] = old_length[a];
    }
    ctx->graded = was_graded && upload() == SLLBM_OK;
    ctx->err = msg;
    return rc;
}

int sllbm_set_displacement(sllbm_ctx *ctx, const double *d)
{
    if (!ctx) return SLLBM_EINVAL;
    if (ctx->d2) return refuse_2d(ctx, "sllbm_set_displacement");
    if (ctx->graded) return fail(ctx, SLLBM_EINVAL, "set_displacement: the mesh has graded cells");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "set_displacement");
    auto drop = [&]() {
        (void)hipFree(ctx->d_mcell);
        (void)hipFree(ctx->d_mt);
        (void)hipFree(ctx->d_mw);
        (void)hipFree(ctx->d_cjac);
        (void)hipFree(ctx->d_mwin);
        (void)hipFree(ctx->d_minv);
        (void)hipFree(ctx->d_minv_start);
        (void)hipFree(ctx->d_mpart);
        ctx->d_mcell = nullptr;
        ctx->d_mt = nullptr;
        ctx->d_mw = nullptr;
        ctx->d_cjac = nullptr;
        ctx->d_mwin = nullptr;
        ctx->mwin_nodes = 0;
        ctx->d_minv = nullptr;
        ctx->d_minv_start = nullptr;
        ctx->d_mpart = nullptr;
        ctx->mqchunk = 0;
        ctx->mapped = false;
    };
    if (!d) {
        drop();
        return SLLBM_OK;
    }
    const int64_t N = ctx->geo.nodes;
    for (int64_t k = 0; k < 3 * N; ++k)
        if (!std::isfinite(d[k])) return fail(ctx, SLLBM_EINVAL, "set_displacement: non-finite displacement");
    std::vector<int32_t> cell;
    std::vector<double> tloc, nodew, cjac;
    std::string why;
    if (!build_mapped_tables(ctx->vs, ctx->geo.p, ctx->geo.nel, ctx->cfg.length, d, ctx->cfg.dt, cell, tloc, nodew,
                             cjac, why))
        return fail(ctx, SLLBM_EINVAL, why);
    std::vector<int32_t> mwin;
    const int tile[3] = {MAPPED_TX, MAPPED_TY, MAPPED_TZ};
    const int win_nodes = build_mapped_windows(ctx->vs.q, ctx->geo.p, ctx->geo.nel, cell, tile,
                                               MAPPED_WINDOW_BYTES / (2 * static_cast<int>(ctx->elem)), mwin);
    const int ncells = ctx->geo.nel[0] * ctx->geo.nel[1] * ctx->geo.nel[2];
    std::vector<int32_t> minv, minv_start;
    build_mapped_inverse(ctx->vs.q, N, ncells, cell, minv, minv_start);
    const int qchunk = mapped_t_chunk(ctx->vs.q, ctx->geo.p, ncells, ctx->elem);
    const int k3 = (ctx->geo.p + 1) * (ctx->geo.p + 1) * (ctx->geo.p + 1);
    const size_t pbytes = static_cast<size_t>(qchunk) * ncells * 2 * k3 * ctx->elem;
    int32_t *dc = nullptr, *dwin = nullptr, *dinv = nullptr, *dinvs = nullptr;
    void *dt = nullptr, *dpart = nullptr;
    double *dw = nullptr, *dj = nullptr;
    auto free_new = [&]() {
        (void)hipFree(dc);
        (void)hipFree(dt);
        (void)hipFree(dw);
        (void)hipFree(dj);
        (void)hipFree(dwin);
        (void)hipFree(dinv);
        (void)hipFree(dinvs);
        (void)hipFree(dpart);
    };
    // local coordinates in the storage type
    std::vector<float> tloc32;
    const void *tsrc = tloc.data();
    if (!is_fp64(ctx)) {
        tloc32.assign(tloc.begin(), tloc.end());
        tsrc = tloc32.data();
    }
    const size_t tbytes = tloc.size() * ctx->elem;
    if ((e = dalloc(&dc, cell.size() * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&dt, tbytes)) != hipSuccess ||
        (e = dalloc(&dw, nodew.size() * sizeof(double))) != hipSuccess ||
        (e = dalloc(&dj, cjac.size() * sizeof(double))) != hipSuccess ||
        (e = dalloc(&dwin, mwin.size() * sizeof(int32_t))) != hipSuccess ||
        (e = dalloc(&dinv, minv.size() * sizeof(int32_t))) != hipSuccess ||
        (e = dalloc(&dinvs, minv_start.size() * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&dpart, pbytes)) != hipSuccess) {
        free_new();
        return fail(ctx, SLLBM_ENOMEM, std::string("distorted-mesh tables: ") + hipGetErrorString(e));
    }
    if ((e = hipMemcpy(dc, cell.data(), cell.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(dt, tsrc, tbytes, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(dw, nodew.data(), nodew.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(dj, cjac.data(), cjac.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(dwin, mwin.data(), mwin.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(dinv, minv.data(), minv.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(dinvs, minv_start.data(), minv_start.size() * sizeof(int32_t), hipMemcpyHostToDevice)) !=
            hipSuccess) {
        free_new();
        return hip_fail(ctx, e, "distorted-mesh table upload");
    }
    drop();
    ctx->d_mcell = dc;
    ctx->d_mt = dt;
    ctx->d_mw = dw;
    ctx->d_cjac = dj;
    ctx->d_mwin = dwin;
    ctx->mwin_nodes = win_nodes;
    ctx->d_minv = dinv;
    ctx->d_minv_start = dinvs;
    ctx->d_mpart = dpart;
    ctx->mqchunk = qchunk;
    const int p = ctx->geo.p;
    glc_points(p, ctx->glc.t);
    for (int k = 0; k <= p; ++k) {
        double den = 1.0;
        for (int m = 0; m <= p; ++m)
            if (m != k) den *= ctx->glc.t[k] - ctx->glc.t[m];
        ctx->glc.inv_den[k] = 1.0 / den;
    }
    ctx->mapped = true;
    return SLLBM_OK;
}

int sllbm_set_viscosity(sllbm_ctx *ctx, double mu_inf)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!(mu_inf > 0.0) || !std::isfinite(mu_inf)) return fail(ctx, SLLBM_EINVAL, "mu_inf must be positive");
    ctx->cfg.mu_inf = mu_inf;
    ctx->cp.mu_inf = mu_inf;
    return SLLBM_OK;
}

int sllbm_init_equilibrium(sllbm_ctx *ctx, const double *rho, const double *u, const double *T)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!rho || !u || !T) return fail(ctx, SLLBM_EINVAL, "NULL field");
    DeviceGuard guard(ctx->cfg.device);
    void *st = ctx->buf[ctx->cur];
    hipError_t e;
    if (ctx->d2)
        e = is_fp64(ctx) ? Launch2D<double>::init_equilibrium(ctx->geo, ctx->cp, rho, u, T, static_cast<double *>(st),
                                                              ctx->stream)
                         : Launch2D<float>::init_equilibrium(ctx->geo, ctx->cp, rho, u, T, static_cast<float *>(st),
                                                             ctx->stream);
    else
        e = is_fp64(ctx) ? Launch<double>::init_equilibrium(ctx->geo, ctx->cp, rho, u, T, static_cast<double *>(st),
                                                            ctx->stream)
                         : Launch<float>::init_equilibrium(ctx->geo, ctx->cp, rho, u, T, static_cast<float *>(st),
                                                           ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "init_equilibrium");
    ctx->has_state = true;
    return SLLBM_OK;
}

int sllbm_set_state(sllbm_ctx *ctx, const void *state)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!state) return fail(ctx, SLLBM_EINVAL, "NULL state");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = hipMemcpyAsync(ctx->buf[ctx->cur], state, sllbm_state_bytes(ctx), hipMemcpyDeviceToDevice,
                                  ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "set_state");
    ctx->has_state = true;
    return SLLBM_OK;
}

int sllbm_get_state(sllbm_ctx *ctx, void *state)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!state) return fail(ctx, SLLBM_EINVAL, "NULL state");
    if (!ctx->has_state) return fail(ctx, SLLBM_ESTATE, "no state set");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e =
        hipMemcpyAsync(state, ctx->buf[ctx->cur], sllbm_state_bytes(ctx), hipMemcpyDeviceToDevice, ctx->stream);
    return check_launch(ctx, e, "get_state");
}

static hipError_t collide_into(sllbm_ctx *c, const void *in, void *out)
{
    if (c->d2) {
        if (is_fp64(c))
            return Launch2D<double>::collide_into(c->geo, c->cp, static_cast<const double *>(in),
                                                  static_cast<double *>(out), c->stream);
        return Launch2D<float>::collide_into(c->geo, c->cp, static_cast<const float *>(in), static_cast<float *>(out),
                                             c->stream);
    }
    if (is_fp64(c))
        return Launch<double>::collide_into(c->geo, c->cp, static_cast<const double *>(in), static_cast<double *>(out),
                                            c->stream);
    return Launch<float>::collide_into(c->geo, c->cp, static_cast<const float *>(in), static_cast<float *>(out),
                                       c->stream);
}

static hipError_t stream_into(sllbm_ctx *c, const void *in, void *out)
{
    if (c->mapped) {
        if (is_fp64(c))
            return launch_stream_mapped<double>(c->geo, mapped_tables(c), static_cast<const double *>(in),
                                                static_cast<double *>(out), c->stream);
        return launch_stream_mapped<float>(c->geo, mapped_tables(c), static_cast<const float *>(in),
                                           static_cast<float *>(out), c->stream);
    }
    if (c->d2) {
        if (is_fp64(c))
            return launch_stream_2d<double>(c->geo, cell_tables<double>(c), static_cast<const double *>(in),
                                            static_cast<double *>(out), c->stream);
        return launch_stream_2d<float>(c->geo, cell_tables<float>(c), static_cast<const float *>(in),
                                       static_cast<float *>(out), c->stream);
    }
    if (c->graded) {
        if (is_fp64(c))
            return launch_stream_graded<double>(c->geo, node_tables<double>(c, 0), static_cast<const double *>(in),
                                                static_cast<double *>(out), c->stream);
        return launch_stream_graded<float>(c->geo, node_tables<float>(c, 0), static_cast<const float *>(in),
                                           static_cast<float *>(out), c->stream);
    }
    if (is_fp64(c))
        return launch_stream_z<double>(c->geo, cell_tables<double>(c), static_cast<const double *>(in),
                                       static_cast<double *>(out), c->stream);
    return launch_stream_z<float>(c->geo, cell_tables<float>(c), static_cast<const float *>(in),
                                  static_cast<float *>(out), c->stream);
}

// S^T: the transposed z-march (equal cells) or the graded march over the
// transposed per-node tables
static hipError_t stream_t_into(sllbm_ctx *c, const void *in, void *out)
{
    if (c->mapped) {
        if (is_fp64(c))
            return launch_stream_mapped_t<double>(c->geo, mapped_tables(c), static_cast<const double *>(in),
                                                  static_cast<double *>(out), c->stream);
        return launch_stream_mapped_t<float>(c->geo, mapped_tables(c), static_cast<const float *>(in),
                                             static_cast<float *>(out), c->stream);
    }
    if (c->graded) {
        if (is_fp64(c))
            return launch_stream_graded<double>(c->geo, node_tables<double>(c, 1), static_cast<const double *>(in),
                                                static_cast<double *>(out), c->stream);
        return launch_stream_graded<float>(c->geo, node_tables<float>(c, 1), static_cast<const float *>(in),
                                           static_cast<float *>(out), c->stream);
    }
    if (is_fp64(c))
        return launch_stream_zt<double>(c->geo, cell_tables<double>(c), static_cast<const double *>(in),
                                        static_cast<double *>(out), c->stream);
    return launch_stream_zt<float>(c->geo, cell_tables<float>(c), static_cast<const float *>(in),
                                   static_cast<float *>(out), c->stream);
}

// n steps X <- S(C(X)): collision in place and streaming into the other
// buffer, which becomes the state; with a record, collision into the spare
// buffer and streaming into record slot s, from which the next step collides.
static int step_impl(sllbm_ctx *ctx, int32_t n, char *record, int64_t stride)
{
    if (!ctx) return SLLBM_EINVAL;
    if (n < 0) return fail(ctx, SLLBM_EINVAL, "negative step count");
    if (!ctx->has_state) return fail(ctx, SLLBM_ESTATE, "no state set");
    if (n == 0) return SLLBM_OK;
    DeviceGuard guard(ctx->cfg.device);
    void *state = ctx->buf[ctx->cur], *post = other(ctx);
    // event pair around a launch of kind k, if timing is on and events remain
    auto mark = [&](int k, int half) {
        if (ctx->timing && ctx->nev[k] < static_cast<int>(ctx->ev[k].size()) / 2) {
            (void)hipEventRecord(ctx->ev[k][2 * ctx->nev[k] + half], ctx->stream);
            if (half) ++ctx->nev[k];
        }
    };
    for (int32_t s = 0; s < n; ++s) {
        hipError_t e;
        if (!record) {
            // collide the state in place, stream it into the other buffer, swap:
            // each kernel then reads and writes one buffer's worth of lines
            mark(0, 0);
            if ((e = collide_into(ctx, state, state)) != hipSuccess) return hip_fail(ctx, e, "collide");
            mark(0, 1);
            mark(1, 0);
            if ((e = stream_into(ctx, state, post)) != hipSuccess) return hip_fail(ctx, e, "stream");
            mark(1, 1);
            ctx->cur = 1 - ctx->cur;
            state = ctx->buf[ctx->cur];
            post = other(ctx);
            continue;
        }
        const void *src = s > 0 ? record + static_cast<int64_t>(s - 1) * stride : state;
        void *dst = record + static_cast<int64_t>(s) * stride;
        mark(0, 0);
        if ((e = collide_into(ctx, src, post)) != hipSuccess) return hip_fail(ctx, e, "collide");
        mark(0, 1);
        mark(1, 0);
        if ((e = stream_into(ctx, post, dst)) != hipSuccess) return hip_fail(ctx, e, "stream");
        mark(1, 1);
    }
    if (record) {
        hipError_t e = hipMemcpyAsync(state, record + static_cast<int64_t>(n - 1) * stride, sllbm_state_bytes(ctx),
                                      hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "record copy");
    }
    return SLLBM_OK;
}

int sllbm_step(sllbm_ctx *ctx, int32_t n) { return step_impl(ctx, n, nullptr, 0); }

int sllbm_set_kernel_timing(sllbm_ctx *ctx, int32_t on)
{
    if (!ctx) return SLLBM_EINVAL;
    DeviceGuard guard(ctx->cfg.device);
    if (on && ctx->ev[0].empty()) {
        for (int k = 0; k < 2; ++k) {
            ctx->ev[k].resize(2 * 4096);
            for (auto &e : ctx->ev[k]) {
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) {
                    e = nullptr;
                    return hip_fail(ctx, r, "hipEventCreate");
                }
            }
        }
    }
    ctx->timing = on != 0;
    ctx->nev[0] = ctx->nev[1] = 0;
    return SLLBM_OK;
}

int sllbm_kernel_times(sllbm_ctx *ctx, double *out)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!out) return fail(ctx, SLLBM_EINVAL, "NULL out");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "synchronize");
    for (int k = 0; k < 2; ++k) {
        double total = 0.0;
        for (int j = 0; j < ctx->nev[k]; ++j) {
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, ctx->ev[k][2 * j], ctx->ev[k][2 * j + 1])) != hipSuccess)
                return hip_fail(ctx, e, "hipEventElapsedTime");
            total += ms;
        }
        out[2 * k] = total;
        out[2 * k + 1] = ctx->nev[k];
        ctx->nev[k] = 0;
    }
    return SLLBM_OK;
}

int sllbm_step_record(sllbm_ctx *ctx, int32_t n, void *states, int64_t stride_bytes)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!states && n > 0) return fail(ctx, SLLBM_EINVAL, "NULL record buffer");
    if (n > 1 && stride_bytes < sllbm_state_bytes(ctx)) return fail(ctx, SLLBM_EINVAL, "record stride too small");
    return step_impl(ctx, n, static_cast<char *>(states), stride_bytes);
}

int sllbm_moments(sllbm_ctx *ctx, double *rho, double *u, double *T)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!ctx->has_state) return fail(ctx, SLLBM_ESTATE, "no state set");
    DeviceGuard guard(ctx->cfg.device);
    const void *st = ctx->buf[ctx->cur];
    hipError_t e;
    if (ctx->d2)
        e = is_fp64(ctx) ? Launch2D<double>::moments(ctx->geo, ctx->cp, static_cast<const double *>(st), rho, u, T,
                                                     ctx->stream)
                         : Launch2D<float>::moments(ctx->geo, ctx->cp, static_cast<const float *>(st), rho, u, T,
                                                    ctx->stream);
    else
        e = is_fp64(ctx) ? Launch<double>::moments(ctx->geo, ctx->cp, static_cast<const double *>(st), rho, u, T,
                                                   ctx->stream)
                         : Launch<float>::moments(ctx->geo, ctx->cp, static_cast<const float *>(st), rho, u, T,
                                                  ctx->stream);
    return check_launch(ctx, e, "moments");
}

int sllbm_totals(sllbm_ctx *ctx, double *out)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!out) return fail(ctx, SLLBM_EINVAL, "NULL out");
    if (!ctx->has_state) return fail(ctx, SLLBM_ESTATE, "no state set");
    DeviceGuard guard(ctx->cfg.device);
    const void *st = ctx->buf[ctx->cur];
    hipError_t e;
    if (ctx->d2)
        e = is_fp64(ctx) ? Launch2D<double>::totals(ctx->geo, static_cast<const double *>(st), ctx->d_nodew,
                                                    ctx->d_partials, RED_BLOCKS, ctx->d_small, ctx->stream)
                         : Launch2D<float>::totals(ctx->geo, static_cast<const float *>(st), ctx->d_nodew,
                                                   ctx->d_partials, RED_BLOCKS, ctx->d_small, ctx->stream);
    else
        e = is_fp64(ctx) ? Launch<double>::totals(ctx->geo, ctx->cp, static_cast<const double *>(st), ctx->d_nodew,
                                                  ctx->mapped ? ctx->d_mw : nullptr, ctx->d_partials, RED_BLOCKS,
                                                  ctx->d_small, ctx->stream)
                         : Launch<float>::totals(ctx->geo, ctx->cp, static_cast<const float *>(st), ctx->d_nodew,
                                                 ctx->mapped ? ctx->d_mw : nullptr, ctx->d_partials, RED_BLOCKS,
                                                 ctx->d_small, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "totals");
    if ((e = hipMemcpyAsync(out, ctx->d_small, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
        return hip_fail(ctx, e, "totals copy");
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(out[k])) return fail(ctx, SLLBM_ENONFINITE, "non-finite totals");
    return SLLBM_OK;
}

int sllbm_stream(sllbm_ctx *ctx, const void *in, void *out, int32_t transpose)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!in || !out || in == out) return fail(ctx, SLLBM_EINVAL, "bad stream buffers");
    if (transpose && ctx->d2) return refuse_2d(ctx, "transposed streaming");
    DeviceGuard guard(ctx->cfg.device);
    if (!transpose) return check_launch(ctx, stream_into(ctx, in, out), "stream");
    return check_launch(ctx, stream_t_into(ctx, in, out), "stream");
}

int sllbm_collide(sllbm_ctx *ctx, void *state)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!state) return fail(ctx, SLLBM_EINVAL, "NULL state");
    DeviceGuard guard(ctx->cfg.device);
    return check_launch(ctx, collide_into(ctx, state, state), "collide");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Reverse mode
// ---------------------------------------------------------------------------
extern "C" {

int sllbm_loss(sllbm_ctx *ctx, const void *state, double *out)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!state || !out) return fail(ctx, SLLBM_EINVAL, "NULL argument");
    if (ctx->d2) return refuse_2d(ctx, "sllbm_loss");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = is_fp64(ctx)
        ? Launch<double>::loss(ctx->geo, static_cast<const double *>(state), ctx->d_dmat, ctx->d_ccw, ctx->h,
                               graded_hw(ctx), mapped_jac(ctx), ctx->d_scr_rho, ctx->d_scr_u, ctx->d_partials,
                               RED_BLOCKS, ctx->d_small, ctx->stream)
        : Launch<float>::loss(ctx->geo, static_cast<const float *>(state), ctx->d_dmat, ctx->d_ccw, ctx->h,
                              graded_hw(ctx), mapped_jac(ctx), ctx->d_scr_rho, ctx->d_scr_u, ctx->d_partials,
                              RED_BLOCKS, ctx->d_small, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "loss");
    if ((e = hipMemcpyAsync(out, ctx->d_small, sizeof(double), hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
        return hip_fail(ctx, e, "loss copy");
    if (!std::isfinite(*out)) return fail(ctx, SLLBM_ENONFINITE, "non-finite loss");
    return SLLBM_OK;
}

int sllbm_diagnostics(sllbm_ctx *ctx, const void *state, double *out)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!out) return fail(ctx, SLLBM_EINVAL, "NULL out");
    if (ctx->d2) return refuse_2d(ctx, "sllbm_diagnostics");
    if (!state && !ctx->has_state) return fail(ctx, SLLBM_ESTATE, "no state set");
    DeviceGuard guard(ctx->cfg.device);
    const void *st = state ? state : ctx->buf[ctx->cur];
    hipError_t e = is_fp64(ctx)
        ? Launch<double>::diagnostics(ctx->geo, ctx->cp, static_cast<const double *>(st), ctx->d_dmat, ctx->d_ccw,
                                      ctx->h, graded_hw(ctx), mapped_jac(ctx), ctx->d_scr_rho, ctx->d_scr_u,
                                      ctx->d_scr_T, ctx->d_partials, RED_BLOCKS, ctx->d_small, ctx->stream)
        : Launch<float>::diagnostics(ctx->geo, ctx->cp, static_cast<const float *>(st), ctx->d_dmat, ctx->d_ccw,
                                     ctx->h, graded_hw(ctx), mapped_jac(ctx), ctx->d_scr_rho, ctx->d_scr_u,
                                     ctx->d_scr_T, ctx->d_partials, RED_BLOCKS, ctx->d_small, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "diagnostics");
    if ((e = hipMemcpyAsync(out, ctx->d_small, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
        return hip_fail(ctx, e, "diagnostics copy");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(out[k])) return fail(ctx, SLLBM_ENONFINITE, "non-finite diagnostics");
    return SLLBM_OK;
}

int sllbm_loss_grad(sllbm_ctx *ctx, const void *state, void *lam)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!state || !lam || state == lam) return fail(ctx, SLLBM_EINVAL, "bad loss_grad buffers");
    if (ctx->d2) return refuse_2d(ctx, "sllbm_loss_grad");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = is_fp64(ctx)
        ? Launch<double>::loss_grad(ctx->geo, static_cast<const double *>(state), ctx->d_dmat, ctx->d_ccw,
                                    ctx->d_nodew, ctx->h, graded_hw(ctx), mapped_jac(ctx),
                                    ctx->mapped ? ctx->d_mw : nullptr, ctx->d_scr_rho, ctx->d_scr_u, ctx->d_scr_div,
                                    ctx->d_partials, RED_BLOCKS, static_cast<double *>(lam), ctx->stream)
        : Launch<float>::loss_grad(ctx->geo, static_cast<const float *>(state), ctx->d_dmat, ctx->d_ccw,
                                   ctx->d_nodew, ctx->h, graded_hw(ctx), mapped_jac(ctx),
                                   ctx->mapped ? ctx->d_mw : nullptr, ctx->d_scr_rho, ctx->d_scr_u, ctx->d_scr_div,
                                   ctx->d_partials, RED_BLOCKS, static_cast<float *>(lam), ctx->stream);
    return check_launch(ctx, e, "loss_grad");
}

int sllbm_adjoint_step(sllbm_ctx *ctx, const void *state_n, const void *lam_next, void *lam_out, double *dmu)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!state_n || !lam_next || !lam_out) return fail(ctx, SLLBM_EINVAL, "NULL argument");
    if (lam_out == lam_next || lam_out == state_n) return fail(ctx, SLLBM_EINVAL, "lam_out aliases an input");
    if (ctx->d2) return refuse_2d(ctx, "sllbm_adjoint_step");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = stream_t_into(ctx, lam_next, lam_out);
    if (e != hipSuccess) return hip_fail(ctx, e, "adjoint_step (transposed streaming)");
    e = is_fp64(ctx)
        ? Launch<double>::collide_vjp(ctx->geo, ctx->cp, static_cast<const double *>(state_n),
                                      static_cast<double *>(lam_out), ctx->d_adj_part, ADJ_BLOCKS, dmu, ctx->stream)
        : Launch<float>::collide_vjp(ctx->geo, ctx->cp, static_cast<const float *>(state_n),
                                     static_cast<float *>(lam_out), ctx->d_adj_part, ADJ_BLOCKS, dmu, ctx->stream);
    return check_launch(ctx, e, "adjoint_step (collision VJP)");
}

int sllbm_moments_vjp(sllbm_ctx *ctx, const double *drho, const double *du, const double *dT, void *lam)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!lam) return fail(ctx, SLLBM_EINVAL, "NULL lam");
    if (ctx->d2) return refuse_2d(ctx, "sllbm_moments_vjp");
    if (!ctx->has_state) return fail(ctx, SLLBM_ESTATE, "no state set");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = is_fp64(ctx)
        ? Launch<double>::moments_vjp(ctx->geo, ctx->cp, static_cast<const double *>(ctx->buf[ctx->cur]), drho, du,
                                      dT, static_cast<double *>(lam), ctx->stream)
        : Launch<float>::moments_vjp(ctx->geo, ctx->cp, static_cast<const float *>(ctx->buf[ctx->cur]), drho, du, dT,
                                     static_cast<float *>(lam), ctx->stream);
    return check_launch(ctx, e, "moments_vjp");
}

int sllbm_init_equilibrium_vjp(sllbm_ctx *ctx, const double *rho, const double *u, const double *T,
                               const void *lam0, double *drho, double *du, double *dT)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!rho || !u || !T || !lam0) return fail(ctx, SLLBM_EINVAL, "NULL argument");
    if (ctx->d2) return refuse_2d(ctx, "sllbm_init_equilibrium_vjp");
    DeviceGuard guard(ctx->cfg.device);
    hipError_t e = is_fp64(ctx)
        ? Launch<double>::init_equilibrium_vjp(ctx->geo, ctx->cp, rho, u, T, static_cast<const double *>(lam0),
                                               drho, du, dT, ctx->stream)
        : Launch<float>::init_equilibrium_vjp(ctx->geo, ctx->cp, rho, u, T, static_cast<const float *>(lam0), drho,
                                              du, dT, ctx->stream);
    return check_launch(ctx, e, "init_equilibrium_vjp");
}

int sllbm_superpose(sllbm_ctx *ctx, const double *base, const double *basis, int32_t m, const double *amps,
                    double *out)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!base || !out || (m > 0 && (!basis || !amps))) return fail(ctx, SLLBM_EINVAL, "NULL argument");
    if (m < 0 || m > MAX_MODES) return fail(ctx, SLLBM_EINVAL, "mode count must be in 0..64");
    DeviceGuard guard(ctx->cfg.device);
    ModeAmplitudes am{};
    for (int j = 0; j < m; ++j) am.a[j] = amps[j];
    const int64_t n = static_cast<int64_t>(ctx->d2 ? 2 : 3) * ctx->geo.nodes;
    return check_launch(ctx, launch_superpose(n, m, am, base, basis, out, ctx->stream), "superpose");
}

int sllbm_project(sllbm_ctx *ctx, const double *basis, int32_t m, const double *v, double *out)
{
    if (!ctx) return SLLBM_EINVAL;
    if (!v || !out || (m > 0 && !basis)) return fail(ctx, SLLBM_EINVAL, "NULL argument");
    if (m < 0 || m > MAX_MODES) return fail(ctx, SLLBM_EINVAL, "mode count must be in 0..64");
    DeviceGuard guard(ctx->cfg.device);
    const int64_t n = static_cast<int64_t>(ctx->d2 ? 2 : 3) * ctx->geo.nodes;
    hipError_t e = hipSuccess;
    for (int m0 = 0; m0 < m; m0 += 8) {
        const int mc = std::min(8, m - m0);
        if ((e = launch_project_chunk(n, m0, mc, basis, v, ctx->d_partials, RED_BLOCKS, ctx->d_small, ctx->stream)) !=
            hipSuccess)
            return hip_fail(ctx, e, "project");
        if ((e = hipMemcpyAsync(out + m0, ctx->d_small, mc * sizeof(double), hipMemcpyDeviceToHost, ctx->stream)) !=
            hipSuccess)
            return hip_fail(ctx, e, "project copy");
    }
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "project");
    return SLLBM_OK;
}

}  // extern "C"
