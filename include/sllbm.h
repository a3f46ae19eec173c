/*
 * sllbm.h -- C ABI of the MI355X (gfx950) semi-Lagrangian lattice Boltzmann
 * library: the per-time-step update of the 45-velocity f and g populations
 * of the compressible SLLBM (Wilde, Kraemer, Reith, Foysi, arXiv:2012.05537)
 * on a periodic hexahedral mesh of equal cells (or of axis-aligned cells of
 * unequal width, sllbm_set_mesh) with Gauss-Lobatto-Chebyshev support points,
 * and its two-dimensional form with the 19-velocity set (SLLBM_D2Q19, the
 * lattice of the shock-tube and 2-D Riemann cases of Sec. III A-B).
 *
 * Two dimensions (velocity_set = SLLBM_D2Q19): D = 2, n_el[2] = 1 and
 * N_z = 1 (length[2] is not used); Q = 19 replaces 45 below; velocity
 * fields u are [2][N]; totals report zero z momentum.  The calls of the
 * adjoint section, sllbm_loss, sllbm_diagnostics, sllbm_set_mesh and the
 * transposed sllbm_stream return EINVAL on such a context.
 *
 * Conventions shared by every call
 * --------------------------------
 *  Units      lattice units: c_s = 1, T0 = 1, gas constant 1, D = 3 (2 for
 *             SLLBM_D2Q19), C_v = 1/(gamma - 1).
 *  Nodes      the unique periodic support points: N_a = n_el[a] * order per
 *             axis, N = N_x N_y N_z.  Node (gx, gy, gz) has linear index
 *             (gz * N_y + gy) * N_x + gx; along an axis, node g = e*order + l
 *             (cell e, local point l in [0, order)) sits at
 *             x = e*h + h*(1 - cos(pi*l/order))/2, h = length/n_el (Sec. II A).
 *  Velocities the 45 abscissae in the order returned by sllbm_velocity_set().
 *  State      one buffer of 2*45*N values of the storage type (double for
 *             SLLBM_FP64, float for SLLBM_FP32_MIXED): f at [i*N + n], then
 *             g at [(45 + i)*N + n].  A "state" passed through this ABI is
 *             always the pre-collision populations h_i(x, t) of Eq. (5).
 *  Fields     rho [N], u [3][N] (component-major), T [N], all double.
 *  Pointers   "device" pointers must be device memory on the context's
 *             device; "host" pointers are ordinary host memory.  The caller
 *             owns every pointer it passes; the library never keeps one past
 *             the call.  The library owns its internal state buffers and tables.
 *  Ordering   every call except sllbm_totals, sllbm_loss, sllbm_create and
 *             sllbm_destroy is asynchronous on the stream set with
 *             sllbm_set_stream (default: the null stream).
 *  Errors     0 on success, else one of the SLLBM_E* codes; no exception
 *             crosses the ABI.  sllbm_last_error() returns the message of the
 *             last failure on this context (or of a failed create, for NULL).
 *  Threads    a context is not thread-safe; distinct contexts are independent.
 */
#ifndef SLLBM_H
#define SLLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SLLBM_OK 0
#define SLLBM_EINVAL 1      /* bad argument or configuration */
#define SLLBM_ENOMEM 2      /* device allocation failed */
#define SLLBM_EDEVICE 3     /* HIP runtime error or no usable gfx950 device */
#define SLLBM_ESTATE 4      /* call not valid in the current state */
#define SLLBM_ENONFINITE 5  /* a non-finite value was found */

#define SLLBM_D3Q45 45
#define SLLBM_D2Q19 19

#define SLLBM_SUTHERLAND 0  /* mu = mu_inf (1+S) T^1.5/(T+S), S = 0.40417 (Sec. III C) */
#define SLLBM_CONSTANT 1    /* mu = mu_inf */

#define SLLBM_FP64 0        /* double populations and arithmetic */
#define SLLBM_FP32_MIXED 1  /* float populations, interpolation and relaxation;
                               double moments, transport coefficients,
                               equilibrium coefficients and centred third moments */

typedef struct sllbm_ctx sllbm_ctx;

typedef struct {
    int32_t n_el[3];        /* cells per axis, >= 1 */
    int32_t order;          /* GLC interpolation order p, 1..6 (Eq. (8)) */
    int32_t velocity_set;   /* SLLBM_D3Q45 or SLLBM_D2Q19 */
    int32_t viscosity_law;  /* SLLBM_SUTHERLAND or SLLBM_CONSTANT */
    int32_t precision;      /* SLLBM_FP64 or SLLBM_FP32_MIXED */
    int32_t device;         /* HIP device ordinal */
    double length[3];       /* domain edge lengths, > 0 */
    double dt;              /* time step, > 0 */
    double gamma;           /* heat capacity ratio, > 1 */
    double prandtl;         /* Prandtl number of the quasi-equilibrium term, > 0 */
    double mu_inf;          /* viscosity at T = 1, > 0 */
} sllbm_config;

/* Create a context (Sec. II A "at the beginning of the simulation": the
 * departure point of every (node, velocity) pair is located once, and the
 * per-axis cell offsets and 1-D Lagrange weights are uploaded).  Allocates
 * two state buffers on cfg->device.  *out is NULL on failure.
 * Errors: EINVAL (bad config), EDEVICE (no gfx950 device), ENOMEM. */
int sllbm_create(const sllbm_config *cfg, sllbm_ctx **out);

/* Free the context and its device memory.  NULL is accepted. */
int sllbm_destroy(sllbm_ctx *ctx);

/* Stream (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream) on
 * which every later call is ordered.  NULL selects the null stream. */
int sllbm_set_stream(sllbm_ctx *ctx, void *hip_stream);

/* Message of the last error on ctx (ctx may be NULL: last failed create). */
const char *sllbm_last_error(const sllbm_ctx *ctx);

/* Number of unique nodes N; -1 for a NULL context. */
int64_t sllbm_num_nodes(const sllbm_ctx *ctx);

/* Bytes of one state buffer (2 * 45 * N * sizeof(storage type)). */
int64_t sllbm_state_bytes(const sllbm_ctx *ctx);

/* The D3Q45 velocity set (Sec. II B, degree-nine cubature): xi[45][3] and
 * w[45] (host).  Returns 45. */
int sllbm_velocity_set(double *xi, double *w);

/* The velocity set velocity_set (SLLBM_D3Q45 or SLLBM_D2Q19, both exact to
 * degree nine for the weight exp(-|xi|^2/2), Sec. II B) in the order the
 * state uses: xi[Q][3] (z = 0 for D2Q19) and w[Q] (host).  Returns Q, or
 * -1 for an unknown set or a NULL pointer. */
int sllbm_lattice(int32_t velocity_set, double *xi, double *w);

/* 1-D node coordinates along each axis (host arrays of N_x, N_y, N_z). */
int sllbm_node_coords(const sllbm_ctx *ctx, double *x, double *y, double *z);

/* Change mu_inf (the "relaxation time" parameter; tau - 1/2 = mu/(P dt)). */
int sllbm_set_viscosity(sllbm_ctx *ctx, double mu_inf);

/* Graded mesh (Sec. II A: departure points are traced through the
 * neighbouring cells; with unequal cells the per-cell interpolation matrices
 * are no longer shared, subsection "Numerical efficiency").  widths_a: host
 * array of n_el[a] positive cell widths along axis a, or NULL to keep equal
 * cells on that axis (at least one must be given); a given axis gets length
 * sum(widths_a), node g = e*order + l of it sits at F_e + w_e t_l (F_e =
 * w_0 + ... + w_{e-1}).  The departure cell of every (node, velocity, axis)
 * is located once here and per-node tables (and their transposes, for S^T)
 * are uploaded; the state is kept.  Afterwards every call uses the graded
 * mesh (streaming in both directions, steps, adjoint steps; totals, loss,
 * loss gradient and diagnostics with each cell's own width).  Synchronises
 * the context's stream.  On failure the previous mesh stays.
 * Errors: EINVAL (no widths, a non-positive width, or a grading so strong
 * that the source window of a 32 x 8 tile exceeds 4096 nodes or the 160 KB
 * of LDS, or that one node is read by more than 24 nodes of an axis),
 * ENOMEM, EDEVICE. */
int sllbm_set_mesh(sllbm_ctx *ctx, const double *widths_x, const double *widths_y, const double *widths_z);

/* Distorted mesh (Sec. II A: departure points traced once through the
 * cells; the general, non-factorising case of subsection "Numerical
 * efficiency").  d: host array [3][N] of periodic node displacements added to
 * the equal-cell GLC positions; each cell becomes the degree-p
 * (isoparametric) image of its reference cube, and populations are
 * interpolated in reference coordinates.  For every velocity and node the
 * departure point x + d - xi dt is located by Newton's method on the cell
 * maps, and its cell and local coordinates are uploaded (28 bytes per
 * velocity and node); totals then weight every node with the |det J| of the
 * cells that hold it.  d = NULL returns to the undistorted mesh.  The state is
 * kept; node coordinates stay those of the reference grid.  The transposed
 * streaming (and so sllbm_adjoint_step) sums every support value's adjoint
 * in a fixed order (per departure cell, then over the cells that share a
 * node; no atomics), so it is bitwise reproducible; for it the call also
 * uploads the nodes of every velocity grouped by departure cell (4 bytes per
 * velocity and node) and allocates partial sums of at most one state's
 * size.  The loss, its gradient and the diagnostics take derivatives
 * in physical coordinates through each cell's map (d u/d x = (d u/d r) J^-1,
 * J = I + dD/dr at the cell's support points) and weight the quadrature with
 * |det J|; J^-1 and |det J| of every cell point are uploaded here (80 bytes
 * per cell point).  Synchronises the context's stream.
 * Errors: EINVAL (2-D context, graded cells, non-finite d, a cell map that
 * folds over (det J <= 0 at a support point), a departure search that does
 * not converge), ENOMEM, EDEVICE; on error the previous mesh stays. */
int sllbm_set_displacement(sllbm_ctx *ctx, const double *d);

/* State := equilibrium of the given fields (Eq. (6); g^eq = (2C_v - D) T f^eq).
 * rho, u ([D][N]), T: device.  Errors: EINVAL on NULL. */
int sllbm_init_equilibrium(sllbm_ctx *ctx, const double *rho, const double *u, const double *T);

/* State := caller's pre-collision populations (device, storage type). */
int sllbm_set_state(sllbm_ctx *ctx, const void *state);

/* Copy the current pre-collision populations to the caller (device). */
int sllbm_get_state(sllbm_ctx *ctx, void *state);

/* Advance n >= 0 time steps of Eq. (5) with the quasi-equilibrium collision
 * of App. D: each step collides every node (one kernel, into a second
 * buffer), then streams every population by the semi-Lagrangian
 * interpolation of Eqs. (8)-(9) back into the state (a second kernel). */
int sllbm_step(sllbm_ctx *ctx, int32_t n);

/* As sllbm_step, and also writes the pre-collision state after each of the
 * n steps to states + k*stride_bytes (device), k = 0..n-1. */
int sllbm_step_record(sllbm_ctx *ctx, int32_t n, void *states, int64_t stride_bytes);

/* Kernel timing of the step loop.  With on != 0, every collision and
 * streaming launch of sllbm_step / sllbm_step_record is bracketed by HIP
 * events on the context's stream (up to 4096 launches of each kind are
 * recorded; later ones are not).  sllbm_kernel_times synchronises the
 * stream and writes to host out[4]: total milliseconds of the collision
 * launches, their count, total milliseconds of the streaming launches, their
 * count; it then clears the record.  on == 0 stops recording. */
int sllbm_set_kernel_timing(sllbm_ctx *ctx, int32_t on);
int sllbm_kernel_times(sllbm_ctx *ctx, double *out);

/* rho, u ([D][N]), T of the current state at every node, Eq. (7) (device,
 * double).  T from 2 rho E = rho |u|^2 + 2 C_v rho T.  Any pointer may be NULL. */
int sllbm_moments(sllbm_ctx *ctx, double *rho, double *u, double *T);

/* Domain integrals of rho, rho u_x, rho u_y, rho u_z and rho E with
 * Clenshaw-Curtis weights of the GLC points (host out[5]).  Deterministic
 * (fixed-order two-stage FP64 reduction).  Synchronises the stream.
 * Returns ENONFINITE (and still fills out) if any value is not finite. */
int sllbm_totals(sllbm_ctx *ctx, double *out);

/* Taylor-Green diagnostics of Sec. III C as domain integrals, on a caller
 * state (device) or, if state is NULL, on the current state:
 *   out[0] = kinetic energy           int (1/2) rho |u|^2
 *   out[1] = solenoidal dissipation   int mu(T) |curl u|^2
 *   out[2] = dilatational dissipation (4/3) int mu(T) (div u)^2
 * mu(T) is the context's viscosity law (mu_inf plays the paper's 1/(rho_ref
 * Re)); derivatives are those of each cell's own interpolation polynomial,
 * integrals the tensor Clenshaw-Curtis rule of each cell (host out[3]).
 * Deterministic; synchronises the stream; ENONFINITE if a value is not finite. */
int sllbm_diagnostics(sllbm_ctx *ctx, const void *state, double *out);

/* ---- adjoint (reverse mode of the step map) ----------------------------- */

/* Flow functional on a caller state (device):
 *   L = sum over cells of the tensor Clenshaw-Curtis quadrature of
 *       (1/2) rho |u|^2 + (div u)^2,
 * div u from each cell's own interpolation polynomial (Sec. III C).
 * Result to host *out; synchronises the stream. */
int sllbm_loss(sllbm_ctx *ctx, const void *state, double *out);

/* dL/d(state) of sllbm_loss, written to lam (device, storage type). */
int sllbm_loss_grad(sllbm_ctx *ctx, const void *state, void *lam);

/* One reverse step.  With X_{n+1} = S(C(X_n)) (C: collision, S: streaming),
 * lam_out = (dX_{n+1}/dX_n)^T lam_next = J_C(X_n)^T S^T lam_next, where S^T
 * is applied as a gather over the transposed 1-D interpolation tables
 * (no atomics).  state_n, lam_next, lam_out: device, storage type; lam_out
 * must not alias lam_next.  If dmu is not NULL, the derivative with respect
 * to mu_inf, sum over nodes of lam_next . S (dC/dmu_inf), is added to *dmu
 * (device double). */
int sllbm_adjoint_step(sllbm_ctx *ctx, const void *state_n, const void *lam_next, void *lam_out,
                       double *dmu);

/* Reverse of sllbm_moments at the current state: given adjoints drho [N],
 * du [3][N] and dT [N] (device double; any may be NULL = zero), write
 * lam = (d(rho, u, T)/d(state))^T (drho, du, dT) (device, storage type),
 * through rho = sum f, rho u = sum f xi and 2 rho E = sum (f |xi|^2 + g)
 * of Eq. (7).  Requires a state. */
int sllbm_moments_vjp(sllbm_ctx *ctx, const double *drho, const double *du, const double *dT, void *lam);

/* Reverse of sllbm_init_equilibrium: given lam0 = dL/d(state), write
 * dL/drho, dL/du ([3][N]) and dL/dT at the fields (rho, u, T).  All device;
 * drho, du, dT may be NULL. */
int sllbm_init_equilibrium_vjp(sllbm_ctx *ctx, const double *rho, const double *u, const double *T,
                               const void *lam0, double *drho, double *du, double *dT);

/* Mode algebra of the gradient workload: velocity modes added to a base
 * flow (the perturbed Taylor-Green initial state of Sec. III C used for
 * gradients).  base, out: device double [D][N] (D = 3, or 2 for D2Q19);
 * basis: device double [m][D][N]; amps: host double [m]; 0 <= m <= 64.
 *   sllbm_superpose: out = base + sum_j amps[j] basis[j]  (asynchronous;
 *                    out may equal base).
 *   sllbm_project:   out[j] = sum over the D*N components of basis[j] v
 *                    (host out[m]); deterministic fixed-order reduction;
 *                    synchronises the stream.
 * EINVAL for NULL pointers or m out of range. */
int sllbm_superpose(sllbm_ctx *ctx, const double *base, const double *basis, int32_t m, const double *amps,
                    double *out);
int sllbm_project(sllbm_ctx *ctx, const double *basis, int32_t m, const double *v, double *out);

/* ---- building blocks exposed for testing -------------------------------- */

/* Streaming only (Eq. (9)) of a caller state: out = S(in) (forward) or
 * out = S^T(in) (transpose != 0).  Device, storage type, no aliasing. */
int sllbm_stream(sllbm_ctx *ctx, const void *in, void *out, int32_t transpose);

/* Collision only (Eq. (5) right-hand side with App. D) of a caller state,
 * in place (device, storage type). */
int sllbm_collide(sllbm_ctx *ctx, void *state);

/* ---- allocation-free entry point ---------------------------------------- */

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the totals
 * of sllbm_totals (Clenshaw-Curtis integrals of rho, rho u_x, rho u_y,
 * rho u_z, rho E) of a caller state, without a context.
 *   cfg    host; the equal-cell periodic mesh and lattice of the state
 *          (n_el, order, length, velocity_set, precision, device; the other
 *          fields are not read).
 *   state  device, [2][Q][N] of cfg's storage type, on cfg->device.
 *   out    device, 5 doubles, written in the order of sllbm_totals.
 *   stream the hipStream_t to run on (NULL: the null stream); asynchronous,
 *          no finiteness check.
 * The library allocates nothing here: the reduction partials and node weights
 * live in a static device array of 256 KB per device (held until the process
 * ends), which limits the grid to N_x + N_y + N_z <= 24576 nodes (EINVAL
 * beyond).  Calls that overlap on one device share that array and race.
 * Same kernels and summation order as sllbm_totals, so the same bits.
 * Errors: EINVAL (configuration, NULL pointer, size), EDEVICE (runtime);
 * the message is sllbm_last_error(NULL). */
int sllbm_totals_noalloc(const sllbm_config *cfg, const void *state, double *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SLLBM_H */
