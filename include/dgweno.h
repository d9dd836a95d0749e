/*
 * dgweno.h - C ABI of the MI355X (gfx950) library for the dissipative-WENO
 * stabilised Runge-Kutta discontinuous Galerkin scheme of
 *   J. Vedral, "Dissipative WENO stabilization of high-order discontinuous
 *   Galerkin methods for hyperbolic problems", arXiv 2309.12019.
 *
 * Problem (Sec. 2, eq. ivp): u_t + div F(u) = 0 for a scalar u (or, with
 * DG_FLUX_EULER, the 1D Euler system) on a uniform Cartesian mesh of square
 * cells (1D or 2D), with
 *   DG_FLUX_LINADV : F(u) = v(x) u,  v = (vel_x - omega (y - rot_cy),
 *                                         vel_y + omega (x - rot_cx))
 *   DG_FLUX_BURGERS: F(u) = a u^2 / 2, a = (vel_x, vel_y)
 *   DG_FLUX_KPP    : F(u) = (sin u, cos u), the non-convex flux of Sec. 5.5
 *                    (2D only; LLF wave speed max |F'(w) . n| over w between
 *                    the two states, exactly; p + 2 quadrature points)
 *   DG_FLUX_EULER  : the 1D Euler equations of Sec. 5.6, a system for
 *                    U = (rho, rho v, rho E) with F = (rho v, rho v^2 + p,
 *                    (rho E + p) v), p = 0.4 (rho E - rho v^2 / 2); LLF wave
 *                    speed max(|v| + c) of the two states, lambda_e the
 *                    largest |v| + c at the p + 2 volume Gauss points,
 *                    gamma_e from the density coefficients alone (the same
 *                    for all three components); a non-periodic end is a
 *                    reflecting wall (mirror state (rho, -rho v, rho E);
 *                    bc_value unused).  Per-stage kernel only.
 * discretised in the broken space V_p (Sec. 2): tensor Legendre polynomials
 * of degree p per axis on every cell.  The library evaluates
 *   dU/dt = M^{-1} (R(U) - s(U))
 * where R is the DG residual of eq. (weak2) with the local Lax-Friedrichs
 * flux (Sec. 2), s the dissipative term of eq. (astab) with
 * nu_e = lambda_e h / (2p) (eq. visc), and gamma_e the WENO smoothness sensor
 * of eqs. (sensor)/(gensensor) (Sec. 4); it advances U with the SSP-RK3 step
 * of eq. (ssp), or the second- or fourth-order SSP step (rk_order).
 *
 * Data layout of a state U (caller-owned device memory, FP64, contiguous):
 *   U[cell * n_loc + j], cell = ix + nx * iy (x fastest), n_loc = (p+1)^dim,
 *   j = a + (p+1) * b where a is the x-degree and b the y-degree of the
 *   Legendre product P_a(xi) P_b(eta) on the reference cell [-1,1]^dim.
 *   DG_FLUX_EULER: n_loc = 3 (p+1), j = k (p+1) + a for component k
 *   (rho, rho v, rho E) and degree a.
 *
 * Conventions for every entry point:
 *   - Return 0 on success, a negative DG_E* code on failure; the message of
 *     the last failure on the calling thread is returned by dg_last_error().
 *   - Argument errors are detected before any device work is queued.
 *   - Pointers named "device" are device memory owned by the caller; the
 *     library never frees them.  Work is queued on the context's stream
 *     (dg_mesh_desc.stream, 0 = the default stream) and is asynchronous
 *     unless stated otherwise.
 *   - A context is not thread-safe; separate contexts are independent.
 */
#ifndef DGWENO_H
#define DGWENO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum dg_status {
  DG_OK = 0,
  DG_EINVAL = -1,       /* invalid argument (checked on the host) */
  DG_ENOMEM = -2,       /* device allocation failed */
  DG_EDEVICE = -3,      /* a HIP runtime call failed */
  DG_ENONFINITE = -4,   /* a state contained NaN or Inf (dg_check_finite) */
  DG_EUNSUPPORTED = -5  /* valid but not built (e.g. an unsupported size) */
};

enum dg_flux { DG_FLUX_LINADV = 0, DG_FLUX_BURGERS = 1, DG_FLUX_KPP = 2, DG_FLUX_EULER = 3 };

/* Scheme labels of Sec. 5: DG (no stabilisation), LO (gamma_e = 1 in
 * eq. astab, i.e. the low-order operator of eq. lostab), WENO (gamma_e from
 * the smoothness sensor of eqs. sensor/gensensor).  ZHAO: gamma_e from the
 * sensor of Zhao et al. that Sec. 5.6 compares with, built on the same HWENO
 * weights: sum_l |omega_l / omega~_l - 1|^theta / (|1 / min_l omega~_l -
 * 1|^theta + m_e) over the candidates that exist (0 for a cell without face
 * neighbours); q and b do not apply.  The adjoint covers DG, LO and WENO. */
enum dg_mode { DG_MODE_DG = 0, DG_MODE_LO = 1, DG_MODE_WENO = 2, DG_MODE_ZHAO = 3 };

/* State outside non-periodic boundary faces.  CONSTANT: bc_value.  RIEMANN
 * (2D Burgers, both axes non-periodic): the exact solution in R^2 of the
 * four-quadrant problem of Sec. 5.4 (u_t + div((1,1) u^2/2) = 0 with -0.2 | -1
 * above 0.5 | 0.8, split at x = y = 1/2), evaluated at the boundary face's
 * Gauss points at the time of each stage's input state (the paper takes its
 * inflow data from that solution; here every boundary face does).  The time
 * comes from the context's clock (dg_set_time). */
enum dg_bc { DG_BC_CONSTANT = 0, DG_BC_RIEMANN = 1 };

typedef struct dg_mesh_desc {
  int32_t dim;               /* 1 or 2 */
  int32_t nx, ny;            /* cells along x and y (ny ignored for dim 1) */
  double x0, x1, y0, y1;     /* domain box; 2D cells must be square */
  int32_t periodic_x, periodic_y;   /* 1: periodic wrap along that axis */
  int32_t p;                 /* polynomial degree, 1..4 */
  int32_t flux;              /* enum dg_flux */
  double vel_x, vel_y;       /* constant velocity (LINADV) or direction a (BURGERS) */
  double omega, rot_cx, rot_cy;     /* rotation part of the LINADV velocity (2D) */
  double bc_value;           /* exterior state u^+ on non-periodic boundary faces */
  int32_t mode;              /* enum dg_mode */
  double q;                  /* sensor exponent q >= 1 (eq. sensor) */
  double b;                  /* sensor threshold b in [0,1] (eq. gensensor) */
  double w_nb;               /* linear weight of each neighbour candidate (Sec. 5) */
  double weno_eps, weno_pow; /* alpha_l = w_l / (eps + beta_l)^pow */
  double lambda_override;    /* > 0: lambda_e := this value in every cell */
  void* stream;              /* hipStream_t the context queues work on (0 = default) */
  double zhao_theta;         /* exponent theta of the ZHAO sensor, > 0 (Sec. 5.6: 1) */
  int32_t rk_order;          /* SSP Runge-Kutta order of dg_step/dg_run: 3 (eq. ssp,
                                default), 2 or 4 (Sec. 5.1 runs order p + 1) */
  int32_t bc_kind;           /* enum dg_bc */
  /* Gauss-Legendre points per axis (the paper leaves its quadrature to the
   * finite element library it uses).  0 selects the built rule: volume and
   * faces exact for the polynomial part of the integrands, p + 1 for
   * LINADV, ceil(3p/2) (1D) or ceil((3p+1)/2) (2D) for BURGERS, p + 2 for
   * KPP and EULER; projection p + 2.  The rules are compile-time tables: any
   * other value is DG_EUNSUPPORTED (DG_EINVAL outside 0..8). */
  int32_t quad_vol, quad_face, quad_proj;
  /* dg_stable_dt's reading of "CFL" (the paper never states its step):
   * 0 scaled (default), dt = cfl h / ((2p+1) lambda_max); 1 literal,
   * dt = cfl h / lambda_max. */
  int32_t cfl_mode;
  /* 1: dg_step and dg_run count the non-finite entries of U on the device
   * once their steps are queued, wait for them, and return DG_ENONFINITE if
   * there are any (the call then synchronises the stream); 0 (default): no
   * check. */
  int32_t check_finite;
  /* HIP device the context runs on: -1 (default) the device current at
   * dg_init_mesh; otherwise that device, made current for the duration of
   * every call on the context and restored afterwards. */
  int32_t device;
} dg_mesh_desc;

typedef struct dg_ctx dg_ctx;   /* opaque, owned by the library */

/* Fill a descriptor with the defaults: 1D, 64 cells on [0,1] periodic, p = 2,
 * LINADV with vel_x = 1, mode WENO, q = 1, b = 0, w_nb = 0.01, eps = 1e-6,
 * pow = 2 (the values of Sec. 5), no lambda override, default stream,
 * zhao_theta = 1, rk_order = 3, bc_kind CONSTANT, built quadrature rules,
 * cfl_mode 0, no finite check, device -1.  Never fails. */
void dg_default_desc(dg_mesh_desc* desc);

/* Validate `desc` and create a context for the problem of Sec. 2 (the
 * conservation law on the mesh T_h, discretised in the broken space V_p of
 * degree p) on the descriptor's HIP device: mesh, compile-time tables for
 * degree p, and two stage buffers of n_cells * n_loc doubles for the stages
 * of eq. (ssp) (three for rk_order 4; the only allocations the context makes
 * besides the adjoint's, on first use).
 * Errors: DG_EINVAL (bad field, null pointer, non-square 2D cells),
 * DG_EUNSUPPORTED (a quadrature rule that is not built), DG_ENOMEM,
 * DG_EDEVICE.  On failure *out is set to NULL. */
int dg_init_mesh(const dg_mesh_desc* desc, dg_ctx** out);

/* Release the context and its device buffers (synchronises its stream). */
void dg_destroy(dg_ctx* ctx);

/* Sizes of the discrete problem (host outputs; any may be NULL). */
int dg_sizes(const dg_ctx* ctx, int64_t* n_cells, int32_t* n_loc, int32_t* n_proj_nodes);

/* Physical coordinates of the projection nodes, written to host memory
 * xy[cell][node][dim] (n_cells * n_proj_nodes * dim doubles): the
 * (p+2)^dim tensor Gauss-Legendre nodes of every cell, x fastest. */
int dg_proj_nodes(const dg_ctx* ctx, double* xy_host);

/* L2 projection of initial data onto V_p (Sec. 2, eq. fesol):
 * U_j = (int phi_j u0 dx) / (int phi_j^2 dx), the integral taken with the
 * projection rule.  u_at_nodes (device, [cell][node]) holds u0 at the nodes
 * from dg_proj_nodes ([cell][component][node] for DG_FLUX_EULER, the
 * conserved variables); U (device) receives the coefficients. */
int dg_project_ic(dg_ctx* ctx, const double* u_at_nodes, double* U);

/* The context's clock: the time of the state that dg_step and dg_run
 * advance.  It starts at 0; dg_step adds dt, dg_run nsteps * dt (step k of a
 * run starts at t + k dt), and dg_rhs evaluates at it.  It matters only for
 * bc_kind RIEMANN.  dg_set_time: t finite. */
int dg_set_time(dg_ctx* ctx, double t);
int dg_get_time(const dg_ctx* ctx, double* t);

/* Semi-discrete operator (eq. weak2 plus eq. astab): dUdt = M^{-1}(R(U) - s(U)).
 * U, dUdt: device [n_cells * n_loc]; gamma: device [n_cells] receiving
 * gamma_e of every cell (0 for DG, 1 for LO), or NULL.  U and dUdt must not
 * overlap. */
int dg_rhs(dg_ctx* ctx, const double* U, double* dUdt, double* gamma);

/* One SSP Runge-Kutta step of size dt, in place on U (device): by default
 * the three-stage third-order method of eq. ssp; with rk_order 2 the two-stage
 * second-order method, with rk_order 4 the five-stage fourth-order method of
 * Spiteri and Ruuth (Sec. 5.1 uses order p + 1 for its convergence study; the
 * paper does not name the fourth-order scheme).  gamma_e and lambda_e are
 * re-evaluated in every stage (Sec. 3, the stabilisation is part of the
 * semi-discrete operator).  The five-stage method evaluates the operator six
 * times per step (its last stage needs L(U^(3)) a second time).  dt must be
 * finite and > 0.  With check_finite, DG_ENONFINITE if U holds NaN or Inf
 * after the step. */
int dg_step(dg_ctx* ctx, double* U, double dt);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): one SSP step of the
 * descriptor's order, as dg_step, without a context.  desc is validated as
 * for dg_init_mesh; work is queued on desc->stream; t is the time of U (it
 * enters through bc_kind RIEMANN only).  The stage states live in a static
 * device array of the library (three buffers of 2^20 doubles, 24 MiB, held
 * on every device the library runs on until the process ends); nothing is
 * allocated.  Every call on a device shares that device's array: calls that
 * overlap on one device (other streams, other threads) race.  The stage
 * kernels are dg_step's per-stage kernels, so results equal dg_step's bit
 * for bit.  Errors: DG_EINVAL for a bad descriptor, U NULL, dt not finite
 * and > 0, t not finite, or n_cells * n_loc above 2^20 (checked before any
 * device call); DG_EDEVICE. */
int dg_step_static(const dg_mesh_desc* desc, double* U, double dt, double t);

/* nsteps SSP steps of size dt (eq. ssp, or the order rk_order selects), in
 * place on U (device): the fully discrete scheme of Sec. 2 run over a fixed
 * step, the stabilisation of Secs. 3 and 4 re-evaluated in every stage.
 * The stage launches (3, 2 or 6 per step; one fused launch per step where
 * dg_set_fused selects it) are recorded once into a HIP graph (cached for the
 * same U, dt and chunk length) and replayed on the context stream.  With
 * bc_kind RIEMANN the stages read their times (on which the exterior state
 * depends) as offsets from a device copy of the context clock, which a
 * one-thread launch sets before each replay, so the same graph serves any
 * time.  nsteps >= 0.  With check_finite, DG_ENONFINITE if U holds NaN or Inf
 * after the run. */
int dg_run(dg_ctx* ctx, double* U, double dt, int32_t nsteps);

/* Stable step for the fixed-step reading of "CFL" (the configurations quote
 * a CFL number; the paper states no step): dt = cfl * h / ((2p+1) *
 * lambda_max) (cfl_mode 0) or cfl * h / lambda_max (cfl_mode 1), where
 * lambda_max is the largest lambda_e of eq. (visc) of U (device) over the
 * mesh.  Synchronous; writes the host double *dt_host. */
int dg_stable_dt(dg_ctx* ctx, const double* U, double cfl, double* dt_host);

/* Check U (device) for NaN/Inf: counted on the device, summed on the host.
 * Synchronous.  Returns DG_OK, or DG_ENONFINITE and the number of non-finite
 * entries in *count (may be NULL). */
int dg_check_finite(dg_ctx* ctx, const double* U, int64_t* count);

/* Not part of the method: a plain streaming device copy dst[0..n) =
 * src[0..n) queued on `stream` (NULL: the default stream), 16 bytes per lane
 * where both pointers are 16-byte aligned.  Its bandwidth is the measured
 * ceiling the stage kernels' HBM traffic is read against.  src, dst: device,
 * caller-owned, must not overlap.  Errors: DG_EINVAL for n < 0, NULL pointers
 * with n > 0, or overlapping ranges. */
int dg_stream_copy(const double* src, double* dst, int64_t n, void* stream);

/* Launch shape of the stage kernel: cells per workgroup, one of the compiled
 * tiles: 1D tx in {256, 64} (ty ignored), 2D (tx, ty) in {(16,16), (8,8)}.
 * The result does not depend on the tile (per-cell arithmetic is identical).
 * Default at dg_init_mesh: 256 (1D), 16x16 (2D; 8x8 if 16x16 exceeds LDS or
 * the mesh has fewer 16x16 tiles than the GPU has compute units, for degrees
 * 3 and 4, and for the KPP flux below four 16x16 tiles per compute unit).  With the KPP flux an
 * 8x8 tile runs on 4 to 16 waves, which evaluate the sine and cosine at the
 * tile's volume and face nodes apart from the cells' sums.
 * Errors: DG_EINVAL for another shape, DG_EUNSUPPORTED if it exceeds LDS. */
int dg_set_tile(dg_ctx* ctx, int32_t tx, int32_t ty);
int dg_get_tile(const dg_ctx* ctx, int32_t* tx, int32_t* ty);

/* Fused step kernel (eq. (ssp), all three stages in one launch): a tile
 * loads U^n on itself and three rings of cells around it and evaluates the
 * stages on shrinking rings in LDS, so one step moves U^n and U^(n+1) through
 * HBM once.  Same per-cell arithmetic as the per-stage kernel, so results are
 * bitwise the same.  The Euler system has a step kernel of its own (three
 * components per cell, walls handled by the cell code).  Used by dg_step and
 * dg_run.  mode: -1 automatic (default: on in 1D (for the Euler system up
 * to four 256-cell tiles per compute unit), and in 2D for meshes of at most
 * one 16x16 tile per compute unit, where per-stage launches are latency
 * bound, and of at most four for degree 1 and for degree-2 Burgers, except
 * for the KPP flux), 0 off, 1 on.  Errors:
 * DG_EINVAL for another mode, DG_EUNSUPPORTED for mode 1 when the three
 * tiles exceed LDS (2D degree 4), rk_order is not 3 or bc_kind is not
 * CONSTANT; in those cases the automatic mode never uses it.  dg_get_fused
 * writes 1 if steps use it.
 * Mode 0 also makes the adjoint (below) launch its two passes of every stage
 * separately instead of sharing launches between consecutive stages; the
 * result is bitwise the same either way. */
int dg_set_fused(dg_ctx* ctx, int32_t mode);
int dg_get_fused(const dg_ctx* ctx, int32_t* active);

/* Launch shape of the fused step kernel (eq. (ssp)): 1D 256 cells (ty
 * ignored); 2D 16 columns of 16 or 8 rows, (tx, ty) in {(16,16), (16,8)}.
 * The result does not depend on it (per-cell arithmetic is identical).
 * Default, chosen per mesh until set: 16x8 on 2D meshes of at most a quarter
 * as many 16x16 tiles as the GPU has compute units, or of more than one per
 * compute unit at degree 2 (at degree 1: up to three); else 16x16.  Takes
 * effect while steps use the fused kernel.
 * Errors: DG_EINVAL for another shape. */
int dg_set_step_tile(dg_ctx* ctx, int32_t tx, int32_t ty);
int dg_get_step_tile(const dg_ctx* ctx, int32_t* tx, int32_t* ty);

/* Replace the stream the context queues work on. */
int dg_set_stream(dg_ctx* ctx, void* stream);

/* Message of the last failure on the calling thread ("" if none). */
const char* dg_last_error(void);

/* ------------------------------------------------------------------------
 * Discrete adjoint (reverse mode of the fully discrete scheme).
 *
 * The derivative is that of the computed map, including the HWENO weights,
 * the sensor min(1, ratio)^q and its threshold, lambda_e and the LLF wave
 * speed; where a max/min switches the derivative of the active branch is
 * used (ties: split evenly).  The first adjoint call on a context allocates
 * two state-sized buffers and two sensor-record buffers (DG_EUNSUPPORTED if
 * the adjoint kernels' tile exceeds LDS).  Every adjoint call returns
 * DG_EUNSUPPORTED for mode ZHAO, for the KPP and Euler fluxes and for bc_kind
 * RIEMANN;
 * the step and run adjoints also for rk_order other than 3.
 * ------------------------------------------------------------------------ */

/* out = J(U)^T v: the transpose Jacobian of dU/dt = L(U) (dg_rhs) applied to
 * v.  U, v, out: device [n_cells * n_loc]; out must not overlap U or v. */
int dg_rhs_vjp(dg_ctx* ctx, const double* U, const double* v, double* out);

/* lam_in = (d step(Un) / d Un)^T lam_out for one SSP-RK3 step of size dt
 * (eq. ssp); the stage states are recomputed from Un.  lam_in may alias
 * lam_out but not Un. */
int dg_step_adjoint(dg_ctx* ctx, const double* Un, double dt, const double* lam_out, double* lam_in);

/* Checkpointed gradient of a function of U^N with respect to U^0 over
 * nsteps steps, with at most nsnaps stored states (binomial checkpointing:
 * each reverse sub-range advances to a checkpoint chosen so the remainder
 * can be reversed with one slot fewer within the same number of sweeps).
 * ckpt: caller-owned device buffer of (nsnaps + 2) * n_cells * n_loc doubles
 * (slot 0 holds U^0, the last slot is working space).  stages: NULL, or a
 * device buffer of 2 * nsteps * n_cells * n_loc doubles that receives the RK
 * stage states U^(1), U^(2) of every step the forward sweep advances (with
 * nsnaps >= nsteps - 1 that is every step); the backward then skips their
 * recomputation.  ckpt and stages must not change between the two calls, and
 * both calls take the same stages argument.
 * dg_adjoint_forward: U^0 -> U^N (written to UT), storing checkpoints.
 * dg_adjoint_backward: lam holds dJ/dU^N on entry and dJ/dU^0 on exit. */
int dg_adjoint_forward(dg_ctx* ctx, const double* U0, double* UT, double dt, int32_t nsteps, int32_t nsnaps,
                       double* ckpt, double* stages);
int dg_adjoint_backward(dg_ctx* ctx, double dt, int32_t nsteps, int32_t nsnaps, double* ckpt,
                        const double* stages, double* lam);

/* Branch records of a run, for finite-difference checks of the adjoint: the
 * computed map is differentiable except where a branch of the method
 * switches: min(1, ratio) and the threshold b of the sensor (eqs.
 * sensor/gensensor), the node of the largest |F'| in lambda_e (eq. visc) and
 * the larger trace in the LLF wave speed (Sec. 2).  This runs nsteps SSP-RK3
 * steps of U in place, as dg_run (same per-stage kernels, launched directly,
 * bitwise the same result), and folds for every cell the branches its
 * operator evaluations took in every stage into three 32-bit hashes,
 * sig[k * n_cells + cell] (device, caller-owned, 3 * n_cells uint32; cleared
 * by the call): k = 0 the sensor, 1 lambda_e, 2 the LLF wave speeds.  Two
 * runs whose records differ in a cell crossed a kink of the map there; two
 * equal records mean no recorded branch switched (up to hash collisions).
 * DG_EUNSUPPORTED outside the adjoint's coverage (see above). */
int dg_run_signature(dg_ctx* ctx, double* U, double dt, int32_t nsteps, uint32_t* sig);

/* Host-only statistics of the checkpoint schedule: stats[6] = {forward-sweep
 * steps, recomputed steps, stores, adjoint steps, highest slot, actions}. */
int dg_revolve_stats(int32_t nsteps, int32_t nsnaps, int64_t* stats);

/* Host-side validation of a descriptor (the checks dg_init_mesh performs
 * before any device call).  DG_OK or DG_EINVAL. */
int dg_validate_desc(const dg_mesh_desc* desc);

/* ------------------------------------------------------------------------
 * Batched execution of independent problems.
 *
 * Many problems of uneven mesh size and degree advance together: problems
 * are grouped into kernel classes (dim, p, flux, mode); every RK stage of a
 * class is one launch over the class's tile list (one workgroup per tile,
 * or a persistent grid that walks the list), and a run
 * of N steps is one HIP graph in which the classes form independent chains on
 * up to four concurrent branches.  Each problem's arithmetic is that of the
 * single-problem path (same per-cell code, same tables), so a problem's
 * result does not depend on the batch it is part of.
 * ------------------------------------------------------------------------ */
typedef struct dg_batch dg_batch;

/* Create a batch from `count` descriptors (each validated as for
 * dg_init_mesh; DG_EUNSUPPORTED for rk_order other than 3, bc_kind RIEMANN
 * or the Euler flux; all work runs on
 * descs[0].stream).  Allocates the problem
 * table, tile lists and two stage arenas of the batch's total size. */
int dg_batch_create(const dg_mesh_desc* descs, int32_t count, dg_batch** out);
void dg_batch_destroy(dg_batch* batch);

/* Layout of the caller-owned state arena: problem i occupies doubles
 * [offsets[i], offsets[i+1]) in the single-problem layout.  offsets: host
 * array of count+1 int64 (may be NULL); total: host int64 (may be NULL). */
int dg_batch_layout(const dg_batch* batch, int64_t* offsets, int64_t* total);

/* nsteps SSP-RK3 steps of every problem, problem i with step dts[i] (host
 * array of count doubles, each finite and > 0), in place on the arena
 * (device).  The graph is recorded once per (arena, dts, nsteps) and
 * replayed. */
int dg_batch_run(dg_batch* batch, double* arena, const double* dts, int32_t nsteps);

/* Reference schedule for comparisons: the same steps with the plain stage
 * kernel, one launch per problem per RK stage, problems in order, on the
 * batch stream, no graph.  Arguments as for dg_batch_run. */
int dg_batch_run_sequential(dg_batch* batch, double* arena, const double* dts, int32_t nsteps);

/* Schedule of class `cls` (0 <= cls < number of classes): tile shape (as in
 * dg_set_tile), persistent grid of grid_per_cu workgroups per compute unit
 * (1..64; 0: one workgroup per tile, without the persistent loop), and tile
 * order (0: problems by decreasing size, 1: increasing, 2: problems
 * interleaved round robin).  DG_EINVAL outside those ranges. */
int dg_batch_num_classes(const dg_batch* batch, int32_t* n);
int dg_batch_set_schedule(dg_batch* batch, int32_t cls, int32_t tx, int32_t ty, int32_t grid_per_cu,
                          int32_t order);
/* info[10] = {dim, p, flux, mode, problems, tx, ty, grid_per_cu, order, branch} */
int dg_batch_get_schedule(const dg_batch* batch, int32_t cls, int32_t* info);
/* Number of concurrent graph branches (1..4); classes are assigned to them
 * longest-first onto the least loaded branch. */
int dg_batch_set_branches(dg_batch* batch, int32_t branches);

/* Autotuner: for every class, time `reps` stage launches (reading the arena,
 * writing only internal buffers: the state is not modified) for every tile
 * shape, grid size and tile order, keep the fastest; then choose the branch
 * count from timed stages.  Synchronous.  dts as for dg_batch_run.  report
 * (host, may be NULL) receives a text summary of at most report_len bytes. */
int dg_batch_tune(dg_batch* batch, double* arena, const double* dts, int32_t reps, char* report,
                  int32_t report_len);

#ifdef __cplusplus
}
#endif
#endif /* DGWENO_H */
