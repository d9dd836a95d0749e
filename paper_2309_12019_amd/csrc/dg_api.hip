// C-ABI of the library (declared in include/dgweno.h): argument validation,
// context and buffer ownership, kernel dispatch, graph capture of dg_run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/dgweno.h"
#include "dg_euler.hpp"
#include "dg_launch.hpp"

using dgk::LaunchFn;
using dgk::LaunchReq;
using dgk::StageArgs;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(DG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Makes `dev` the current HIP device for a scope (no-op when it already is)
// and restores the previous one.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    int cur = -1;
    if (dev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != dev && hipSetDevice(dev) == hipSuccess) prev = cur;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

LaunchFn launcher(int dim, int p) {
  static const LaunchFn tab[2][4] = {{dgk_launch_1_1, dgk_launch_1_2, dgk_launch_1_3, dgk_launch_1_4},
                                     {dgk_launch_2_1, dgk_launch_2_2, dgk_launch_2_3, dgk_launch_2_4}};
  return tab[dim - 1][p - 1];
}

struct GraphKey {
  const double* U;
  double dt;
  int steps;
  bool operator<(const GraphKey& o) const { return std::tie(U, dt, steps) < std::tie(o.U, o.dt, o.steps); }
};

}  // namespace

struct dg_ctx {
  dg_mesh_desc d;
  int dev = 0;             // HIP device of the context
  int nl = 0;
  long long ncells = 0;
  int tx = 0, ty = 1;
  int max_lds = 65536;
  int cus = 256;
  int fused_mode = -1;   // fused step kernel: -1 automatic, 0 off, 1 on
  bool fused = false;    // whether steps use the fused kernel
  int sty = dgk::kStepTile2D;  // 2D fused step tile: 16 columns of sty rows (16 or 8)
  bool sty_set = false;        // sty set by dg_set_step_tile (else chosen per mesh)
  double h = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;  // private stream used only to record graphs
  double* U1 = nullptr;
  double* U2 = nullptr;
  double* U3 = nullptr;           // third stage buffer (five-stage method only)
  double* tclock = nullptr;       // BC_RIEMANN: device copy of the time a run or step starts from; the
                                  // stages take their times as offsets from it (graphs replay at any time)
  double t = 0.0;                 // the context's clock: time of the state dg_step/dg_run advance
  double* red = nullptr;          // per-block partial results of reductions
  size_t red_len = 0;
  LaunchFn launch = nullptr;
  std::map<GraphKey, hipGraphExec_t> graphs;
  // adjoint buffers, allocated on first use
  double* A1 = nullptr;   // cotangent of U^(2)
  double* A2 = nullptr;   // cotangent of U^(1)
  double* Zmem = nullptr;  // both record buffers (one allocation)
  double* Z = nullptr;     // sensor records
  double* Z2 = nullptr;    // second record buffer: launches that read one set and write another
};

// ---------------------------------------------------------------------------
// Stage buffers of dg_step_static, for callers that cannot allocate: three
// buffers of kStaticStageDoubles doubles in one file-scope device array
// (24 MiB, held on every device the library runs on until the process
// ends).  Host code never uses the array's name as an address: its address on
// each device comes from hipGetSymbolAddress, taken once per device.
// ---------------------------------------------------------------------------
constexpr long long kStaticStageDoubles = 1LL << 20;
static __device__ __align__(256) double scratch[3 * kStaticStageDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device (looked up on first use there).
int scratch_on_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(DG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_EUNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                                                 kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(DG_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

}  // namespace

namespace {

StageArgs base_args(const dg_ctx* c) {
  StageArgs A{};
  const dg_mesh_desc& d = c->d;
  A.nx = d.nx;
  A.ny = d.dim == 2 ? d.ny : 1;
  A.per_x = d.periodic_x != 0;
  A.per_y = d.dim == 2 && d.periodic_y != 0;
  A.h = c->h;
  A.g2h = 2.0 / c->h;
  dgk::stage_lfac(d.dim, d.p, A.g2h, A.lfac);
  A.x0 = d.x0;
  A.y0 = d.dim == 2 ? d.y0 : 0.0;
  A.vx = d.vel_x;
  A.vy = d.dim == 2 ? d.vel_y : 0.0;
  A.omega = d.dim == 2 ? d.omega : 0.0;
  A.cx = d.rot_cx;
  A.cy = d.rot_cy;
  A.anorm = d.dim == 2 ? std::hypot(d.vel_x, d.vel_y) : std::fabs(d.vel_x);
  A.bc = d.bc_value;
  A.q = d.q;
  A.bthr = d.b;
  A.wnb = d.w_nb;
  A.eps = d.weno_eps;
  A.wpow = d.weno_pow;
  A.lam_over = d.lambda_override;
  A.theta = d.zhao_theta;
  A.bc_kind = d.bc_kind;
  A.tx = c->tx;
  A.ty = d.dim == 2 ? c->ty : 1;
  return A;
}

size_t stage_lds_bytes(int dim, int nl, int p, int flux, int tx, int ty) {
  return sizeof(double) * (size_t)dgk::stage_kernel_lds_doubles(dim, nl, p, flux, tx, dim == 2 ? ty : 1);
}

// BC_RIEMANN: the device clock := t (on st, before the stages that read it)
int set_clock(dg_ctx* c, hipStream_t st, double t) {
  if (!c->tclock) return DG_OK;
  const hipError_t e = dgk_set_clock(c->tclock, t, st);
  return e == hipSuccess ? DG_OK : hip_fail(e, "clock");
}

// one stage: out = a*un + b*(uin + dt*L(uin)), or out = L(uin) when rhs_only;
// t is the time of uin (it enters through the BC_RIEMANN exterior state only;
// there, with the context's clock, t is the offset from the clock's time)
int stage(dg_ctx* c, hipStream_t st, const double* uin, const double* un, double* out, double* gamma,
          double a, double b, double dt, int rhs_only, double t = 0.0) {
  LaunchReq r{};
  r.kind = dgk::LAUNCH_STAGE;
  r.flux = c->d.flux;
  r.mode = c->d.mode;
  r.args = base_args(c);
  r.args.tclock = c->tclock;
  // 8x8 tiles of several waves on meshes of a few tiles per compute unit:
  // the KPP flux by split_waves; the others four waves up to three tiles
  // per compute unit (per step, 192^2 P2 rotation 17.1 -> 15.7 us at 2.25
  // tiles per CU, but 256^2 20.4 -> 23.1 at four)
  if (c->d.dim == 2 && c->tx == 8) {
    const long long t8 = (long long)((c->d.nx + 7) / 8) * ((c->d.ny + 7) / 8);
    if (c->d.flux == DG_FLUX_KPP)
      r.waves = dgk::split_waves(t8, c->cus, c->d.p);
    else
      r.waves = t8 <= 3LL * c->cus ? 4 : 1;
  }
  r.args.uin = uin;
  r.args.un = un;
  r.args.out = out;
  r.args.gamma = gamma;
  r.args.a = a;
  r.args.b = b;
  r.args.dt = dt;
  r.args.rhs_only = rhs_only;
  r.args.t = t;
  r.stream = st;
  hipError_t e = c->launch(&r);
  if (e != hipSuccess) return hip_fail(e, "stage kernel launch");
  return DG_OK;
}

// eq. (ssp): U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1)); U = 1/3 U + 2/3 (U2 + dt L(U2)).
// The stage states go to U1, U2 (default: the context's buffers).
// One SSP-RK3 step from Un into Uout (Uout may be Un: the last stage reads
// U^n and writes the same element from one thread); the stage states go to
// U1, U2 (the handle's scratch unless given).  The step starts at time t; the
// stages' operators are taken at t, t + dt and t + dt/2.
int rk3_step_to(dg_ctx* c, hipStream_t st, const double* Un, double* Uout, double dt, double* U1 = nullptr,
                double* U2 = nullptr, double t = 0.0) {
  int rc;
  U1 = U1 ? U1 : c->U1;
  U2 = U2 ? U2 : c->U2;
  if ((rc = stage(c, st, Un, Un, U1, nullptr, 0.0, 1.0, dt, 0, t))) return rc;
  if ((rc = stage(c, st, U1, Un, U2, nullptr, 0.75, 0.25, dt, 0, t + dt))) return rc;
  return stage(c, st, U2, Un, Uout, nullptr, 1.0 / 3.0, 2.0 / 3.0, dt, 0, t + 0.5 * dt);
}

// One fused SSP-RK3 step (one launch) from Un into Uout != Un.
int step_fused(dg_ctx* c, hipStream_t st, const double* Un, double* Uout, double dt) {
  LaunchReq r{};
  r.kind = dgk::LAUNCH_STEP;
  r.flux = c->d.flux;
  r.mode = c->d.mode;
  r.args = base_args(c);
  r.args.uin = Un;
  r.args.un = Un;
  r.args.out = Uout;
  r.args.dt = dt;
  r.args.tx = c->d.dim == 1 ? dgk::kStepTile1D : dgk::kStepTile2D;
  r.args.ty = c->d.dim == 1 ? 1 : c->sty;
  r.stream = st;
  hipError_t e = c->launch(&r);
  if (e != hipSuccess) return hip_fail(e, "step kernel launch");
  return DG_OK;
}

// The second-order SSP step in place from time t: U1 = U + dt L(U, t);
// U = 1/2 U + 1/2 (U1 + dt L(U1, t + dt)).
int rk2_step(dg_ctx* c, hipStream_t st, double* U, double dt, double t) {
  int rc;
  if ((rc = stage(c, st, U, U, c->U1, nullptr, 0.0, 1.0, dt, 0, t))) return rc;
  return stage(c, st, c->U1, U, U, nullptr, 0.5, 0.5, dt, 0, t + dt);
}

// Shu-Osher coefficients of the five-stage fourth-order SSP method (Spiteri
// and Ruuth): U_k = sum_j alpha_kj U_j + beta_kj dt L(U_j).
constexpr double kA10 = 1.0, kB10 = 0.391752226571890;
constexpr double kA20 = 0.444370493651235, kA21 = 0.555629506348765, kB21 = 0.368410593050371;
constexpr double kA30 = 0.620101851488403, kA32 = 0.379898148511597, kB32 = 0.251891774271694;
constexpr double kA40 = 0.178079954393132, kA43 = 0.821920045606868, kB43 = 0.544974750228521;
constexpr double kA52 = 0.517231671970585, kA53 = 0.096059710526147, kB53 = 0.063692468666290;
constexpr double kA54 = 0.386708617503269, kB54 = 0.226007483236906;

// The five-stage step in place, as stage launches of the form
// out = a un + b (uin + dt' L(uin)) with dt' = dt beta / alpha.  The last
// stage needs L(U3) and L(U4); L(U3) is evaluated twice (for U4 and for the
// partial sum W = a52 U2 + a53 U3 + b53 dt L(U3)) so that every launch
// remains one stage kernel.  Buffers: U1 <- U1, U3; U2 <- U2, W; U3 <- U4.
// The stage states' times follow from the same combination applied to t' = 1.
int rk54_step(dg_ctx* c, hipStream_t st, double* U, double dt, double t0) {
  int rc;
  double *A = c->U1, *B = c->U2, *C = c->U3;
  const double t1 = kA10 * t0 + kB10 * dt;
  const double t2 = (kA20 * t0 + kA21 * t1) + kB21 * dt;
  const double t3 = (kA30 * t0 + kA32 * t2) + kB32 * dt;
  const double t4 = (kA40 * t0 + kA43 * t3) + kB43 * dt;
  if ((rc = stage(c, st, U, U, A, nullptr, 0.0, kA10, dt * kB10 / kA10, 0, t0))) return rc;  // U1
  if ((rc = stage(c, st, A, U, B, nullptr, kA20, kA21, dt * kB21 / kA21, 0, t1))) return rc;  // U2
  if ((rc = stage(c, st, B, U, A, nullptr, kA30, kA32, dt * kB32 / kA32, 0, t2))) return rc;  // U3
  if ((rc = stage(c, st, A, U, C, nullptr, kA40, kA43, dt * kB43 / kA43, 0, t3))) return rc;  // U4
  if ((rc = stage(c, st, A, B, B, nullptr, kA52, kA53, dt * kB53 / kA53, 0, t3))) return rc;  // W
  return stage(c, st, C, B, U, nullptr, 1.0, kA54, dt * kB54 / kA54, 0, t4);                 // U^{n+1}
}

// One SSP step of the descriptor's order on U in place from time t (stage kernels).
int ssp_step(dg_ctx* c, hipStream_t st, double* U, double dt, double t) {
  if (c->d.rk_order == 2) return rk2_step(c, st, U, dt, t);
  if (c->d.rk_order == 4) return rk54_step(c, st, U, dt, t);
  return rk3_step_to(c, st, U, U, dt, nullptr, nullptr, t);
}

// len SSP steps on U in place.  With the fused kernel (three-stage method
// only) the steps alternate between U and the scratch buffer U1 (the kernel
// cannot write the array it reads), and an odd count ends with one copy back
// into U.  Step s starts at time t0 + s dt.
int rk_steps(dg_ctx* c, hipStream_t st, double* U, double dt, int len, double t0 = 0.0) {
  if (!c->fused) {
    for (int s = 0; s < len; ++s) {
      int rc = ssp_step(c, st, U, dt, t0 + s * dt);
      if (rc) return rc;
    }
    return DG_OK;
  }
  double* cur = U;
  double* other = c->U1;
  for (int s = 0; s < len; ++s) {
    int rc = step_fused(c, st, cur, other, dt);
    if (rc) return rc;
    std::swap(cur, other);
  }
  if (cur != U) {
    hipError_t e = hipMemcpyAsync(U, cur, sizeof(double) * (size_t)c->ncells * c->nl, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "step copy");
  }
  return DG_OK;
}

int rk3_step(dg_ctx* c, hipStream_t st, double* U, double dt, double* U1 = nullptr, double* U2 = nullptr) {
  if (!U1 && !U2) return rk_steps(c, st, U, dt, 1);
  return rk3_step_to(c, st, U, U, dt, U1, U2);
}

int validate(const dg_mesh_desc* d) {
  if (!d) return fail(DG_EINVAL, "desc is NULL");
  if (d->dim != 1 && d->dim != 2) return fail(DG_EINVAL, "dim must be 1 or 2 (got %d)", d->dim);
  if (d->p < 1 || d->p > 4) return fail(DG_EINVAL, "p must be in 1..4 (got %d)", d->p);
  if (d->nx < 1) return fail(DG_EINVAL, "nx must be >= 1 (got %d)", d->nx);
  if (d->dim == 2 && d->ny < 1) return fail(DG_EINVAL, "ny must be >= 1 (got %d)", d->ny);
  if ((long long)d->nx * (d->dim == 2 ? d->ny : 1) > (1LL << 31) - 1)
    return fail(DG_EINVAL, "mesh too large");
  if (!(d->x1 > d->x0) || !std::isfinite(d->x0) || !std::isfinite(d->x1))
    return fail(DG_EINVAL, "need x0 < x1 (finite)");
  if (d->dim == 2) {
    if (!(d->y1 > d->y0) || !std::isfinite(d->y0) || !std::isfinite(d->y1))
      return fail(DG_EINVAL, "need y0 < y1 (finite)");
    const double hx = (d->x1 - d->x0) / d->nx, hy = (d->y1 - d->y0) / d->ny;
    if (std::fabs(hx - hy) > 1e-12 * hx) return fail(DG_EINVAL, "2D cells must be square (hx=%g hy=%g)", hx, hy);
  }
  if (d->flux != DG_FLUX_LINADV && d->flux != DG_FLUX_BURGERS && d->flux != DG_FLUX_KPP &&
      d->flux != DG_FLUX_EULER)
    return fail(DG_EINVAL, "unknown flux %d", d->flux);
  if (d->flux == DG_FLUX_EULER && d->dim != 1) return fail(DG_EINVAL, "the Euler system is one-dimensional here");
  if (d->flux == DG_FLUX_KPP && d->dim != 2) return fail(DG_EINVAL, "the KPP flux is two-dimensional");
  if (d->mode != DG_MODE_DG && d->mode != DG_MODE_LO && d->mode != DG_MODE_WENO && d->mode != DG_MODE_ZHAO)
    return fail(DG_EINVAL, "unknown mode %d", d->mode);
  if (!(d->zhao_theta > 0.0) || !std::isfinite(d->zhao_theta)) return fail(DG_EINVAL, "zhao_theta must be > 0");
  if (d->rk_order < 2 || d->rk_order > 4) return fail(DG_EINVAL, "rk_order must be 2, 3 or 4 (got %d)", d->rk_order);
  if (d->bc_kind != DG_BC_CONSTANT && d->bc_kind != DG_BC_RIEMANN)
    return fail(DG_EINVAL, "unknown bc_kind %d", d->bc_kind);
  if (d->bc_kind == DG_BC_RIEMANN &&
      (d->dim != 2 || d->flux != DG_FLUX_BURGERS || d->periodic_x || d->periodic_y))
    return fail(DG_EINVAL, "bc_kind RIEMANN needs 2D Burgers with non-periodic boundaries");
  if (!(d->q >= 1.0) || !std::isfinite(d->q)) return fail(DG_EINVAL, "q must be >= 1");
  if (!(d->b >= 0.0 && d->b <= 1.0)) return fail(DG_EINVAL, "b must be in [0,1]");
  const int m = 2 * d->dim;
  if (!(d->w_nb > 0.0) || !(m * d->w_nb < 1.0)) return fail(DG_EINVAL, "need 0 < w_nb < 1/(2 dim)");
  if (!(d->weno_eps > 0.0) || !std::isfinite(d->weno_eps)) return fail(DG_EINVAL, "weno_eps must be > 0");
  if (!(d->weno_pow > 0.0) || !std::isfinite(d->weno_pow)) return fail(DG_EINVAL, "weno_pow must be > 0");
  if (!std::isfinite(d->lambda_override) || d->lambda_override < 0)
    return fail(DG_EINVAL, "lambda_override must be >= 0");
  const double vals[] = {d->vel_x, d->vel_y, d->omega, d->rot_cx, d->rot_cy, d->bc_value};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(DG_EINVAL, "non-finite flux parameter");
  // quadrature: 0 or the compile-time rule of this flux and degree
  const int qv = dgk::quad_points(d->dim, d->p, d->flux);
  const int32_t qs[3] = {d->quad_vol, d->quad_face, d->quad_proj};
  const int built[3] = {qv, qv, d->p + 2};
  const char* which[3] = {"quad_vol", "quad_face", "quad_proj"};
  for (int k = 0; k < 3; ++k) {
    if (qs[k] < 0 || qs[k] > dgk::kMaxQ) return fail(DG_EINVAL, "%s must be 0 or 1..%d (got %d)", which[k], dgk::kMaxQ, qs[k]);
    if (qs[k] != 0 && qs[k] != built[k])
      return fail(DG_EUNSUPPORTED, "%s = %d is not built: the rule for this flux and degree has %d points", which[k],
                  qs[k], built[k]);
  }
  if (d->cfl_mode != 0 && d->cfl_mode != 1) return fail(DG_EINVAL, "cfl_mode must be 0 or 1 (got %d)", d->cfl_mode);
  if (d->check_finite != 0 && d->check_finite != 1)
    return fail(DG_EINVAL, "check_finite must be 0 or 1 (got %d)", d->check_finite);
  if (d->device < -1) return fail(DG_EINVAL, "device must be -1 or a device index (got %d)", d->device);
  return DG_OK;
}

// With check_finite: count the non-finite entries of U (queued after the
// caller's work on the context stream, then waited for).
int finite_or_fail(dg_ctx* c, const double* U);

int check_tile(const dg_ctx* c, int tx, int ty) {
  const int dim = c->d.dim;
  bool ok = false;
  if (dim == 1) {
    for (int t : dgk::kTiles1D) ok |= tx == t;
    ty = 1;
  } else {
    for (auto& t : dgk::kTiles2D) ok |= tx == t[0] && ty == t[1];
  }
  if (!ok)
    return fail(DG_EINVAL, dim == 1 ? "1D tile must be 256 or 64 cells (got %d)"
                                     : "2D tile must be 16x16 or 8x8 (got %dx%d)", tx, ty);
  if (stage_lds_bytes(dim, c->nl, c->d.p, c->d.flux, tx, ty) > (size_t)c->max_lds)
    return fail(DG_EUNSUPPORTED, "tile %dx%d needs %zu bytes of LDS (limit %d)", tx, ty,
                stage_lds_bytes(dim, c->nl, c->d.p, c->d.flux, tx, ty), c->max_lds);
  return DG_OK;
}

int zrec_size(int dim, int nl) { return dgk::zrec_doubles(dim, nl); }

int ensure_adjoint(dg_ctx* c) {
  if (c->d.flux == DG_FLUX_EULER) return fail(DG_EUNSUPPORTED, "the adjoint does not cover the Euler system");
  if (c->d.bc_kind != DG_BC_CONSTANT)
    return fail(DG_EUNSUPPORTED, "the adjoint does not cover the exact-solution exterior state");
  if (c->d.mode == DG_MODE_ZHAO) return fail(DG_EUNSUPPORTED, "the adjoint does not cover the ZHAO sensor");
  if (c->d.flux == DG_FLUX_KPP) return fail(DG_EUNSUPPORTED, "the adjoint does not cover the KPP flux");
  if (c->A1) return DG_OK;
  // the adjoint kernels' tiles hold the state and the cotangent
  const int atx = c->d.dim == 2 ? dgk::kAdjTileX : c->tx, aty = c->d.dim == 2 ? dgk::kAdjTileY : 1;
  const size_t alds = 2 * sizeof(double) * (size_t)dgk::tile_lds_doubles(c->d.dim, c->nl, atx, aty);
  if (alds > (size_t)c->max_lds)
    return fail(DG_EUNSUPPORTED, "the adjoint tile needs %zu bytes of LDS (limit %d)", alds, c->max_lds);
  const size_t n = (size_t)c->ncells * c->nl;
  const size_t nz = (size_t)c->ncells * zrec_size(c->d.dim, c->nl);
  hipError_t e;
  if ((e = hipMalloc(&c->A1, n * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->A2, n * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->Zmem, 2 * nz * sizeof(double))) != hipSuccess) {
    if (c->A1) (void)hipFree(c->A1);
    if (c->A2) (void)hipFree(c->A2);
    c->A1 = c->A2 = nullptr;
    c->Zmem = c->Z = c->Z2 = nullptr;
    return fail(DG_ENOMEM, "adjoint buffers: %s", hipGetErrorString(e));
  }
  c->Z = c->Zmem;
  c->Z2 = c->Zmem + nz;
  return DG_OK;
}

// One adjoint launch (kind: pass A, pass B, or pass B + the next pass A):
// records z of U seeded with v (pass A); out = alpha v + beta J(U)^T v +
// g1 X + g2 Y from the records z (pass B); then the records znext of unext
// seeded with out (pass B + A).
int adj_launch(dg_ctx* c, hipStream_t st, int kind, const double* U, const double* v, double* z, double* out,
               double alpha, double beta, const double* X, double g1, const double* Y, double g2,
               const double* unext = nullptr, double* znext = nullptr) {
  LaunchReq r{};
  r.kind = kind;
  r.flux = c->d.flux;
  r.mode = c->d.mode;
  r.stream = st;
  r.adj.s = base_args(c);
  r.adj.s.uin = U;
  r.adj.v = v;
  r.adj.z = z;
  r.adj.out = out;
  r.adj.X = X;
  r.adj.Y = Y;
  r.adj.alpha = alpha;
  r.adj.beta = beta;
  r.adj.g1 = g1;
  r.adj.g2 = g2;
  r.adj.unext = unext;
  r.adj.znext = znext;
  hipError_t e = c->launch(&r);
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return DG_OK;
}

// out = alpha v + beta J(U)^T v + g1 X + g2 Y (pass A, when the operator has a
// sensor, then pass B)
int adjoint_stage(dg_ctx* c, hipStream_t st, const double* U, const double* v, double* out, double alpha,
                  double beta, const double* X, double g1, const double* Y, double g2) {
  int rc;
  if (c->d.mode == DG_MODE_WENO &&
      (rc = adj_launch(c, st, dgk::LAUNCH_ADJ_SENSOR, U, v, c->Z, nullptr, 0, 0, nullptr, 0, nullptr, 0)))
    return rc;
  return adj_launch(c, st, dgk::LAUNCH_ADJ_GRAD, U, v, c->Z, out, alpha, beta, X, g1, Y, g2);
}

// Whether the adjoint runs pass B of a stage and pass A of the stage before
// it in one launch (the stabilised operator; switched off with the fused
// step kernel, for comparison).
bool adj_fused(const dg_ctx* c) { return c->d.mode == DG_MODE_WENO && c->fused_mode != 0; }

// lam_in = (d step(Un) / d Un)^T lam_out for eq. (ssp).  The stage states
// U^(1), U^(2) are recomputed from Un unless given (S1, S2).
// With adj_fused: `zpend` says that the records of U^(2) seeded with lam_out
// are already in c->Z (written by the previous adjoint step's last launch);
// `next_S2`, when given, is U^(2) of the step reversed next, whose records
// (seeded with lam_in) the last launch writes for that step.
int rk3_adjoint(dg_ctx* c, hipStream_t st, const double* Un, double dt, const double* lam_out, double* lam_in,
                const double* S1 = nullptr, const double* S2 = nullptr, bool zpend = false,
                const double* next_S2 = nullptr) {
  int rc;
  if (!S1 || !S2) {
    if ((rc = stage(c, st, Un, Un, c->U1, nullptr, 0.0, 1.0, dt, 0))) return rc;
    if ((rc = stage(c, st, c->U1, Un, c->U2, nullptr, 0.75, 0.25, dt, 0))) return rc;
    S1 = c->U1;
    S2 = c->U2;
  }
  const double a2 = 0.75, b2 = 0.25, a3 = 1.0 / 3.0, b3 = 2.0 / 3.0;
  if (!adj_fused(c)) {
    // stage 3: U = a3 Un + b3 (U2 + dt L(U2))  ->  lam_U2 = b3 mu + b3 dt J(U2)^T mu
    if ((rc = adjoint_stage(c, st, S2, lam_out, c->A1, b3, b3 * dt, nullptr, 0, nullptr, 0))) return rc;
    // stage 2: U2 = a2 Un + b2 (U1 + dt L(U1))
    if ((rc = adjoint_stage(c, st, S1, c->A1, c->A2, b2, b2 * dt, nullptr, 0, nullptr, 0))) return rc;
    // stage 1: U1 = Un + dt L(Un); lam_n = lam_U1 + dt J(Un)^T lam_U1 + a2 lam_U2 + a3 mu
    return adjoint_stage(c, st, Un, c->A2, lam_in, 1.0, dt, c->A1, a2, lam_out, a3);
  }
  using dgk::LAUNCH_ADJ_GRAD;
  using dgk::LAUNCH_ADJ_GRAD_SENSOR;
  using dgk::LAUNCH_ADJ_SENSOR;
  // the same three stage adjoints, each pass B sharing a launch with the pass
  // A of the stage before it (records alternate between c->Z and c->Z2)
  if (!zpend && (rc = adj_launch(c, st, LAUNCH_ADJ_SENSOR, S2, lam_out, c->Z, nullptr, 0, 0, nullptr, 0, nullptr, 0)))
    return rc;
  if ((rc = adj_launch(c, st, LAUNCH_ADJ_GRAD_SENSOR, S2, lam_out, c->Z, c->A1, b3, b3 * dt, nullptr, 0, nullptr, 0,
                       S1, c->Z2)))
    return rc;
  if ((rc = adj_launch(c, st, LAUNCH_ADJ_GRAD_SENSOR, S1, c->A1, c->Z2, c->A2, b2, b2 * dt, nullptr, 0, nullptr, 0,
                       Un, c->Z)))
    return rc;
  if (!next_S2) return adj_launch(c, st, LAUNCH_ADJ_GRAD, Un, c->A2, c->Z, lam_in, 1.0, dt, c->A1, a2, lam_out, a3);
  rc = adj_launch(c, st, LAUNCH_ADJ_GRAD_SENSOR, Un, c->A2, c->Z, lam_in, 1.0, dt, c->A1, a2, lam_out, a3, next_S2,
                  c->Z2);
  std::swap(c->Z, c->Z2);  // the next step finds its first records in c->Z
  return rc;
}

// ---- binomial checkpointing (revolve-style) --------------------------------
enum { RV_RESTORE = 0, RV_ADVANCE = 1, RV_STORE = 2, RV_ADJOINT = 3 };
struct RvAction {
  int op, a;
};

long long binom_capped(int n, int k) {
  if (k < 0 || k > n) return 0;
  long long r = 1;
  for (int i = 1; i <= k; ++i) {
    r = r * (n - k + i) / i;
    if (r > (1LL << 40)) return 1LL << 40;
  }
  return r;
}

// Reverse steps [lo, hi) given the state at lo in slot `slot_lo` and `s` free
// slots: advance m steps and checkpoint, reverse the tail with s-1 slots, then
// the head with s.  m = n - C(s-1+t, s-1) with t the smallest number of sweeps
// such that C(s+t, s) >= n (the binomial bound of reversal with s snapshots).
void rv_plan(int lo, int hi, int s, int slot_lo, std::vector<int>& freeslots, std::vector<RvAction>& out) {
  const int n = hi - lo;
  if (n == 1) {
    out.push_back({RV_RESTORE, slot_lo});
    out.push_back({RV_ADJOINT, lo});
    return;
  }
  if (s == 0 || freeslots.empty()) {
    for (int k = hi - 1; k >= lo; --k) {
      out.push_back({RV_RESTORE, slot_lo});
      if (k > lo) out.push_back({RV_ADVANCE, k - lo});
      out.push_back({RV_ADJOINT, k});
    }
    return;
  }
  int t = 1;
  while (binom_capped(s + t, s) < n) ++t;
  long long m = n - binom_capped(s - 1 + t, s - 1);
  if (m < 1) m = 1;
  if (m > n - 1) m = n - 1;
  const int slot = freeslots.back();
  freeslots.pop_back();
  out.push_back({RV_RESTORE, slot_lo});
  out.push_back({RV_ADVANCE, (int)m});
  out.push_back({RV_STORE, slot});
  rv_plan(lo + (int)m, hi, s - 1, slot, freeslots, out);
  freeslots.push_back(slot);
  rv_plan(lo, lo + (int)m, s, slot_lo, freeslots, out);
}

std::vector<RvAction> rv_schedule(int nsteps, int nsnaps) {
  std::vector<int> freeslots;
  for (int k = nsnaps; k >= 1; --k) freeslots.push_back(k);
  std::vector<RvAction> out;
  rv_plan(0, nsteps, nsnaps, 0, freeslots, out);
  return out;
}

// index of the first action of the reverse sweep: the restore that precedes
// the first adjoint step
size_t rv_split(const std::vector<RvAction>& a) {
  size_t i = 0;
  while (i < a.size() && a[i].op != RV_ADJOINT) ++i;
  while (i > 0 && a[i].op != RV_RESTORE) --i;
  return i;
}

void drop_graphs(dg_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

// Steps whose stage states the forward sweep records: every step advanced
// before the first reverse action (the step index of each slot is tracked
// through the stores and restores), and the final step to U^N.
std::vector<char> rv_stage_steps(const std::vector<RvAction>& a, int nsteps, int nsnaps) {
  std::vector<char> have(nsteps, 0);
  std::vector<int> slot_step(nsnaps + 1, 0);
  const size_t split = rv_split(a);
  int cur = 0;
  for (size_t i = 0; i < split; ++i) {
    if (a[i].op == RV_RESTORE) cur = slot_step[a[i].a];
    if (a[i].op == RV_STORE) slot_step[a[i].a] = cur;
    if (a[i].op == RV_ADVANCE)
      for (int k = 0; k < a[i].a; ++k) have[cur++] = 1;
  }
  have[nsteps - 1] = 1;
  return have;
}

}  // namespace

extern "C" {

void dg_default_desc(dg_mesh_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->dim = 1;
  d->nx = 64;
  d->ny = 1;
  d->x0 = 0.0;
  d->x1 = 1.0;
  d->y0 = 0.0;
  d->y1 = 1.0;
  d->periodic_x = 1;
  d->periodic_y = 1;
  d->p = 2;
  d->flux = DG_FLUX_LINADV;
  d->vel_x = 1.0;
  d->rot_cx = 0.5;
  d->rot_cy = 0.5;
  d->mode = DG_MODE_WENO;
  d->q = 1.0;
  d->b = 0.0;
  d->w_nb = 1e-2;
  d->weno_eps = 1e-6;
  d->weno_pow = 2.0;
  d->zhao_theta = 1.0;
  d->rk_order = 3;
  d->bc_kind = DG_BC_CONSTANT;
  d->device = -1;
}

const char* dg_last_error(void) { return g_err; }

int dgk_fail(int code, const char* msg) { return fail(code, "%s", msg); }

int dg_validate_desc(const dg_mesh_desc* desc) {
  g_err[0] = 0;
  return validate(desc);
}

// Whether the fused step kernel fits this problem (its three LDS tiles), and
// the automatic choice (measured on MI355X): in 1D always (1.4-1.8x at 4096 to
// 10^6 cells); in 2D while the mesh has at most one 16x16 tile per compute
// unit (1.2-1.5x at 128^2 and 256^2), since with more tiles the recomputed
// rings and the one-workgroup-per-CU occupancy of the fused kernel cost more
// than the launches and HBM passes it saves (0.7-0.86x from 384^2 up).
// Default tile of the per-stage kernel: 256 cells in 1D; in 2D 16x16 unless
// its LDS exceeds the limit, and 8x8 when the mesh has fewer 16x16 tiles
// than compute units (four times the workgroups: 128^2 P2 25.0 -> 20.4 us
// per step for the four-quadrant problem, 20.7 -> 16.2 for Burgers).  The
// KPP flux takes 8x8 (its kernel of 4 to 16 waves per tile) below four
// 16x16 tiles per compute unit: P2 stage 19.6 -> 6.4 us at 128^2, 20.2 ->
// 13.3 at 256^2, 40.6 -> 35.6 at 448^2; at 512^2 both take 42.7 us, and
// beyond the 16x16 kernel is faster (131 against 160 us at 1024^2).
//   Degrees 3 and 4 take 8x8 tiles on every mesh: their registers allow two
// waves per SIMD (p = 3) or one (p = 4), and four independent one-wave
// workgroups per compute unit hide more latency than one four-wave tile
// whose waves wait for each other at its barrier.  Per stage, 16x16 -> 8x8:
// rotation p = 4 59.7 -> 50.7 us at 512^2, 235 -> 179 at 1024^2; p = 3
// 23.6 -> 20.1 at 384^2, 29.1 -> 27.7 at 512^2; Burgers p = 3 111.6 ->
// 106.7 at 1024^2 (the one loss: rotation p = 3 at 1024^2, 104.3 -> 106.2).
void default_tile(dg_ctx* c) {
  if (c->d.dim == 1) {
    c->tx = 256;
    c->ty = 1;
    return;
  }
  c->tx = c->ty = 16;
  const long long t16 = (long long)((c->d.nx + 15) / 16) * ((c->d.ny + 15) / 16);
  if (stage_lds_bytes(2, c->nl, c->d.p, c->d.flux, 16, 16) > (size_t)c->max_lds || t16 < (long long)c->cus ||
      c->d.p >= 3 || (c->d.flux == DG_FLUX_KPP && t16 < 4LL * c->cus))
    c->tx = c->ty = 8;
}

bool fused_fits(const dg_ctx* c) {
  if (c->d.rk_order != 3) return false;            // the fused kernel is the three-stage method
  if (c->d.bc_kind != DG_BC_CONSTANT) return false;  // its rings take the constant exterior state
  if (c->d.flux == DG_FLUX_EULER)                    // the Euler system's own step kernel
    return sizeof(double) * (size_t)dgk::euler_step_lds_doubles(c->d.p) <= (size_t)c->max_lds;
  if (c->d.dim == 2 && c->d.p == 4) return false;  // not built (its 16x16 tiles exceed LDS)
  const int tx = c->d.dim == 1 ? dgk::kStepTile1D : dgk::kStepTile2D;
  const int ty = c->d.dim == 1 ? 1 : dgk::kStepTile2D;  // the larger of the two 2D tiles
  return sizeof(double) * (size_t)dgk::step_lds_doubles(c->d.dim, c->nl, tx, ty) <= (size_t)c->max_lds;
}

long long step_tiles16(const dg_ctx* c) {
  return (long long)((c->d.nx + 15) / 16) * ((c->d.ny + 15) / 16);
}

// The 2D fused step tile.  16x8 tiles (up to two workgroups of four waves per
// compute unit up to P2) spread a small mesh over more compute units and,
// past one 16x16 tile per compute unit, fill the GPU in finer steps; between
// a quarter of and one 16x16 tile per compute unit, 16x16 tiles (one
// workgroup of eight waves per compute unit, fewer ring cells per output
// cell) are faster, and so they are at P3 on larger meshes (94 KB of LDS
// leave one four-wave 16x8 workgroup per compute unit).  Measured per step
// (WENO, rotation / Burgers), 16x16 -> 16x8: P2 128^2 12.0 -> 10.5 / 13.4 ->
// 11.2 us; 256^2 13.8 -> 15.1 / 15.4 -> 16.9; 384^2 35.0 -> 32.1 / 39.9 ->
// 31.6; 512^2 48.2 -> 47.6 / 54.4 -> 47.6; P3 128^2 21.1 -> 16.7 / 22.9 ->
// 18.1; P3 384^2 63.1 -> 79.0 (rotation).  At P1 a 16x16 tile needs only
// 39 KB and is not held to one workgroup per compute unit: 16x8 wins at
// 384^2 (15.9 -> 15.0) but not at 512^2 (20.9 -> 22.2), so P1 keeps 16x16
// from three 16x16 tiles per compute unit on.
void resolve_step_tile(dg_ctx* c) {
  if (c->d.dim != 2 || c->sty_set) return;
  const long long t16 = step_tiles16(c), cus = c->cus;
  const bool beyond = t16 > cus && (c->d.p == 2 || (c->d.p == 1 && t16 <= 3 * cus));
  c->sty = (4 * t16 <= cus || beyond) ? dgk::kStepTile2DHalf : dgk::kStepTile2D;
}

void resolve_fused(dg_ctx* c) {
  resolve_step_tile(c);
  if (c->fused_mode == 0 || !fused_fits(c)) {
    c->fused = false;
    return;
  }
  if (c->fused_mode == 1) {
    c->fused = true;
    return;
  }
  // the KPP flux: the per-stage kernel spreads the sine and cosine of every
  // node over up to 16 waves per tile; the fused kernel evaluates them for
  // each cell on one thread and recomputes the rings (128^2 P2: 84 us per
  // step fused, 18.6 us per-stage)
  if (c->d.flux == DG_FLUX_KPP) {
    c->fused = false;
    return;
  }
  // the Euler system: its fused step up to four 256-cell tiles per compute
  // unit (Sod, per step: 128 cells 11.1 -> 8.2 us, 2^18 cells 40.4 -> 35.6),
  // but not beyond, where its 56 KB of LDS per tile leaves two workgroups
  // per compute unit (2^20 cells: 115 against 124 us)
  if (c->d.flux == DG_FLUX_EULER) {
    c->fused = (c->d.nx + dgk::kEulerStepTile - 1) / dgk::kEulerStepTile <= 4LL * c->cus;
    return;
  }
  // 2D: up to one 16x16 tile per compute unit the per-stage launches are
  // latency-bound and the fused step wins (up to 1.5x); beyond, the
  // per-stage kernel streams, and the fused kernel's recomputed rings cost
  // about what its saved traffic gains.  On the tile resolve_step_tile picks
  // it still wins up to four 16x16 tiles per compute unit for P1 and for P2
  // Burgers (per step, per-stage ->
  // fused: P1 rotation 384^2 16.7 -> 15.0 us, 512^2 22.0 -> 20.9; P2 Burgers
  // 384^2 35.2 -> 31.6, 448^2 42.9 -> 40.6, 512^2 49.7 -> 47.6), but not for
  // P2 rotation (384^2 31.7 -> 32.1, 448^2 38.9 -> 41.8) or P3 (384^2 58.6
  // -> 63.1 on 16x16).
  if (c->d.dim == 1) {
    c->fused = true;
    return;
  }
  const long long t16 = step_tiles16(c), cus = c->cus;
  c->fused = t16 <= cus || (t16 <= 4 * cus && (c->d.p == 1 || (c->d.p == 2 && c->d.flux == DG_FLUX_BURGERS)));
}

int dg_init_mesh(const dg_mesh_desc* desc, dg_ctx** out) {
  g_err[0] = 0;
  if (!out) return fail(DG_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(desc);
  if (rc) return rc;
  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) return fail(DG_ENOMEM, "host allocation failed");
  c->d = *desc;
  if (c->d.dim == 1) c->d.ny = 1;
  c->nl = c->d.dim == 1 ? c->d.p + 1 : (c->d.p + 1) * (c->d.p + 1);
  if (c->d.flux == DG_FLUX_EULER) c->nl *= 3;   // (rho, rho v, rho E) per coefficient
  c->ncells = (long long)c->d.nx * c->d.ny;
  c->h = (c->d.x1 - c->d.x0) / c->d.nx;
  c->stream = static_cast<hipStream_t>(desc->stream);
  c->launch = launcher(c->d.dim, c->d.p);
  int dev = 0, ndev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && desc->device >= 0) {
    e = hipGetDeviceCount(&ndev);
    if (e == hipSuccess && desc->device >= ndev) {
      delete c;
      return fail(DG_EINVAL, "device %d: only %d devices", desc->device, ndev);
    }
    dev = desc->device;
  }
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDevice");
  }
  c->dev = dev;
  DeviceGuard guard(dev);
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
    c->max_lds = lds;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) c->cus = cus;
  default_tile(c);
  resolve_fused(c);
  const size_t bytes = sizeof(double) * (size_t)c->ncells * c->nl;
  if ((e = hipMalloc(&c->U1, bytes)) != hipSuccess || (e = hipMalloc(&c->U2, bytes)) != hipSuccess ||
      (c->d.rk_order == 4 && (e = hipMalloc(&c->U3, bytes)) != hipSuccess)) {
    dg_destroy(c);
    return fail(DG_ENOMEM, "stage buffers (%zu bytes each): %s", bytes, hipGetErrorString(e));
  }
  c->red_len = (size_t)((c->ncells + 255) / 256) + 1;
  if ((e = hipMalloc(&c->red, sizeof(double) * c->red_len)) != hipSuccess) {
    dg_destroy(c);
    return fail(DG_ENOMEM, "reduction buffer: %s", hipGetErrorString(e));
  }
  if (c->d.bc_kind == DG_BC_RIEMANN && (e = hipMalloc(&c->tclock, sizeof(double))) != hipSuccess) {
    dg_destroy(c);
    return fail(DG_ENOMEM, "clock: %s", hipGetErrorString(e));
  }
  if ((e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking)) != hipSuccess) {
    dg_destroy(c);
    return hip_fail(e, "hipStreamCreate");
  }
  *out = c;
  return DG_OK;
}

void dg_destroy(dg_ctx* c) {
  if (!c) return;
  DeviceGuard guard(c->dev);
  if (c->stream || c->U1) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  if (c->U1) (void)hipFree(c->U1);
  if (c->U2) (void)hipFree(c->U2);
  if (c->U3) (void)hipFree(c->U3);
  if (c->tclock) (void)hipFree(c->tclock);
  if (c->red) (void)hipFree(c->red);
  if (c->A1) (void)hipFree(c->A1);
  if (c->A2) (void)hipFree(c->A2);
  if (c->Zmem) (void)hipFree(c->Zmem);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  delete c;
}

int dg_sizes(const dg_ctx* c, int64_t* n_cells, int32_t* n_loc, int32_t* n_proj_nodes) {
  if (!c) return fail(DG_EINVAL, "ctx is NULL");
  if (n_cells) *n_cells = c->ncells;
  if (n_loc) *n_loc = c->nl;
  if (n_proj_nodes) *n_proj_nodes = c->d.dim == 1 ? c->d.p + 2 : (c->d.p + 2) * (c->d.p + 2);
  return DG_OK;
}

int dg_proj_nodes(const dg_ctx* c, double* xy) {
  if (!c || !xy) return fail(DG_EINVAL, "NULL argument");
  const int p = c->d.p, Q = p + 2;
  double gx[8] = {0};
  // projection rule: Q = p + 2 Gauss points (compile-time tables per degree)
  switch (Q) {
    case 3: { constexpr auto g = dgk::make_gauss<3>(); for (int i = 0; i < 3; ++i) gx[i] = g.x[i]; break; }
    case 4: { constexpr auto g = dgk::make_gauss<4>(); for (int i = 0; i < 4; ++i) gx[i] = g.x[i]; break; }
    case 5: { constexpr auto g = dgk::make_gauss<5>(); for (int i = 0; i < 5; ++i) gx[i] = g.x[i]; break; }
    case 6: { constexpr auto g = dgk::make_gauss<6>(); for (int i = 0; i < 6; ++i) gx[i] = g.x[i]; break; }
    default: return fail(DG_EUNSUPPORTED, "projection rule");
  }
  const double hh = 0.5 * c->h;
  const int dim = c->d.dim;
  size_t k = 0;
  for (long long e = 0; e < c->ncells; ++e) {
    const long long ix = e % c->d.nx, iy = e / c->d.nx;
    const double xc = c->d.x0 + (ix + 0.5) * c->h;
    const double yc = c->d.y0 + (iy + 0.5) * c->h;
    if (dim == 1) {
      for (int q = 0; q < Q; ++q) xy[k++] = xc + hh * gx[q];
    } else {
      for (int qy = 0; qy < Q; ++qy)
        for (int qx = 0; qx < Q; ++qx) {
          xy[k++] = xc + hh * gx[qx];
          xy[k++] = yc + hh * gx[qy];
        }
    }
  }
  return DG_OK;
}

int dg_project_ic(dg_ctx* c, const double* u_at_nodes, double* U) {
  if (!c || !u_at_nodes || !U) return fail(DG_EINVAL, "NULL argument");
  DeviceGuard guard(c->dev);
  LaunchReq r{};
  r.kind = dgk::LAUNCH_PROJECT;
  r.src = u_at_nodes;
  r.dst = U;
  // the Euler state projects component by component ([cell][component][...])
  r.ncells = c->ncells * (c->d.flux == DG_FLUX_EULER ? 3 : 1);
  r.stream = c->stream;
  hipError_t e = c->launch(&r);
  return e == hipSuccess ? DG_OK : hip_fail(e, "projection launch");
}

int dg_rhs(dg_ctx* c, const double* U, double* dUdt, double* gamma) {
  if (!c || !U || !dUdt) return fail(DG_EINVAL, "NULL argument");
  DeviceGuard guard(c->dev);
  if (U == dUdt) return fail(DG_EINVAL, "U and dUdt must not overlap");
  const int rc = set_clock(c, c->stream, c->t);
  if (rc) return rc;
  return stage(c, c->stream, U, nullptr, dUdt, gamma, 0.0, 1.0, 0.0, 1, c->tclock ? 0.0 : c->t);
}

int dg_step(dg_ctx* c, double* U, double dt) {
  if (!c || !U) return fail(DG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite and > 0");
  DeviceGuard guard(c->dev);
  int rc = set_clock(c, c->stream, c->t);
  if (rc == DG_OK) rc = rk_steps(c, c->stream, U, dt, 1, c->tclock ? 0.0 : c->t);
  if (rc == DG_OK) c->t += dt;
  if (rc == DG_OK && c->d.check_finite) return finite_or_fail(c, U);
  return rc;
}

int dg_step_static(const dg_mesh_desc* desc, double* U, double dt, double t) {
  g_err[0] = 0;
  int rc = validate(desc);
  if (rc) return rc;
  if (!U) return fail(DG_EINVAL, "U is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(t)) return fail(DG_EINVAL, "t must be finite");
  // the same problem a context would hold, on the stack: no stage buffers of
  // its own, no tables (the kernels' tables are compile-time constants)
  dg_ctx c;
  c.d = *desc;
  if (c.d.dim == 1) c.d.ny = 1;
  c.nl = c.d.dim == 1 ? c.d.p + 1 : (c.d.p + 1) * (c.d.p + 1);
  if (c.d.flux == DG_FLUX_EULER) c.nl *= 3;
  c.ncells = (long long)c.d.nx * c.d.ny;
  const long long ndof = c.ncells * c.nl;
  if (ndof > kStaticStageDoubles)
    return fail(DG_EINVAL, "dg_step_static: %lld coefficients exceed its static stage buffers (%lld)", ndof,
                kStaticStageDoubles);
  c.h = (c.d.x1 - c.d.x0) / c.d.nx;
  c.stream = static_cast<hipStream_t>(desc->stream);
  c.launch = launcher(c.d.dim, c.d.p);
  c.fused = false;   // the per-stage kernels (the fused kernel needs a second state buffer)
  int dev = 0, lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
    c.max_lds = lds;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) c.cus = cus;
  default_tile(&c);
  double* base = nullptr;
  if ((rc = scratch_on_current_device(&base))) return rc;
  c.U1 = base;
  c.U2 = base + kStaticStageDoubles;
  c.U3 = base + 2 * kStaticStageDoubles;
  return ssp_step(&c, c.stream, U, dt, t);
}

int dg_set_time(dg_ctx* c, double t) {
  if (!c) return fail(DG_EINVAL, "ctx is NULL");
  if (!std::isfinite(t)) return fail(DG_EINVAL, "t must be finite");
  c->t = t;
  return DG_OK;
}

int dg_get_time(const dg_ctx* c, double* t) {
  if (!c || !t) return fail(DG_EINVAL, "NULL argument");
  *t = c->t;
  return DG_OK;
}

// The executable graph of `len` SSP-RK3 steps on U with step dt: from the
// cache, else captured on the private capture stream and instantiated.
static int run_graph(dg_ctx* c, double* U, double dt, int len, hipGraphExec_t* out) {
  GraphKey key{U, dt, len};
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    *out = it->second;
    return DG_OK;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  int rc = DG_OK;
  rc = rk_steps(c, c->capture, U, dt, len);
  e = hipStreamEndCapture(c->capture, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  c->graphs[key] = exec;
  *out = exec;
  return DG_OK;
}

static int run_steps(dg_ctx* c, double* U, double dt, int32_t nsteps);

int dg_run(dg_ctx* c, double* U, double dt, int32_t nsteps) {
  if (!c || !U) return fail(DG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return DG_OK;
  DeviceGuard guard(c->dev);
  const int rc = run_steps(c, U, dt, nsteps);
  if (rc == DG_OK && c->d.check_finite) return finite_or_fail(c, U);
  return rc;
}

// dg_run's steps (arguments checked by the caller)
static int run_steps(dg_ctx* c, double* U, double dt, int32_t nsteps) {
  // whole chunks of up to 64 steps replay one captured graph; a remainder
  // replays a second graph of its own length (both cached per (U, dt, length)).
  // Under BC_RIEMANN the stages read their times from the device clock,
  // set before each replay to the time that replay starts from.
  const int chunk = nsteps < 64 ? nsteps : 64;
  const int reps = nsteps / chunk, rest = nsteps % chunk;
  hipGraphExec_t exec = nullptr, tail = nullptr;
  if (c->graphs.size() >= 15) drop_graphs(c);  // bounded cache; room for two entries
  int rc = run_graph(c, U, dt, chunk, &exec);
  if (rc == DG_OK && rest) rc = run_graph(c, U, dt, rest, &tail);
  if (rc) return rc;
  for (int i = 0; i < reps; ++i) {
    if ((rc = set_clock(c, c->stream, c->t + (double)i * chunk * dt))) return rc;
    hipError_t e = hipGraphLaunch(exec, c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  if (rest) {
    if ((rc = set_clock(c, c->stream, c->t + (double)reps * chunk * dt))) return rc;
    hipError_t e = hipGraphLaunch(tail, c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  c->t += nsteps * dt;
  return DG_OK;
}

int dg_run_signature(dg_ctx* c, double* U, double dt, int32_t nsteps, uint32_t* sig) {
  if (!c || !U || !sig) return fail(DG_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if ((c->d.flux != DG_FLUX_LINADV && c->d.flux != DG_FLUX_BURGERS) || c->d.mode == DG_MODE_ZHAO ||
      c->d.bc_kind != DG_BC_CONSTANT || c->d.rk_order != 3)
    return fail(DG_EUNSUPPORTED, "branch records cover what the adjoint covers: linear and Burgers fluxes, "
                                 "modes DG/LO/WENO, the constant exterior state, SSP-RK3");
  DeviceGuard guard(c->dev);
  hipError_t e = hipMemsetAsync(sig, 0, sizeof(uint32_t) * 3 * (size_t)c->ncells, c->stream);
  if (e != hipSuccess) return hip_fail(e, "branch record clear");
  auto record = [&](const double* uin) -> int {
    LaunchReq r{};
    r.kind = dgk::LAUNCH_SIGNATURE;
    r.flux = c->d.flux;
    r.mode = c->d.mode;
    r.args = base_args(c);
    r.args.uin = uin;
    r.sig = sig;
    r.stream = c->stream;
    const hipError_t le = c->launch(&r);
    return le == hipSuccess ? DG_OK : hip_fail(le, "branch record launch");
  };
  const double as[3] = {0.0, 0.75, 1.0 / 3.0}, bs[3] = {1.0, 0.25, 2.0 / 3.0};
  double* in[3] = {U, c->U1, c->U2};
  double* out[3] = {c->U1, c->U2, U};
  for (int s = 0; s < nsteps; ++s)
    for (int k = 0; k < 3; ++k) {
      int rc = record(in[k]);
      if (rc == DG_OK) rc = stage(c, c->stream, in[k], U, out[k], nullptr, as[k], bs[k], dt, 0, c->t);
      if (rc) return rc;
    }
  c->t += nsteps * dt;
  return DG_OK;
}

int dg_stable_dt(dg_ctx* c, const double* U, double cfl, double* dt_host) {
  if (!c || !U || !dt_host) return fail(DG_EINVAL, "NULL argument");
  DeviceGuard guard(c->dev);
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(DG_EINVAL, "cfl must be finite and > 0");
  LaunchReq r{};
  r.kind = dgk::LAUNCH_LAMBDA;
  r.flux = c->d.flux;
  r.args = base_args(c);
  r.src = U;
  r.dst = c->red;
  r.ncells = c->ncells;
  r.stream = c->stream;
  hipError_t e = c->launch(&r);
  if (e != hipSuccess) return hip_fail(e, "lambda launch");
  const size_t nb = (size_t)((c->ncells + 255) / 256);
  std::vector<double> h(nb);
  if ((e = hipMemcpyAsync(h.data(), c->red, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return hip_fail(e, "lambda readback");
  double lam = 0.0;
  for (double v : h) lam = v > lam ? v : lam;
  if (!(lam > 0.0) || !std::isfinite(lam)) return fail(DG_ENONFINITE, "maximal wave speed is %g", lam);
  *dt_host = c->d.cfl_mode == 1 ? cfl * c->h / lam : cfl * c->h / ((2 * c->d.p + 1) * lam);
  return DG_OK;
}

int dg_check_finite(dg_ctx* c, const double* U, int64_t* count) {
  if (!c || !U) return fail(DG_EINVAL, "NULL argument");
  DeviceGuard guard(c->dev);
  const long long n = (long long)c->ncells * c->nl;
  // per-block counts on the device (grid-stride), summed here
  long long nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  if (nb > (long long)c->red_len) nb = (long long)c->red_len;
  hipError_t e = dgk_count_nonfinite(U, n, c->red, (int)nb, c->stream);
  if (e != hipSuccess) return hip_fail(e, "finite-check launch");
  std::vector<double> h((size_t)nb);
  if ((e = hipMemcpyAsync(h.data(), c->red, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, c->stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return hip_fail(e, "finite-check readback");
  double bad = 0.0;
  for (double v : h) bad += v;
  if (count) *count = (int64_t)bad;
  return bad > 0.0 ? fail(DG_ENONFINITE, "%lld non-finite entries", (long long)bad) : DG_OK;
}

}  // extern "C"

namespace {
int finite_or_fail(dg_ctx* c, const double* U) {
  int64_t bad = 0;
  const int rc = dg_check_finite(c, U, &bad);
  if (rc == DG_ENONFINITE) return fail(DG_ENONFINITE, "%lld non-finite entries after the steps", (long long)bad);
  return rc;
}
}  // namespace

extern "C" {

int dg_stream_copy(const double* src, double* dst, int64_t n, void* stream) {
  if (n < 0) return fail(DG_EINVAL, "n must be >= 0");
  if (n > 0 && (!src || !dst)) return fail(DG_EINVAL, "NULL argument");
  const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
  if (n > 0 && s0 < d0 + (uintptr_t)n * sizeof(double) && d0 < s0 + (uintptr_t)n * sizeof(double))
    return fail(DG_EINVAL, "src and dst overlap");
  hipError_t e = dgk_stream_copy(src, dst, (long long)n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "copy launch");
  return DG_OK;
}

int dg_set_tile(dg_ctx* c, int32_t tx, int32_t ty) {
  if (!c) return fail(DG_EINVAL, "ctx is NULL");
  int rc = check_tile(c, tx, ty);
  if (rc) return rc;
  c->tx = tx;
  c->ty = c->d.dim == 2 ? ty : 1;
  drop_graphs(c);
  return DG_OK;
}

int dg_set_fused(dg_ctx* c, int32_t mode) {
  if (!c) return fail(DG_EINVAL, "ctx is NULL");
  if (mode < -1 || mode > 1) return fail(DG_EINVAL, "mode must be -1 (automatic), 0 (off) or 1 (on)");
  if (mode == 1 && c->d.rk_order != 3)
    return fail(DG_EUNSUPPORTED, "the fused step kernel implements the three-stage SSP method only");
  if (mode == 1 && c->d.bc_kind != DG_BC_CONSTANT)
    return fail(DG_EUNSUPPORTED, "the fused step kernel takes the constant exterior state only");
  if (mode == 1 && !fused_fits(c))
    return fail(DG_EUNSUPPORTED, "the fused step kernel's LDS tiles exceed the device limit for this degree");
  c->fused_mode = mode;
  resolve_fused(c);
  drop_graphs(c);
  return DG_OK;
}

int dg_set_step_tile(dg_ctx* c, int32_t tx, int32_t ty) {
  if (!c) return fail(DG_EINVAL, "ctx is NULL");
  if (c->d.dim == 1) {
    if (tx != dgk::kStepTile1D) return fail(DG_EINVAL, "1D step tile must be %d cells (got %d)", dgk::kStepTile1D, tx);
    return DG_OK;
  }
  if (tx != dgk::kStepTile2D || (ty != dgk::kStepTile2D && ty != dgk::kStepTile2DHalf))
    return fail(DG_EINVAL, "2D step tile must be 16x16 or 16x8 (got %dx%d)", tx, ty);
  c->sty = ty;
  c->sty_set = true;
  drop_graphs(c);
  return DG_OK;
}

int dg_get_step_tile(const dg_ctx* c, int32_t* tx, int32_t* ty) {
  if (!c) return fail(DG_EINVAL, "ctx is NULL");
  const bool d1 = c->d.dim == 1;
  if (tx) *tx = d1 ? (c->d.flux == DG_FLUX_EULER ? dgk::kEulerStepTile : dgk::kStepTile1D) : dgk::kStepTile2D;
  if (ty) *ty = d1 ? 1 : c->sty;
  return DG_OK;
}

int dg_get_fused(const dg_ctx* c, int32_t* active) {
  if (!c || !active) return fail(DG_EINVAL, "NULL argument");
  *active = c->fused ? 1 : 0;
  return DG_OK;
}

int dg_get_tile(const dg_ctx* c, int32_t* tx, int32_t* ty) {
  if (!c) return fail(DG_EINVAL, "ctx is NULL");
  if (tx) *tx = c->tx;
  if (ty) *ty = c->ty;
  return DG_OK;
}

int dg_rhs_vjp(dg_ctx* c, const double* U, const double* v, double* out) {
  if (!c || !U || !v || !out) return fail(DG_EINVAL, "NULL argument");
  DeviceGuard guard(c->dev);
  if (out == U || out == v) return fail(DG_EINVAL, "out must not overlap U or v");
  int rc = ensure_adjoint(c);
  if (rc) return rc;
  return adjoint_stage(c, c->stream, U, v, out, 0.0, 1.0, nullptr, 0, nullptr, 0);
}

int dg_step_adjoint(dg_ctx* c, const double* Un, double dt, const double* lam_out, double* lam_in) {
  if (!c || !Un || !lam_out || !lam_in) return fail(DG_EINVAL, "NULL argument");
  DeviceGuard guard(c->dev);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite and > 0");
  if (lam_in == Un) return fail(DG_EINVAL, "lam_in must not overlap Un");
  if (c->d.rk_order != 3) return fail(DG_EUNSUPPORTED, "the step adjoint covers the three-stage SSP method only");
  int rc = ensure_adjoint(c);
  if (rc) return rc;
  return rk3_adjoint(c, c->stream, Un, dt, lam_out, lam_in);
}

int dg_revolve_stats(int32_t nsteps, int32_t nsnaps, int64_t* stats) {
  if (nsteps < 1 || nsnaps < 0 || !stats) return fail(DG_EINVAL, "need nsteps >= 1, nsnaps >= 0, stats");
  auto a = rv_schedule(nsteps, nsnaps);
  const size_t split = rv_split(a);
  int64_t fwd_steps = 0, rec_steps = 0, stores = 0, adj = 0, maxslot = 0;
  int64_t last_adj = nsteps;
  for (size_t i = 0; i < a.size(); ++i) {
    if (a[i].op == RV_ADVANCE) (i < split ? fwd_steps : rec_steps) += a[i].a;
    if (a[i].op == RV_STORE) {
      ++stores;
      maxslot = a[i].a > maxslot ? a[i].a : maxslot;
    }
    if (a[i].op == RV_ADJOINT) {
      if (a[i].a != last_adj - 1) return fail(DG_EINVAL, "internal: adjoint steps out of order");
      last_adj = a[i].a;
      ++adj;
    }
  }
  stats[0] = fwd_steps;   // steps advanced by the forward sweep (before the final step)
  stats[1] = rec_steps;   // steps recomputed during the reverse sweep
  stats[2] = stores;      // checkpoint stores
  stats[3] = adj;         // adjoint steps (== nsteps)
  stats[4] = maxslot;     // highest checkpoint slot used (<= nsnaps)
  stats[5] = (int64_t)a.size();
  return DG_OK;
}


int dg_adjoint_forward(dg_ctx* c, const double* U0, double* UT, double dt, int32_t nsteps, int32_t nsnaps,
                       double* ckpt, double* stages) {
  if (!c || !U0 || !UT || !ckpt) return fail(DG_EINVAL, "NULL argument");
  DeviceGuard guard(c->dev);
  if (c->d.rk_order != 3) return fail(DG_EUNSUPPORTED, "the step adjoint covers the three-stage SSP method only");
  if (c->d.bc_kind != DG_BC_CONSTANT)
    return fail(DG_EUNSUPPORTED, "the adjoint does not cover the exact-solution exterior state");
  if (c->d.flux == DG_FLUX_EULER) return fail(DG_EUNSUPPORTED, "the adjoint does not cover the Euler system");
  if (c->d.mode == DG_MODE_ZHAO) return fail(DG_EUNSUPPORTED, "the adjoint does not cover the ZHAO sensor");
  if (c->d.flux == DG_FLUX_KPP) return fail(DG_EUNSUPPORTED, "the adjoint does not cover the KPP flux");
  if (nsteps < 1 || nsnaps < 0) return fail(DG_EINVAL, "need nsteps >= 1 and nsnaps >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite and > 0");
  const size_t n = (size_t)c->ncells * c->nl;
  double* work = ckpt + (size_t)(nsnaps + 1) * n;
  hipError_t e = hipMemcpyAsync(ckpt, U0, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
  auto a = rv_schedule(nsteps, nsnaps);
  const size_t split = rv_split(a);
  auto S1 = [&](int k) { return stages ? stages + (size_t)(2 * k) * n : nullptr; };
  auto S2 = [&](int k) { return stages ? stages + (size_t)(2 * k + 1) * n : nullptr; };
  int rc = DG_OK;
  int cur = 0;                 // step index of the current state
  const double* state = ckpt;  // where the current state lives (a slot or the work buffer)
  std::vector<int> slot_step(nsnaps + 1, 0);
  for (size_t i = 0; i < split && rc == DG_OK; ++i) {
    if (a[i].op == RV_RESTORE) {
      state = ckpt + (size_t)a[i].a * n;  // read in place; nothing is copied
      cur = slot_step[a[i].a];
    } else if (a[i].op == RV_STORE) {
      double* dst = ckpt + (size_t)a[i].a * n;
      if (state != dst) {
        e = hipMemcpyAsync(dst, state, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
        state = dst;
      }
      slot_step[a[i].a] = cur;
    } else if (a[i].op == RV_ADVANCE) {
      // the last step of an advance that is stored writes straight into its slot
      const bool stored = i + 1 < split && a[i + 1].op == RV_STORE;
      for (int k = 0; k < a[i].a && rc == DG_OK; ++k, ++cur) {
        double* dst = (stored && k == a[i].a - 1) ? ckpt + (size_t)a[i + 1].a * n : work;
        rc = rk3_step_to(c, c->stream, state, dst, dt, S1(cur), S2(cur));
        state = dst;
      }
    }
  }
  if (rc) return rc;
  // the state at nsteps-1 is restored by the first reverse action; reach U_T from it
  const int slot = a[split].a;
  int k0 = 0;
  for (size_t i = split; i < a.size() && a[i].op != RV_ADJOINT; ++i)
    if (a[i].op == RV_ADVANCE) k0 += a[i].a;
  state = ckpt + (size_t)slot * n;
  for (int k = 0; k < k0 + 1 && rc == DG_OK; ++k) {
    const int step = nsteps - 1 - k0 + k;
    rc = rk3_step_to(c, c->stream, state, UT, dt, k == k0 ? S1(step) : nullptr, k == k0 ? S2(step) : nullptr);
    state = UT;
  }
  return rc;
}

int dg_adjoint_backward(dg_ctx* c, double dt, int32_t nsteps, int32_t nsnaps, double* ckpt, const double* stages,
                        double* lam) {
  if (!c || !ckpt || !lam) return fail(DG_EINVAL, "NULL argument");
  DeviceGuard guard(c->dev);
  if (c->d.rk_order != 3) return fail(DG_EUNSUPPORTED, "the step adjoint covers the three-stage SSP method only");
  if (nsteps < 1 || nsnaps < 0) return fail(DG_EINVAL, "need nsteps >= 1 and nsnaps >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite and > 0");
  int rc = ensure_adjoint(c);
  if (rc) return rc;
  const size_t n = (size_t)c->ncells * c->nl;
  double* work = ckpt + (size_t)(nsnaps + 1) * n;
  auto a = rv_schedule(nsteps, nsnaps);
  std::vector<char> have = stages ? rv_stage_steps(a, nsteps, nsnaps) : std::vector<char>(nsteps, 0);
  hipError_t e = hipSuccess;
  const double* state = work;  // where the current state lives (a slot or the work buffer)
  bool zpend = false;          // the next adjoint step's first records are in place
  for (size_t i = rv_split(a); i < a.size() && rc == DG_OK; ++i) {
    switch (a[i].op) {
      case RV_RESTORE:
        state = ckpt + (size_t)a[i].a * n;  // read in place
        break;
      case RV_STORE:
        if (state != ckpt + (size_t)a[i].a * n) {
          e = hipMemcpyAsync(ckpt + (size_t)a[i].a * n, state, n * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream);
          state = ckpt + (size_t)a[i].a * n;
        }
        break;
      case RV_ADVANCE:
        // the first step out of a slot writes into the work buffer
        for (int k = 0; k < a[i].a && rc == DG_OK; ++k) {
          if (state != work) {
            rc = rk3_step_to(c, c->stream, state, work, dt);
            state = work;
          } else {
            rc = rk3_step(c, c->stream, work, dt);
          }
        }
        break;
      case RV_ADJOINT: {
        // lam <- (d step / d U^k)^T lam
        const int k = a[i].a;
        // the stage states of the step reversed next, when kept, let the last
        // launch of this step also start that one
        const double* next_S2 =
            adj_fused(c) && k > 0 && have[k - 1] ? stages + (size_t)(2 * (k - 1) + 1) * n : nullptr;
        if (have[k])
          rc = rk3_adjoint(c, c->stream, state, dt, lam, lam, stages + (size_t)(2 * k) * n,
                           stages + (size_t)(2 * k + 1) * n, zpend, next_S2);
        else
          rc = rk3_adjoint(c, c->stream, state, dt, lam, lam, nullptr, nullptr, zpend, next_S2);
        zpend = next_S2 != nullptr;
        break;
      }
    }
    if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
  }
  return rc;
}

int dg_set_stream(dg_ctx* c, void* stream) {
  if (!c) return fail(DG_EINVAL, "ctx is NULL");
  c->stream = static_cast<hipStream_t>(stream);
  c->d.stream = stream;
  return DG_OK;
}

}  // extern "C"
