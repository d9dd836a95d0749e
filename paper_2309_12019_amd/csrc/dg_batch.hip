// Batched execution of many independent problems (C ABI in include/dgweno.h).
//
// Problems are grouped into kernel classes (dimension, degree, flux, mode).
// One persistent launch per class and RK stage walks that class's tile list
// with a grid stride; a whole run of N steps is one HIP graph whose classes
// form independent chains spread over up to four concurrent branches.  The
// schedule (tile shape, grid size and tile order per class, number of
// branches) is chosen by dg_batch_tune from timed trial launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/dgweno.h"
#include "dg_batch_plan.hpp"
#include "dg_launch.hpp"

using dgk::BatchProblem;
using dgk::BatchStageArgs;
using dgk::BatchTile;
using dgk::LaunchFn;
using dgk::LaunchReq;
using dgk::StageArgs;

extern "C" int dgk_fail(int code, const char* msg);  // dg_api.hip: sets dg_last_error

namespace {

int bfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return dgk_fail(code, buf);
}

LaunchFn launcher(int dim, int p) {
  static const LaunchFn tab[2][4] = {{dgk_launch_1_1, dgk_launch_1_2, dgk_launch_1_3, dgk_launch_1_4},
                                     {dgk_launch_2_1, dgk_launch_2_2, dgk_launch_2_3, dgk_launch_2_4}};
  return tab[dim - 1][p - 1];
}

constexpr int kMaxBranches = 4;

struct Class {
  int dim, p, flux, mode, nl;
  std::vector<int> probs;     // problem indices
  // schedule
  int tx = 0, ty = 1, grid_per_cu = 0, order = 0, branch = 0;  // grid_per_cu 0: one workgroup per tile
  // device tile list for the current schedule, allocated once at creation
  // with room for the longest list any supported tile shape gives
  BatchTile* d_tiles = nullptr;
  long long cap = 0;
  int ntiles = 0;
  double cost_us = 0.0;       // measured per-stage time (tuner)
};

}  // namespace

struct dg_batch {
  std::vector<dg_mesh_desc> d;
  std::vector<dgk::BatchMesh> mesh;  // the plan's view of each problem
  std::vector<long long> off;       // count + 1
  std::vector<StageArgs> args;      // per problem (pointers unset)
  std::vector<Class> cls;
  BatchProblem* d_probs = nullptr;  // per problem
  double* U1 = nullptr;
  double* U2 = nullptr;
  double* dts_dev_unused = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t cap[kMaxBranches] = {};
  hipEvent_t ev[kMaxBranches + 1] = {};
  int branches = 1;
  int cus = 256;
  int max_lds = 65536;
  std::vector<double> dts;          // dts the graph was recorded with
  const double* graph_arena = nullptr;
  int graph_steps = 0;
  hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(dg_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
}

int nl_of(const dg_mesh_desc& d) { return d.dim == 1 ? d.p + 1 : (d.p + 1) * (d.p + 1); }

size_t lds_bytes(int dim, int nl, int flux, int tx, int ty) {
  return sizeof(double) * (size_t)dgk::stage_lds_doubles(dim, nl, flux, tx, dim == 2 ? ty : 1);
}

// Build the tile list of a class for its current schedule and upload it into
// the class's device list (no allocation).  Work already queued on the
// batch's streams may still read the list, so they are drained first.
int build_tiles(dg_batch* b, Class& c) {
  std::vector<BatchTile> all;
  dgk::batch_tile_list(b->mesh, c.probs, c.tx, c.ty, c.order, all);
  if ((long long)all.size() > c.cap) return bfail(DG_EINVAL, "tile list exceeds its capacity");
  hipError_t e = hipStreamSynchronize(b->stream);
  for (int k = 0; k < kMaxBranches && e == hipSuccess; ++k)
    if (b->cap[k]) e = hipStreamSynchronize(b->cap[k]);
  if (e != hipSuccess) return bfail(DG_EDEVICE, "stream synchronisation: %s", hipGetErrorString(e));
  c.ntiles = (int)all.size();
  e = hipMemcpy(c.d_tiles, all.data(), sizeof(BatchTile) * all.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bfail(DG_EDEVICE, "tile list upload: %s", hipGetErrorString(e));
  return DG_OK;
}

int class_grid(const dg_batch* b, const Class& c) { return dgk::batch_grid(c.grid_per_cu, b->cus, c.ntiles); }

// one RK stage of one class: out = a*un + b*(uin + dt*L(uin)) per problem
int class_stage(dg_batch* b, Class& c, hipStream_t st, const double* uin, const double* un, double* out, double a,
                double bb) {
  LaunchReq r{};
  r.kind = dgk::LAUNCH_BATCH;
  r.flux = c.flux;
  r.mode = c.mode;
  r.args.tx = c.tx;
  r.args.ty = c.ty;
  r.ncells = class_grid(b, c);
  r.batch_one = c.grid_per_cu == 0;
  r.stream = st;
  r.batch.probs = b->d_probs;
  r.batch.tiles = c.d_tiles;
  r.batch.ntiles = c.ntiles;
  r.batch.uin = uin;
  r.batch.un = un;
  r.batch.out = out;
  r.batch.a = a;
  r.batch.b = bb;
  hipError_t e = launcher(c.dim, c.p)(&r);
  if (e != hipSuccess) return bfail(DG_EDEVICE, "batch stage launch: %s", hipGetErrorString(e));
  return DG_OK;
}

int class_step(dg_batch* b, Class& c, hipStream_t st, double* U) {
  int rc;
  if ((rc = class_stage(b, c, st, U, U, b->U1, 0.0, 1.0))) return rc;
  if ((rc = class_stage(b, c, st, b->U1, U, b->U2, 0.75, 0.25))) return rc;
  return class_stage(b, c, st, b->U2, U, U, 1.0 / 3.0, 2.0 / 3.0);
}

int upload_problems(dg_batch* b, const double* dts) {
  std::vector<BatchProblem> h(b->d.size());
  for (size_t i = 0; i < h.size(); ++i) {
    h[i].off = b->off[i];
    h[i].args = b->args[i];
    h[i].args.dt = dts ? dts[i] : 0.0;
  }
  hipError_t e = hipMemcpy(b->d_probs, h.data(), sizeof(BatchProblem) * h.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bfail(DG_EDEVICE, "problem table upload: %s", hipGetErrorString(e));
  return DG_OK;
}

StageArgs args_of(const dg_mesh_desc& d) {
  StageArgs A{};
  A.nx = d.nx;
  A.ny = d.dim == 2 ? d.ny : 1;
  A.per_x = d.periodic_x != 0;
  A.per_y = d.dim == 2 && d.periodic_y != 0;
  A.h = (d.x1 - d.x0) / d.nx;
  A.g2h = 2.0 / A.h;
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
  return A;
}

// assign classes to branches: longest measured (or estimated) cost first onto
// the least loaded branch
void assign_branches(dg_batch* b) {
  std::vector<int> idx(b->cls.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return b->cls[x].cost_us > b->cls[y].cost_us; });
  std::vector<double> load(b->branches, 0.0);
  for (int i : idx) {
    int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->cls[i].branch = k;
    load[k] += b->cls[i].cost_us;
  }
}

}  // namespace

extern "C" {

int dg_batch_create(const dg_mesh_desc* descs, int32_t count, dg_batch** out) {
  if (!out) return bfail(DG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs || count < 1) return bfail(DG_EINVAL, "need at least one descriptor");
  // validate each problem through the single-problem path (host checks only)
  for (int i = 0; i < count; ++i) {
    dg_mesh_desc d = descs[i];
    int rc = dg_validate_desc(&d);
    if (rc) return rc;
    if (d.rk_order != 3) return bfail(DG_EUNSUPPORTED, "problem %d: batched runs use the three-stage SSP method only", i);
    if (d.bc_kind != DG_BC_CONSTANT)
      return bfail(DG_EUNSUPPORTED, "problem %d: batched runs take the constant exterior state only", i);
    if (d.flux == DG_FLUX_EULER) return bfail(DG_EUNSUPPORTED, "problem %d: batched runs take scalar states only", i);
  }
  dg_batch* b = new (std::nothrow) dg_batch();
  if (!b) return bfail(DG_ENOMEM, "host allocation failed");
  b->d.assign(descs, descs + count);
  b->stream = static_cast<hipStream_t>(descs[0].stream);
  for (int i = 0; i < count; ++i) {
    dg_mesh_desc& d = b->d[i];
    if (d.dim == 1) d.ny = 1;
    b->mesh.push_back(dgk::BatchMesh{d.dim, d.nx, d.ny, d.p, d.flux, d.mode});
    b->args.push_back(args_of(d));
  }
  b->off = dgk::batch_offsets(b->mesh);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) == hipSuccess) {
      b->cus = pr.multiProcessorCount;
      b->max_lds = (int)pr.sharedMemPerBlock;
    }
  }
  // classes
  for (const auto& probs : dgk::batch_classes(b->mesh)) {
    const dg_mesh_desc& d = b->d[probs[0]];
    Class c;
    c.dim = d.dim;
    c.p = d.p;
    c.flux = d.flux;
    c.mode = d.mode;
    c.nl = nl_of(d);
    c.tx = d.dim == 1 ? 256 : 16;
    c.ty = d.dim == 1 ? 1 : 16;
    if (lds_bytes(c.dim, c.nl, c.flux, c.tx, c.ty) > (size_t)b->max_lds) c.tx = c.ty = 8;
    c.probs = probs;
    c.cap = dgk::batch_tile_capacity(b->mesh, probs);
    b->cls.push_back(c);
  }
  const size_t total = (size_t)b->off[count];
  if ((e = hipMalloc(&b->U1, total * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&b->U2, total * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&b->d_probs, sizeof(BatchProblem) * count)) != hipSuccess) {
    dg_batch_destroy(b);
    return bfail(DG_ENOMEM, "batch buffers: %s", hipGetErrorString(e));
  }
  for (auto& c : b->cls) {
    if ((e = hipMalloc(&c.d_tiles, sizeof(BatchTile) * (size_t)c.cap)) != hipSuccess) {
      dg_batch_destroy(b);
      return bfail(DG_ENOMEM, "tile lists: %s", hipGetErrorString(e));
    }
  }
  for (int k = 0; k < kMaxBranches; ++k) {
    if ((e = hipStreamCreateWithFlags(&b->cap[k], hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming)) != hipSuccess) {
      dg_batch_destroy(b);
      return bfail(DG_EDEVICE, "streams: %s", hipGetErrorString(e));
    }
  }
  if ((e = hipEventCreateWithFlags(&b->ev[kMaxBranches], hipEventDisableTiming)) != hipSuccess) {
    dg_batch_destroy(b);
    return bfail(DG_EDEVICE, "events: %s", hipGetErrorString(e));
  }
  for (auto& c : b->cls) {
    // estimated cost for the initial branch assignment: DOFs of the class
    for (int i : c.probs) c.cost_us += (double)(b->off[i + 1] - b->off[i]);
    int rc = build_tiles(b, c);
    if (rc) {
      dg_batch_destroy(b);
      return rc;
    }
  }
  b->branches = std::min<int>(kMaxBranches, (int)b->cls.size());
  assign_branches(b);
  *out = b;
  return DG_OK;
}

void dg_batch_destroy(dg_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (auto& c : b->cls)
    if (c.d_tiles) (void)hipFree(c.d_tiles);
  if (b->U1) (void)hipFree(b->U1);
  if (b->U2) (void)hipFree(b->U2);
  if (b->d_probs) (void)hipFree(b->d_probs);
  for (int k = 0; k < kMaxBranches; ++k) {
    if (b->cap[k]) (void)hipStreamDestroy(b->cap[k]);
    if (b->ev[k]) (void)hipEventDestroy(b->ev[k]);
  }
  if (b->ev[kMaxBranches]) (void)hipEventDestroy(b->ev[kMaxBranches]);
  delete b;
}

int dg_batch_layout(const dg_batch* b, int64_t* offsets, int64_t* total) {
  if (!b) return bfail(DG_EINVAL, "batch is NULL");
  if (offsets)
    for (size_t i = 0; i < b->off.size(); ++i) offsets[i] = b->off[i];
  if (total) *total = b->off.back();
  return DG_OK;
}

int dg_batch_num_classes(const dg_batch* b, int32_t* n) {
  if (!b || !n) return bfail(DG_EINVAL, "NULL argument");
  *n = (int32_t)b->cls.size();
  return DG_OK;
}

int dg_batch_get_schedule(const dg_batch* b, int32_t cls, int32_t* info) {
  if (!b || !info) return bfail(DG_EINVAL, "NULL argument");
  if (cls < 0 || cls >= (int)b->cls.size()) return bfail(DG_EINVAL, "class %d out of range", cls);
  const Class& c = b->cls[cls];
  const int32_t v[10] = {c.dim, c.p, c.flux, c.mode, (int32_t)c.probs.size(), c.tx, c.ty, c.grid_per_cu, c.order,
                         c.branch};
  std::memcpy(info, v, sizeof(v));
  return DG_OK;
}

int dg_batch_set_schedule(dg_batch* b, int32_t cls, int32_t tx, int32_t ty, int32_t grid_per_cu, int32_t order) {
  if (!b) return bfail(DG_EINVAL, "batch is NULL");
  if (cls < 0 || cls >= (int)b->cls.size()) return bfail(DG_EINVAL, "class %d out of range", cls);
  Class& c = b->cls[cls];
  bool ok = false;
  if (c.dim == 1) {
    for (int t : dgk::kTiles1D) ok |= tx == t;
    ty = 1;
  } else {
    for (auto& t : dgk::kTiles2D) ok |= tx == t[0] && ty == t[1];
  }
  if (!ok) return bfail(DG_EINVAL, "unsupported tile %dx%d", tx, ty);
  if (lds_bytes(c.dim, c.nl, c.flux, tx, ty) > (size_t)b->max_lds) return bfail(DG_EUNSUPPORTED, "tile exceeds LDS");
  if (grid_per_cu < 0 || grid_per_cu > 64)
    return bfail(DG_EINVAL, "grid_per_cu must be in 0..64 (0: one workgroup per tile)");
  if (order < 0 || order > 2) return bfail(DG_EINVAL, "order must be 0, 1 or 2");
  c.tx = tx;
  c.ty = ty;
  c.grid_per_cu = grid_per_cu;
  c.order = order;
  drop_graph(b);
  return build_tiles(b, c);
}

int dg_batch_set_branches(dg_batch* b, int32_t branches) {
  if (!b) return bfail(DG_EINVAL, "batch is NULL");
  if (branches < 1 || branches > kMaxBranches) return bfail(DG_EINVAL, "branches must be in 1..%d", kMaxBranches);
  b->branches = branches;
  assign_branches(b);
  drop_graph(b);
  return DG_OK;
}

int dg_batch_run(dg_batch* b, double* arena, const double* dts, int32_t nsteps) {
  if (!b || !arena || !dts) return bfail(DG_EINVAL, "NULL argument");
  if (nsteps < 0) return bfail(DG_EINVAL, "nsteps must be >= 0");
  for (size_t i = 0; i < b->d.size(); ++i)
    if (!(dts[i] > 0.0) || !std::isfinite(dts[i])) return bfail(DG_EINVAL, "dt of problem %zu is invalid", i);
  if (nsteps == 0) return DG_OK;
  const bool same = b->exec && b->graph_arena == arena && b->graph_steps == nsteps &&
                    std::equal(b->dts.begin(), b->dts.end(), dts);
  if (!same) {
    drop_graph(b);
    // the problem table carries dt; upload before recording (the graph reads it)
    (void)hipStreamSynchronize(b->stream);
    int rc = upload_problems(b, dts);
    if (rc) return rc;
    hipError_t e = hipStreamBeginCapture(b->cap[0], hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(DG_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    // fork the other branches off the origin stream
    (void)hipEventRecord(b->ev[kMaxBranches], b->cap[0]);
    for (int k = 1; k < b->branches; ++k) (void)hipStreamWaitEvent(b->cap[k], b->ev[kMaxBranches], 0);
    rc = DG_OK;
    for (int s = 0; s < nsteps && rc == DG_OK; ++s)
      for (auto& c : b->cls) {
        rc = class_step(b, c, b->cap[c.branch], arena);
        if (rc) break;
      }
    // join
    for (int k = 1; k < b->branches; ++k) {
      (void)hipEventRecord(b->ev[k], b->cap[k]);
      (void)hipStreamWaitEvent(b->cap[0], b->ev[k], 0);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap[0], &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return bfail(DG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return bfail(DG_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    b->graph_arena = arena;
    b->graph_steps = nsteps;
    b->dts.assign(dts, dts + b->d.size());
  }
  hipError_t e = hipGraphLaunch(b->exec, b->stream);
  if (e != hipSuccess) return bfail(DG_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
  return DG_OK;
}

// Reference schedule for comparisons: the plain per-problem stage kernel, one
// launch per problem per RK stage, problems in order, on the batch stream, no
// graph.  Same per-cell arithmetic as dg_batch_run.
int dg_batch_run_sequential(dg_batch* b, double* arena, const double* dts, int32_t nsteps) {
  if (!b || !arena || !dts) return bfail(DG_EINVAL, "NULL argument");
  if (nsteps < 0) return bfail(DG_EINVAL, "nsteps must be >= 0");
  for (size_t i = 0; i < b->d.size(); ++i)
    if (!(dts[i] > 0.0) || !std::isfinite(dts[i])) return bfail(DG_EINVAL, "dt of problem %zu is invalid", i);
  const double as[3] = {0.0, 0.75, 1.0 / 3.0}, bs[3] = {1.0, 0.25, 2.0 / 3.0};
  for (int s = 0; s < nsteps; ++s)
    for (size_t i = 0; i < b->d.size(); ++i) {
      const dg_mesh_desc& d = b->d[i];
      const long long off = b->off[i];
      double* U = arena + off;
      double* U1 = b->U1 + off;
      double* U2 = b->U2 + off;
      const double* in[3] = {U, U1, U2};
      double* out[3] = {U1, U2, U};
      for (int k = 0; k < 3; ++k) {
        LaunchReq r{};
        r.kind = dgk::LAUNCH_STAGE;
        r.flux = d.flux;
        r.mode = d.mode;
        r.args = b->args[i];
        r.args.tx = d.dim == 1 ? 256 : 16;
        r.args.ty = d.dim == 1 ? 1 : 16;
        if (lds_bytes(d.dim, nl_of(d), d.flux, r.args.tx, r.args.ty) > (size_t)b->max_lds) r.args.tx = r.args.ty = 8;
        r.args.uin = in[k];
        r.args.un = U;
        r.args.out = out[k];
        r.args.a = as[k];
        r.args.b = bs[k];
        r.args.dt = dts[i];
        r.stream = b->stream;
        hipError_t e = launcher(d.dim, d.p)(&r);
        if (e != hipSuccess) return bfail(DG_EDEVICE, "stage launch: %s", hipGetErrorString(e));
      }
    }
  return DG_OK;
}

// Autotuner.  For every class: time its stage-1 launch (reads the arena,
// writes the internal stage buffer, so the state is untouched) for every tile
// shape, persistent grid size and tile order, keep the fastest; then assign
// classes to branches by their measured cost and time whole steps for 1..4
// branches, keeping the fastest.  Synchronous.  `report` (may be NULL)
// receives a text summary.
int dg_batch_tune(dg_batch* b, double* arena, const double* dts, int32_t reps, char* report, int32_t report_len) {
  if (!b || !arena || !dts) return bfail(DG_EINVAL, "NULL argument");
  if (reps < 1) return bfail(DG_EINVAL, "reps must be >= 1");
  int rc = upload_problems(b, dts);
  if (rc) return rc;
  drop_graph(b);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  std::string rep;
  hipStream_t st = b->cap[0];
  for (size_t ci = 0; ci < b->cls.size(); ++ci) {
    Class& c = b->cls[ci];
    std::vector<std::pair<int, int>> tiles;
    if (c.dim == 1)
      for (int t : dgk::kTiles1D) tiles.push_back({t, 1});
    else
      for (auto& t : dgk::kTiles2D) tiles.push_back({t[0], t[1]});
    float best = 1e30f;
    int bt = c.tx, bty = c.ty, bg = c.grid_per_cu, bo = c.order;
    for (auto& tt : tiles) {
      if (lds_bytes(c.dim, c.nl, c.flux, tt.first, tt.second) > (size_t)b->max_lds) continue;
      for (int order : {0, 2}) {
        c.tx = tt.first;
        c.ty = tt.second;
        c.order = order;
        if ((rc = build_tiles(b, c))) return rc;
        for (int g : {0, 1, 2, 4, 8}) {
          c.grid_per_cu = g;
          if ((rc = class_stage(b, c, st, arena, arena, b->U1, 0.0, 1.0))) return rc;  // warm-up
          (void)hipEventRecord(e0, st);
          for (int r = 0; r < reps; ++r)
            if ((rc = class_stage(b, c, st, arena, arena, b->U1, 0.0, 1.0))) return rc;
          (void)hipEventRecord(e1, st);
          (void)hipEventSynchronize(e1);
          float ms = 0;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (ms < best) {
            best = ms;
            bt = tt.first;
            bty = tt.second;
            bg = g;
            bo = order;
          }
        }
      }
    }
    c.tx = bt;
    c.ty = bty;
    c.grid_per_cu = bg;
    c.order = bo;
    c.cost_us = 1e3 * best / reps;
    if ((rc = build_tiles(b, c))) return rc;
    char line[200];
    snprintf(line, sizeof(line), "class %zu (dim %d p %d flux %d, %zu problems): tile %dx%d grid %dx%d order %d: %.1f us\n",
             ci, c.dim, c.p, c.flux, c.probs.size(), c.tx, c.ty, c.grid_per_cu, b->cus, c.order, c.cost_us);
    rep += line;
  }
  // branches: time 2 full steps (on the internal buffers: stage 1 from the
  // arena into U1, stages 2-3 on copies) for each branch count
  int bestb = 1;
  float bestt = 1e30f;
  for (int nb = 1; nb <= std::min<int>(kMaxBranches, (int)b->cls.size()); ++nb) {
    b->branches = nb;
    assign_branches(b);
    (void)hipStreamSynchronize(st);
    (void)hipEventRecord(b->ev[kMaxBranches], st);
    for (int k = 1; k < nb; ++k) (void)hipStreamWaitEvent(b->cap[k], b->ev[kMaxBranches], 0);
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r)
      for (auto& c : b->cls)
        if ((rc = class_stage(b, c, b->cap[c.branch], arena, arena, b->U1, 0.0, 1.0))) return rc;
    for (int k = 1; k < nb; ++k) {
      (void)hipEventRecord(b->ev[k], b->cap[k]);
      (void)hipStreamWaitEvent(st, b->ev[k], 0);
    }
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    char line[120];
    snprintf(line, sizeof(line), "branches %d: %.1f us per stage\n", nb, 1e3 * ms / reps);
    rep += line;
    if (ms < bestt * 0.97f) {
      bestt = ms;
      bestb = nb;
    }
  }
  b->branches = bestb;
  assign_branches(b);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (report && report_len > 0) {
    std::strncpy(report, rep.c_str(), (size_t)report_len - 1);
    report[report_len - 1] = 0;
  }
  return DG_OK;
}

}  // extern "C"
