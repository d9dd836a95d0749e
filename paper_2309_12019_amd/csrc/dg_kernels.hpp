// Device code of the dissipative-WENO RKDG scheme: the per-stage kernel, the
// fused SSP-RK3 step kernel, the batched stage kernel and the projection and
// wave-speed kernels.
//
// One thread owns one cell.  A workgroup owns a tile of tx x ty cells; each
// thread loads its own cell's coefficients into registers (cell-major in HBM)
// and publishes them into a coefficient-major LDS tile (lanes reading one
// coefficient of consecutive cells hit consecutive banks), the first threads
// load the one-cell face halo, and each thread evaluates for its cell
//   * the HWENO reconstruction and smoothness sensor gamma_e (Sec. 4),
//   * the volume integral of eq. (weak2) by sum factorisation,
//   * the four (two in 1D) face integrals with the LLF flux (Sec. 2),
//   * lambda_e, nu_e = lambda_e h / (2p) and the dissipation of eq. (astab),
//   * the inverse of the (diagonal) mass matrix,
// and writes either dU/dt or the SSP-RK3 stage combination (eq. ssp)
//   out = a U^n + b (U^(k-1) + dt dU/dt)
// straight to HBM.  The fused step kernel runs the three stages of a step on
// shrinking rings of a larger tile held in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "dg_tables.hpp"

namespace dgk {

enum { FLUX_LINADV = 0, FLUX_BURGERS = 1, FLUX_KPP = 2, FLUX_EULER = 3 };  // KPP: 2D; EULER: 1D system
enum { MODE_DG = 0, MODE_LO = 1, MODE_WENO = 2, MODE_ZHAO = 3 };
// exterior state at non-periodic faces: the constant bc, or (2D Burgers only)
// the exact solution of the four-quadrant problem of Sec. 5.4 at time t
enum { BC_CONSTANT = 0, BC_RIEMANN = 1 };

struct StageArgs {
  const double* uin;  // operator input U^(k-1), [cells][NL]
  const double* un;   // U^n for the RK combination (unused when a == 0)
  double* out;        // [cells][NL]
  double* gamma;      // optional [cells]
  double a, b, dt;    // out = a U^n + b (U^(k-1) + dt L); rhs_only: out = L
  int rhs_only;
  int nx, ny;         // ny = 1 in 1D
  int per_x, per_y;
  double h, x0, y0;
  double vx, vy, omega, cx, cy;  // LINADV velocity; BURGERS direction (vx, vy)
  double anorm;                  // ||(vx, vy)||_2 (BURGERS wave speed factor)
  double bc;                     // exterior state at non-periodic faces (BC_CONSTANT)
  double t;                      // time of uin (the exterior state of BC_RIEMANN)
  int bc_kind;                   // BC_CONSTANT or BC_RIEMANN
  double q, bthr, wnb, eps, wpow, lam_over;
  double theta;                  // exponent of the Zhao et al. sensor (MODE_ZHAO)
  int tx, ty;                    // tile (one of the compiled shapes; ty = 1 in 1D)
  const double* tclock;          // BC_RIEMANN: if set, uin's time is *tclock + t (t an offset)
  double g2h;                    // 2 / h, formed on the host (the same correctly rounded quotient)
  double lfac[25];               // (2/h) minv_a minv_b per coefficient a + (p+1) b (1D: (2/h) minv_a),
                                 // formed on the host in the same order (stage_lfac)
};

// The factors of the mass inverse and 2/h that turn a cell's weak-form sums
// into dU/dt, per coefficient, in the order the kernels multiplied them.
template <int P>
inline void stage_lfac_p(int dim, double g2h, double* lf) {
  constexpr DegTab<P> t = make_deg<P>();
  constexpr int N = P + 1;
  for (int bb = 0; bb < (dim == 2 ? N : 1); ++bb)
    for (int a = 0; a < N; ++a) lf[a + N * bb] = dim == 2 ? (g2h * t.minv[a]) * t.minv[bb] : g2h * t.minv[a];
}
inline void stage_lfac(int dim, int p, double g2h, double* lf) {
  switch (p) {
    case 1: stage_lfac_p<1>(dim, g2h, lf); break;
    case 2: stage_lfac_p<2>(dim, g2h, lf); break;
    case 3: stage_lfac_p<3>(dim, g2h, lf); break;
    default: stage_lfac_p<4>(dim, g2h, lf); break;
  }
}

// Tile geometry: TX x TY cells per workgroup (TY = 1 in 1D) plus a one-cell
// face halo.  LDS holds the tile coefficient-major: plane j (one per basis
// function) stores coefficient j of every slot; the plane stride is odd so
// lanes reading consecutive slots of one plane hit consecutive banks.
template <int DIM, int TX, int TY>
struct TileGeom {
  static constexpr int W = TX + 2;                  // slots per row
  static constexpr int H = DIM == 2 ? TY + 2 : 1;   // slot rows
  static constexpr int NS = W * H;
  static constexpr int S = NS | 1;                  // plane stride (doubles)
  static constexpr int NT = DIM == 2 ? TX * TY : TX;
};

// supported tiles (all multiples of 64 cells)
constexpr int kTiles1D[2] = {256, 64};
constexpr int kTiles2D[2][2] = {{16, 16}, {8, 8}};

__host__ __device__ inline int tile_lds_doubles(int dim, int nl, int tx, int ty) {
  const int ns = dim == 1 ? tx + 2 : (tx + 2) * (ty + 2);
  return nl * (ns | 1);   // the tile with its face halo
}

// Shared faces.  In a 2D tile of at least four waves the per-stage and
// batched kernels can evaluate the flux moments of every face of the tile
// once, in a face phase, and keep them in LDS after the tile: the x faces
// ((TX + 1) per row, row-major) in N planes of stride XS, then the y faces
// (TX per row of faces, TY + 1 rows) in N planes of stride YS.  A cell's own
// four face evaluations compute each interior face twice.  The face phase
// costs a second barrier and LDS; it pays where the flux is expensive (the
// Burgers and KPP fluxes) at p = 2, and is used there only.  (A one-wave 8 x 8
// tile has as many face rounds either way.)
__host__ __device__ constexpr bool shares_faces(int dim, int p, int flux, int tx, int ty) {
  return dim == 2 && p == 2 && (flux == FLUX_BURGERS || flux == FLUX_KPP) && tx * ty >= 256;
}

template <int TX, int TY>
struct FaceGeom {
  static constexpr int NXF = (TX + 1) * TY;  // x faces
  static constexpr int NYF = TX * (TY + 1);  // y faces
  static constexpr int XS = NXF | 1, YS = NYF | 1;
};

__host__ __device__ inline int face_lds_doubles(int n, int tx, int ty) {
  return n * ((((tx + 1) * ty) | 1) + ((tx * (ty + 1)) | 1));
}

// LDS of the per-stage and batched stage kernels: the tile, and the shared
// faces where the tile has them (nl = (p + 1)^dim)
__host__ __device__ inline int stage_lds_doubles(int dim, int nl, int flux, int tx, int ty) {
  int n = 1;
  while ((dim == 2 ? n * n : n) < nl) ++n;
  const int t = tile_lds_doubles(dim, nl, tx, ty);
  return shares_faces(dim, n - 1, flux, tx, ty) ? t + face_lds_doubles(n, tx, ty) : t;
}

// The face thread t of a tile evaluates in round k (0..3) of the face phase:
// round 0 x face t, round 1 y face t (every thread), round 2 x face NT + lane
// on wave `rot` only, round 3 y face NT + lane on wave (rot + NW / 2) mod NW
// only (NW waves of 64 lanes, NT = TX TY threads): the faces left over after
// a full round of the workgroup (a column of x faces, a row of y faces).
// Returns false where the thread has no face in that round; axis = k & 1.
template <int TX, int TY>
__host__ __device__ inline bool face_task(int t, int rot, int k, int& e) {
  constexpr int NT = TX * TY, NW = NT / 64;
  if (k < 2) {
    e = t;
    return true;
  }
  e = NT + (t & 63);
  const int w = t >> 6;
  if (k == 2) return w == rot && e < (TX + 1) * TY;
  return w == (rot + NW / 2) % NW && e < TX * (TY + 1);
}

// Face e of a tile's shared faces: axis 0 the x faces (e < (TX + 1) TY), 1
// the y faces (e < TX (TY + 1)).  Returns the LDS slot of the cell below the
// face (the cell above is slot + 1 for x faces, slot + W for y faces) and in
// (gx, gy) that cell's mesh coordinates before wrapping.  The faces of tile
// cell (lx, ly): x faces ly (TX + 1) + lx (-x) and the next (+x), y faces
// ly TX + lx (-y) and that + TX (+y).
template <int TX, int TY>
__host__ __device__ inline int face_slot(int axis, int e, int ix0, int iy0, int& gx, int& gy) {
  constexpr int W = TX + 2;
  if (axis == 0) {
    const int fx = e % (TX + 1), ly = e / (TX + 1);
    gx = ix0 - 1 + fx;
    gy = iy0 + ly;
    return (ly + 1) * W + fx;
  }
  const int lx = e % TX, fy = e / TX;
  gx = ix0 + lx;
  gy = iy0 - 1 + fy;
  return fy * W + lx + 1;
}

// Workgroup barrier around LDS traffic between lanes.  For workgroups of a
// single wave (8x8 and 64-cell tiles) the compiler removes s_barrier, and with
// it the ordering of one lane's LDS accesses relative to another lane's: it
// may move a lane's LDS reads of its neighbours' slots above the writes of
// those slots, which it sees as different addresses.  The asm statement is a
// full compiler memory barrier and waits for the wave's LDS operations, so
// LDS writes before it and reads after it keep their order in every case.
__device__ inline void tile_barrier() {
  __syncthreads();
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// x, hidden from the optimiser: a value computed in two phases of a kernel
// would otherwise be shared between them and held in registers in between
__device__ inline int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// XCD-aware tile order.  The dispatcher hands workgroup k (x fastest) to
// XCD k mod 8, and each XCD has its own L2.  Workgroup k takes tile
// xcd_tile(k, g) of the g tiles (row-major), a bijection under which every
// XCD works through one contiguous band of tiles in order: the halos a tile
// shares with its neighbours are then read on one XCD and hit its L2 instead
// of being fetched again by another.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_tile(int k, int g) {
  const int q = g / kXcds, r = g % kXcds, x = k % kXcds, i = k / kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// x mod n for x in [-1, n + tile]: cheap for the common single wrap
__host__ __device__ inline int wrap_index(int x, int n) {
  if (x < 0) return x + n;
  while (x >= n) x -= n;
  return x;
}

// 1/x to near full precision: hardware estimate and two Newton steps
__device__ inline double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// general powers (cold paths: exponents other than the defaults)
__device__ __noinline__ double pow_cold(double x, double y) { return pow(x, y); }
// sin and cos of the KPP flux, out of line: inlined at every quadrature node
// their argument reduction would set the register count of the whole kernel.
// sincos_inl is the same routine inlined, for code that holds few registers
// around the call (the node tasks of kpp_split_tile): the same results.
__device__ inline void sincos_inl(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __noinline__ void sincos_cold(double x, double* s, double* c) { sincos_inl(x, s, c); }

// sqrt(x) for x > 0: hardware estimate and one Newton correction
__device__ inline double sqrt_pos(double x) {
  const double s = __builtin_amdgcn_sqrt(x);
  const double e = fma(-s, s, x);
  return fma(0.5 * rcp(s), e, s);
}

// Per-cell arithmetic.  `b` points at this cell's slot in LDS plane 0;
// coefficient j of the cell sits at b[j*S], of its face neighbour f at
// b[j*S + off(f)] with off = -1, +1, -W, +W (faces -x, +x, -y, +y).
// Non-periodic boundary slots hold the constant exterior state, so the
// face traces need no special case.
// Exact solution in R^2 of the four-quadrant Burgers problem of Sec. 5.4,
// u_t + div((1, 1) u^2 / 2) = 0 with -0.2 | -1 above 0.5 | 0.8 (split at
// x = y = 1/2), at (x, y) and time t > 0.  Along each line c = x - y the
// problem is one-dimensional (flux u^2 in x + y); its waves, located by
// z = 2x - 1 for c >= 0 and by w = 2y - 1 for c < 0:
//   c >= 0: a fan 0.5 -> 0.8 over t <= z <= 1.6t and a shock 0.8 | -1 at
//     z = 2c - 0.2t; the shock reaches the fan's head at t = 10c/9, crosses
//     the fan along z = 3.6 sqrt(10c/9) sqrt(t) - 2t, leaves it at t = 1.6c
//     and goes on as 0.5 | -1 at z = 2.4c - 0.5t;
//   c < 0 (d = -c): shocks 0.5 | -0.2 at w = 0.3t and -0.2 | -1 at
//     w = 2d - 1.2t, which merge at t = 4d/3 into 0.5 | -1 at
//     w = 16d/15 - 0.5t.
__device__ inline double riemann_exact(double x, double y, double t) {
  const double c = x - y;
  if (c >= 0.0) {
    const double z = 2.0 * x - 1.0, t1 = c * (10.0 / 9.0), t2 = 1.6 * c;
    if (t <= t1) {
      if (z <= t) return 0.5;
      if (z < 1.6 * t) return z / (2.0 * t);
      return z < 2.0 * c - 0.2 * t ? 0.8 : -1.0;
    }
    if (t <= t2) {
      if (z <= t) return 0.5;
      return z < 3.6 * sqrt(t1) * sqrt(t) - 2.0 * t ? z / (2.0 * t) : -1.0;
    }
    return z < 2.4 * c - 0.5 * t ? 0.5 : -1.0;
  }
  const double d = -c, w = 2.0 * y - 1.0;
  if (t <= d * (4.0 / 3.0)) {
    if (w < 0.3 * t) return 0.5;
    return w < 2.0 * d - 1.2 * t ? -0.2 : -1.0;
  }
  return w < d * (16.0 / 15.0) - 0.5 * t ? 0.5 : -1.0;
}

template <int DIM, int P, int FLUX, int MODE, int S, int W>
struct Cell {
  using TB = Tables<DIM, P, FLUX>;
  static constexpr int N = P + 1;
  static constexpr int NL = TB::NL;
  static constexpr int Q = TB::Q;
  static constexpr int NF = 2 * DIM;

  __device__ static constexpr int off(int f) { return f == 0 ? -1 : f == 1 ? 1 : f == 2 ? -W : W; }

  // BC_RIEMANN exterior slots: a slot outside one boundary holds, in planes
  // 0..Q-1, the exact solution at the Q Gauss points of the one face that
  // reads it (node order of the face loop) at uin's time (A.t, or *A.tclock
  // + A.t); a slot outside two boundaries (used by no face) holds zeros;
  // slots inside are left alone.
  __device__ static inline void riemann_slot(const StageArgs& A, int gx, int gy, double (&v)[NL]) {
    static_assert(Q <= NL, "the face nodes must fit the slot's planes");
    const bool ox = (unsigned)gx >= (unsigned)A.nx, oy = (unsigned)gy >= (unsigned)A.ny;
    if (!ox && !oy) return;
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = 0.0;
    if (ox && oy) return;
    const double t = A.tclock ? *A.tclock + A.t : A.t;
    const double hh = 0.5 * A.h;
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      double x, y;
      if (ox) {
        x = gx < 0 ? A.x0 : A.x0 + A.nx * A.h;
        y = fma(hh, TB::nd.x[r], A.y0 + (gy + 0.5) * A.h);
      } else {
        y = gy < 0 ? A.y0 : A.y0 + A.ny * A.h;
        x = fma(hh, TB::nd.x[r], A.x0 + (gx + 0.5) * A.h);
      }
      v[r] = riemann_exact(x, y, t);
    }
  }

  // whether the sensor's B is diagonal (up to P2), and whether i is the
  // first index of the group of diagonal entries equal to B[i][i]
  __host__ __device__ static constexpr bool sn_diagonal() {
    for (int i = 0; i < NL; ++i)
      for (int j = 0; j < NL; ++j)
        if (i != j && TB::sn.B[i][j] != 0.0) return false;
    return true;
  }
  __host__ __device__ static constexpr bool sn_group_head(int i) {
    for (int j = 1; j < i; ++j)
      if (TB::sn.B[j][j] == TB::sn.B[i][i]) return false;
    return TB::sn.B[i][i] != 0.0;
  }

  // v^T B v with the sensor's quadratic form over the non-constant
  // coefficients, zero entries skipped at compile time (the first term of
  // every sum is a product: no zero to add to).  A diagonal B takes equal
  // entries once, B_g times the sum of v_i^2 over the group g (in 2D the
  // axis swap maps B to itself, so its entries come in pairs).
  __device__ static inline double qform(const double (&v)[NL]) {
    if constexpr (sn_diagonal()) {
      double acc = 0.0;
      bool started = false;
#pragma unroll
      for (int i = 1; i < NL; ++i) {
        if (sn_group_head(i)) {
          double sq = v[i] * v[i];
#pragma unroll
          for (int j = i + 1; j < NL; ++j)
            if (TB::sn.B[j][j] == TB::sn.B[i][i]) sq = fma(v[j], v[j], sq);
          acc = started ? fma(TB::sn.B[i][i], sq, acc) : TB::sn.B[i][i] * sq;
          started = true;
        }
      }
      return acc;
    }
    double acc = 0.0;
    bool started = false;
#pragma unroll
    for (int i = 1; i < NL; ++i) {
      double ri = 0.0;
      bool any = false;
#pragma unroll
      for (int j = i; j < NL; ++j) {
        if (TB::sn.B[i][j] != 0.0) {
          ri = any ? fma((j == i ? 1.0 : 2.0) * TB::sn.B[i][j], v[j], ri)
                   : ((j == i ? 1.0 : 2.0) * TB::sn.B[i][j]) * v[j];
          any = true;
        }
      }
      if (any) {
        acc = started ? fma(v[i], ri, acc) : v[i] * ri;
        started = true;
      }
    }
    return acc;
  }

  // neighbour f continued into this cell, in this cell's basis (non-constant
  // coefficients only): P_a(xi -/+ 2) = sum_b T[s][a][b] P_b(xi).  T[s][a][a]
  // = 1 (equal leading coefficients), so coefficient c of a row starts as
  // the neighbour's own coefficient c, and the higher ones add to it.
  template <int F>
  __device__ static inline void candidate(const double* b, double (&cd)[NL]) {
    constexpr int si = F & 1;
    constexpr int o = off(F);
    cd[0] = 0.0;  // the constant coefficient is not used
    if constexpr (DIM == 1 || F < 2) {
      constexpr int R = DIM == 1 ? 1 : N;
#pragma unroll
      for (int e = 0; e < R; ++e)
#pragma unroll
        for (int a = 0; a < N; ++a) {
          const double cn = b[(a + N * e) * S + o];
#pragma unroll
          for (int c = 0; c <= a; ++c)
            if (TB::dg.T[si][a][c] != 0.0 && (c + N * e) != 0)
              cd[c + N * e] = c == a ? TB::dg.T[si][a][c] * cn : fma(TB::dg.T[si][a][c], cn, cd[c + N * e]);
        }
    } else {
#pragma unroll
      for (int e = 0; e < N; ++e)
#pragma unroll
        for (int a = 0; a < N; ++a) {
          const double cn = b[(a + N * e) * S + o];
#pragma unroll
          for (int c = 0; c <= e; ++c)
            if (TB::dg.T[si][e][c] != 0.0 && (a + N * c) != 0)
              cd[a + N * c] = c == e ? TB::dg.T[si][e][c] * cn : fma(TB::dg.T[si][e][c], cn, cd[a + N * c]);
        }
    }
  }

  template <int F>
  __device__ static inline void cand_any(int f, const double* b, double (&cd)[NL]) {
    if constexpr (F < NF) {
      if (f == F)
        candidate<F>(b, cd);
      else
        cand_any<F + 1>(f, b, cd);
    }
  }

  __device__ static inline double weight(const StageArgs& A, double beta) {
    const double t = A.eps + beta;
    if (A.wpow == 2.0) {
      const double r = rcp(t);
      return r * r;
    }
    return pow_cold(t, -A.wpow);
  }

  // gamma_e of eqs. (sensor)/(gensensor) with the HWENO reconstruction.
  // One pass over the candidates: each candidate's indicator gives its
  // unnormalised weight alpha_l at once, so c* = sum_l alpha_l c^(l) / sum alpha
  // accumulates while the candidate is in registers.  SB: one candidate live
  // at a time (see below); without it the compiler may keep the neighbours'
  // coefficients in registers for the faces, where registers are not what
  // limits the occupancy.
  template <bool SB>
  __device__ static inline double sensor(const StageArgs& A, const double* b, const bool (&has)[NF],
                                         const double (&c)[NL]) {
    const double beta0 = qform(c);
    int m = 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) m += has[f];
    const double a0 = (1.0 - m * A.wnb) * weight(A, beta0);
    double asum = a0;
    double acc[NL];  // sum_l alpha_l c^(l), non-constant coefficients
#pragma unroll
    for (int j = 1; j < NL; ++j) acc[j] = a0 * c[j];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double cd[NL];
      cand_any<0>(f, b, cd);
      const double al = has[f] ? A.wnb * weight(A, qform(cd)) : 0.0;
      asum += al;
#pragma unroll
      for (int j = 1; j < NL; ++j) acc[j] = fma(al, cd[j], acc[j]);
      // keep one candidate live at a time (the scheduler would otherwise
      // hoist every candidate's LDS reads and double the register count)
      if constexpr (SB) __builtin_amdgcn_sched_barrier(0);
    }
    const double inv = rcp(asum);
    // c - c*: the constant coefficient of every candidate is c_0, and the
    // quadratic form ignores it
    double cs[NL];
    cs[0] = 0.0;
#pragma unroll
    for (int j = 1; j < NL; ++j) cs[j] = fma(-inv, acc[j], c[j]);
    const double num2 = qform(cs);
    double ratio;
    if (num2 == 0.0)
      ratio = 0.0;
    else if (beta0 == 0.0)
      ratio = __builtin_inf();
    else
      ratio = sqrt_pos(num2 * rcp(beta0));
    if (!(ratio >= A.bthr)) return 0.0;
    const double r1 = fmin(1.0, ratio);
    return A.q == 1.0 ? r1 : pow_cold(r1, A.q);
  }

  // Every face flux is taken in one orientation: n = +e_axis, from the cell
  // below the face (state ul) to the cell above it (state uh).  The cell above
  // uses H(uh, ul, -n) = -H(ul, uh, n) (the LLF flux is conservative), so both
  // cells of a face, and a tile's shared face phase, compute the same face
  // moments bit for bit.  The roundings are fixed by explicit fma.
  //
  // KPP flux F(u) = (sin u, cos u) of Sec. 5.5: H(ul, uh, e_axis) with
  // s+ = max |F'(w) . n| over w between the states, i.e. max |cos w| (x
  // faces) or |sin w| (y faces): 1 where that interval holds a peak (k pi,
  // resp. pi/2 + k pi), else the larger end value
  template <bool INL = false>
  __device__ static inline double llf_kpp(int axis, double ul, double uh) {
    constexpr double kPi = 3.141592653589793238462643383279502884;
    double sl, cl, sh, ch;
    if constexpr (INL) {
      sincos_inl(ul, &sl, &cl);
      sincos_inl(uh, &sh, &ch);
    } else {
      sincos_cold(ul, &sl, &cl);
      sincos_cold(uh, &sh, &ch);
    }
    const double Fl = axis == 0 ? sl : cl, Fh = axis == 0 ? sh : ch;
    const double dl = axis == 0 ? fabs(cl) : fabs(sl), dh = axis == 0 ? fabs(ch) : fabs(sh);
    const double shift = axis == 0 ? 0.0 : 0.5 * kPi;
    const bool peak = floor((fmax(ul, uh) - shift) / kPi) >= ceil((fmin(ul, uh) - shift) / kPi);
    const double splus = peak ? 1.0 : fmax(dl, dh);
    return fma(-0.5 * splus, uh - ul, 0.5 * (Fl + Fh));
  }

  // LLF flux H(ul, uh, e_axis) of Sec. 2 for the linear and Burgers fluxes;
  // v: the velocity component along the axis (linear) or the axis component
  // of the Burgers direction
  __device__ static inline double llf(double v, double ul, double uh) {
    if constexpr (FLUX == FLUX_LINADV) {
      return fma(-0.5 * fabs(v), uh - ul, (0.5 * v) * (ul + uh));
    } else {
      // -0.5 |v| is exact: the product equals -0.5 (|v| max) bit for bit
      const double nsp = (-0.5 * fabs(v)) * fmax(fabs(ul), fabs(uh));
      return fma(nsp, uh - ul, (0.25 * v) * fma(ul, ul, uh * uh));
    }
  }

  // Velocity component along `axis` at the Q Gauss points of a line of
  // faces normal to it (linear flux): v_x on the row of cells i (it depends
  // on y only), v_y on the column i (x only); the Burgers direction
  // otherwise.
  __device__ static inline void line_velocity(const StageArgs& A, int axis, int i, double (&v)[Q]) {
    const double hh = 0.5 * A.h;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if constexpr (FLUX == FLUX_LINADV) {
        if (axis == 0) {
          const double yc = fma(i + 0.5, A.h, A.y0);
          v[k] = fma(-A.omega, fma(hh, TB::nd.x[k], yc) - A.cy, A.vx);
        } else {
          const double xc = fma(i + 0.5, A.h, A.x0);
          v[k] = fma(A.omega, fma(hh, TB::nd.x[k], xc) - A.cx, A.vy);
        }
      } else {
        v[k] = axis == 0 ? A.vx : A.vy;
      }
    }
  }

  // Trace of a cell on one of its faces normal to `axis`, in the face's
  // Legendre basis: t_k = sum_i P_i(+-1) c(i, k), c(i, k) the coefficient of
  // P_i along the axis times P_k along the face (in 1D the single value).
  // UPPER: the cell above the face (its -axis side, P_i(-1) = (-1)^i); else
  // the cell below (P_i(+1) = 1).  coef(j) returns coefficient j.
  template <bool UPPER, class Coef>
  __device__ static inline void trace(int axis, Coef coef, double (&t)[DIM == 2 ? N : 1]) {
    // (P_0 = 1 at both ends: the sum starts with the i = 0 coefficient)
    if constexpr (DIM == 1) {
      double acc = coef(0);
#pragma unroll
      for (int a = 1; a < N; ++a) acc = fma(UPPER ? TB::dg.sgn[a] : 1.0, coef(a), acc);
      t[0] = acc;
    } else {
#pragma unroll
      for (int k = 0; k < N; ++k) {
        double acc = coef(axis == 0 ? N * k : k);
#pragma unroll
        for (int i = 1; i < N; ++i)
          acc = fma(UPPER ? TB::dg.sgn[i] : 1.0, coef(axis == 0 ? i + N * k : k + N * i), acc);
        t[k] = acc;
      }
    }
  }

  // One x node line of the 2D sum factorisation: s1[bb] = sum_a c(a, bb)
  // P_a(x_qx), and the value at node (qx, qy) from it.  coef(j) returns
  // coefficient j.  The volume integral and the KPP node tasks of
  // kpp_split_tile evaluate u_h at a node with these, bit for bit alike.
  template <class Coef>
  __device__ static inline void xline(Coef coef, int qx, double (&s1)[N]) {
#pragma unroll
    for (int bb = 0; bb < N; ++bb) {
      double t = coef(N * bb);
#pragma unroll
      for (int a = 1; a < N; ++a) t = fma(coef(a + N * bb), TB::nd.L[a][qx], t);
      s1[bb] = t;
    }
  }
  __device__ static inline double ynode(const double (&s1)[N], int qy) {
    double u = s1[0];
#pragma unroll
    for (int bb = 1; bb < N; ++bb) u = fma(s1[bb], TB::nd.L[bb][qy], u);
    return u;
  }

  // The moments g[k] = sum_r w_r P_k(x_r) H_r of a 2D face from the face
  // flux at its Q Gauss points (line_moments: mirrored node pairs)
  __device__ static inline void face_sum(const double (&H)[Q], double (&g)[N]) { line_moments<false>(H, g); }

  // The two states at Gauss point r of a 2D face from the traces
  __device__ static inline void face_node(const double (&tl)[N], const double (&th)[N], int r, double& ul,
                                          double& uh) {
    ul = tl[0];
    uh = th[0];
#pragma unroll
    for (int k = 1; k < N; ++k) {
      ul = fma(tl[k], TB::nd.L[k][r], ul);
      uh = fma(th[k], TB::nd.L[k][r], uh);
    }
  }

  // Moments g_k = sum_r w_r L_k(x_r) H(ul(x_r), uh(x_r), e_axis) of a 2D face
  // from the traces of the cells below (tl) and above (th) it; v as from
  // line_velocity.  XBC: where xl (xh) is set, the state below (above) at
  // point r is ext[r * S] instead (the BC_RIEMANN exterior slot).
  template <bool XBC, bool INL = false>
  __device__ static inline void face_moments(int axis, const double (&tl)[N], const double (&th)[N],
                                             const double (&v)[Q], bool xl, bool xh, const double* ext,
                                             double (&g)[N]) {
    double H[Q];
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      double ul, uh;
      face_node(tl, th, r, ul, uh);
      if constexpr (XBC && FLUX == FLUX_BURGERS) {
        if (xl) ul = ext[r * S];
        if (xh) uh = ext[r * S];
      }
      if constexpr (FLUX == FLUX_KPP)
        H[r] = llf_kpp<INL>(axis, ul, uh);
      else
        H[r] = llf(v[r], ul, uh);
    }
    face_sum(H, g);
  }

  // Adds face f's term - int_f phi H(u^-, u^+, n) to R from the face's
  // moments: the cell below the face (f = 1, 3) subtracts them, the cell
  // above (f = 0, 2) adds them with P_i(-1) = (-1)^i.
  __device__ static inline void add_face(int f, const double (&g)[DIM == 2 ? N : 1], double (&R)[NL]) {
    const bool below = f & 1;
    if constexpr (DIM == 1) {
#pragma unroll
      for (int a = 0; a < N; ++a) R[a] = fma(below ? -1.0 : TB::dg.sgn[a], g[0], R[a]);
    } else {
      const int axis = f >> 1;
#pragma unroll
      for (int k = 0; k < N; ++k)
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const int j = axis == 0 ? i + N * k : k + N * i;
          R[j] = fma(below ? -1.0 : TB::dg.sgn[i], g[k], R[j]);
        }
    }
  }

  // The sensor of Zhao et al. that Sec. 5.6 compares with: the deviation of
  // the nonlinear HWENO weights (the same alpha_l as in sensor()) from the
  // linear ones, sum_l |omega_l / omega~_l - 1|^theta over the candidates
  // that exist, over |1 / min_l omega~_l - 1|^theta + m_e; 0 without face
  // neighbours.
  template <bool SB>
  __device__ static inline double zhao(const StageArgs& A, const double* b, const bool (&has)[NF],
                                       const double (&c)[NL]) {
    int m = 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) m += has[f];
    if (m == 0) return 0.0;
    const double lin0 = 1.0 - m * A.wnb;
    double al[NF + 1];
    al[0] = lin0 * weight(A, qform(c));
    double asum = al[0];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double cd[NL];
      cand_any<0>(f, b, cd);
      al[f + 1] = has[f] ? A.wnb * weight(A, qform(cd)) : 0.0;
      asum += al[f + 1];
      if constexpr (SB) __builtin_amdgcn_sched_barrier(0);
    }
    const double inv = rcp(asum);
    auto pw = [&](double x) { return A.theta == 1.0 ? x : pow_cold(x, A.theta); };
    double dev = pw(fabs(al[0] * inv / lin0 - 1.0));
#pragma unroll
    for (int f = 0; f < NF; ++f)
      if (has[f]) dev += pw(fabs(al[f + 1] * inv / A.wnb - 1.0));
    return dev / (pw(fabs(1.0 / fmin(lin0, A.wnb) - 1.0)) + m);
  }

  // gamma_e of the cell at mesh coordinates (ix, iy) in this stabilisation mode
  template <bool SB>
  __device__ static inline double gamma_of(const StageArgs& A, const double* b, const double (&c)[NL], int ix,
                                           int iy) {
    if constexpr (MODE == MODE_DG) {
      return 0.0;
    } else if constexpr (MODE == MODE_LO) {
      return 1.0;
    } else {
      bool has[NF];
      has[0] = A.per_x || ix > 0;
      has[1] = A.per_x || ix < A.nx - 1;
      if constexpr (DIM == 2) {
        has[2] = A.per_y || iy > 0;
        has[3] = A.per_y || iy < A.ny - 1;
      }
      if constexpr (MODE == MODE_ZHAO)
        return zhao<SB>(A, b, has, c);
      else
        return sensor<SB>(A, b, has, c);
    }
  }

  // dU/dt of one cell and gamma_e; c holds the cell's own coefficients (the
  // same values as its LDS slot b), the neighbours are read from LDS.  SB as
  // for sensor(); the arithmetic is the same either way.  The three parts
  // (gamma_of, residual, finish) may also run on different threads.
  // XBC: compile the BC_RIEMANN exterior state in (the per-stage kernel only).
  template <bool SB = true, bool XBC = false>
  __device__ static inline void rhs(const StageArgs& A, const double* b, const double (&c)[NL], int ix, int iy,
                                    double (&L)[NL], double& gam_out) {
    const double gam = gamma_of<SB>(A, b, c, ix, iy);
    gam_out = gam;
    double R[NL], lam;
    residual<XBC>(A, b, c, ix, iy, R, lam);
    finish(A, c, gam, lam, R, L);
  }

  // The moments of face f of the cell (0: -x, 1: +x, 2: -y, 3: +y), oriented
  // from the cell below the face to the cell above it: this cell's
  // coefficients from registers, the neighbour's from its LDS slot.
  template <bool XBC = false>
  __device__ static inline void cell_face(const StageArgs& A, const double* b, const double (&c)[NL], int ix, int iy,
                                          int f, double (&g)[DIM == 2 ? N : 1]) {
    const bool below = f & 1;  // this cell lies below the face
    const int axis = f >> 1;
    const int o = off(f);
    auto own = [&](int j) { return c[j]; };
    auto nbr = [&](int j) { return b[j * S + o]; };
    constexpr int NT_ = DIM == 2 ? N : 1;
    double tl[NT_], th[NT_];
    if (below) {
      trace<false>(axis, own, tl);
      trace<true>(axis, nbr, th);
    } else {
      trace<false>(axis, nbr, tl);
      trace<true>(axis, own, th);
    }
    if constexpr (DIM == 1) {
      g[0] = llf(A.vx, tl[0], th[0]);
    } else {
      double v[Q];
      line_velocity(A, axis, axis == 0 ? iy : ix, v);
      // a boundary face under BC_RIEMANN reads the exterior state at its
      // nodes from the neighbour's slot
      bool xb = false;
      if constexpr (XBC && FLUX == FLUX_BURGERS) {
        if (A.bc_kind == BC_RIEMANN)
          xb = f == 0 ? ix == 0 : f == 1 ? ix == A.nx - 1 : f == 2 ? iy == 0 : iy == A.ny - 1;
      }
      face_moments<XBC>(axis, tl, th, v, xb && !below, xb && below, b + o, g);
    }
  }

  // g[bb] = sum_q w_q T_bb(x_q) f_q over the Q Gauss nodes of a line, T_bb
  // = P_bb (DER = false) or P_bb' (DER = true, bb >= 1), with the mirror
  // symmetry of the rule: T_bb(-x) = +/- T_bb(x), so f enters as the sum
  // or the difference of each node pair (the first term of each sum a
  // product; terms with a zero table entry dropped at compile time)
  __host__ __device__ static constexpr bool nodes_mirrored() {
    for (int r = 0; r < Q; ++r) {
      const int m = Q - 1 - r;
      if (TB::nd.x[r] != -TB::nd.x[m] || TB::nd.w[r] != TB::nd.w[m]) return false;
      for (int k = 0; k < N; ++k) {
        const double sg = k % 2 ? -1.0 : 1.0;
        if (TB::nd.L[k][r] != sg * TB::nd.L[k][m] || TB::nd.D[k][r] != -sg * TB::nd.D[k][m]) return false;
      }
    }
    return true;
  }
  template <bool DER>
  __device__ static inline void line_moments(const double (&f)[Q], double (&g)[N]) {
    // the pair sums stay plain adds: fused with the products that form f
    // (as the compiler may choose, kernel by kernel) they would round
    // differently in different kernels
#pragma clang fp contract(off)
    static_assert(nodes_mirrored(), "the Gauss tables must be mirror-symmetric bit for bit");
    constexpr int H = Q / 2;
    double sp[H + 1], dp[H + 1];
#pragma unroll
    for (int r = 0; r < H; ++r) {
      sp[r] = f[r] + f[Q - 1 - r];
      dp[r] = f[r] - f[Q - 1 - r];
    }
    if constexpr (Q % 2 == 1) {
      sp[H] = f[H];
      dp[H] = 0.0;  // odd functions vanish at the middle node (not used)
    }
#pragma unroll
    for (int bb = DER ? 1 : 0; bb < N; ++bb) {
      // parity of T_bb: even for P_bb with bb even, for P_bb' with bb odd
      const bool even = DER ? (bb % 2 == 1) : (bb % 2 == 0);
      const int nr = even ? (Q + 1) / 2 : H;
      double acc = 0.0;
      bool started = false;
#pragma unroll
      for (int r = 0; r < nr; ++r) {
        const double k = TB::nd.w[r] * (DER ? TB::nd.D[bb][r] : TB::nd.L[bb][r]);
        if (k != 0.0) {
          const double v = even ? sp[r] : dp[r];
          acc = started ? fma(k, v, acc) : k * v;
          started = true;
        }
      }
      g[bb] = acc;
    }
  }

  // Volume minus face terms of the weak form (R) and the cell's wave speed
  // lambda_e (before the override); the faces in the order -x, +x, -y, +y.
  // FACES = false: the volume terms only (a tile's shared faces are added
  // by the caller, in the same order).  VS > 0 (2D KPP): the flux pair at
  // volume node (qx, qy) was evaluated beforehand, sin u at
  // vol[(qx Q + qy) VS] and cos u at vol[(Q^2 + qx Q + qy) VS].
  template <bool XBC = false, bool FACES = true, int VS = 0>
  __device__ static inline void residual(const StageArgs& A, const double* b, const double (&c)[NL], int ix, int iy,
                                         double (&R)[NL], double& lam, const double* vol = nullptr) {
    // (every sum starts with a product: R is assigned, not cleared, at the
    // first node)
    if constexpr (DIM == 1) {
      R[0] = 0.0;
      double umax = 0.0;
#pragma unroll
      for (int qn = 0; qn < Q; ++qn) {
        double u = c[0];
#pragma unroll
        for (int a = 1; a < N; ++a) u = fma(c[a], TB::nd.L[a][qn], u);
        double F;
        if constexpr (FLUX == FLUX_LINADV) {
          F = A.vx * u;
        } else {
          F = A.vx * (0.5 * u * u);
          umax = fmax(umax, fabs(u));
        }
        const double wF = TB::nd.w[qn] * F;
#pragma unroll
        for (int a = 1; a < N; ++a) R[a] = qn == 0 ? TB::nd.D[a][qn] * wF : fma(TB::nd.D[a][qn], wF, R[a]);
      }
      lam = FLUX == FLUX_LINADV ? fabs(A.vx) : A.anorm * umax;
    } else {
      // velocity components along the node lines (linear flux): v_x depends
      // on y only, v_y on x only
      double vxl[Q], vyl[Q];
      line_velocity(A, 0, iy, vxl);
      line_velocity(A, 1, ix, vyl);
      // int grad(phi) . F(u_h), sum factorised over x nodes.  Burgers: the
      // node sums take u^2, and the factors v_x / 2, v_y / 2 are applied once
      // per x node
      double umax = 0.0;
      const double hvx = 0.5 * A.vx, hvy = 0.5 * A.vy;
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        double s1[N];
        xline([&](int j) { return c[j]; }, qx, s1);
        // the flux at the Q nodes of this x node's line
        constexpr bool SAMEF = FLUX == FLUX_BURGERS;  // Fy = Fx (u^2)
        double fx[Q], fy[SAMEF ? 1 : Q];
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          const double u = ynode(s1, qy);
          if constexpr (FLUX == FLUX_LINADV) {
            fx[qy] = vxl[qy] * u;
            fy[qy] = vyl[qx] * u;
          } else if constexpr (FLUX == FLUX_KPP) {
            if constexpr (VS > 0) {
              fx[qy] = vol[(qx * Q + qy) * VS];
              fy[qy] = vol[(Q * Q + qx * Q + qy) * VS];
            } else {
              double sn, cs;  // (scalars: the call does not pin the arrays to memory)
              sincos_cold(u, &sn, &cs);
              fx[qy] = sn;
              fy[qy] = cs;
            }
          } else {
            fx[qy] = u * u;
            umax = fmax(umax, fabs(u));
          }
        }
        // gx[bb] = sum_qy w L_bb F_x, gy[bb] = sum_qy w P_bb' F_y over the
        // line, folded over mirrored node pairs (qy, Q-1-qy): the Gauss
        // nodes and weights are symmetric and P_bb has the parity of bb, so
        // even functions take the pair's sum and odd ones its difference
        // (the middle node of an odd rule only the even ones)
        double gx[N], gy[N];
        line_moments<false>(fx, gx);
        if constexpr (SAMEF)
          line_moments<true>(fx, gy);
        else
          line_moments<true>(fy, gy);
        if constexpr (FLUX == FLUX_BURGERS) {
#pragma unroll
          for (int bb = 0; bb < N; ++bb) {
            gx[bb] *= hvx;
            if (bb > 0) gy[bb] *= hvy;
          }
        }
        const double wq = TB::nd.w[qx];
#pragma unroll
        for (int bb = 0; bb < N; ++bb)
#pragma unroll
          for (int a = 0; a < N; ++a) {
            double t = qx == 0 ? 0.0 : R[a + N * bb];
            bool started = qx > 0;
            if (a > 0) {
              const double k = wq * TB::nd.D[a][qx];
              t = started ? fma(k, gx[bb], t) : k * gx[bb];
              started = true;
            }
            if (bb > 0) {
              const double k = wq * TB::nd.L[a][qx];
              t = started ? fma(k, gy[bb], t) : k * gy[bb];
            }
            R[a + N * bb] = t;
          }
      }
      if constexpr (FLUX == FLUX_LINADV) {
        // |v|^2 = v_x(y)^2 + v_y(x)^2 separates over the node grid
        double mx = 0.0, my = 0.0;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          mx = fmax(mx, vxl[k] * vxl[k]);
          my = fmax(my, vyl[k] * vyl[k]);
        }
        lam = sqrt_pos(mx + my);
      } else if constexpr (FLUX == FLUX_KPP) {
        lam = 1.0;  // ||F'(u)||_2 = ||(cos u, -sin u)||_2
      } else {
        lam = A.anorm * umax;
      }
    }
    if constexpr (FACES) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        double g[DIM == 2 ? N : 1];
        cell_face<XBC>(A, b, c, ix, iy, f, g);
        add_face(f, g, R);
      }
    }
  }

  // Branch record of the cell's evaluation, for checks of the discrete
  // adjoint by finite differences: the decisions the operator takes where the
  // computed map is not differentiable, each folded into its own 32-bit hash.
  //   v[0] the sensor (eqs. sensor/gensensor): gamma_e >= 1 (min(1, ratio) at
  //        its cap) and gamma_e == 0 (below the threshold b);
  //   v[1] lambda_e of eq. (visc) for Burgers: the volume node of the largest
  //        |u| (strict running maximum, as in volume) and the sign of u there;
  //   v[2] the LLF wave speed for Burgers (Sec. 2): at every face node which
  //        of |u_below|, |u_above| is larger, and their signs.
  // The node values and traces are computed with the same explicit fma chains
  // as the operator (trace, face_node), so the decisions are its own.  The
  // linear flux has no such point in U (its wave speeds depend on x only).
  __device__ static inline void branches(const StageArgs& A, const double* b, const double (&c)[NL], double gam,
                                         uint32_t (&v)[3]) {
    auto fold = [](uint32_t h, uint32_t x) { return (h ^ x) * 16777619u; };
    v[0] = v[1] = v[2] = 2166136261u;
    if constexpr (MODE == MODE_WENO) v[0] = fold(v[0], (gam >= 1.0 ? 1u : 0u) | (gam == 0.0 ? 2u : 0u));
    if constexpr (FLUX == FLUX_BURGERS) {
      double umax = 0.0;
      uint32_t arg = 0xffffu, sgn = 0;
      if constexpr (DIM == 1) {
#pragma unroll
        for (int qn = 0; qn < Q; ++qn) {
          double u = c[0];
#pragma unroll
          for (int a = 1; a < N; ++a) u = fma(c[a], TB::nd.L[a][qn], u);
          if (fabs(u) > umax) {
            umax = fabs(u);
            arg = qn;
            sgn = u < 0.0;
          }
        }
      } else {
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) {
          double s1[N];
#pragma unroll
          for (int bb = 0; bb < N; ++bb) {
            double t = c[N * bb];
#pragma unroll
            for (int a = 1; a < N; ++a) t = fma(c[a + N * bb], TB::nd.L[a][qx], t);
            s1[bb] = t;
          }
#pragma unroll
          for (int qy = 0; qy < Q; ++qy) {
            double u = s1[0];
#pragma unroll
            for (int bb = 1; bb < N; ++bb) u = fma(s1[bb], TB::nd.L[bb][qy], u);
            if (fabs(u) > umax) {
              umax = fabs(u);
              arg = qx * Q + qy;
              sgn = u < 0.0;
            }
          }
        }
      }
      v[1] = fold(v[1], arg | (sgn << 16));
      // faces: the traces and node values of cell_face
      auto rec = [&](double ul, double uh) {
        v[2] = fold(v[2], (fabs(ul) > fabs(uh) ? 1u : 0u) | (ul < 0.0 ? 2u : 0u) | (uh < 0.0 ? 4u : 0u));
      };
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const bool below = f & 1;
        const int axis = f >> 1;
        auto own = [&](int j) { return c[j]; };
        auto nbr = [&](int j) { return b[j * S + off(f)]; };
        constexpr int NT_ = DIM == 2 ? N : 1;
        double tl[NT_], th[NT_];
        if (below) {
          trace<false>(axis, own, tl);
          trace<true>(axis, nbr, th);
        } else {
          trace<false>(axis, nbr, tl);
          trace<true>(axis, own, th);
        }
        if constexpr (DIM == 1) {
          rec(tl[0], th[0]);
        } else {
#pragma unroll
          for (int r = 0; r < Q; ++r) {
            double ul, uh;
            face_node(tl, th, r, ul, uh);
            rec(ul, uh);
          }
        }
      }
    }
  }

  // (2/h) minv_a minv_b (1D: (2/h) minv_a): up to P2 the host's product
  // (the same value; saves the multiplications in every thread), from P3 on
  // formed here (read from the arguments, its 16-25 values cost the P3 and
  // P4 kernels registers)
  __device__ static inline double lfac(const StageArgs& A, int a, int bb) {
    if constexpr (P <= 2)
      return A.lfac[a + N * bb];
    else
      return DIM == 2 ? A.g2h * TB::dg.minv[a] * TB::dg.minv[bb] : A.g2h * TB::dg.minv[a];
  }

  // Dissipation gamma nu int grad(phi).grad(u_h) and M^-1:
  // L = (2/h) Mhat^-1 [ vol - face - (gamma lambda / p) Khat c ]
  __device__ static inline void finish(const StageArgs& A, const double (&c)[NL], double gam, double lam,
                                       const double (&R)[NL], double (&L)[NL]) {
    if (A.lam_over > 0.0) lam = A.lam_over;
    const double kd = gam * lam * (1.0 / P);
    if constexpr (DIM == 1) {
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double kc = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2)
          if (TB::dg.S[a][a2] != 0.0) kc = fma(TB::dg.S[a][a2], c[a2], kc);
        L[a] = lfac(A, a, 0) * fma(-kd, kc, R[a]);
      }
    } else {
#pragma unroll
      for (int bb = 0; bb < N; ++bb)
#pragma unroll
        for (int a = 0; a < N; ++a) {
          double kc = 0.0;
#pragma unroll
          for (int a2 = 0; a2 < N; ++a2)
            if (TB::dg.S[a][a2] != 0.0) kc = fma(TB::dg.S[a][a2] * TB::dg.mhat[bb], c[a2 + N * bb], kc);
#pragma unroll
          for (int b2 = 0; b2 < N; ++b2)
            if (TB::dg.S[bb][b2] != 0.0) kc = fma(TB::dg.S[bb][b2] * TB::dg.mhat[a], c[a + N * b2], kc);
          L[a + N * bb] = lfac(A, a, bb) * fma(-kd, kc, R[a + N * bb]);
        }
    }
  }
};

// Global cell index of slot (gx, gy) relative to the mesh, with periodic wrap;
// false if the slot lies outside a non-periodic boundary.
// (In 1D the row index is ignored.)
template <int DIM>
__host__ __device__ inline bool slot_cell(const StageArgs& A, int gx, int gy, size_t& cell) {
  const int nx = A.nx, ny = DIM == 2 ? A.ny : 1;
  if (DIM == 1) gy = 0;
  if ((unsigned)gx >= (unsigned)nx) {
    if (!A.per_x) return false;
    gx = wrap_index(gx, nx);
  }
  if (DIM == 2 && (unsigned)gy >= (unsigned)ny) {
    if (!A.per_y) return false;
    gy = wrap_index(gy, ny);
  }
  cell = (size_t)gy * nx + gx;
  return true;
}

// The KPP flux on 8 x 8 tiles (kpp_split_tile): 4 to 16 waves per tile.  LDS:
// the tile, then the flux pair at every volume node of every cell (plane
// node, sin u then cos u, 64 cells each: 2 Q^2 planes), then the LLF flux
// at every node of every face (x faces, then y faces; per axis Q planes of
// the 72 faces in face_slot's order).
__host__ __device__ constexpr bool splits_nodes(int dim, int flux, int tx, int ty) {
  return dim == 2 && flux == FLUX_KPP && tx == 8 && ty == 8;
}
__host__ __device__ inline int split_lds_doubles(int nl, int q) {
  return tile_lds_doubles(2, nl, 8, 8) + 2 * q * q * 64 + 2 * 72 * q;
}
// Volume node task v (< 64 q^2) of kpp_split_tile: tile cell v mod 64 at
// node (qx, qy), v / 64 = qx q + qy.  Returns the index of its sin u in the
// node planes (cos u: + 64 q^2); slot: the cell's LDS slot.
__host__ __device__ inline int split_vol_task(int v, int q, int& slot, int& qx, int& qy) {
  const int lc = v & 63, node = v >> 6;
  qx = node / q;
  qy = node % q;
  slot = ((lc >> 3) + 1) * 10 + (lc & 7) + 1;
  return node * 64 + lc;
}
// Face node task i (< 144 q): axis, Gauss point r and face e (face_slot's
// order); returns its index in the face node planes
__host__ __device__ inline int split_face_task(int i, int q, int& axis, int& r, int& e) {
  axis = i >= 72 * q;
  const int j = i - axis * 72 * q;
  r = j / 72;
  e = j % 72;
  return (axis * q + r) * 72 + e;
}
// Face f (0: -x, 1: +x, 2: -y, 3: +y) of tile cell lc, as a face of its axis
__host__ __device__ inline int split_cell_face(int lc, int f) {
  const int lx = lc % 8, ly = lc / 8;
  return f < 2 ? ly * 9 + lx + (f & 1) : ly * 8 + lx + (f & 1) * 8;
}
// LDS of the per-stage kernels on this tile (2D 8x8: the larger of the
// one-wave and the four-wave kernel, roles_tile)
__host__ __device__ inline int stage_kernel_lds_doubles(int dim, int nl, int p, int flux, int tx, int ty) {
  if (splits_nodes(dim, flux, tx, ty)) return split_lds_doubles(nl, quad_points(dim, p, flux));
  const int one = stage_lds_doubles(dim, nl, flux, tx, ty);
  if (dim == 2 && tx == 8 && ty == 8) {
    const int four = tile_lds_doubles(2, nl, 8, 8) + face_lds_doubles(p + 1, 8, 8) + 64;
    return four > one ? four : one;
  }
  return one;
}

// The slots thread t of the tile at (ix0, iy0) loads: its own cell's slot
// (always) and at most one slot of the halo ring (no corners: the stencil has
// face neighbours only).  gx, gy are mesh coordinates before wrapping; in 1D
// the row is 0.
template <int DIM, int TX, int TY>
__host__ __device__ inline bool tile_slots(int t, int ix0, int iy0, int& sc, int& gx, int& gy, int& hslot, int& hgx,
                                           int& hgy) {
  using G = TileGeom<DIM, TX, TY>;
  const int lx = DIM == 2 ? t % TX : t, ly = DIM == 2 ? t / TX : 0;
  sc = DIM == 2 ? (ly + 1) * G::W + lx + 1 : lx + 1;
  gx = ix0 + lx;
  gy = DIM == 2 ? iy0 + ly : 0;
  int sx, sy;
  if constexpr (DIM == 1) {
    if (t >= 2) return false;
    sx = t == 0 ? 0 : TX + 1;
    sy = 0;
  } else {
    if (t >= 2 * TX + 2 * TY) return false;
    if (t < TX) {
      sx = t + 1;
      sy = 0;
    } else if (t < 2 * TX) {
      sx = t - TX + 1;
      sy = TY + 1;
    } else if (t < 2 * TX + TY) {
      sx = 0;
      sy = t - 2 * TX + 1;
    } else {
      sx = TX + 1;
      sy = t - 2 * TX - TY + 1;
    }
  }
  hslot = sy * G::W + sx;
  hgx = ix0 - 1 + sx;
  hgy = DIM == 2 ? iy0 - 1 + sy : 0;
  return true;
}

// Mesh index of the face neighbour f (0: -x, 1: +x, 2: -y, 3: +y) of cell
// (ix, iy), wrapping periodically; callers use it only where the neighbour
// exists (periodic axis or interior face).
__host__ __device__ inline size_t neighbour_cell(int ix, int iy, int f, int nx, int ny) {
  if (f == 0) ix = ix == 0 ? nx - 1 : ix - 1;
  if (f == 1) ix = ix == nx - 1 ? 0 : ix + 1;
  if (f == 2) iy = iy == 0 ? ny - 1 : iy - 1;
  if (f == 3) iy = iy == ny - 1 ? 0 : iy + 1;
  return (size_t)iy * nx + ix;
}

// The NL coefficients of the cell at mesh coordinates (gx, gy) before
// wrapping, or the constant exterior state outside a non-periodic boundary.
template <int DIM, int NL>
__device__ inline void load_cell(const StageArgs& A, int gx, int gy, double (&v)[NL]) {
  size_t cell;
  if (slot_cell<DIM>(A, gx, gy, cell)) {
    const double* src = A.uin + cell * NL;
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = src[j];
  } else {
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = j == 0 ? A.bc : 0.0;
  }
}

// Load one slot into the coefficient-major LDS tile.
template <int DIM, int NL, int S>
__device__ inline void load_slot(const StageArgs& A, double* lds, int slot, int gx, int gy) {
  double v[NL];
  load_cell<DIM, NL>(A, gx, gy, v);
#pragma unroll
  for (int j = 0; j < NL; ++j) lds[j * S + slot] = v[j];
}

// One tile of the fused stage: TX*TY threads, one per cell.  Each thread
// loads its own cell's coefficients into registers (a wave covers a
// contiguous span of the cell-major state) and publishes them in the
// coefficient-major LDS tile (NL * S doubles) for its neighbours; the first
// threads also load the halo ring.  After one barrier each thread evaluates
// its cell from registers (own) and LDS (face neighbours), reads U^n of its
// cell and writes the RK combination straight to HBM.  Tiles that share
// faces (shares_faces) first evaluate every face once into LDS (a second
// barrier); the cells then add their faces' moments in the order of the
// per-cell evaluation, so the result is the same bit for bit.
// XBC: compile the BC_RIEMANN exterior state in (2D Burgers per-stage kernel).
template <int DIM, int P, int FLUX, int MODE, int TX, int TY, bool XBC = false>
__device__ inline void stage_tile(const StageArgs& A, double* lds, int ix0, int iy0) {
  using G = TileGeom<DIM, TX, TY>;
  using C = Cell<DIM, P, FLUX, MODE, G::S, G::W>;
  constexpr int NL = C::NL;
  constexpr int S = G::S;
  const int nx = A.nx, ny = DIM == 2 ? A.ny : 1;
  const bool comb = !A.rhs_only && A.a != 0.0;

  const int t = threadIdx.x;
  int sc, gx, gy, hs, hgx, hgy;
  const bool halo = tile_slots<DIM, TX, TY>(t, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
  const bool active = gx < nx && gy < ny;
  const size_t cell = (size_t)gy * nx + gx;
  // own slot (cells past a ragged edge hold the wrapped or exterior state)
  double c[NL];
  load_cell<DIM, NL>(A, gx, gy, c);
  bool xbc = false;  // exterior slots from the exact solution (BC_RIEMANN)
  if constexpr (XBC) {
    xbc = A.bc_kind == BC_RIEMANN;
    if (xbc) {
      C::riemann_slot(A, gx, gy, c);
      if (halo) {
        double v[NL];
        load_cell<DIM, NL>(A, hgx, hgy, v);
        C::riemann_slot(A, hgx, hgy, v);
#pragma unroll
        for (int j = 0; j < NL; ++j) lds[j * S + hs] = v[j];
      }
    }
  }
  if (!xbc && halo) load_slot<DIM, NL, S>(A, lds, hs, hgx, hgy);
#pragma unroll
  for (int j = 0; j < NL; ++j) lds[j * S + sc] = c[j];
  tile_barrier();
  constexpr bool SHARE = shares_faces(DIM, P, FLUX, TX, TY);
  using FG = FaceGeom<TX, TY>;
  constexpr int N = P + 1;
  double* const fxl = lds + NL * S;      // shared x faces (SHARE)
  double* const fyl = fxl + N * FG::XS;  // shared y faces
  if constexpr (SHARE) {
    // face phase: every x face of the tile, then every y face, one per
    // thread and round (face_task); the two waves that take the faces left
    // over change with the tile, so that no SIMD takes them on every tile.
    // Few registers are live here: the KPP flux takes its sine and cosine
    // inline (16x16 P2 stage 175 -> 129 us at 1024^2)
    constexpr int NT = TX * TY, NW = NT / 64;
    static_assert(NT % 64 == 0 && FG::NXF - NT <= 64 && FG::NYF - NT <= 64, "one extra round of faces");
    auto face = [&](int axis, int e) {
      int fgx, fgy;
      const int lo = face_slot<TX, TY>(axis, e, ix0, iy0, fgx, fgy);
      const int hi = lo + (axis == 0 ? 1 : G::W);
      double tl[N], th[N], v[C::Q], g[N];
      C::template trace<false>(axis, [&](int j) { return lds[j * S + lo]; }, tl);
      C::template trace<true>(axis, [&](int j) { return lds[j * S + hi]; }, th);
      C::line_velocity(A, axis, opaque(axis == 0 ? fgy : fgx), v);
      bool xl = false, xh = false;
      if constexpr (XBC) {
        if (xbc) {
          const int l = axis == 0 ? fgx : fgy, n = axis == 0 ? nx : ny;
          xl = l == -1;
          xh = l == n - 1;
        }
      }
      C::template face_moments<XBC, true>(axis, tl, th, v, xl, xh, lds + (xl ? lo : hi), g);
      double* dst = axis == 0 ? fxl + e : fyl + e;
#pragma unroll
      for (int k = 0; k < N; ++k) dst[k * (axis == 0 ? FG::XS : FG::YS)] = g[k];
    };
    const int rot = (int)(((unsigned)ix0 / TX + (unsigned)iy0 / TY) % NW);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int e;
      if (face_task<TX, TY>(t, rot, k, e)) face(k & 1, e);
    }
    tile_barrier();
  }
  if (active) {
    double L[NL], gam;
    if constexpr (SHARE) {
      gam = C::template gamma_of<true>(A, lds + sc, c, gx, gy);
      double R[NL], lam;
      C::template residual<false, false>(A, lds + sc, c, gx, gy, R, lam);
      const int lx = t % TX, ly = t / TX;
      const int ex = ly * (TX + 1) + lx, ey = ly * TX + lx;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const double* src = f < 2 ? fxl + ex + (f & 1) : fyl + ey + (f & 1) * TX;
        double g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) g[k] = src[k * (f < 2 ? FG::XS : FG::YS)];
        C::add_face(f, g, R);
      }
      C::finish(A, c, gam, lam, R, L);
    } else {
      C::template rhs<true, XBC>(A, lds + sc, c, gx, gy, L, gam);
    }
    if (A.gamma) A.gamma[cell] = gam;
    double* dst = A.out + cell * NL;
    if (A.rhs_only) {
#pragma unroll
      for (int j = 0; j < NL; ++j) dst[j] = L[j];
    } else {
      double un[NL];
      if (comb) {
#pragma unroll
        for (int j = 0; j < NL; ++j) un[j] = A.un[cell * NL + j];
      }
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        double v = A.b * fma(A.dt, L[j], c[j]);
        if (comb) v = fma(A.a, un[j], v);
        dst[j] = v;
      }
    }
  }
}

// The fused stage kernel.  Grid: (ceil(nx/TX), ceil(ny/TY)), one tile each,
// in the XCD-aware order of xcd_tile.  XBC: the BC_RIEMANN exterior state
// compiled in (2D Burgers; launched for that exterior state only, since the
// checks cost every cell ~4 % of its instructions).
template <int DIM, int P, int FLUX, int MODE, int TX, int TY, bool XBC = false>
__global__ void __launch_bounds__(DIM == 2 ? TX * TY : TX) stage_kernel(const StageArgs A) {
  extern __shared__ double lds[];
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bx = tile % gridDim.x, by = tile / gridDim.x;
  stage_tile<DIM, P, FLUX, MODE, TX, TY, XBC && DIM == 2 && FLUX == FLUX_BURGERS>(A, lds, bx * TX,
                                                                                DIM == 2 ? by * TY : 0);
}

// Small meshes on 8 x 8 tiles (the linear and Burgers fluxes): four waves
// per tile.  With few tiles per compute unit (the library takes this kernel
// up to three), one-wave tiles leave SIMDs idle and every lane runs its
// cell's whole stage as one dependent chain; here the parts of the stage
// run side by side on the tile's four waves:
//   * wave 0 loads the tile (as stage_tile does) and evaluates the volume
//     terms and lambda_e of its 64 cells (residual without faces);
//   * wave 1 evaluates gamma_e of the same cells (their coefficients read
//     back from LDS), into LDS;
//   * waves 2 and 3 evaluate each of the tile's 144 faces once, into LDS,
//     as the shared-face phase of stage_tile does;
// then, after a barrier, wave 0 adds each cell's four faces in the order of
// the per-cell evaluation, finishes and stores: the same functions in the
// same order as stage_tile, so the same result bit for bit.
// XBC: the BC_RIEMANN exterior state compiled in (2D Burgers).
constexpr int kRoleThreads = 256;
__host__ __device__ inline int roles_lds_doubles(int nl, int n) {
  return tile_lds_doubles(2, nl, 8, 8) + face_lds_doubles(n, 8, 8) + 64;
}
// Face task i (< 144) of waves 2 and 3: axis and face index (face_slot's order)
__host__ __device__ inline void roles_face_task(int i, int& axis, int& e) {
  axis = i >= 72;
  e = axis ? i - 72 : i;
}
template <int P, int FLUX, int MODE, bool XBC>
__device__ inline void roles_tile(const StageArgs& A, double* lds, int ix0, int iy0) {
  constexpr int TX = 8, TY = 8;
  using G = TileGeom<2, TX, TY>;
  using C = Cell<2, P, FLUX, MODE, G::S, G::W>;
  using FG = FaceGeom<TX, TY>;
  constexpr int NL = C::NL, N = C::N, S = G::S;
  static_assert(FLUX == FLUX_LINADV || FLUX == FLUX_BURGERS, "the KPP flux has kpp_split_tile");
  static_assert(FG::NXF == 72 && FG::NYF == 72, "roles_face_task assumes 8 x 8 tiles");
  double* const fxl = lds + NL * S;      // x faces
  double* const fyl = fxl + N * FG::XS;  // y faces
  double* const gaml = fyl + N * FG::YS;  // gamma_e of the tile's cells
  const int nx = A.nx, ny = A.ny;
  const int t = threadIdx.x;
  const int lc = t & 63, w = t >> 6;
  int sc, gx, gy, hs, hgx, hgy;
  const bool halo = tile_slots<2, TX, TY>(lc, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
  const bool active = gx < nx && gy < ny;
  bool xbc = false;  // exterior slots from the exact solution (BC_RIEMANN)
  if constexpr (XBC) xbc = A.bc_kind == BC_RIEMANN;
  double c[NL];
  if (w == 0) {
    load_cell<2, NL>(A, gx, gy, c);
    if constexpr (XBC) {
      if (xbc) {
        C::riemann_slot(A, gx, gy, c);
        if (halo) {
          double v[NL];
          load_cell<2, NL>(A, hgx, hgy, v);
          C::riemann_slot(A, hgx, hgy, v);
#pragma unroll
          for (int j = 0; j < NL; ++j) lds[j * S + hs] = v[j];
        }
      }
    }
    if (!xbc && halo) load_slot<2, NL, S>(A, lds, hs, hgx, hgy);
#pragma unroll
    for (int j = 0; j < NL; ++j) lds[j * S + sc] = c[j];
  }
  tile_barrier();
  double R[NL], lam = 0.0;
  if (w == 0) {
    if (active) C::template residual<false, false>(A, lds + sc, c, gx, gy, R, lam);
  } else if (w == 1) {
    if (active) {
      double cc[NL];
#pragma unroll
      for (int j = 0; j < NL; ++j) cc[j] = lds[j * S + sc];
      gaml[lc] = C::template gamma_of<true>(A, lds + sc, cc, gx, gy);
    }
  } else {
    for (int i = t - 128; i < FG::NXF + FG::NYF; i += kRoleThreads - 128) {
      int axis, e;
      roles_face_task(i, axis, e);
      int fgx, fgy;
      const int lo = face_slot<TX, TY>(axis, e, ix0, iy0, fgx, fgy);
      const int hi = lo + (axis == 0 ? 1 : G::W);
      double tl[N], th[N], v[C::Q], g[N];
      C::template trace<false>(axis, [&](int q) { return lds[q * S + lo]; }, tl);
      C::template trace<true>(axis, [&](int q) { return lds[q * S + hi]; }, th);
      C::line_velocity(A, axis, axis == 0 ? fgy : fgx, v);
      bool xl = false, xh = false;
      if constexpr (XBC) {
        if (xbc) {
          const int l = axis == 0 ? fgx : fgy, n = axis == 0 ? nx : ny;
          xl = l == -1;
          xh = l == n - 1;
        }
      }
      C::template face_moments<XBC>(axis, tl, th, v, xl, xh, lds + (xl ? lo : hi), g);
      double* dst = axis == 0 ? fxl + e : fyl + e;
#pragma unroll
      for (int k = 0; k < N; ++k) dst[k * (axis == 0 ? FG::XS : FG::YS)] = g[k];
    }
  }
  tile_barrier();
  if (w != 0 || !active) return;
  const int lx = lc % TX, ly = lc / TX;
  const int ex = ly * (TX + 1) + lx, ey = ly * TX + lx;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double* src = f < 2 ? fxl + ex + (f & 1) : fyl + ey + (f & 1) * TX;
    double g[N];
#pragma unroll
    for (int k = 0; k < N; ++k) g[k] = src[k * (f < 2 ? FG::XS : FG::YS)];
    C::add_face(f, g, R);
  }
  double L[NL];
  C::finish(A, c, gaml[lc], lam, R, L);
  const size_t cell = (size_t)gy * nx + gx;
  if (A.gamma) A.gamma[cell] = gaml[lc];
  double* dst = A.out + cell * NL;
  if (A.rhs_only) {
#pragma unroll
    for (int j = 0; j < NL; ++j) dst[j] = L[j];
  } else {
    const bool comb = A.a != 0.0;
    double un[NL];
    if (comb) {
#pragma unroll
      for (int j = 0; j < NL; ++j) un[j] = A.un[cell * NL + j];
    }
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      double v = A.b * fma(A.dt, L[j], c[j]);
      if (comb) v = fma(A.a, un[j], v);
      dst[j] = v;
    }
  }
}

// Grid as for stage_kernel on 8 x 8 tiles, kRoleThreads threads.
template <int P, int FLUX, int MODE, bool XBC>
__global__ void __launch_bounds__(kRoleThreads) roles_kernel(const StageArgs A) {
  extern __shared__ double lds[];
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bx = tile % gridDim.x, by = tile / gridDim.x;
  roles_tile<P, FLUX, MODE, XBC && FLUX == FLUX_BURGERS>(A, lds, bx * 8, by * 8);
}

// The per-stage KPP kernel on 8 x 8 tiles.  The sine and cosine at every
// volume and face node dominate this stage, and a one-wave 8 x 8 tile per
// workgroup leaves most SIMDs idle on small meshes (a 128^2 mesh is 256
// tiles).  Here a tile has NTH / 64 waves (4, 8 or 16):
//   * wave 0 owns the 64 cells: it loads the tile into LDS as stage_tile
//     does, evaluates gamma_e (the sensor reads the tile only), and after
//     the node phase sums the volume and face integrals, finishes and
//     stores its cells;
//   * in the node phase the waves evaluate the node fluxes: (sin u, cos u)
//     at the Q^2 volume nodes of every cell and the LLF flux at the Q nodes
//     of every face of the tile (each face once), into LDS.  Wave 0 takes V0
//     rounds of volume nodes beside the sensor (split_v0); the other waves
//     take every face node, then the remaining volume nodes.
// u_h at a node, the face traces and the fluxes are computed by the same
// functions as in the per-cell path (xline/ynode, trace/face_node,
// llf_kpp), and wave 0 sums them in the same order (residual with VS = 64,
// face_sum, add_face), so the result is the same bit for bit.  The node
// tasks hold few registers, so they take the sine and cosine inline
// (sincos_inl: no call frame in scratch memory; 7.8 -> 6.3 us per stage at
// 128^2 P2, 17.1 -> 13.1 at 256^2).
template <int P, int MODE, int V0, int NTH>
__device__ inline void kpp_split_tile(const StageArgs& A, double* lds, int ix0, int iy0) {
  constexpr int TX = 8, TY = 8;
  using G = TileGeom<2, TX, TY>;
  using C = Cell<2, P, FLUX_KPP, MODE, G::S, G::W>;
  constexpr int NL = C::NL, N = C::N, Q = C::Q, S = G::S;
  constexpr int NV = 64 * Q * Q;  // volume node tasks
  constexpr int NFA = 72;         // faces per axis ((TX + 1) TY = TX (TY + 1))
  constexpr int NFN = 2 * NFA * Q;  // face node tasks
  static_assert(V0 >= 0 && V0 <= Q * Q, "wave 0 takes whole rounds of volume nodes");
  static_assert(G::W == 10 && FaceGeom<TX, TY>::NXF == NFA && FaceGeom<TX, TY>::NYF == NFA,
                "split_vol_task and split_face_task assume 8 x 8 tiles");
  constexpr int H0 = 64;  // the first thread of the node tasks
  static_assert(NTH % 64 == 0 && NTH > H0, "whole waves, at least one for the node tasks");
  double* const vol = lds + NL * S;
  double* const fnl = vol + 2 * Q * Q * 64;
  const int nx = A.nx, ny = A.ny;
  const int t = threadIdx.x;
  const bool owner = t < 64;

  int sc = 0, gx = 0, gy = 0;
  double c[NL];
  if (owner) {
    int hs, hgx, hgy;
    const bool halo = tile_slots<2, TX, TY>(t, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
    load_cell<2, NL>(A, gx, gy, c);
    if (halo) load_slot<2, NL, S>(A, lds, hs, hgx, hgy);
#pragma unroll
    for (int j = 0; j < NL; ++j) lds[j * S + sc] = c[j];
  }
  tile_barrier();
  auto vol_node = [&](int v) {
    int slot, qx, qy;
    const int o = split_vol_task(v, Q, slot, qx, qy);
    double s1[N];
    C::xline([&](int j) { return lds[j * S + slot]; }, qx, s1);
    double Fx, Fy;
    sincos_inl(C::ynode(s1, qy), &Fx, &Fy);
    vol[o] = Fx;
    vol[o + Q * Q * 64] = Fy;
  };
  const bool active = owner && gx < nx && gy < ny;
  double gam = 0.0;
  if (owner) {
    if (active) gam = C::template gamma_of<true>(A, lds + sc, c, gx, gy);
    for (int k = 0; k < V0; ++k) vol_node(k * 64 + t);
  } else {
    const int u = t - H0;
    for (int i = u; i < NFN; i += NTH - H0) {
      int axis, r, e;
      const int o = split_face_task(i, Q, axis, r, e);
      int fgx, fgy;
      const int lo = face_slot<TX, TY>(axis, e, ix0, iy0, fgx, fgy);
      const int hi = lo + (axis == 0 ? 1 : G::W);
      double tl[N], th[N];
      C::template trace<false>(axis, [&](int q) { return lds[q * S + lo]; }, tl);
      C::template trace<true>(axis, [&](int q) { return lds[q * S + hi]; }, th);
      double ul, uh;
      C::face_node(tl, th, r, ul, uh);
      fnl[o] = C::template llf_kpp<true>(axis, ul, uh);
    }
    for (int v = V0 * 64 + u; v < NV; v += NTH - H0) vol_node(v);
  }
  tile_barrier();
  if (!active) return;
  double R[NL], lam;
  const int lc = t;
  C::template residual<false, false, 64>(A, lds + sc, c, gx, gy, R, lam, vol + lc);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int axis = f >> 1;
    const int e = split_cell_face(lc, f);
    double H[Q], g[N];
#pragma unroll
    for (int r = 0; r < Q; ++r) H[r] = fnl[(axis * Q + r) * NFA + e];
    C::face_sum(H, g);
    C::add_face(f, g, R);
  }
  double L[NL];
  C::finish(A, c, gam, lam, R, L);
  const size_t cell = (size_t)gy * nx + gx;
  if (A.gamma) A.gamma[cell] = gam;
  double* dst = A.out + cell * NL;
  if (A.rhs_only) {
#pragma unroll
    for (int j = 0; j < NL; ++j) dst[j] = L[j];
  } else {
    const bool comb = A.a != 0.0;
    double un[NL];
    if (comb) {
#pragma unroll
      for (int j = 0; j < NL; ++j) un[j] = A.un[cell * NL + j];
    }
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      double v = A.b * fma(A.dt, L[j], c[j]);
      if (comb) v = fma(A.a, un[j], v);
      dst[j] = v;
    }
  }
}

// Volume node rounds of wave 0 in kpp_split_tile with nth threads: Q^2 / 2
// at four waves, Q^2 / 8 at eight, Q^2 / 16 at sixteen (measured at p = 2
// with the sensor, per stage: four waves 7.24 us at 128^2 and 12.9 at 256^2
// against 7.4-7.8 and 12.9-13.4 for 0-10 rounds; eight waves 8.42 at 176^2
// against 8.49-8.73; sixteen 6.07 at 128^2 against 6.25-6.36)
__host__ __device__ constexpr int split_v0(int p, int nth) {
  return (p + 2) * (p + 2) / (nth <= 256 ? 2 : nth <= 512 ? 8 : 16);
}

// Waves per tile of kpp_split_kernel for a mesh of `tiles` 8x8 tiles on
// `cus` compute units: sixteen while every tile has a compute unit of its
// own, eight up to two tiles per compute unit, else four (more workgroups
// then share each compute unit); at most what the degree's registers allow
// without spilling (split_max_waves: 128 VGPRs at sixteen waves, 256 at
// eight; p = 3 needs ~200, p = 4 ~256)
__host__ __device__ constexpr int split_max_waves(int p) { return p <= 2 ? 16 : p == 3 ? 8 : 4; }
__host__ __device__ constexpr int split_waves(long long tiles, int cus, int p) {
  const int w = tiles <= cus ? 16 : tiles <= 2LL * cus ? 8 : 4;
  return w < split_max_waves(p) ? w : split_max_waves(p);
}

// Grid as for stage_kernel on 8 x 8 tiles, NTH threads.
template <int P, int MODE, int NTH>
__global__ void __launch_bounds__(NTH) kpp_split_kernel(const StageArgs A) {
  extern __shared__ double lds[];
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bx = tile % gridDim.x, by = tile / gridDim.x;
  kpp_split_tile<P, MODE, split_v0(P, NTH), NTH>(A, lds, bx * 8, by * 8);
}

// Branch records of the stage input (Cell::branches) of every cell, folded
// into sig[k * cells + cell] (k = 0 sensor, 1 wave speed lambda_e, 2 LLF):
// the tile is loaded as in stage_tile's general path; nothing is written but
// the records.  Grid as for stage_kernel.
template <int DIM, int P, int FLUX, int MODE, int TX, int TY>
__global__ void __launch_bounds__(DIM == 2 ? TX * TY : TX) signature_kernel(const StageArgs A, uint32_t* sig) {
  extern __shared__ double lds[];
  using G = TileGeom<DIM, TX, TY>;
  using C = Cell<DIM, P, FLUX, MODE, G::S, G::W>;
  constexpr int NL = C::NL;
  constexpr int S = G::S;
  const int ix0 = blockIdx.x * TX, iy0 = DIM == 2 ? blockIdx.y * TY : 0;
  const int nx = A.nx, ny = DIM == 2 ? A.ny : 1;
  const int t = threadIdx.x;
  int sc, gx, gy, hs, hgx, hgy;
  const bool halo = tile_slots<DIM, TX, TY>(t, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
  double c[NL];
  load_cell<DIM, NL>(A, gx, gy, c);
  if (halo) load_slot<DIM, NL, S>(A, lds, hs, hgx, hgy);
#pragma unroll
  for (int j = 0; j < NL; ++j) lds[j * S + sc] = c[j];
  tile_barrier();
  if (gx < nx && gy < ny) {
    const size_t cell = (size_t)gy * nx + gx, ncells = (size_t)nx * ny;
    const double gam = C::template gamma_of<true>(A, lds + sc, c, gx, gy);
    uint32_t v[3];
    C::branches(A, lds + sc, c, gam, v);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint32_t h = sig[k * ncells + cell];
      sig[k * ncells + cell] = ((h << 7) | (h >> 25)) ^ v[k];
    }
  }
}

// ---------------------------------------------------------------------------
// Fused SSP-RK3 step: the three stages of eq. (ssp) in one launch.  A tile of
// TX x TY cells (TY = 1 in 1D) loads U^n on itself and three rings of cells
// around it (tile A); stage 1 evaluates U^(1) on the tile and two rings (tile
// B), stage 2 U^(2) on the tile and one ring (tile C), stage 3 U^(n+1) on the
// tile, straight to HBM.  Every cell value of every stage is computed with
// the same per-cell arithmetic as the per-stage kernel, so the result is the
// same bit for bit; the rings are recomputed by each tile that needs them.
// Slots outside a non-periodic boundary hold the exterior state in every
// stage, as in the per-stage kernel.
// ---------------------------------------------------------------------------
template <int DIM, int TX, int TY>
struct StepGeom {
  static constexpr int R = DIM == 2 ? TY : 1;
  // tile with k rings: width, rows, slots, plane stride (odd)
  template <int K>
  struct T {
    static constexpr int W = TX + 2 * K;
    static constexpr int H = DIM == 2 ? TY + 2 * K : 1;
    static constexpr int N = W * H;
    static constexpr int S = N | 1;
  };
  using A = T<3>;
  using B = T<2>;
  using C = T<1>;
  static constexpr int NT = DIM == 2 ? 2 * TX * TY : TX + 64;  // threads (= step_threads)
};

__host__ __device__ constexpr int step_threads(int dim, int tx, int ty) { return dim == 2 ? 2 * tx * ty : tx + 64; }

__host__ __device__ inline int step_lds_doubles(int dim, int nl, int tx, int ty) {
  int tot = 0;
  for (int k = 1; k <= 3; ++k) {
    const int w = tx + 2 * k, h = dim == 2 ? ty + 2 * k : 1;
    tot += (w * h) | 1;
  }
  return nl * tot + step_threads(dim, tx, ty) / 2;  // + the gamma exchange of split stages
}

// A stage of the fused step whose output tile has at most half as many
// cells as the workgroup has threads leaves waves idle (stage 3 of a 16x16
// tile: 256 cells, 512 threads).  Such a stage splits cells over two
// threads: one evaluates gamma_e, the other the residual, then (after a
// barrier) the dissipation, mass inverse and RK combination.  The first
// split_full(n, nt) cells (a multiple of 64) are evaluated whole by one
// thread each; the rest are split, each role on whole waves, so that no wave
// holds two roles.  n when nothing splits: then every thread takes whole
// cells, as in the per-stage kernel.
__host__ __device__ constexpr int split_full(int n, int nt) {
  for (int f = 0; f <= nt / 2 && f < n; f += 64) {
    const int ws = (n - f + 63) / 64;
    if (64 * (f / 64 + 2 * ws) <= nt) return f;
  }
  return n;
}

// Role of thread t in a stage of n output cells and nt threads when the
// stage splits (split_full(n, nt) < n): 0 the whole cell o, 1 gamma of cell o,
// 2 the rest of cell o; o >= n: no cell.  The split cells' gamma goes to slot
// o - split_full(n, nt) of the exchange buffer (at most nt / 2 slots).
__host__ __device__ constexpr void split_role(int t, int n, int nt, int& role, int& o) {
  const int f = split_full(n, nt), ws = (n - f + 63) / 64;
  role = t < f ? 0 : (t < f + 64 * ws ? 1 : 2);
  o = role == 2 ? t - 64 * ws : t;
}

// Mesh cell of coordinates (gx, gy) before wrapping, any distance outside the
// mesh: wrapped coordinates on periodic axes; false outside a non-periodic
// boundary.  (In 1D the row is 0.)
template <int DIM>
__host__ __device__ inline bool step_cell(const StageArgs& A, int gx, int gy, int& wx, int& wy) {
  const int nx = A.nx, ny = DIM == 2 ? A.ny : 1;
  if (DIM == 1) gy = 0;
  if (gx < 0 || gx >= nx) {
    if (!A.per_x) return false;
    gx %= nx;
    if (gx < 0) gx += nx;
  }
  if (DIM == 2 && (gy < 0 || gy >= ny)) {
    if (!A.per_y) return false;
    gy %= ny;
    if (gy < 0) gy += ny;
  }
  wx = gx;
  wy = gy;
  return true;
}

// Output slot o of the stage whose output tile has KO rings: its local
// coordinates, the slot of the same cell in the input tile (KO + 1 rings) and
// in tile A (3 rings), and its mesh coordinates before wrapping.
template <int DIM, int TX, int TY, int KO>
__host__ __device__ inline void step_slot(int o, int ix0, int iy0, int& islot, int& aslot, int& gx, int& gy) {
  using G = StepGeom<DIM, TX, TY>;
  using TO = typename G::template T<KO>;
  using TI = typename G::template T<KO + 1>;
  const int ox = o % TO::W, oy = o / TO::W;
  gx = ix0 - KO + ox;
  gy = DIM == 2 ? iy0 - KO + oy : 0;
  if constexpr (DIM == 2) {
    islot = (oy + 1) * TI::W + ox + 1;
    aslot = (oy + 3 - KO) * G::A::W + ox + 3 - KO;
  } else {
    islot = ox + 1;
    aslot = ox + 3 - KO;
  }
}

// One stage of the fused step: for every cell of the output tile (KO rings)
// evaluate the operator on the input tile (KO + 1 rings) and combine
// a U^n + b (U^(k-1) + dt L); KO = 0 writes the tile's mesh cells to HBM.
template <int DIM, int P, int FLUX, int MODE, int TX, int TY, int KO>
__device__ inline void step_stage(const StageArgs& A, const double* tin, const double* ta, double* tout, int ix0,
                                  int iy0, double a, double b, double* gx_lds) {
  using G = StepGeom<DIM, TX, TY>;
  using TI = typename G::template T<KO + 1>;
  using TO = typename G::template T<KO>;
  using C = Cell<DIM, P, FLUX, MODE, TI::S, TI::W>;
  constexpr int NL = C::NL;
  // 2D: LDS allows one workgroup per CU, so up to P = 2 the registers freed
  // by the scheduling barrier do not raise the occupancy
  constexpr bool SB = DIM == 1 || P > 2;
  constexpr int NF_ = split_full(TO::N, G::NT);  // cells evaluated whole
  constexpr bool SPLIT = (MODE == MODE_WENO || MODE == MODE_ZHAO) && NF_ < TO::N;
  const int nx = A.nx, ny = DIM == 2 ? A.ny : 1;

  // RK combination of cell o and its store (to the output tile, or to HBM)
  auto store = [&](int o, int aslot, int wx, int wy, const double (&c)[NL], const double (&L)[NL]) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      double v = b * fma(A.dt, L[j], c[j]);
      if (a != 0.0) v = fma(a, ta[j * G::A::S + aslot], v);
      if constexpr (KO == 0)
        A.out[((size_t)wy * nx + wx) * NL + j] = v;
      else
        tout[j * TO::S + o] = v;
    }
  };
  // the slots of cell o; false if it has no equation (past a ragged edge, or
  // outside a non-periodic boundary, where `ext` writes the exterior state)
  auto locate = [&](int o, bool ext, int& islot, int& aslot, int& wx, int& wy) {
    int gx, gy;
    step_slot<DIM, TX, TY, KO>(o, ix0, iy0, islot, aslot, gx, gy);
    if constexpr (KO == 0) {
      if (gx >= nx || gy >= ny) return false;
    }
    if (!step_cell<DIM>(A, gx, gy, wx, wy)) {
      if (ext) {
#pragma unroll
        for (int j = 0; j < NL; ++j) tout[j * TO::S + o] = j == 0 ? A.bc : 0.0;
      }
      return false;
    }
    return true;
  };

  if constexpr (!SPLIT) {
#pragma unroll 1
    for (int o = threadIdx.x; o < TO::N; o += G::NT) {
      int islot, aslot, wx, wy;
      if (!locate(o, true, islot, aslot, wx, wy)) continue;
      double c[NL], L[NL], gam;
#pragma unroll
      for (int j = 0; j < NL; ++j) c[j] = tin[j * TI::S + islot];
      C::template rhs<SB>(A, tin + islot, c, wx, wy, L, gam);
      store(o, aslot, wx, wy, c, L);
    }
  } else {
    // roles by thread: [0, NF_) whole cells; the next waves gamma of the split
    // cells; the waves after those the rest of the same cells
    int role, o;
    split_role(threadIdx.x, TO::N, G::NT, role, o);
    int islot = 0, aslot = 0, wx = 0, wy = 0;
    const bool valid = o < TO::N && locate(o, role != 1, islot, aslot, wx, wy);
    double c[NL], R[NL], lam = 0.0;
    if (valid) {
#pragma unroll
      for (int j = 0; j < NL; ++j) c[j] = tin[j * TI::S + islot];
      if (role == 0) {
        double L[NL], gam;
        C::template rhs<SB>(A, tin + islot, c, wx, wy, L, gam);
        store(o, aslot, wx, wy, c, L);
      } else if (role == 1) {
        gx_lds[o - NF_] = C::template gamma_of<SB>(A, tin + islot, c, wx, wy);
      } else {
        C::residual(A, tin + islot, c, wx, wy, R, lam);
      }
    }
    tile_barrier();  // every thread: gamma of the split cells is in LDS
    if (valid && role == 2) {
      double L[NL];
      C::finish(A, c, gx_lds[o - NF_], lam, R, L);
      store(o, aslot, wx, wy, c, L);
    }
  }
}

// The fused step kernel.  Grid: (ceil(nx/TX), ceil(ny/TY)), tiles in the
// order of xcd_tile; StepGeom::NT threads; LDS: step_lds_doubles.  A.uin = U^n, A.out = U^(n+1), two
// different arrays (tiles run concurrently and read U^n of their neighbours).
template <int DIM, int P, int FLUX, int MODE, int TX, int TY>
__global__ void __launch_bounds__(step_threads(DIM, TX, TY)) step_kernel(const StageArgs A) {
  using G = StepGeom<DIM, TX, TY>;
  constexpr int NL = DIM == 1 ? P + 1 : (P + 1) * (P + 1);
  extern __shared__ double lds[];
  double* ta = lds;
  double* tb = ta + NL * G::A::S;
  double* tc = tb + NL * G::B::S;
  double* gx = tc + NL * G::C::S;  // gamma of the split cells of a stage (NT / 2)
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int ix0 = (tile % gridDim.x) * TX, iy0 = DIM == 2 ? (tile / gridDim.x) * TY : 0;
  // U^n on the tile and three rings
#pragma unroll 1
  for (int o = threadIdx.x; o < G::A::N; o += G::NT) {
    const int ox = o % G::A::W, oy = o / G::A::W;
    int wx, wy;
    double v[NL];
    if (step_cell<DIM>(A, ix0 - 3 + ox, DIM == 2 ? iy0 - 3 + oy : 0, wx, wy)) {
      const double* src = A.uin + ((size_t)wy * A.nx + wx) * NL;
#pragma unroll
      for (int j = 0; j < NL; ++j) v[j] = src[j];
    } else {
#pragma unroll
      for (int j = 0; j < NL; ++j) v[j] = j == 0 ? A.bc : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NL; ++j) ta[j * G::A::S + o] = v[j];
  }
  tile_barrier();
  step_stage<DIM, P, FLUX, MODE, TX, TY, 2>(A, ta, ta, tb, ix0, iy0, 0.0, 1.0, gx);
  tile_barrier();
  step_stage<DIM, P, FLUX, MODE, TX, TY, 1>(A, tb, ta, tc, ix0, iy0, 0.75, 0.25, gx);
  tile_barrier();
  step_stage<DIM, P, FLUX, MODE, TX, TY, 0>(A, tc, ta, nullptr, ix0, iy0, 1.0 / 3.0, 2.0 / 3.0, gx);
}

// ---------------------------------------------------------------------------
// Batched stage: many independent problems of one kernel class (dimension,
// degree, flux, mode, tile) in one persistent launch.  Each workgroup walks
// the tile list with a grid stride (the list order is the schedule); a tile
// names its problem, whose entry holds the problem's parameters and the
// offset of its state in the batch arena.
// ---------------------------------------------------------------------------
struct BatchProblem {
  long long off;   // first double of the problem's state in the arena
  StageArgs args;  // mesh, flux, sensor parameters and dt (pointers unused)
};
struct BatchTile {
  int prob, ix0, iy0, pad;
};
struct BatchStageArgs {
  const BatchProblem* probs;
  const BatchTile* tiles;
  int ntiles;
  const double* uin;
  const double* un;
  double* out;
  double a, b;
};

template <int DIM, int P, int FLUX, int MODE, int TX, int TY>
__device__ inline void batch_tile(const BatchStageArgs& B, double* lds, int k) {
  const BatchTile tl = B.tiles[k];
  StageArgs A = B.probs[tl.prob].args;
  const long long off = B.probs[tl.prob].off;
  A.uin = B.uin + off;
  A.un = B.un + off;
  A.out = B.out + off;
  A.gamma = nullptr;
  A.a = B.a;
  A.b = B.b;
  A.rhs_only = 0;
  stage_tile<DIM, P, FLUX, MODE, TX, TY>(A, lds, tl.ix0, tl.iy0);
}

// ONE: one workgroup per tile (grid = the number of tiles), no tile loop;
// a loop makes the compiler keep the arithmetic's loop-invariant values in
// registers across tiles (tens of VGPRs more), which this form avoids.
template <int DIM, int P, int FLUX, int MODE, int TX, int TY, bool ONE = false>
__global__ void __launch_bounds__(DIM == 2 ? TX * TY : TX) batch_stage_kernel(const BatchStageArgs B) {
  extern __shared__ double lds[];
  if constexpr (ONE) {
    if ((int)blockIdx.x < B.ntiles) batch_tile<DIM, P, FLUX, MODE, TX, TY>(B, lds, blockIdx.x);
  } else {
    for (int k = blockIdx.x; k < B.ntiles; k += gridDim.x) {
      batch_tile<DIM, P, FLUX, MODE, TX, TY>(B, lds, k);
      tile_barrier();  // the next tile reuses LDS
    }
  }
}

// ---------------------------------------------------------------------------
// L2 projection of nodal values: c_j = Mhat_j^{-1} sum_q w_q phi_j(x_q) u_q,
// (p+2)^d Gauss nodes per cell, x fastest.  One thread per cell.
// ---------------------------------------------------------------------------
template <int DIM, int P>
__global__ void __launch_bounds__(256) project_kernel(const double* __restrict__ u, double* __restrict__ U,
                                                       long long ncells) {
  constexpr int N = P + 1, QP = P + 2;
  constexpr int NL = DIM == 1 ? N : N * N;
  constexpr int NQ = DIM == 1 ? QP : QP * QP;
  constexpr NodeTab<P, QP> nd = make_nodes<P, QP>();
  constexpr DegTab<P> dg = make_deg<P>();
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncells) return;
  const double* ue = u + e * NQ;
  double c[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) c[j] = 0.0;
  if constexpr (DIM == 1) {
#pragma unroll
    for (int q = 0; q < QP; ++q) {
      const double wu = nd.w[q] * ue[q];
#pragma unroll
      for (int a = 0; a < N; ++a) c[a] = fma(nd.L[a][q], wu, c[a]);
    }
#pragma unroll
    for (int a = 0; a < N; ++a) U[e * NL + a] = dg.minv[a] * c[a];
  } else {
#pragma unroll
    for (int qy = 0; qy < QP; ++qy) {
      double s1[N];
#pragma unroll
      for (int a = 0; a < N; ++a) s1[a] = 0.0;
#pragma unroll
      for (int qx = 0; qx < QP; ++qx) {
        const double wu = nd.w[qx] * ue[qx + QP * qy];
#pragma unroll
        for (int a = 0; a < N; ++a) s1[a] = fma(nd.L[a][qx], wu, s1[a]);
      }
#pragma unroll
      for (int b = 0; b < N; ++b)
#pragma unroll
        for (int a = 0; a < N; ++a) c[a + N * b] = fma(nd.w[qy] * nd.L[b][qy], s1[a], c[a + N * b]);
    }
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
      for (int a = 0; a < N; ++a) U[e * NL + a + N * b] = dg.minv[a] * dg.minv[b] * c[a + N * b];
  }
}

// lambda_e per cell, reduced to one maximum per block (for the stable step)
template <int DIM, int P, int FLUX>
__global__ void __launch_bounds__(256) lambda_kernel(const StageArgs A, const double* __restrict__ U,
                                                      double* __restrict__ block_max) {
  using TB = Tables<DIM, P, FLUX>;
  constexpr int N = P + 1, NL = TB::NL, Q = TB::Q;
  __shared__ double red[256];
  const long long ncells = (long long)A.nx * (DIM == 2 ? A.ny : 1);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double lam = 0.0;
  if (e < ncells) {
    const int ix = (int)(e % A.nx), iy = (int)(e / A.nx);
    const double hh = 0.5 * A.h;
    if (A.lam_over > 0.0) {
      lam = A.lam_over;
    } else if constexpr (FLUX == FLUX_KPP) {
      lam = 1.0;  // ||(cos u, -sin u)||_2
    } else if constexpr (FLUX == FLUX_LINADV) {
      if constexpr (DIM == 1) {
        lam = fabs(A.vx);
      } else {
        const double xc = A.x0 + (ix + 0.5) * A.h, yc = A.y0 + (iy + 0.5) * A.h;
        double m = 0.0;
        for (int qx = 0; qx < Q; ++qx)
          for (int qy = 0; qy < Q; ++qy) {
            const double vx = A.vx - A.omega * (yc + hh * TB::nd.x[qy] - A.cy);
            const double vy = A.vy + A.omega * (xc + hh * TB::nd.x[qx] - A.cx);
            m = fmax(m, vx * vx + vy * vy);
          }
        lam = sqrt(m);
      }
    } else {
      double m = 0.0;
      const double* c = U + e * NL;
      if constexpr (DIM == 1) {
        for (int q = 0; q < Q; ++q) {
          double u = 0.0;
          for (int a = 0; a < N; ++a) u = fma(c[a], TB::nd.L[a][q], u);
          m = fmax(m, fabs(u));
        }
      } else {
        for (int qx = 0; qx < Q; ++qx)
          for (int qy = 0; qy < Q; ++qy) {
            double u = 0.0;
            for (int b = 0; b < N; ++b)
              for (int a = 0; a < N; ++a) u = fma(c[a + N * b], TB::nd.L[a][qx] * TB::nd.L[b][qy], u);
            m = fmax(m, fabs(u));
          }
      }
      lam = A.anorm * m;
    }
  }
  red[threadIdx.x] = lam;
  tile_barrier();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    tile_barrier();
  }
  if (threadIdx.x == 0) block_max[blockIdx.x] = red[0];
}

}  // namespace dgk
