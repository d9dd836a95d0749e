// Device code: the discrete adjoint of the stabilised DG operator.
//
// For a cotangent v of dU/dt = L(U) the kernels compute J(U)^T v, the
// gradient of <v, L(U)> with respect to U, in gather form (each cell
// assembles its own gradient; no atomics).  With g_e = (2/h) Mhat^-1 v_e,
//   <v, L(U)> = sum_e g_e . ( vol_e - face_e - (gamma_e lambda_e / p) Khat c_e )
// and the gradient with respect to c_e collects
//   * volume:  sum_q w_q (grad g_e . F'(u_q)) phi(q)
//   * faces:   - sum_r w_r (g_e^- - g_nb^+) dH/du^- phi(r) over the cell's faces
//              (conservation, H_nb = -H_e, folds the neighbour's equation in)
//   * dissipation: - (gamma lambda / p) Khat g_e, and through lambda_e
//   * sensor: gamma_e depends on c_e and on the face neighbours (candidates).
// The sensor part needs the neighbours' sensor state, so it runs as a
// separate pass: pass A reverses each cell's sensor with the seed
//   gamma_bar_e = -(lambda_e / p) g_e . Khat c_e
// and stores a compact record (dbar = d<.>/d(c - c*), omega_l, beta_bar_l,
// gamma_e); pass B gathers the records of the cell and its face neighbours,
// rebuilding each candidate cotangent from the cell's own coefficients.
#pragma once

#include "dg_kernels.hpp"

namespace dgk {

struct AdjArgs {
  StageArgs s;        // geometry, flux, sensor parameters; s.uin = U (state)
  const double* v;    // cotangent of L(U), [cells][NL]
  double* z;          // sensor records, field-major: field k of cell e at z[k * cells + e]
  double* out;        // pass B: out = alpha v + beta J^T v + g1 X + g2 Y
  const double* X;    // optional [cells][NL]
  const double* Y;    // optional [cells][NL]
  double alpha, beta, g1, g2;
  const double* unext;  // pass B + A launch: the state whose sensor is reversed next
  double* znext;        // pass B + A launch: its records (not the buffer z)
};

// Doubles per cell in the sensor record (the layout is ZRec's).
__host__ __device__ constexpr int zrec_doubles(int dim, int nl) { return nl + 2 * (2 * dim + 1) + 1; }

template <int DIM, int P>
struct ZRec {
  static constexpr int NL = DIM == 1 ? P + 1 : (P + 1) * (P + 1);
  static constexpr int NF = 2 * DIM;
  // fields dbar[NL], omega[NF+1], beta_bar[NF+1], gamma; stored field-major
  // (one plane of cells per field) so that a wave's stores and its reads of a
  // neighbour's field are contiguous
  static constexpr int OM = NL, BB = NL + NF + 1, GA = NL + 2 * (NF + 1);
  static constexpr int SIZE = GA + 1;
  static_assert(SIZE == zrec_doubles(DIM, NL), "record layout");
};

template <int DIM, int P, int FLUX, int MODE, int S, int W>
struct AdjCell {
  using C = Cell<DIM, P, FLUX, MODE, S, W>;
  using TB = typename C::TB;
  using Z = ZRec<DIM, P>;
  static constexpr int N = P + 1;
  static constexpr int NL = C::NL;
  static constexpr int Q = C::Q;
  static constexpr int NF = 2 * DIM;

  // o = B v (sensor quadratic form as a matrix; compile-time sparse)
  __device__ static inline void bvec(const double (&v)[NL], double (&o)[NL]) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 1; j < NL; ++j)
        if (TB::sn.B[i][j] != 0.0) t = fma(TB::sn.B[i][j], v[j], t);
      o[i] = t;
    }
  }

  // candidate of direction F built from coefficients in registers
  template <int F>
  __device__ static inline void cand_regs(const double (&cn)[NL], double (&cd)[NL]) {
    constexpr int si = F & 1;
#pragma unroll
    for (int j = 0; j < NL; ++j) cd[j] = 0.0;
    if constexpr (DIM == 1 || F < 2) {
      constexpr int R = DIM == 1 ? 1 : N;
#pragma unroll
      for (int e = 0; e < R; ++e)
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int c = 0; c <= a; ++c)
            if (TB::dg.T[si][a][c] != 0.0 && (c + N * e) != 0)
              cd[c + N * e] = fma(TB::dg.T[si][a][c], cn[a + N * e], cd[c + N * e]);
    } else {
#pragma unroll
      for (int e = 0; e < N; ++e)
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int c = 0; c <= e; ++c)
            if (TB::dg.T[si][e][c] != 0.0 && (a + N * c) != 0)
              cd[a + N * c] = fma(TB::dg.T[si][e][c], cn[a + N * e], cd[a + N * c]);
    }
  }

  // acc += (candidate map of direction F)^T cb
  template <int F>
  __device__ static inline void cand_T(const double (&cb)[NL], double (&acc)[NL]) {
    constexpr int si = F & 1;
    if constexpr (DIM == 1 || F < 2) {
      constexpr int R = DIM == 1 ? 1 : N;
#pragma unroll
      for (int e = 0; e < R; ++e)
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int c = 0; c <= a; ++c)
            if (TB::dg.T[si][a][c] != 0.0 && (c + N * e) != 0)
              acc[a + N * e] = fma(TB::dg.T[si][a][c], cb[c + N * e], acc[a + N * e]);
    } else {
#pragma unroll
      for (int e = 0; e < N; ++e)
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int c = 0; c <= e; ++c)
            if (TB::dg.T[si][e][c] != 0.0 && (a + N * c) != 0)
              acc[a + N * e] = fma(TB::dg.T[si][e][c], cb[a + N * c], acc[a + N * e]);
    }
  }

  // g = (2/h) Mhat^-1 v
  __device__ static inline void scale_g(const StageArgs& A, const double (&v)[NL], double (&g)[NL]) {
    const double g2h = A.g2h;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int a = j % N, bb = j / N;
      g[j] = (g2h * (DIM == 1 ? TB::dg.minv[j] : TB::dg.minv[a] * TB::dg.minv[bb])) * v[j];
    }
  }

  // kappa = g . Khat c
  __device__ static inline double kappa(const double (&g)[NL], const double (&c)[NL]) {
    double k = 0.0;
    if constexpr (DIM == 1) {
#pragma unroll
      for (int a = 0; a < N; ++a)
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2)
          if (TB::dg.S[a][a2] != 0.0) k = fma(TB::dg.S[a][a2] * g[a], c[a2], k);
    } else {
#pragma unroll
      for (int bb = 0; bb < N; ++bb)
#pragma unroll
        for (int a = 0; a < N; ++a) {
#pragma unroll
          for (int a2 = 0; a2 < N; ++a2)
            if (TB::dg.S[a][a2] != 0.0) k = fma(TB::dg.S[a][a2] * TB::dg.mhat[bb] * g[a + N * bb], c[a2 + N * bb], k);
#pragma unroll
          for (int b2 = 0; b2 < N; ++b2)
            if (TB::dg.S[bb][b2] != 0.0) k = fma(TB::dg.S[bb][b2] * TB::dg.mhat[a] * g[a + N * bb], c[a + N * b2], k);
        }
    }
    return k;
  }

  // o -= s Khat g
  __device__ static inline void sub_khat(double s, const double (&g)[NL], double (&o)[NL]) {
    if constexpr (DIM == 1) {
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double t = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2)
          if (TB::dg.S[a][a2] != 0.0) t = fma(TB::dg.S[a][a2], g[a2], t);
        o[a] = fma(-s, t, o[a]);
      }
    } else {
#pragma unroll
      for (int bb = 0; bb < N; ++bb)
#pragma unroll
        for (int a = 0; a < N; ++a) {
          double t = 0.0;
#pragma unroll
          for (int a2 = 0; a2 < N; ++a2)
            if (TB::dg.S[a][a2] != 0.0) t = fma(TB::dg.S[a][a2] * TB::dg.mhat[bb], g[a2 + N * bb], t);
#pragma unroll
          for (int b2 = 0; b2 < N; ++b2)
            if (TB::dg.S[bb][b2] != 0.0) t = fma(TB::dg.S[bb][b2] * TB::dg.mhat[a], g[a + N * b2], t);
          o[a + N * bb] = fma(-s, t, o[a + N * bb]);
        }
    }
  }

  // lambda_e and, for the Burgers flux, the node where |u| is largest
  __device__ static inline double lambda(const StageArgs& A, const double (&c)[NL], double xc, double yc,
                                         int& qmax, double& umax_signed) {
    qmax = -1;
    umax_signed = 0.0;
    const double hh = 0.5 * A.h;
    if constexpr (FLUX == FLUX_LINADV) {
      if constexpr (DIM == 1) {
        return fabs(A.vx);
      } else {
        double mx = 0.0, my = 0.0;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const double vx = A.vx - A.omega * (fma(hh, TB::nd.x[k], yc) - A.cy);
          const double vy = A.vy + A.omega * (fma(hh, TB::nd.x[k], xc) - A.cx);
          mx = fmax(mx, vx * vx);
          my = fmax(my, vy * vy);
        }
        return sqrt_pos(mx + my);
      }
    } else {
      double m = 0.0;
      if constexpr (DIM == 1) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          double u = c[0];
#pragma unroll
          for (int a = 1; a < N; ++a) u = fma(c[a], TB::nd.L[a][q], u);
          if (fabs(u) > m) {
            m = fabs(u);
            qmax = q;
            umax_signed = u;
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
            if (fabs(u) > m) {
              m = fabs(u);
              qmax = qx + Q * qy;
              umax_signed = u;
            }
          }
        }
      }
      return A.anorm * m;
    }
  }

  // phi_j at volume node qmax (select chains, no dynamic table indexing)
  __device__ static inline void basis_at(int qmax, double (&phi)[NL]) {
    if constexpr (DIM == 1) {
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) t = q == qmax ? TB::nd.L[a][q] : t;
        phi[a] = t;
      }
    } else {
      const int qx = qmax % Q, qy = qmax / Q;
      double lx[N], ly[N];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double tx = 0.0, ty = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          tx = q == qx ? TB::nd.L[a][q] : tx;
          ty = q == qy ? TB::nd.L[a][q] : ty;
        }
        lx[a] = tx;
        ly[a] = ty;
      }
#pragma unroll
      for (int bb = 0; bb < N; ++bb)
#pragma unroll
        for (int a = 0; a < N; ++a) phi[a + N * bb] = lx[a] * ly[bb];
    }
  }

  // Pass A: the sensor of one cell, forward and reverse, seeded with
  // gamma_bar = -(lambda / p) g . Khat c.  Writes the cell's record.
  // SB: scheduling barriers between the candidates (one candidate live at a
  // time; off where the kernel's register budget is set by other work).
  template <bool SB>
  __device__ static inline void sensor_adjoint(const StageArgs& A, const double* b, const double (&c)[NL], int ix,
                                               int iy, const double (&v)[NL], double* zrec, size_t zs) {
    bool has[NF];
    has[0] = A.per_x || ix > 0;
    has[1] = A.per_x || ix < A.nx - 1;
    if constexpr (DIM == 2) {
      has[2] = A.per_y || iy > 0;
      has[3] = A.per_y || iy < A.ny - 1;
    }
    // forward
    double beta[NF + 1], al[NF + 1];
    double cd[NL];
    beta[0] = C::qform(c);
    int m = 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      C::template cand_any<0>(f, b, cd);
      beta[f + 1] = C::qform(cd);
      al[f + 1] = has[f] ? A.wnb * C::weight(A, beta[f + 1]) : 0.0;
      m += has[f];
      if constexpr (SB) __builtin_amdgcn_sched_barrier(0);
    }
    al[0] = (1.0 - m * A.wnb) * C::weight(A, beta[0]);
    double ssum = 0.0;
#pragma unroll
    for (int l = 0; l <= NF; ++l) ssum += al[l];
    const double inv = rcp(ssum);
    double om[NF + 1];
#pragma unroll
    for (int l = 0; l <= NF; ++l) om[l] = al[l] * inv;
    // d = c - c* (non-constant coefficients; the quadratic form ignores d_0)
    double d[NL];
    d[0] = 0.0;
#pragma unroll
    for (int j = 1; j < NL; ++j) d[j] = om[0] * c[j];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      C::template cand_any<0>(f, b, cd);
#pragma unroll
      for (int j = 1; j < NL; ++j) d[j] = fma(om[f + 1], cd[j], d[j]);
      if constexpr (SB) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 1; j < NL; ++j) d[j] = c[j] - d[j];
    const double num2 = C::qform(d);
    const double den2 = beta[0];
    double ratio;
    if (num2 == 0.0)
      ratio = 0.0;
    else if (den2 == 0.0)
      ratio = __builtin_inf();
    else
      ratio = sqrt_pos(num2 * rcp(den2));
    double gam = 0.0;
    if (ratio >= A.bthr) {
      const double r1 = fmin(1.0, ratio);
      gam = A.q == 1.0 ? r1 : pow_cold(r1, A.q);
    }
    // seed: gamma_bar = -(lambda/p) g . Khat c
    double g[NL];
    scale_g(A, v, g);
    int qm;
    double um;
    const double xc = A.x0 + (ix + 0.5) * A.h;
    const double yc = DIM == 2 ? A.y0 + (iy + 0.5) * A.h : 0.0;
    double lam = lambda(A, c, xc, yc, qm, um);
    if (A.lam_over > 0.0) lam = A.lam_over;
    const double gbar = -(lam * (1.0 / P)) * kappa(g, c);
    // reverse
    double rbar = 0.0;
    if (num2 > 0.0 && den2 > 0.0 && ratio >= A.bthr && ratio <= 1.0)
      rbar = A.q == 1.0 ? gbar : gbar * A.q * pow_cold(ratio, A.q - 1.0);
    double num2b = 0.0, den2b = 0.0;
    if (rbar != 0.0) {
      const double id = rcp(den2);
      num2b = rbar * 0.5 * rcp(ratio) * id;
      den2b = -rbar * 0.5 * ratio * id;
    }
    double db[NL];
    bvec(d, db);
#pragma unroll
    for (int j = 0; j < NL; ++j) db[j] *= 2.0 * num2b;
    // omega_bar_l = -dbar . cand_l
    double omb[NF + 1];
    {
      double t = 0.0;
#pragma unroll
      for (int j = 1; j < NL; ++j) t = fma(db[j], c[j], t);
      omb[0] = -t;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      C::template cand_any<0>(f, b, cd);
      double t = 0.0;
#pragma unroll
      for (int j = 1; j < NL; ++j) t = fma(db[j], cd[j], t);
      omb[f + 1] = -t;
      if constexpr (SB) __builtin_amdgcn_sched_barrier(0);
    }
    double dot = 0.0;
#pragma unroll
    for (int l = 0; l <= NF; ++l) dot = fma(omb[l], om[l], dot);
    double bb[NF + 1];
#pragma unroll
    for (int l = 0; l <= NF; ++l) {
      const double alb = (omb[l] - dot) * inv;
      // d alpha / d beta = -pow alpha / (eps + beta)
      bb[l] = al[l] == 0.0 ? 0.0 : alb * (-A.wpow) * al[l] * rcp(A.eps + beta[l]);
    }
    bb[0] += den2b;
#pragma unroll
    for (int j = 0; j < NL; ++j) zrec[j * zs] = db[j];
#pragma unroll
    for (int l = 0; l <= NF; ++l) {
      zrec[(Z::OM + l) * zs] = om[l];
      zrec[(Z::BB + l) * zs] = bb[l];
    }
    zrec[Z::GA * zs] = gam;
  }

  // numerical flux derivative dH/du^-
  __device__ static inline double dllf(double s, double vax, double um, double up) {
    if constexpr (FLUX == FLUX_LINADV) {
      const double vn = s * vax;
      return 0.5 * vn + 0.5 * fabs(vn);
    } else {
      const double an = s * vax;
      const double aum = fabs(um), aup = fabs(up);
      const double sp = fabs(an) * fmax(aum, aup);
      // d max(|um|, |up|)/d um: whole derivative to the larger, half each on a tie
      const double dsel = aum > aup ? 1.0 : (aum == aup ? 0.5 : 0.0);
      const double sgn = um > 0.0 ? 1.0 : (um < 0.0 ? -1.0 : 0.0);
      return 0.5 * an * um + 0.5 * sp - 0.5 * (up - um) * fabs(an) * dsel * sgn;
    }
  }

  // Face F (2D) of pass B: - sum_r w_r (g^- - g_nb^+) dH/du^- phi(r) into G
  template <int F>
  __device__ static inline void face2d(const StageArgs& A, const double* b, const double* bv, const double (&c)[NL],
                                       const double (&g)[NL], const double (&vxl)[Q], const double (&vyl)[Q],
                                       double (&G)[NL]) {
    const double g2h = A.g2h;
    constexpr int axis = F >> 1;
    constexpr bool plus = F & 1;
    const double s = plus ? 1.0 : -1.0;
    double tm[N], tp[N], sm[N], sp[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double t = 0.0, tn = 0.0, gt = 0.0, gn = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int j = axis == 0 ? i + N * k : k + N * i;
        const double so = plus ? 1.0 : TB::dg.sgn[i];
        const double sn = plus ? TB::dg.sgn[i] : 1.0;
        t = fma(so, c[j], t);
        tn = fma(sn, b[j * S + C::off(F)], tn);
        gt = fma(so, g[j], gt);
        gn = fma(sn * g2h * TB::dg.minv[i] * TB::dg.minv[k], bv[j * S + C::off(F)], gn);
      }
      tm[k] = t;
      tp[k] = tn;
      sm[k] = gt;
      sp[k] = gn;
    }
    double acc[N];
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k] = 0.0;
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      double um = tm[0], up = tp[0], gm = sm[0], gp = sp[0];
#pragma unroll
      for (int k = 1; k < N; ++k) {
        um = fma(tm[k], TB::nd.L[k][r], um);
        up = fma(tp[k], TB::nd.L[k][r], up);
        gm = fma(sm[k], TB::nd.L[k][r], gm);
        gp = fma(sp[k], TB::nd.L[k][r], gp);
      }
      const double vax = axis == 0 ? vxl[r] : vyl[r];
      const double dl = TB::nd.w[r] * (gm - gp) * dllf(s, vax, um, up);
#pragma unroll
      for (int k = 0; k < N; ++k) acc[k] = fma(TB::nd.L[k][r], dl, acc[k]);
    }
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int j = axis == 0 ? i + N * k : k + N * i;
        const double so = plus ? 1.0 : TB::dg.sgn[i];
        G[j] = fma(-so, acc[k], G[j]);
      }
  }

  // Pass B: J^T v of one cell (gather form), combined into the output
  __device__ static inline void grad(const AdjArgs& Ad, const double* b, const double* bv, const double (&c)[NL],
                                     const double (&v)[NL], int ix, int iy, size_t cell, double (&G)[NL]) {
    const StageArgs& A = Ad.s;
    const size_t zs = (size_t)A.nx * (DIM == 2 ? A.ny : 1);  // record field stride
    double g[NL];
    scale_g(A, v, g);
#pragma unroll
    for (int j = 0; j < NL; ++j) G[j] = 0.0;
    bool has[NF];
    has[0] = A.per_x || ix > 0;
    has[1] = A.per_x || ix < A.nx - 1;
    if constexpr (DIM == 2) {
      has[2] = A.per_y || iy > 0;
      has[3] = A.per_y || iy < A.ny - 1;
    }
    const double hh = 0.5 * A.h;
    const double xc = A.x0 + (ix + 0.5) * A.h;
    const double yc = DIM == 2 ? A.y0 + (iy + 0.5) * A.h : 0.0;
    const double g2h = A.g2h;

    // ---- volume: sum_q w_q (grad g . F'(u_q)) phi(q); for the Burgers flux
    // the same node values give lambda_e and its node (the order and the
    // arithmetic of lambda(), so the result is the same)
    double vmax = 0.0, vmax_u = 0.0;
    int vmax_q = -1;
    if constexpr (DIM == 1) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        double u = c[0], gd = 0.0;
#pragma unroll
        for (int a = 1; a < N; ++a) {
          u = fma(c[a], TB::nd.L[a][q], u);
          gd = fma(g[a], TB::nd.D[a][q], gd);
        }
        if (FLUX == FLUX_BURGERS && fabs(u) > vmax) {
          vmax = fabs(u);
          vmax_q = q;
          vmax_u = u;
        }
        const double fp = FLUX == FLUX_LINADV ? A.vx : A.vx * u;
        const double sq = TB::nd.w[q] * gd * fp;
#pragma unroll
        for (int a = 0; a < N; ++a) G[a] = fma(TB::nd.L[a][q], sq, G[a]);
      }
    } else {
      double vxl[Q], vyl[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if constexpr (FLUX == FLUX_LINADV) {
          vxl[k] = A.vx - A.omega * (fma(hh, TB::nd.x[k], yc) - A.cy);
          vyl[k] = A.vy + A.omega * (fma(hh, TB::nd.x[k], xc) - A.cx);
        } else {
          vxl[k] = A.vx;
          vyl[k] = A.vy;
        }
      }
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        double s1[N], gx1[N], gy1[N];
#pragma unroll
        for (int bb = 0; bb < N; ++bb) {
          double t = c[N * bb], tx = 0.0, ty = g[N * bb];
#pragma unroll
          for (int a = 1; a < N; ++a) {
            t = fma(c[a + N * bb], TB::nd.L[a][qx], t);
            tx = fma(g[a + N * bb], TB::nd.D[a][qx], tx);
            ty = fma(g[a + N * bb], TB::nd.L[a][qx], ty);
          }
          s1[bb] = t;
          gx1[bb] = tx;
          gy1[bb] = ty;
        }
        double acc[N];
#pragma unroll
        for (int bb = 0; bb < N; ++bb) acc[bb] = 0.0;
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          double u = s1[0], gx = gx1[0], gy = 0.0;
#pragma unroll
          for (int bb = 1; bb < N; ++bb) {
            u = fma(s1[bb], TB::nd.L[bb][qy], u);
            gx = fma(gx1[bb], TB::nd.L[bb][qy], gx);
            gy = fma(gy1[bb], TB::nd.D[bb][qy], gy);
          }
          if (FLUX == FLUX_BURGERS && fabs(u) > vmax) {
            vmax = fabs(u);
            vmax_q = qx + Q * qy;
            vmax_u = u;
          }
          double fx, fy;
          if constexpr (FLUX == FLUX_LINADV) {
            fx = vxl[qy];
            fy = vyl[qx];
          } else {
            fx = A.vx * u;
            fy = A.vy * u;
          }
          const double sq = TB::nd.w[qy] * fma(gx, fx, gy * fy);
#pragma unroll
          for (int bb = 0; bb < N; ++bb) acc[bb] = fma(TB::nd.L[bb][qy], sq, acc[bb]);
        }
        const double wq = TB::nd.w[qx];
#pragma unroll
        for (int bb = 0; bb < N; ++bb)
#pragma unroll
          for (int a = 0; a < N; ++a) G[a + N * bb] = fma(wq * TB::nd.L[a][qx], acc[bb], G[a + N * bb]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    // ---- faces: - sum_r w_r (g^- - g_nb^+) dH/du^- phi(r)
    if constexpr (DIM == 1) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const double s = f ? 1.0 : -1.0;
        double um = 0.0, up = 0.0, gm = 0.0, gp = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
          const double so = f ? 1.0 : TB::dg.sgn[a];
          const double sn = f ? TB::dg.sgn[a] : 1.0;
          um = fma(so, c[a], um);
          up = fma(sn, b[a * S + C::off(f)], up);
          gm = fma(so, g[a], gm);
          gp = fma(sn * g2h * TB::dg.minv[a], bv[a * S + C::off(f)], gp);
        }
        const double dl = (gm - gp) * dllf(s, A.vx, um, up);
#pragma unroll
        for (int a = 0; a < N; ++a) G[a] = fma(f ? -1.0 : -TB::dg.sgn[a], dl, G[a]);
      }
    } else {
      double vxl[Q], vyl[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if constexpr (FLUX == FLUX_LINADV) {
          vxl[k] = A.vx - A.omega * (fma(hh, TB::nd.x[k], yc) - A.cy);
          vyl[k] = A.vy + A.omega * (fma(hh, TB::nd.x[k], xc) - A.cx);
        } else {
          vxl[k] = A.vx;
          vyl[k] = A.vy;
        }
      }
      // one face live at a time (keeps the register count down)
      face2d<0>(A, b, bv, c, g, vxl, vyl, G);
      __builtin_amdgcn_sched_barrier(0);
      face2d<1>(A, b, bv, c, g, vxl, vyl, G);
      __builtin_amdgcn_sched_barrier(0);
      face2d<2>(A, b, bv, c, g, vxl, vyl, G);
      __builtin_amdgcn_sched_barrier(0);
      face2d<3>(A, b, bv, c, g, vxl, vyl, G);
      __builtin_amdgcn_sched_barrier(0);
    }

    // ---- dissipation: - kd Khat g, and through lambda_e
    if constexpr (MODE != MODE_DG) {
      double gam = 1.0;
      const double* zo = nullptr;
      if constexpr (MODE == MODE_WENO) {
        zo = Ad.z + cell;
        gam = zo[Z::GA * zs];
      }
      int qm;
      double um, lam;
      if constexpr (FLUX == FLUX_BURGERS) {
        qm = vmax_q;
        um = vmax_u;
        lam = A.anorm * vmax;
      } else {
        lam = lambda(A, c, xc, yc, qm, um);
      }
      const bool over = A.lam_over > 0.0;
      if (over) lam = A.lam_over;
      sub_khat(gam * lam * (1.0 / P), g, G);
      if constexpr (FLUX == FLUX_BURGERS) {
        if (!over && qm >= 0 && gam != 0.0) {
          const double kap = kappa(g, c);
          const double coef = -(gam * kap * (1.0 / P)) * A.anorm * (um > 0.0 ? 1.0 : -1.0);
          double phi[NL];
          basis_at(qm, phi);
#pragma unroll
          for (int j = 0; j < NL; ++j) G[j] = fma(coef, phi[j], G[j]);
        }
      }
      // ---- sensor records: own and the face neighbours'
      if constexpr (MODE == MODE_WENO) {
        double d[NL], bc[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) d[j] = zo[j * zs];
        bvec(c, bc);
        const double om0 = zo[Z::OM * zs], bb0 = zo[Z::BB * zs];
#pragma unroll
        for (int j = 1; j < NL; ++j) G[j] = fma(1.0 - om0, d[j], fma(2.0 * bb0, bc[j], G[j]));
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          if (!has[f]) continue;
          // neighbour across face f; this cell is its candidate of face f^1
          const double* zn = Ad.z + neighbour_cell(ix, iy, f, A.nx, DIM == 2 ? A.ny : 1);
          const int fo = f ^ 1;
          double cd[NL], cb[NL];
          if (fo == 0) cand_regs<0>(c, cd);
          if (fo == 1) cand_regs<1>(c, cd);
          if constexpr (DIM == 2) {
            if (fo == 2) cand_regs<2>(c, cd);
            if (fo == 3) cand_regs<3>(c, cd);
          }
          double bcd[NL];
          bvec(cd, bcd);
          const double omf = zn[(Z::OM + fo + 1) * zs], bbf = zn[(Z::BB + fo + 1) * zs];
#pragma unroll
          for (int j = 0; j < NL; ++j) cb[j] = j == 0 ? 0.0 : fma(-omf, zn[j * zs], 2.0 * bbf * bcd[j]);
          if (fo == 0) cand_T<0>(cb, G);
          if (fo == 1) cand_T<1>(cb, G);
          if constexpr (DIM == 2) {
            if (fo == 2) cand_T<2>(cb, G);
            if (fo == 3) cand_T<3>(cb, G);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }
};

// The cotangent of the cell at (gx, gy) before wrapping; zero outside a
// non-periodic boundary (no equation there).
template <int DIM, int NL>
__device__ inline void load_cell_v(const AdjArgs& Ad, int gx, int gy, double (&v)[NL]) {
  size_t cell;
  if (slot_cell<DIM>(Ad.s, gx, gy, cell)) {
    const double* src = Ad.v + cell * NL;
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = src[j];
  } else {
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = 0.0;
  }
}

// The coefficients of the cell at (gx, gy) before wrapping in the state U, or
// the exterior state outside a non-periodic boundary.
template <int DIM, int NL>
__device__ inline void load_cell_at(const StageArgs& A, const double* U, int gx, int gy, double (&v)[NL]) {
  size_t cell;
  if (slot_cell<DIM>(A, gx, gy, cell)) {
    const double* src = U + cell * NL;
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = src[j];
  } else {
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = j == 0 ? A.bc : 0.0;
  }
}

// Pass A kernel: sensor records.  LDS: NL * S doubles (state tile + halo).
// Each thread keeps its own cell's coefficients and cotangent in registers
// and publishes the coefficients for its neighbours.
template <int DIM, int P, int FLUX, int MODE, int TX, int TY>
__global__ void __launch_bounds__(DIM == 2 ? TX * TY : TX) adj_sensor_kernel(const AdjArgs Ad) {
  using G = TileGeom<DIM, TX, TY>;
  using AC = AdjCell<DIM, P, FLUX, MODE, G::S, G::W>;
  constexpr int NL = AC::NL, S = G::S;
  extern __shared__ double lds[];
  const StageArgs& A = Ad.s;
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);  // XCD-aware order
  const int ix0 = (tile % gridDim.x) * TX, iy0 = DIM == 2 ? (tile / gridDim.x) * TY : 0;
  const int t = threadIdx.x;
  int sc, gx, gy, hs, hgx, hgy;
  const bool halo = tile_slots<DIM, TX, TY>(t, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
  const bool active = gx < A.nx && gy < (DIM == 2 ? A.ny : 1);
  const size_t cell = (size_t)gy * A.nx + gx;
  double c[NL], v[NL];
  load_cell<DIM, NL>(A, gx, gy, c);
  if (halo) load_slot<DIM, NL, S>(A, lds, hs, hgx, hgy);
  if (active) {
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = Ad.v[cell * NL + j];
  }
#pragma unroll
  for (int j = 0; j < NL; ++j) lds[j * S + sc] = c[j];
  tile_barrier();
  if (!active) return;
  AC::template sensor_adjoint<true>(A, lds + sc, c, gx, gy, v, Ad.z + cell, (size_t)A.nx * (DIM == 2 ? A.ny : 1));
}

// Pass B kernel: J^T v and the combination.  LDS: 2 * NL * S doubles (state
// and cotangent tiles); own values stay in registers.
template <int DIM, int P, int FLUX, int MODE, int TX, int TY>
__global__ void __launch_bounds__(DIM == 2 ? TX * TY : TX) adj_grad_kernel(const AdjArgs Ad) {
  using G = TileGeom<DIM, TX, TY>;
  using AC = AdjCell<DIM, P, FLUX, MODE, G::S, G::W>;
  constexpr int NL = AC::NL, S = G::S;
  extern __shared__ double lds[];
  double* ldsv = lds + NL * S;
  const StageArgs& A = Ad.s;
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);  // XCD-aware order
  const int ix0 = (tile % gridDim.x) * TX, iy0 = DIM == 2 ? (tile / gridDim.x) * TY : 0;
  const int t = threadIdx.x;
  int sc, gx, gy, hs, hgx, hgy;
  const bool halo = tile_slots<DIM, TX, TY>(t, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
  const bool active = gx < A.nx && gy < (DIM == 2 ? A.ny : 1);
  const size_t cell = (size_t)gy * A.nx + gx;
  double c[NL], v[NL];
  load_cell<DIM, NL>(A, gx, gy, c);
  load_cell_v<DIM, NL>(Ad, gx, gy, v);
  if (halo) {
    double hv[NL];
    load_slot<DIM, NL, S>(A, lds, hs, hgx, hgy);
    load_cell_v<DIM, NL>(Ad, hgx, hgy, hv);
#pragma unroll
    for (int j = 0; j < NL; ++j) ldsv[j * S + hs] = hv[j];
  }
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    lds[j * S + sc] = c[j];
    ldsv[j * S + sc] = v[j];
  }
  tile_barrier();
  if (!active) return;
  double Gr[NL];
  AC::grad(Ad, lds + sc, ldsv + sc, c, v, gx, gy, cell, Gr);
  // the combination term by term over the whole cell, then one burst of
  // stores (loads of X and Y are not held behind stores to the same cell)
  double o[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    o[j] = Ad.beta * Gr[j];
    if (Ad.alpha != 0.0) o[j] = fma(Ad.alpha, ldsv[j * S + sc], o[j]);  // LDS: v is dead in registers by now
  }
  if (Ad.X) {
#pragma unroll
    for (int j = 0; j < NL; ++j) o[j] = fma(Ad.g1, Ad.X[cell * NL + j], o[j]);
  }
  if (Ad.Y) {
#pragma unroll
    for (int j = 0; j < NL; ++j) o[j] = fma(Ad.g2, Ad.Y[cell * NL + j], o[j]);
  }
  double* dst = Ad.out + cell * NL;
#pragma unroll
  for (int j = 0; j < NL; ++j) dst[j] = o[j];
}

// Pass B of one RK stage followed by pass A of the stage before it, in one
// launch: out = alpha v + beta J(U)^T v + g1 X + g2 Y with U = Ad.s.uin, then
// the sensor records of U' = Ad.unext seeded with this cell's out (the
// cotangent the next pass B takes as v), written to Ad.znext.  Pass A needs
// the seed of its own cell only, so no other tile's result is waited for.
// The records read (Ad.z) and written (Ad.znext) are different buffers.
// LDS as pass B's; the state plane is reloaded with U' once pass B is done.
template <int DIM, int P, int FLUX, int MODE, int TX, int TY>
__global__ void __launch_bounds__(DIM == 2 ? TX * TY : TX) adj_grad_sensor_kernel(const AdjArgs Ad) {
  using G = TileGeom<DIM, TX, TY>;
  using AC = AdjCell<DIM, P, FLUX, MODE, G::S, G::W>;
  constexpr int NL = AC::NL, S = G::S;
  extern __shared__ double lds[];
  double* ldsv = lds + NL * S;
  const StageArgs& A = Ad.s;
  const int tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);  // XCD-aware order
  const int ix0 = (tile % gridDim.x) * TX, iy0 = DIM == 2 ? (tile / gridDim.x) * TY : 0;
  const int t = threadIdx.x;
  int sc, gx, gy, hs, hgx, hgy;
  const bool halo = tile_slots<DIM, TX, TY>(t, ix0, iy0, sc, gx, gy, hs, hgx, hgy);
  const bool active = gx < A.nx && gy < (DIM == 2 ? A.ny : 1);
  const size_t cell = (size_t)gy * A.nx + gx;
  double c[NL], v[NL];
  load_cell<DIM, NL>(A, gx, gy, c);
  load_cell_v<DIM, NL>(Ad, gx, gy, v);
  if (halo) {
    double hv[NL];
    load_slot<DIM, NL, S>(A, lds, hs, hgx, hgy);
    load_cell_v<DIM, NL>(Ad, hgx, hgy, hv);
#pragma unroll
    for (int j = 0; j < NL; ++j) ldsv[j * S + hs] = hv[j];
  }
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    lds[j * S + sc] = c[j];
    ldsv[j * S + sc] = v[j];
  }
  // U' of the cell and of its halo slot, loaded now so that the loads
  // overlap pass B (up to P = 2; from P = 3 on the registers they would hold
  // through pass B make it spill)
  constexpr bool early = P <= 2;
  double cn[NL], hn[NL];
  if constexpr (early) {
    load_cell_at<DIM, NL>(A, Ad.unext, gx, gy, cn);
    if (halo) load_cell_at<DIM, NL>(A, Ad.unext, hgx, hgy, hn);
  }
  tile_barrier();
  double o[NL];
  if (active) {
    double Gr[NL];
    AC::grad(Ad, lds + sc, ldsv + sc, c, v, gx, gy, cell, Gr);
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      o[j] = Ad.beta * Gr[j];
      if (Ad.alpha != 0.0) o[j] = fma(Ad.alpha, ldsv[j * S + sc], o[j]);
    }
    if (Ad.X) {
#pragma unroll
      for (int j = 0; j < NL; ++j) o[j] = fma(Ad.g1, Ad.X[cell * NL + j], o[j]);
    }
    if (Ad.Y) {
#pragma unroll
      for (int j = 0; j < NL; ++j) o[j] = fma(Ad.g2, Ad.Y[cell * NL + j], o[j]);
    }
    double* dst = Ad.out + cell * NL;
#pragma unroll
    for (int j = 0; j < NL; ++j) dst[j] = o[j];
  }
  if constexpr (!early) {
    load_cell_at<DIM, NL>(A, Ad.unext, gx, gy, cn);
    if (halo) load_cell_at<DIM, NL>(A, Ad.unext, hgx, hgy, hn);
  }
  tile_barrier();  // every thread is done with the state plane
#pragma unroll
  for (int j = 0; j < NL; ++j) lds[j * S + sc] = cn[j];
  if (halo) {
#pragma unroll
    for (int j = 0; j < NL; ++j) lds[j * S + hs] = hn[j];
  }
  tile_barrier();
  // without the candidate barriers up to P = 2 (registers there are set by
  // pass B); from P = 3 on pass A would raise the register count
  if (active)
    AC::template sensor_adjoint<(P > 2)>(A, lds + sc, cn, gx, gy, o, Ad.znext + cell,
                                         (size_t)A.nx * (DIM == 2 ? A.ny : 1));
}

}  // namespace dgk
