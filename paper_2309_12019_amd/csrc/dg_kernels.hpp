// Device code: the fused per-stage kernel of the dissipative-WENO RKDG scheme.
//
// One thread owns one cell.  A workgroup owns a tile of tx x ty cells; it
// stages the tile and its one-cell face halo from HBM into LDS (coalesced,
// cell-major in HBM, transposed to coefficient-major in LDS so that lanes
// reading the same coefficient of consecutive cells hit consecutive banks),
// evaluates for each cell
//   * the HWENO reconstruction and smoothness sensor gamma_e (Sec. 4),
//   * the volume integral of eq. (weak2) by sum factorisation,
//   * the four (two in 1D) face integrals with the LLF flux (Sec. 2),
//   * lambda_e, nu_e = lambda_e h / (2p) and the dissipation of eq. (astab),
//   * the inverse of the (diagonal) mass matrix,
// and writes either dU/dt or the SSP-RK3 stage combination (eq. ssp)
//   out = a U^n + b (U^(k-1) + dt dU/dt)
// back through LDS with coalesced stores.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "dg_tables.hpp"

namespace dgk {

enum { FLUX_LINADV = 0, FLUX_BURGERS = 1 };
enum { MODE_DG = 0, MODE_LO = 1, MODE_WENO = 2 };

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
  double bc;                     // exterior state at non-periodic faces
  double q, bthr, wnb, eps, wpow, lam_over;
  int tx, ty;                    // tile (ty = 1 in 1D)
  int lds_stride;                // doubles between coefficient planes in LDS
};

// number of LDS doubles a tile needs
__host__ __device__ inline int stage_slots(int dim, int tx, int ty) {
  return dim == 1 ? tx + 2 : (tx + 2) * (ty + 2);
}
__host__ __device__ inline int stage_stride(int dim, int tx, int ty) {
  int s = stage_slots(dim, tx, ty);
  return s | 1;  // odd: consecutive coefficient planes start in different banks
}

// Per-cell arithmetic.  `lds` holds the tile, coefficient-major; `sc` is the
// slot of this cell, `W` the slot-row width.
template <int DIM, int P, int FLUX, int MODE>
struct Cell {
  using TB = Tables<DIM, P, FLUX>;
  static constexpr int N = P + 1;
  static constexpr int NL = TB::NL;
  static constexpr int Q = TB::Q;
  static constexpr int NF = 2 * DIM;

  // c^T B c with the sensor's quadratic form (zero entries skipped at compile time)
  __device__ static inline double qform(const double (&v)[NL]) {
    double acc = 0.0;
#pragma unroll
    for (int i = 1; i < NL; ++i) {
      double ri = 0.0;
      bool any = false;
#pragma unroll
      for (int j = i; j < NL; ++j) {
        if (TB::sn.B[i][j] != 0.0) {
          ri = fma((j == i ? 1.0 : 2.0) * TB::sn.B[i][j], v[j], ri);
          any = true;
        }
      }
      if (any) acc = fma(v[i], ri, acc);
    }
    return acc;
  }

  // neighbour on face f (0: -x, 1: +x, 2: -y, 3: +y), continued into this cell
  // and expanded in this cell's basis: P_a(xi -/+ 2) = sum_b T[s][a][b] P_b(xi)
  template <int F>
  __device__ static inline void candidate(const double (&cn)[NL], double (&cd)[NL]) {
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
          for (int b = 0; b <= a; ++b)
            if (TB::dg.T[si][a][b] != 0.0)
              cd[b + N * e] = fma(TB::dg.T[si][a][b], cn[a + N * e], cd[b + N * e]);
    } else {
#pragma unroll
      for (int e = 0; e < N; ++e)
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int b = 0; b <= e; ++b)
            if (TB::dg.T[si][e][b] != 0.0)
              cd[a + N * b] = fma(TB::dg.T[si][e][b], cn[a + N * e], cd[a + N * b]);
    }
  }

  __device__ static inline void load(const double* lds, int S, int slot, double (&v)[NL]) {
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = lds[j * S + slot];
  }

  __device__ static inline double weight_fn(const StageArgs& A, double beta) {
    const double t = A.eps + beta;
    if (A.wpow == 2.0) {
      const double r = 1.0 / t;
      return r * r;
    }
    return pow(t, -A.wpow);
  }

  // gamma_e of eqs. (sensor)/(gensensor) with the HWENO reconstruction
  __device__ static inline double sensor(const StageArgs& A, const double* lds, int S,
                                         const int (&nbs)[NF], const bool (&has)[NF],
                                         const double (&c)[NL]) {
    double beta[NF + 1];
    beta[0] = qform(c);
    int m = 0;
    double cn[NL], cd[NL];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      beta[f + 1] = 0.0;
      if (has[f]) {
        ++m;
        load(lds, S, nbs[f], cn);
        if (f == 0) candidate<0>(cn, cd);
        if (f == 1) candidate<1>(cn, cd);
        if constexpr (DIM == 2) {
          if (f == 2) candidate<2>(cn, cd);
          if (f == 3) candidate<3>(cn, cd);
        }
        beta[f + 1] = qform(cd);
      }
    }
    double al[NF + 1];
    al[0] = (1.0 - m * A.wnb) * weight_fn(A, beta[0]);
    double asum = al[0];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      al[f + 1] = has[f] ? A.wnb * weight_fn(A, beta[f + 1]) : 0.0;
      asum += al[f + 1];
    }
    const double inv = 1.0 / asum;
    // U* = sum_l omega_l U_l ; only the non-constant coefficients matter
    double cs[NL];
    const double w0 = al[0] * inv;
#pragma unroll
    for (int j = 0; j < NL; ++j) cs[j] = w0 * c[j];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (has[f]) {
        const double wl = al[f + 1] * inv;
        load(lds, S, nbs[f], cn);
        if (f == 0) candidate<0>(cn, cd);
        if (f == 1) candidate<1>(cn, cd);
        if constexpr (DIM == 2) {
          if (f == 2) candidate<2>(cn, cd);
          if (f == 3) candidate<3>(cn, cd);
        }
#pragma unroll
        for (int j = 1; j < NL; ++j) cs[j] = fma(wl, cd[j], cs[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < NL; ++j) cs[j] = c[j] - cs[j];
    const double num2 = qform(cs);
    const double den2 = beta[0];
    double ratio;
    if (num2 == 0.0)
      ratio = 0.0;
    else if (den2 == 0.0)
      ratio = __builtin_inf();
    else
      ratio = sqrt(num2) / sqrt(den2);
    if (!(ratio >= A.bthr)) return 0.0;
    const double r1 = fmin(1.0, ratio);
    return A.q == 1.0 ? r1 : pow(r1, A.q);
  }

  // numerical flux H(um, up, n) for n = s e_axis at a face point (Sec. 2, LLF)
  __device__ static inline double llf(const StageArgs& A, int axis, double s, double um,
                                      double up, double x, double y) {
    if constexpr (FLUX == FLUX_LINADV) {
      double v;
      if constexpr (DIM == 1) {
        v = A.vx;
      } else {
        v = axis == 0 ? A.vx - A.omega * (y - A.cy) : A.vy + A.omega * (x - A.cx);
      }
      const double vn = s * v;
      return 0.5 * vn * (um + up) - 0.5 * fabs(vn) * (up - um);
    } else {
      const double an = s * (axis == 0 ? A.vx : A.vy);
      const double sp = fabs(an) * fmax(fabs(um), fabs(up));
      return 0.25 * an * (um * um + up * up) - 0.5 * sp * (up - um);
    }
  }

  // dU/dt of one cell (and gamma_e, lambda_e)
  __device__ static inline void rhs(const StageArgs& A, const double* lds, int S, int sc, int W,
                                    int ix, int iy, double (&L)[NL], double& gam_out) {
    double c[NL];
    load(lds, S, sc, c);
    int nbs[NF];
    bool has[NF];
    nbs[0] = sc - 1;
    nbs[1] = sc + 1;
    has[0] = A.per_x || ix > 0;
    has[1] = A.per_x || ix < A.nx - 1;
    if constexpr (DIM == 2) {
      nbs[2] = sc - W;
      nbs[3] = sc + W;
      has[2] = A.per_y || iy > 0;
      has[3] = A.per_y || iy < A.ny - 1;
    }
    double gam;
    if constexpr (MODE == MODE_DG)
      gam = 0.0;
    else if constexpr (MODE == MODE_LO)
      gam = 1.0;
    else
      gam = sensor(A, lds, S, nbs, has, c);
    gam_out = gam;

    const double hh = 0.5 * A.h;
    const double xc = A.x0 + (ix + 0.5) * A.h;
    const double yc = DIM == 2 ? A.y0 + (iy + 0.5) * A.h : 0.0;
    double R[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) R[j] = 0.0;
    double smax = 0.0;  // max |u| (BURGERS) or max |v|^2 (LINADV) over volume nodes

    // ---- volume integral  int grad(phi) . F(u_h)
    if constexpr (DIM == 1) {
#pragma unroll
      for (int qn = 0; qn < Q; ++qn) {
        double u = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) u = fma(c[a], TB::nd.L[a][qn], u);
        double F;
        if constexpr (FLUX == FLUX_LINADV) {
          F = A.vx * u;
        } else {
          F = A.vx * 0.5 * u * u;
          smax = fmax(smax, fabs(u));
        }
        const double wF = TB::nd.w[qn] * F;
#pragma unroll
        for (int a = 1; a < N; ++a) R[a] = fma(TB::nd.D[a][qn], wF, R[a]);
      }
    } else {
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        double s1[N];  // s1[b] = sum_a c[a + N b] P_a(x_qx)
#pragma unroll
        for (int b = 0; b < N; ++b) {
          double t = 0.0;
#pragma unroll
          for (int a = 0; a < N; ++a) t = fma(c[a + N * b], TB::nd.L[a][qx], t);
          s1[b] = t;
        }
        double gx[N], gy[N];
#pragma unroll
        for (int b = 0; b < N; ++b) gx[b] = gy[b] = 0.0;
        const double xq = xc + hh * TB::nd.x[qx];
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          double u = 0.0;
#pragma unroll
          for (int b = 0; b < N; ++b) u = fma(s1[b], TB::nd.L[b][qy], u);
          double Fx, Fy;
          if constexpr (FLUX == FLUX_LINADV) {
            const double yq = yc + hh * TB::nd.x[qy];
            const double vxq = A.vx - A.omega * (yq - A.cy);
            const double vyq = A.vy + A.omega * (xq - A.cx);
            Fx = vxq * u;
            Fy = vyq * u;
            smax = fmax(smax, vxq * vxq + vyq * vyq);
          } else {
            const double hu2 = 0.5 * u * u;
            Fx = A.vx * hu2;
            Fy = A.vy * hu2;
            smax = fmax(smax, fabs(u));
          }
          const double wFx = TB::nd.w[qy] * Fx, wFy = TB::nd.w[qy] * Fy;
#pragma unroll
          for (int b = 0; b < N; ++b) {
            gx[b] = fma(TB::nd.L[b][qy], wFx, gx[b]);
            if (b > 0) gy[b] = fma(TB::nd.D[b][qy], wFy, gy[b]);
          }
        }
        const double wq = TB::nd.w[qx];
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
          for (int a = 0; a < N; ++a) {
            double t = R[a + N * b];
            if (a > 0) t = fma(wq * TB::nd.D[a][qx], gx[b], t);
            if (b > 0) t = fma(wq * TB::nd.L[a][qx], gy[b], t);
            R[a + N * b] = t;
          }
      }
    }

    // ---- face integrals  - int_dK phi H(u^-, u^+, n)
    if constexpr (DIM == 1) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const double s = f ? 1.0 : -1.0;
        double um = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) um = fma(f ? 1.0 : TB::dg.sgn[a], c[a], um);
        double up = A.bc;
        if (has[f]) {
          up = 0.0;
#pragma unroll
          for (int a = 0; a < N; ++a) up = fma(f ? TB::dg.sgn[a] : 1.0, lds[a * S + nbs[f]], up);
        }
        const double H = llf(A, 0, s, um, up, xc + s * hh, 0.0);
#pragma unroll
        for (int a = 0; a < N; ++a) R[a] = fma(f ? -1.0 : -TB::dg.sgn[a], H, R[a]);
      }
    } else {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const int axis = f >> 1;
        const bool plus = f & 1;
        const double s = plus ? 1.0 : -1.0;
        // trace coefficients along the face (index runs over the other axis)
        double tm[N], tp[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
          double t = 0.0, tn = 0.0;
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const int j = axis == 0 ? i + N * k : k + N * i;
            const double so = plus ? 1.0 : TB::dg.sgn[i];  // P_i(s)
            const double sn = plus ? TB::dg.sgn[i] : 1.0;  // P_i(-s)
            t = fma(so, c[j], t);
            if (has[f]) tn = fma(sn, lds[j * S + nbs[f]], tn);
          }
          tm[k] = t;
          tp[k] = tn;
        }
        double g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) g[k] = 0.0;
#pragma unroll
        for (int r = 0; r < Q; ++r) {
          double um = 0.0, up = 0.0;
#pragma unroll
          for (int k = 0; k < N; ++k) {
            um = fma(tm[k], TB::nd.L[k][r], um);
            up = fma(tp[k], TB::nd.L[k][r], up);
          }
          if (!has[f]) up = A.bc;
          const double t = hh * TB::nd.x[r];
          const double xf = axis == 0 ? xc + s * hh : xc + t;
          const double yf = axis == 0 ? yc + t : yc + s * hh;
          const double wH = TB::nd.w[r] * llf(A, axis, s, um, up, xf, yf);
#pragma unroll
          for (int k = 0; k < N; ++k) g[k] = fma(TB::nd.L[k][r], wH, g[k]);
        }
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const int j = axis == 0 ? i + N * k : k + N * i;
            const double so = plus ? 1.0 : TB::dg.sgn[i];
            R[j] = fma(-so, g[k], R[j]);
          }
      }
    }

    // ---- lambda_e, dissipation gamma nu int grad(phi) . grad(u_h), M^-1
    double lam;
    if (A.lam_over > 0.0) {
      lam = A.lam_over;
    } else if constexpr (FLUX == FLUX_LINADV) {
      lam = DIM == 1 ? fabs(A.vx) : sqrt(smax);
    } else {
      lam = A.anorm * smax;
    }
    // L = (2/h) Mhat^{-1} [ vol - face - (gamma lambda / p) Khat c ]
    const double kd = gam * lam * (1.0 / P);
    const double g2h = 2.0 / A.h;
    if constexpr (DIM == 1) {
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double kc = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2)
          if (TB::dg.S[a][a2] != 0.0) kc = fma(TB::dg.S[a][a2], c[a2], kc);
        L[a] = (g2h * TB::dg.minv[a]) * fma(-kd, kc, R[a]);
      }
    } else {
#pragma unroll
      for (int b = 0; b < N; ++b)
#pragma unroll
        for (int a = 0; a < N; ++a) {
          double kc = 0.0;
#pragma unroll
          for (int a2 = 0; a2 < N; ++a2)
            if (TB::dg.S[a][a2] != 0.0) kc = fma(TB::dg.S[a][a2] * TB::dg.mhat[b], c[a2 + N * b], kc);
#pragma unroll
          for (int b2 = 0; b2 < N; ++b2)
            if (TB::dg.S[b][b2] != 0.0) kc = fma(TB::dg.S[b][b2] * TB::dg.mhat[a], c[a + N * b2], kc);
          L[a + N * b] = (g2h * TB::dg.minv[a] * TB::dg.minv[b]) * fma(-kd, kc, R[a + N * b]);
        }
    }
  }
};

// The fused stage kernel.  Grid: (ceil(nx/tx), ceil(ny/ty)); block: tx*ty
// threads; dynamic LDS: NL * lds_stride doubles.
template <int DIM, int P, int FLUX, int MODE>
__global__ void __launch_bounds__(256) stage_kernel(const StageArgs A) {
  using C = Cell<DIM, P, FLUX, MODE>;
  constexpr int NL = C::NL;
  extern __shared__ double lds[];
  const int tx = A.tx;
  const int ty = DIM == 2 ? A.ty : 1;
  const int W = tx + 2;
  const int nslots = DIM == 2 ? W * (ty + 2) : W;
  const int S = A.lds_stride;
  const int ix0 = blockIdx.x * tx;
  const int iy0 = DIM == 2 ? blockIdx.y * ty : 0;
  const int nx = A.nx, ny = DIM == 2 ? A.ny : 1;

  for (int idx = threadIdx.x; idx < nslots * NL; idx += blockDim.x) {
    const int s = idx / NL;
    const int j = idx - s * NL;
    const int sy = DIM == 2 ? s / W : 0;
    const int sx = s - sy * W;
    int gx = ix0 - 1 + sx;
    int gy = DIM == 2 ? iy0 - 1 + sy : 0;
    bool ok = true;
    if (gx < 0 || gx >= nx) {
      if (A.per_x)
        gx = ((gx % nx) + nx) % nx;
      else
        ok = false;
    }
    if (DIM == 2 && (gy < 0 || gy >= ny)) {
      if (A.per_y)
        gy = ((gy % ny) + ny) % ny;
      else
        ok = false;
    }
    lds[j * S + s] = ok ? A.uin[((size_t)gy * nx + gx) * NL + j] : 0.0;
  }
  __syncthreads();

  const int t = threadIdx.x;
  const int lx = t % tx, ly = t / tx;
  const int ix = ix0 + lx, iy = iy0 + ly;
  const bool active = ly < ty && ix < nx && iy < ny;
  const int sc = DIM == 2 ? (ly + 1) * W + lx + 1 : lx + 1;
  double res[NL];
  if (active) {
    double L[NL], gam;
    C::rhs(A, lds, S, sc, W, ix, iy, L, gam);
    if (A.gamma) A.gamma[(size_t)iy * nx + ix] = gam;
    if (A.rhs_only) {
#pragma unroll
      for (int j = 0; j < NL; ++j) res[j] = L[j];
    } else {
#pragma unroll
      for (int j = 0; j < NL; ++j) res[j] = A.b * fma(A.dt, L[j], lds[j * S + sc]);
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int j = 0; j < NL; ++j) lds[j * S + sc] = res[j];
  }
  __syncthreads();
  const bool comb = !A.rhs_only && A.a != 0.0;
  for (int idx = threadIdx.x; idx < tx * ty * NL; idx += blockDim.x) {
    const int cl = idx / NL;
    const int j = idx - cl * NL;
    const int cyl = cl / tx;
    const int cxl = cl - cyl * tx;
    const int gx = ix0 + cxl, gy = iy0 + cyl;
    if (gx < nx && gy < ny) {
      const size_t g = ((size_t)gy * nx + gx) * NL + j;
      const int slot = DIM == 2 ? (cyl + 1) * W + cxl + 1 : cxl + 1;
      double v = lds[j * S + slot];
      if (comb) v = fma(A.a, A.un[g], v);
      A.out[g] = v;
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
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) block_max[blockIdx.x] = red[0];
}

}  // namespace dgk
