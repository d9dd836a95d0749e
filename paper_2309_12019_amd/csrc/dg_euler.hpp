// Device code of the one-dimensional Euler equations of Sec. 5.6:
// U = (rho, rho v, rho E), F(U) = (rho v, rho v^2 + p, (rho E + p) v),
// p = (gamma - 1)(rho E - rho v^2 / 2), gamma = 1.4, with the same DG
// operator, dissipation and sensor as the scalar path:
//   L_k = (2/h) Mhat^-1 [ vol_k - face_k - (gamma_e lambda_e / p) Khat c_k ]
// for the three components k, gamma_e from the density coefficients alone.
// The LLF wave speed is the larger |v| + c of the two states, lambda_e the
// largest |v| + c over the volume Gauss nodes (p + 2 of them: the flux is
// rational), and a reflecting wall sees the mirror state (rho, -rho v, rho E).
//
// State layout: cell-major, [cell][component][coefficient] (3 (p+1) doubles
// per cell).  A tile of TX cells holds the 3 (p+1) coefficient planes of its
// cells and a one-cell halo in LDS (density planes first, so the scalar
// sensor reads them unchanged).
#pragma once

#include "dg_kernels.hpp"

namespace dgk {

constexpr double kEulerGamma = 1.4;

// F(u) and |v| + c of one state
__device__ inline void euler_flux(const double (&u)[3], double (&F)[3], double& speed) {
  const double v = u[1] / u[0];
  const double p = (kEulerGamma - 1.0) * (u[2] - 0.5 * u[1] * v);
  F[0] = u[1];
  F[1] = fma(u[1], v, p);
  F[2] = (u[2] + p) * v;
  speed = fabs(v) + sqrt(kEulerGamma * p / u[0]);
}

// H . n of the LLF flux for the outward normal n = side
__device__ inline void llf_euler(double side, const double (&um)[3], const double (&up)[3], double (&H)[3]) {
  double Fm[3], Fp[3], sm, sp;
  euler_flux(um, Fm, sm);
  euler_flux(up, Fp, sp);
  const double s = fmax(sm, sp);
#pragma unroll
  for (int k = 0; k < 3; ++k) H[k] = 0.5 * side * (Fm[k] + Fp[k]) - 0.5 * s * (up[k] - um[k]);
}

template <int P, int MODE, int TX>
struct EulerCell {
  using G = TileGeom<1, TX, 1>;
  using C = Cell<1, P, FLUX_EULER, MODE, G::S, G::W>;  // sensor, dissipation, tables
  using TB = typename C::TB;
  static constexpr int N = P + 1;
  static constexpr int Q = TB::Q;
  static constexpr int S = G::S;

  // Volume minus face terms for the three components, and lambda_e.
  // b: the cell's slot in the LDS tile (plane j = k N + a); c[k][a]: own state.
  __device__ static inline void residual(const StageArgs& A, const double* b, const double (&c)[3][N], int ix,
                                         double (&R)[3][N], double& lam) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int a = 0; a < N; ++a) R[k][a] = 0.0;
    lam = 0.0;
    // ---- volume  int phi_a' F(u_h)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      double u[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double t = c[k][0];
#pragma unroll
        for (int a = 1; a < N; ++a) t = fma(c[k][a], TB::nd.L[a][q], t);
        u[k] = t;
      }
      double F[3], sp;
      euler_flux(u, F, sp);
      lam = fmax(lam, sp);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double wF = TB::nd.w[q] * F[k];
#pragma unroll
        for (int a = 1; a < N; ++a) R[k][a] = fma(TB::nd.D[a][q], wF, R[k][a]);
      }
    }
    // ---- faces  - phi_a H . n at x_{e -/+ 1/2}
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const bool wall = !A.per_x && (f ? ix == A.nx - 1 : ix == 0);
      double um[3], up[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double tm = 0.0, tp = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
          const double so = f ? 1.0 : TB::dg.sgn[a];  // P_a at this cell's face
          const double sn = f ? TB::dg.sgn[a] : 1.0;  // P_a at the neighbour's face
          tm = fma(so, c[k][a], tm);
          tp = fma(sn, b[(k * N + a) * S + C::off(f)], tp);
        }
        um[k] = tm;
        up[k] = tp;
      }
      if (wall) {
        up[0] = um[0];
        up[1] = -um[1];
        up[2] = um[2];
      }
      double H[3];
      llf_euler(f ? 1.0 : -1.0, um, up, H);
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < N; ++a) R[k][a] = fma(f ? -1.0 : -TB::dg.sgn[a], H[k], R[k][a]);
    }
  }
};

// One tile of the Euler stage: TX threads, one per cell; the layout and the
// barrier discipline of the scalar stage tile.  out = a U^n + b (U + dt L),
// or out = L when rhs_only; gamma (optional) receives gamma_e.
template <int P, int MODE, int TX>
__device__ inline void euler_stage_tile(const StageArgs& A, double* lds, int ix0) {
  using E = EulerCell<P, MODE, TX>;
  using C = typename E::C;
  constexpr int N = E::N, NLE = 3 * N, S = E::S;
  const bool comb = !A.rhs_only && A.a != 0.0;
  const int t = threadIdx.x;
  int sc, gx, gy, hs, hgx, hgy;
  const bool halo = tile_slots<1, TX, 1>(t, ix0, 0, sc, gx, gy, hs, hgx, hgy);
  const bool active = gx < A.nx;
  double cf[NLE];
  load_cell<1, NLE>(A, gx, 0, cf);
  if (halo) load_slot<1, NLE, S>(A, lds, hs, hgx, 0);
#pragma unroll
  for (int j = 0; j < NLE; ++j) lds[j * S + sc] = cf[j];
  tile_barrier();
  if (active) {
    double c[3][N], rho[N];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int a = 0; a < N; ++a) c[k][a] = cf[k * N + a];
#pragma unroll
    for (int a = 0; a < N; ++a) rho[a] = c[0][a];
    const double gam = C::template gamma_of<true>(A, lds + sc, rho, gx, 0);
    double R[3][N], lam;
    E::residual(A, lds + sc, c, gx, R, lam);
    if (A.gamma) A.gamma[gx] = gam;
    // all three components first, then the cell's 3 (p+1) doubles in one
    // burst: stores spread between the components' arithmetic leave lines
    // partly written in L2 and multiply the HBM write traffic
    double out[NLE];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double L[N];
      C::finish(A, c[k], gam, lam, R[k], L);
#pragma unroll
      for (int a = 0; a < N; ++a)
        out[k * N + a] = A.rhs_only ? L[a] : A.b * fma(A.dt, L[a], c[k][a]);
    }
    if (comb) {
      const double* un = A.un + (size_t)gx * NLE;
#pragma unroll
      for (int j = 0; j < NLE; ++j) out[j] = fma(A.a, un[j], out[j]);
    }
    double* dst = A.out + (size_t)gx * NLE;
#pragma unroll
    for (int j = 0; j < NLE; ++j) dst[j] = out[j];
  }
}

template <int P, int MODE, int TX>
__global__ void __launch_bounds__(TX) euler_stage_kernel(const StageArgs A) {
  extern __shared__ double lds[];
  euler_stage_tile<P, MODE, TX>(A, lds, blockIdx.x * TX);
}

// The fused SSP-RK3 step of the Euler system: all three stages of a step in
// one launch, as the scalar step kernel does.  A tile of kEulerStepTile cells
// loads U^n on itself and three cells each side (tile A), evaluates stage 1
// on the tile and two cells each side (tile B), stage 2 on one cell each
// side (tile C) and stage 3 on the tile, straight to HBM; U^n for the RK
// combinations comes from tile A.  The cell arithmetic is EulerCell's and
// the combination the per-stage kernel's, in the same order, so the result
// is the same bit for bit.  Slots outside a wall hold the constant exterior
// state: the cell code reads them and discards what it read (the wall takes
// the mirror state, the sensor ignores the missing neighbour), so they need
// only be finite.  In 1D the rings cost 6 cells in 256 and a step moves U^n
// and U^(n+1) through HBM once (16 B per DOF instead of 64).
constexpr int kEulerStepTile = 256;
constexpr int kEulerStepThreads = 320;  // stage 1 covers 260 cells in one round
__host__ __device__ inline int euler_step_lds_doubles(int p) {
  constexpr int T = kEulerStepTile;
  return 3 * (p + 1) * (((T + 6) | 1) + ((T + 4) | 1) + ((T + 2) | 1));
}

// One stage of the fused Euler step: output cells o < nout at mesh x index
// gx0 + o, from the input tile tin (interior width TXI, slots TXI + 2; cell o
// at slot o + 1) and U^n in tile A (cell o at slot o + aoff).  LAST: store
// the tile's own in-mesh cells to A.out, else every slot of tout.
template <int P, int MODE, int TXI, bool LAST>
__device__ inline void euler_fused_stage(const StageArgs& A, const double* tin, const double* ta, int aoff,
                                         double* tout, int nout, int gx0, double a, double b) {
  using E = EulerCell<P, MODE, TXI>;
  using C = typename E::C;
  constexpr int N = E::N, NLE = 3 * N, S = E::S;
  constexpr int SA = (kEulerStepTile + 6) | 1;
  constexpr int SO = (TXI + 2 - 2) | 1;  // output tile: two slots fewer
  for (int o = threadIdx.x; o < nout; o += kEulerStepThreads) {
    const int gx = gx0 + o;
    int wx, wy;
    if (!step_cell<1>(A, gx, 0, wx, wy) || (LAST && gx >= A.nx)) {
      if constexpr (!LAST) {
#pragma unroll
        for (int j = 0; j < NLE; ++j) tout[j * SO + o] = j == 0 ? A.bc : 0.0;
      }
      continue;
    }
    const double* bs = tin + (o + 1);
    double c[3][N], rho[N];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int q = 0; q < N; ++q) c[k][q] = bs[(k * N + q) * S];
#pragma unroll
    for (int q = 0; q < N; ++q) rho[q] = c[0][q];
    const double gam = C::template gamma_of<true>(A, bs, rho, wx, 0);
    double R[3][N], lam;
    E::residual(A, bs, c, wx, R, lam);
    double out[NLE];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double L[N];
      C::finish(A, c[k], gam, lam, R[k], L);
#pragma unroll
      for (int q = 0; q < N; ++q) out[k * N + q] = b * fma(A.dt, L[q], c[k][q]);
    }
    if (a != 0.0) {
#pragma unroll
      for (int j = 0; j < NLE; ++j) out[j] = fma(a, ta[j * SA + o + aoff], out[j]);
    }
    if constexpr (LAST) {
      double* dst = A.out + (size_t)wx * NLE;
#pragma unroll
      for (int j = 0; j < NLE; ++j) dst[j] = out[j];
    } else {
#pragma unroll
      for (int j = 0; j < NLE; ++j) tout[j * SO + o] = out[j];
    }
  }
}

// Grid: ceil(nx / kEulerStepTile) tiles, kEulerStepThreads threads, LDS
// euler_step_lds_doubles(P).  A.uin = U^n, A.out = U^(n+1), two different
// arrays (tiles run concurrently and read U^n of their neighbours).
template <int P, int MODE>
__global__ void __launch_bounds__(kEulerStepThreads) euler_step_kernel(const StageArgs A) {
  constexpr int T = kEulerStepTile, NLE = 3 * (P + 1);
  constexpr int SA = (T + 6) | 1, SB = (T + 4) | 1;
  extern __shared__ double lds[];
  double* const ta = lds;
  double* const tb = ta + NLE * SA;
  double* const tc = tb + NLE * SB;
  const int ix0 = xcd_tile(blockIdx.x, gridDim.x) * T;
  // U^n on the tile and three cells each side
  for (int o = threadIdx.x; o < T + 6; o += kEulerStepThreads) {
    int wx, wy;
    double v[NLE];
    if (step_cell<1>(A, ix0 - 3 + o, 0, wx, wy)) {
      const double* src = A.uin + (size_t)wx * NLE;
#pragma unroll
      for (int j = 0; j < NLE; ++j) v[j] = src[j];
    } else {
#pragma unroll
      for (int j = 0; j < NLE; ++j) v[j] = j == 0 ? A.bc : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NLE; ++j) ta[j * SA + o] = v[j];
  }
  tile_barrier();
  euler_fused_stage<P, MODE, T + 4, false>(A, ta, ta, 1, tb, T + 4, ix0 - 2, 0.0, 1.0);
  tile_barrier();
  euler_fused_stage<P, MODE, T + 2, false>(A, tb, ta, 2, tc, T + 2, ix0 - 1, 0.75, 0.25);
  tile_barrier();
  euler_fused_stage<P, MODE, T, true>(A, tc, ta, 3, nullptr, T, ix0, 1.0 / 3.0, 2.0 / 3.0);
}

// Per-block maximum of lambda_e = max over the volume nodes of |v| + c.
template <int P>
__global__ void __launch_bounds__(256) euler_lambda_kernel(const StageArgs A, const double* __restrict__ U,
                                                           double* __restrict__ block_max) {
  using TB = Tables<1, P, FLUX_EULER>;
  constexpr int N = P + 1, Q = TB::Q;
  __shared__ double red[256];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double lam = 0.0;
  if (e < A.nx) {
    if (A.lam_over > 0.0) {
      lam = A.lam_over;
    } else {
      const double* c = U + e * 3 * N;
      for (int q = 0; q < Q; ++q) {
        double u[3], F[3], sp;
        for (int k = 0; k < 3; ++k) {
          double s = 0.0;
          for (int a = 0; a < N; ++a) s = fma(c[k * N + a], TB::nd.L[a][q], s);
          u[k] = s;
        }
        euler_flux(u, F, sp);
        lam = fmax(lam, sp);
      }
    }
  }
  red[threadIdx.x] = lam;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) block_max[blockIdx.x] = red[0];
}

}  // namespace dgk
