/*
 * Plain C oracle of the dissipative-WENO-stabilised RKDG scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Like the PyTorch oracle beside it (dgoracle.py),
 * this file is the slow, obviously-correct reference the HIP library is
 * checked against; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, tables or constants with
 * the HIP library: Gauss rules, Legendre polynomials and every matrix are
 * derived here from their definitions when a problem is created.  It exists
 * because the PyTorch oracle cannot follow the largest workloads (a 1024^2
 * mesh) for hundreds of steps in test time; it computes the same thing,
 * cell by cell, with loops over quadrature points and basis functions.
 *
 * Paper: J. Vedral, "Dissipative WENO stabilization of high-order
 * discontinuous Galerkin methods for hyperbolic problems" (arXiv 2309.12019).
 *
 * Per cell, in the paper's order (FP64; no sum factorisation, no blocking):
 *   Sec. 2, eq. (weak2): R_i = int_K grad(phi_i) . F(u_h) dx
 *                              - int_dK phi_i H(u^-, u^+, n) ds,
 *     H the local Lax-Friedrichs flux of Sec. 2, whose wave speed
 *     s^+ = max over the segment [u^-, u^+] of |F'(w) . n|;
 *   Sec. 4, eqs. (sensor)/(gensensor): gamma_e = min(1, |U - U*|_e / |U|_e)^q
 *     (0 below the threshold b), U* the Hermite-WENO reconstruction from the
 *     cell's own polynomial and its face neighbours' polynomials continued
 *     into the cell with the cell's own mean, nonlinear weights
 *     alpha_l = w~_l / (eps + beta_l)^r with the linear weights of Sec. 5;
 *     or the sensor of Zhao et al. that Sec. 5.6 compares with;
 *   Sec. 3, eqs. (lostab), (visc), (astab): s_i = gamma_e nu_e
 *     int_K grad(phi_i) . grad(u_h) dx, nu_e = lambda_e h / (2p),
 *     lambda_e = max over the volume nodes of ||F'(u_h)||_2 (or an override);
 *   dU/dt = M^-1 (R - s);
 *   Sec. 2, eq. (ssp): the three-stage SSP Runge-Kutta step (and the second-
 *     order and five-stage fourth-order SSP methods of the convergence study,
 *     Sec. 5.1).
 * The readings where the paper is silent are the PyTorch oracle's: the
 * candidates, indicators and weights above; Gauss rules with p+1 points per
 * axis for linear advection, p+2 for KPP, ceil(3p/2) (1D) or ceil((3p+1)/2)
 * (2D) for Burgers; a constant exterior state outside non-periodic faces.
 *
 * Layout: U[cell][j], cell = ix + nx iy, j = a + (p+1) b (tensor Legendre
 * modes on [-1,1]^d, x fastest), as the PyTorch oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { LINADV = 0, BURGERS = 1, KPP = 2 };
enum { MODE_DG = 0, MODE_LO = 1, MODE_WENO = 2, MODE_ZHAO = 3 };

#define MAXN 5            /* p + 1 <= 5 */
#define MAXL 25           /* (p + 1)^2 */
#define MAXQ 8            /* Gauss points per axis */
#define MAXQD (MAXQ * MAXQ)

typedef struct {
  int dim, nx, ny;
  double x0, x1, y0, y1;
  int per_x, per_y;
  int p, flux;
  double vx, vy, omega, cx, cy;  /* velocity v = (vx - omega (y - cy), vy + omega (x - cx)); Burgers: a = (vx, vy) */
  double bc;                     /* exterior state outside non-periodic faces */
  int mode;
  double q, b, wnb, eps, r, theta;
  int rk_order;
  double lam_over;               /* > 0: lambda_e fixed */
  int quad_vol, quad_face;       /* 0: the default rules above */
} orc_problem;

typedef struct {
  orc_problem P;
  int n1, nl, nf, qv, qf, nvq;   /* modes per axis, per cell; faces; rules; volume nodes */
  long ncells;
  double h, J, Jf, g;            /* dx = J dxi, ds = Jf ds_ref, d/dx = g d/dxi */
  /* volume rule: reference points, weights, phi and its derivatives there */
  double vpt[MAXQD][2], vw[MAXQD];
  double V[MAXQD][MAXL], DV[2][MAXQD][MAXL];
  /* faces f = (axis, side) in the order (0,-1), (0,+1), (1,-1), (1,+1):
     points, weights, phi on this side and phi of the neighbour there */
  int fax[4], fside[4];
  double fpt[4][MAXQ][2], fw[4][MAXQ];
  double FV[4][MAXQ][MAXL], FVo[4][MAXQ][MAXL];
  double Minv[MAXL][MAXL];       /* inverse mass matrix */
  double K[MAXL][MAXL];          /* int grad(phi_i) . grad(phi_j) dx */
  double cont[4][MAXL][MAXL];    /* neighbour mode j continued into the cell, in modes i */
  double B[MAXL][MAXL];          /* |v|_e^2 = c^T B c */
  double *L, *W1, *W2;           /* work arrays of one state each */
} orc_ctx;

/* ---------------------------------------------------------------------- */
/* Legendre polynomials and Gauss rules, from their definitions            */
/* ---------------------------------------------------------------------- */

/* m-th derivative of P_a at x for a = 0..n-1 (m <= n), by differentiating
   Bonnet's recursion (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1} m times:
   (k+1) P_{k+1}^(m) = (2k+1) (x P_k^(m) + m P_k^(m-1)) - k P_{k-1}^(m). */
static void legendre_deriv(int n, int m, double x, double* out) {
  double d[MAXQ + 2][MAXQ + 2];   /* d[mm][a] = P_a^(mm)(x) */
  for (int mm = 0; mm <= m; ++mm) {
    for (int a = 0; a < n; ++a) {
      double v;
      if (a == 0)
        v = mm == 0 ? 1.0 : 0.0;
      else if (a == 1)
        v = mm == 0 ? x : (mm == 1 ? 1.0 : 0.0);
      else {
        const int k = a - 1;
        v = (2 * k + 1) * (x * d[mm][k] + (mm > 0 ? mm * d[mm - 1][k] : 0.0)) - k * d[mm][k - 1];
        v /= (k + 1);
      }
      d[mm][a] = v;
    }
  }
  for (int a = 0; a < n; ++a) out[a] = d[m][a];
}

/* Gauss-Legendre rule with Q points on [-1,1]: the roots of P_Q by Newton's
   method, weights 2 / ((1 - x^2) P_Q'(x)^2), ascending nodes. */
static void gauss(int Q, double* x, double* w) {
  double v[MAXQ + 2], dv[MAXQ + 2];
  for (int i = 0; i < Q; ++i) {
    double t = cos(M_PI * (i + 0.75) / (Q + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre_deriv(Q + 1, 0, t, v);
      legendre_deriv(Q + 1, 1, t, dv);
      const double dx = v[Q] / dv[Q];
      t -= dx;
      if (fabs(dx) < 1e-17) break;
    }
    legendre_deriv(Q + 1, 1, t, dv);
    x[Q - 1 - i] = t;   /* the guesses descend */
    w[Q - 1 - i] = 2.0 / ((1.0 - t * t) * dv[Q] * dv[Q]);
  }
}

/* D^k phi_j at a reference point (k = (kx, ky); 1D uses kx only) */
static void basis_eval(const orc_ctx* c, const double* pt, int kx, int ky, double* out) {
  double px[MAXN], py[MAXN];
  legendre_deriv(c->n1, kx, pt[0], px);
  if (c->P.dim == 1) {
    for (int a = 0; a < c->n1; ++a) out[a] = px[a];
    return;
  }
  legendre_deriv(c->n1, ky, pt[1], py);
  for (int bb = 0; bb < c->n1; ++bb)
    for (int a = 0; a < c->n1; ++a) out[a + c->n1 * bb] = px[a] * py[bb];
}

/* inverse of an n x n matrix by Gauss-Jordan elimination with partial pivoting */
static int invert(int n, double A[MAXL][MAXL], double X[MAXL][MAXL]) {
  double a[MAXL][2 * MAXL];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) a[i][j] = j < n ? A[i][j] : (j - n == i ? 1.0 : 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int i = col + 1; i < n; ++i)
      if (fabs(a[i][col]) > fabs(a[piv][col])) piv = i;
    if (a[piv][col] == 0.0) return -1;
    if (piv != col)
      for (int j = 0; j < 2 * n; ++j) {
        const double t = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = t;
      }
    const double d = a[col][col];
    for (int j = 0; j < 2 * n; ++j) a[col][j] /= d;
    for (int i = 0; i < n; ++i)
      if (i != col && a[i][col] != 0.0) {
        const double f = a[i][col];
        for (int j = 0; j < 2 * n; ++j) a[i][j] -= f * a[col][j];
      }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) X[i][j] = a[i][j + n];
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Problem set-up                                                          */
/* ---------------------------------------------------------------------- */

/* Volume Gauss points per axis: exact for the polynomial part of the flux */
static int default_qv(const orc_problem* P) {
  if (P->flux == LINADV) return P->p + 1;
  if (P->flux == KPP) return P->p + 2;
  if (P->dim == 1) return (3 * P->p + 1) / 2;    /* ceil(3p/2) */
  return (3 * P->p + 2) / 2;                     /* ceil((3p+1)/2) */
}

void* orc_create(const orc_problem* P) {
  if (P->dim < 1 || P->dim > 2 || P->p < 1 || P->p > 4 || P->nx < 1 || (P->dim == 2 && P->ny < 1)) return NULL;
  if (P->flux == KPP && P->dim != 2) return NULL;
  if (P->flux < LINADV || P->flux > KPP || P->mode < MODE_DG || P->mode > MODE_ZHAO) return NULL;
  if (P->rk_order != 2 && P->rk_order != 3 && P->rk_order != 4) return NULL;
  orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  if (!c) return NULL;
  c->P = *P;
  const int d = P->dim;
  c->n1 = P->p + 1;
  c->nl = d == 1 ? c->n1 : c->n1 * c->n1;
  c->nf = 2 * d;
  c->qv = P->quad_vol ? P->quad_vol : default_qv(P);
  c->qf = P->quad_face ? P->quad_face : c->qv;
  if (c->qv > MAXQ || c->qf > MAXQ) {
    free(c);
    return NULL;
  }
  c->ncells = (long)P->nx * (d == 2 ? P->ny : 1);
  c->h = (P->x1 - P->x0) / P->nx;
  c->J = d == 1 ? c->h / 2.0 : (c->h / 2.0) * (c->h / 2.0);
  c->Jf = d == 1 ? 1.0 : c->h / 2.0;
  c->g = 2.0 / c->h;

  /* volume rule (x fastest) and the basis there */
  double gx[MAXQ], gw[MAXQ];
  gauss(c->qv, gx, gw);
  c->nvq = d == 1 ? c->qv : c->qv * c->qv;
  for (int qn = 0; qn < c->nvq; ++qn) {
    const int i = qn % c->qv, k = qn / c->qv;
    c->vpt[qn][0] = gx[i];
    c->vpt[qn][1] = d == 2 ? gx[k] : 0.0;
    c->vw[qn] = d == 2 ? gw[i] * gw[k] : gw[i];
    basis_eval(c, c->vpt[qn], 0, 0, c->V[qn]);
    basis_eval(c, c->vpt[qn], 1, 0, c->DV[0][qn]);
    if (d == 2) basis_eval(c, c->vpt[qn], 0, 1, c->DV[1][qn]);
  }
  /* faces */
  gauss(c->qf, gx, gw);
  for (int f = 0; f < c->nf; ++f) {
    const int ax = f / 2, s = f % 2 ? 1 : -1;
    c->fax[f] = ax;
    c->fside[f] = s;
    const int nq = d == 1 ? 1 : c->qf;
    for (int r = 0; r < nq; ++r) {
      double pt[2], po[2];
      pt[ax] = s;
      po[ax] = -s;   /* the same physical point seen from the neighbour */
      if (d == 2) {
        pt[1 - ax] = gx[r];
        po[1 - ax] = gx[r];
      } else {
        pt[1] = po[1] = 0.0;
      }
      c->fpt[f][r][0] = pt[0];
      c->fpt[f][r][1] = pt[1];
      c->fw[f][r] = d == 1 ? 1.0 : gw[r];
      basis_eval(c, pt, 0, 0, c->FV[f][r]);
      basis_eval(c, po, 0, 0, c->FVo[f][r]);
    }
  }
  /* exact rule (p+1 points per axis) for mass, stiffness, continuation and
     the semi-norm: every integrand there is a polynomial of degree <= 2p */
  double ex[MAXQ], ew[MAXQ];
  gauss(c->n1, ex, ew);
  const int neq = d == 1 ? c->n1 : c->n1 * c->n1;
  double ept[MAXQD][2], eww[MAXQD];
  for (int qn = 0; qn < neq; ++qn) {
    const int i = qn % c->n1, k = qn / c->n1;
    ept[qn][0] = ex[i];
    ept[qn][1] = d == 2 ? ex[k] : 0.0;
    eww[qn] = d == 2 ? ew[i] * ew[k] : ew[i];
  }
  double E[MAXQD][MAXL], DE[2][MAXQD][MAXL];
  for (int qn = 0; qn < neq; ++qn) {
    basis_eval(c, ept[qn], 0, 0, E[qn]);
    basis_eval(c, ept[qn], 1, 0, DE[0][qn]);
    if (d == 2) basis_eval(c, ept[qn], 0, 1, DE[1][qn]);
  }
  double M[MAXL][MAXL], Mref[MAXL][MAXL], Mrefinv[MAXL][MAXL];
  for (int i = 0; i < c->nl; ++i)
    for (int j = 0; j < c->nl; ++j) {
      double m = 0.0, k = 0.0;
      for (int qn = 0; qn < neq; ++qn) {
        m += eww[qn] * E[qn][i] * E[qn][j];
        for (int ax = 0; ax < d; ++ax) k += eww[qn] * DE[ax][qn][i] * DE[ax][qn][j];
      }
      Mref[i][j] = m;
      M[i][j] = c->J * m;
      c->K[i][j] = c->J * c->g * c->g * k;
    }
  if (invert(c->nl, M, c->Minv) || invert(c->nl, Mref, Mrefinv)) {
    free(c);
    return NULL;
  }
  /* continuation of the side-s neighbour along `ax`: its polynomial at
     xi - 2 s e_ax, L2-projected onto the cell's space with the exact rule */
  for (int f = 0; f < c->nf; ++f) {
    double rhs[MAXL][MAXL];
    for (int qn = 0; qn < neq; ++qn) {
      double sh[2] = {ept[qn][0], ept[qn][1]};
      sh[c->fax[f]] -= 2.0 * c->fside[f];
      double Es[MAXL];
      basis_eval(c, sh, 0, 0, Es);
      for (int i = 0; i < c->nl; ++i)
        for (int j = 0; j < c->nl; ++j) {
          if (qn == 0) rhs[i][j] = 0.0;
          rhs[i][j] += eww[qn] * E[qn][i] * Es[j];
        }
    }
    for (int i = 0; i < c->nl; ++i)
      for (int j = 0; j < c->nl; ++j) {
        double s = 0.0;
        for (int k = 0; k < c->nl; ++k) s += Mrefinv[i][k] * rhs[k][j];
        c->cont[f][i][j] = s;
      }
  }
  /* scaled Sobolev semi-norm of Sec. 4: |v|_e^2 = sum over 1 <= |k| <= p of
     h^(2|k| - d) int_K |D^k v|^2 dx, with D^k = g^|k| D^k_xi and dx = J dxi */
  for (int i = 0; i < c->nl; ++i)
    for (int j = 0; j < c->nl; ++j) c->B[i][j] = 0.0;
  for (int s = 1; s <= P->p; ++s)
    for (int kx = s; kx >= (d == 1 ? s : 0); --kx) {
      const int ky = d == 1 ? 0 : s - kx;
      const double scale = pow(c->h, 2 * s - d) * pow(c->g, 2 * s) * c->J;
      for (int qn = 0; qn < neq; ++qn) {
        double Dk[MAXL];
        basis_eval(c, ept[qn], kx, ky, Dk);
        for (int i = 0; i < c->nl; ++i)
          for (int j = 0; j < c->nl; ++j) c->B[i][j] += scale * eww[qn] * Dk[i] * Dk[j];
      }
    }
  const size_t n = (size_t)c->ncells * c->nl;
  c->L = (double*)malloc(n * sizeof(double));
  c->W1 = (double*)malloc(n * sizeof(double));
  c->W2 = (double*)malloc(n * sizeof(double));
  if (!c->L || !c->W1 || !c->W2) {
    free(c->L);
    free(c->W1);
    free(c->W2);
    free(c);
    return NULL;
  }
  return c;
}

void orc_destroy(void* h) {
  orc_ctx* c = (orc_ctx*)h;
  if (!c) return;
  free(c->L);
  free(c->W1);
  free(c->W2);
  free(c);
}

int orc_sizes(void* h, long* ncells, int* nloc) {
  const orc_ctx* c = (const orc_ctx*)h;
  *ncells = c->ncells;
  *nloc = c->nl;
  return 0;
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Pointwise physics                                                       */
/* ---------------------------------------------------------------------- */

/* F(u) at the physical point (x, y): component ax */
static double flux_c(const orc_problem* P, int ax, double u, double x, double y) {
  if (P->flux == LINADV) {
    if (P->dim == 1) return P->vx * u;
    return (ax == 0 ? P->vx - P->omega * (y - P->cy) : P->vy + P->omega * (x - P->cx)) * u;
  }
  if (P->flux == KPP) return ax == 0 ? sin(u) : cos(u);
  return (ax == 0 ? P->vx : P->vy) * 0.5 * u * u;
}

/* F'(u) at (x, y): component ax */
static double dflux_c(const orc_problem* P, int ax, double u, double x, double y) {
  if (P->flux == LINADV) {
    if (P->dim == 1) return P->vx;
    return ax == 0 ? P->vx - P->omega * (y - P->cy) : P->vy + P->omega * (x - P->cx);
  }
  if (P->flux == KPP) return ax == 0 ? cos(u) : -sin(u);
  return (ax == 0 ? P->vx : P->vy) * u;
}

/* Local Lax-Friedrichs flux H(u^-, u^+, n), n = side e_ax (Sec. 2).  For the
   linear and Burgers fluxes F'(w) . n is affine in w, so max |F'(w) . n| over
   the segment is attained at an end point.  KPP: |cos w| (x faces) or |sin w|
   (y faces) reaches 1 where the segment holds a point k pi (x) or
   pi/2 + k pi (y), else the larger end value. */
static double llf(const orc_problem* P, int ax, int side, double um, double up, double x, double y) {
  const double Fm = flux_c(P, ax, um, x, y) * side, Fp = flux_c(P, ax, up, x, y) * side;
  const double sm = fabs(dflux_c(P, ax, um, x, y) * side), sp = fabs(dflux_c(P, ax, up, x, y) * side);
  double s = sm > sp ? sm : sp;
  if (P->flux == KPP) {
    const double lo = um < up ? um : up, hi = um < up ? up : um;
    const double shift = ax == 0 ? 0.0 : 0.5 * M_PI;
    if (floor((hi - shift) / M_PI) >= ceil((lo - shift) / M_PI)) s = 1.0;
  }
  return 0.5 * (Fm + Fp) - 0.5 * s * (up - um);
}

/* ---------------------------------------------------------------------- */
/* The operator, one cell at a time                                        */
/* ---------------------------------------------------------------------- */

/* face neighbour f of cell (ix, iy), or -1 outside a non-periodic boundary */
static long neighbour(const orc_ctx* c, int ix, int iy, int f) {
  const orc_problem* P = &c->P;
  const int ny = P->dim == 2 ? P->ny : 1;
  int jx = ix, jy = iy;
  if (c->fax[f] == 0) {
    jx += c->fside[f];
    if (jx < 0 || jx >= P->nx) {
      if (!P->per_x) return -1;
      jx = (jx + P->nx) % P->nx;
    }
  } else {
    jy += c->fside[f];
    if (jy < 0 || jy >= ny) {
      if (!P->per_y) return -1;
      jy = (jy + ny) % ny;
    }
  }
  return (long)jy * P->nx + jx;
}

static double qform(const orc_ctx* c, const double* v) {
  double s = 0.0;
  for (int i = 0; i < c->nl; ++i)
    for (int j = 0; j < c->nl; ++j) s += v[i] * c->B[i][j] * v[j];
  return s;
}

/* gamma_e of the cell (Sec. 4, or the Zhao et al. sensor of Sec. 5.6) */
static double cell_gamma(const orc_ctx* c, const double* U, long e, int ix, int iy) {
  const orc_problem* P = &c->P;
  if (P->mode == MODE_DG) return 0.0;
  if (P->mode == MODE_LO) return 1.0;
  const int nl = c->nl;
  const double* u = U + e * nl;
  double cand[5][MAXL], lin[5], beta[5], alpha[5];
  int exists[5], m = 0;
  /* candidate 0: the cell's own polynomial */
  for (int j = 0; j < nl; ++j) cand[0][j] = u[j];
  exists[0] = 1;
  /* one candidate per face neighbour: its polynomial continued into the
     cell, with the cell's own mean */
  for (int f = 0; f < c->nf; ++f) {
    const long nb = neighbour(c, ix, iy, f);
    exists[f + 1] = nb >= 0;
    m += nb >= 0;
    for (int i = 0; i < nl; ++i) {
      double s = 0.0;
      if (nb >= 0)
        for (int j = 0; j < nl; ++j) s += c->cont[f][i][j] * U[nb * nl + j];
      cand[f + 1][i] = s;
    }
    cand[f + 1][0] = u[0];
  }
  lin[0] = 1.0 - m * P->wnb;
  for (int l = 1; l <= c->nf; ++l) lin[l] = P->wnb;
  double asum = 0.0;
  for (int l = 0; l <= c->nf; ++l) {
    beta[l] = qform(c, cand[l]);
    alpha[l] = exists[l] ? lin[l] / pow(P->eps + beta[l], P->r) : 0.0;
    asum += alpha[l];
  }
  if (P->mode == MODE_ZHAO) {
    if (m == 0) return 0.0;
    double dev = 0.0, lmin = INFINITY;
    for (int l = 0; l <= c->nf; ++l)
      if (exists[l]) {
        dev += pow(fabs((alpha[l] / asum) / lin[l] - 1.0), P->theta);
        if (lin[l] < lmin) lmin = lin[l];
      }
    return dev / (pow(fabs(1.0 / lmin - 1.0), P->theta) + m);
  }
  /* U - U*, U* = sum_l omega_l U_l */
  double diff[MAXL];
  for (int j = 0; j < nl; ++j) {
    double us = 0.0;
    for (int l = 0; l <= c->nf; ++l) us += (alpha[l] / asum) * cand[l][j];
    diff[j] = u[j] - us;
  }
  const double num2 = qform(c, diff), den2 = beta[0];
  double ratio;
  if (!(num2 > 0.0))
    ratio = 0.0;
  else if (!(den2 > 0.0))
    ratio = INFINITY;
  else
    ratio = sqrt(num2) / sqrt(den2);
  double gam = pow(ratio < 1.0 ? ratio : 1.0, P->q);
  if (!(ratio >= P->b)) gam = 0.0;
  return gam;
}

/* dU/dt of cell e and its gamma_e */
static void cell_rhs(const orc_ctx* c, const double* U, long e, double* L, double* gam_out) {
  const orc_problem* P = &c->P;
  const int d = P->dim, nl = c->nl;
  const int ix = (int)(e % P->nx), iy = (int)(e / P->nx);
  const double xc = P->x0 + (ix + 0.5) * c->h;
  const double yc = d == 2 ? P->y0 + (iy + 0.5) * c->h : 0.0;
  const double* u = U + e * nl;
  double R[MAXL];
  for (int i = 0; i < nl; ++i) R[i] = 0.0;

  /* volume term of eq. (weak2) and lambda_e (eq. visc) */
  double lam = 0.0;
  for (int qn = 0; qn < c->nvq; ++qn) {
    const double x = xc + 0.5 * c->h * c->vpt[qn][0];
    const double y = d == 2 ? yc + 0.5 * c->h * c->vpt[qn][1] : 0.0;
    double uq = 0.0;
    for (int j = 0; j < nl; ++j) uq += u[j] * c->V[qn][j];
    double sp2 = 0.0;
    for (int ax = 0; ax < d; ++ax) {
      const double F = flux_c(P, ax, uq, x, y);
      for (int i = 0; i < nl; ++i) R[i] += c->J * c->g * c->vw[qn] * F * c->DV[ax][qn][i];
      const double dF = dflux_c(P, ax, uq, x, y);
      sp2 += dF * dF;
    }
    const double sp = d == 1 ? fabs(dflux_c(P, 0, uq, x, y)) : sqrt(sp2);
    if (sp > lam) lam = sp;
  }
  if (P->lam_over > 0.0) lam = P->lam_over;

  /* face terms with the LLF flux */
  const int nq = d == 1 ? 1 : c->qf;
  for (int f = 0; f < c->nf; ++f) {
    const long nb = neighbour(c, ix, iy, f);
    for (int r = 0; r < nq; ++r) {
      const double x = xc + 0.5 * c->h * c->fpt[f][r][0];
      const double y = d == 2 ? yc + 0.5 * c->h * c->fpt[f][r][1] : 0.0;
      double um = 0.0, up;
      for (int j = 0; j < nl; ++j) um += u[j] * c->FV[f][r][j];
      if (nb >= 0) {
        up = 0.0;
        for (int j = 0; j < nl; ++j) up += U[nb * nl + j] * c->FVo[f][r][j];
      } else {
        up = P->bc;
      }
      const double H = llf(P, c->fax[f], c->fside[f], um, up, x, y);
      for (int i = 0; i < nl; ++i) R[i] -= c->Jf * c->fw[f][r] * H * c->FV[f][r][i];
    }
  }

  /* dissipation of eq. (astab) with nu_e = lambda_e h / (2p) */
  const double gam = cell_gamma(c, U, e, ix, iy);
  const double nu = lam * c->h / (2.0 * P->p);
  for (int i = 0; i < nl; ++i) {
    double Ku = 0.0;
    for (int j = 0; j < nl; ++j) Ku += c->K[i][j] * u[j];
    R[i] -= gam * nu * Ku;
  }
  /* mass inverse */
  for (int i = 0; i < nl; ++i) {
    double s = 0.0;
    for (int j = 0; j < nl; ++j) s += c->Minv[i][j] * R[j];
    L[i] = s;
  }
  if (gam_out) *gam_out = gam;
}

/* dU/dt = M^-1 (R(U) - s(U)) on the whole mesh; gamma optional */
int orc_rhs(void* h, const double* U, double* L, double* gamma) {
  const orc_ctx* c = (const orc_ctx*)h;
  const long n = c->ncells;
#pragma omp parallel for schedule(static)
  for (long e = 0; e < n; ++e) cell_rhs(c, U, e, L + e * c->nl, gamma ? gamma + e : NULL);
  return 0;
}

/* out = a X + b Y + s L (elementwise over the mesh) */
static void combine(long n, double a, const double* X, double b, const double* Y, double s, const double* L,
                    double* out) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) out[i] = a * X[i] + b * Y[i] + s * L[i];
}

/* Shu-Osher form of the five-stage fourth-order SSP method of Spiteri and
   Ruuth (published coefficients): U_k = sum_j (al[k][j] U_j + be[k][j] dt L(U_j)) */
static const double AL5[5][5] = {{1.0, 0, 0, 0, 0},
                                 {0.444370493651235, 0.555629506348765, 0, 0, 0},
                                 {0.620101851488403, 0.0, 0.379898148511597, 0, 0},
                                 {0.178079954393132, 0.0, 0.0, 0.821920045606868, 0},
                                 {0.0, 0.0, 0.517231671970585, 0.096059710526147, 0.386708617503269}};
static const double BE5[5][5] = {{0.391752226571890, 0, 0, 0, 0},
                                 {0.0, 0.368410593050371, 0, 0, 0},
                                 {0.0, 0.0, 0.251891774271694, 0, 0},
                                 {0.0, 0.0, 0.0, 0.544974750228521, 0},
                                 {0.0, 0.0, 0.0, 0.063692468666290, 0.226007483236906}};

/* One SSP Runge-Kutta step of the problem's order, in place */
int orc_step(void* hd, double* U, double dt) {
  orc_ctx* c = (orc_ctx*)hd;
  const long n = c->ncells * c->nl;
  if (c->P.rk_order == 2) {
    orc_rhs(c, U, c->L, NULL);
    combine(n, 1.0, U, 0.0, U, dt, c->L, c->W1);           /* U1 = U + dt L(U) */
    orc_rhs(c, c->W1, c->L, NULL);
    combine(n, 0.5, U, 0.5, c->W1, 0.5 * dt, c->L, U);     /* U/2 + U1/2 + dt/2 L(U1) */
    return 0;
  }
  if (c->P.rk_order == 3) {
    orc_rhs(c, U, c->L, NULL);
    combine(n, 1.0, U, 0.0, U, dt, c->L, c->W1);           /* U1 = U + dt L(U) */
    orc_rhs(c, c->W1, c->L, NULL);
    combine(n, 0.75, U, 0.25, c->W1, 0.25 * dt, c->L, c->W2);   /* U2 = 3/4 U + 1/4 U1 + 1/4 dt L(U1) */
    orc_rhs(c, c->W2, c->L, NULL);
    combine(n, 1.0 / 3.0, U, 2.0 / 3.0, c->W2, (2.0 / 3.0) * dt, c->L, U);  /* eq. (ssp) */
    return 0;
  }
  /* five stages: keep U_0..U_4 and L(U_0)..L(U_4) */
  double* st[6];
  double* Ls[5];
  st[0] = U;
  for (int k = 1; k < 6; ++k) st[k] = NULL;
  for (int k = 0; k < 5; ++k) Ls[k] = NULL;
  int ok = 1;
  for (int k = 1; k < 6 && ok; ++k) ok = (st[k] = (double*)malloc(n * sizeof(double))) != NULL;
  for (int k = 0; k < 5 && ok; ++k) ok = (Ls[k] = (double*)malloc(n * sizeof(double))) != NULL;
  if (ok) {
    orc_rhs(c, U, Ls[0], NULL);
    for (int k = 1; k <= 5; ++k) {
      double* out = st[k];
#pragma omp parallel for schedule(static)
      for (long i = 0; i < n; ++i) {
        double v = 0.0;
        for (int j = 0; j < k; ++j) {
          if (AL5[k - 1][j] != 0.0) v += AL5[k - 1][j] * st[j][i];
          if (BE5[k - 1][j] != 0.0) v += BE5[k - 1][j] * dt * Ls[j][i];
        }
        out[i] = v;
      }
      if (k < 5) orc_rhs(c, out, Ls[k], NULL);
    }
    memcpy(U, st[5], n * sizeof(double));
  }
  for (int k = 1; k < 6; ++k) free(st[k]);
  for (int k = 0; k < 5; ++k) free(Ls[k]);
  return ok ? 0 : -1;
}

int orc_run(void* h, double* U, double dt, int nsteps) {
  for (int s = 0; s < nsteps; ++s)
    if (orc_step(h, U, dt)) return -1;
  return 0;
}
