// Compile-time tables for the tensor Legendre basis on [-1,1]^d.
//
// Everything here is constexpr: the kernels see the values as immediate
// constants, and entries that vanish identically (parity, degree) are known to
// be zero at compile time so the unrolled loops can skip them.
//
// Polynomial tables (Legendre coefficients, derivative Gram matrices, the
// neighbour-continuation matrix, the sensor's quadratic form) are computed in
// exact rational arithmetic and rounded to double once.  Gauss-Legendre rules
// come from Newton's method on the three-term recurrence.
#pragma once

#include <cstdint>

namespace dgk {

constexpr int kMaxP = 4;
constexpr int kMaxQ = 8;

// ---------------------------------------------------------------------------
// exact rationals (small: every table here stays far below 2^62)
// ---------------------------------------------------------------------------
struct Rat {
  long long n = 0, d = 1;
};
constexpr long long iabs(long long a) { return a < 0 ? -a : a; }
constexpr long long igcd(long long a, long long b) {
  a = iabs(a);
  b = iabs(b);
  while (b) {
    long long t = a % b;
    a = b;
    b = t;
  }
  return a ? a : 1;
}
constexpr Rat mk(long long n, long long d = 1) {
  if (d < 0) { n = -n; d = -d; }
  long long g = igcd(n, d);
  return Rat{n / g, d / g};
}
constexpr Rat add(Rat a, Rat b) { return mk(a.n * b.d + b.n * a.d, a.d * b.d); }
constexpr Rat mul(Rat a, Rat b) {
  long long g1 = igcd(a.n, b.d), g2 = igcd(b.n, a.d);
  return mk((a.n / g1) * (b.n / g2), (a.d / g2) * (b.d / g1));
}
constexpr double to_d(Rat a) { return static_cast<double>(a.n) / static_cast<double>(a.d); }

// polynomial with rational coefficients, degree <= 2*kMaxP + 2
constexpr int kPolyLen = 2 * kMaxP + 3;
struct Poly {
  Rat c[kPolyLen] = {};
};

// Legendre P_a via (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}
constexpr Poly legendre(int a) {
  Poly p0{}, p1{};
  p0.c[0] = mk(1);
  p1.c[1] = mk(1);
  if (a == 0) return p0;
  for (int k = 1; k < a; ++k) {
    Poly nx{};
    for (int i = 0; i + 1 < kPolyLen; ++i) nx.c[i + 1] = add(nx.c[i + 1], mul(mk(2 * k + 1, k + 1), p1.c[i]));
    for (int i = 0; i < kPolyLen; ++i) nx.c[i] = add(nx.c[i], mul(mk(-k, k + 1), p0.c[i]));
    p0 = p1;
    p1 = nx;
  }
  return p1;
}
constexpr Poly deriv(Poly p, int k) {
  for (int r = 0; r < k; ++r) {
    Poly q{};
    for (int i = 1; i < kPolyLen; ++i) q.c[i - 1] = mul(mk(i), p.c[i]);
    p = q;
  }
  return p;
}
constexpr Poly pmul(const Poly& a, const Poly& b) {
  Poly r{};
  for (int i = 0; i < kPolyLen; ++i)
    for (int j = 0; i + j < kPolyLen; ++j)
      if (a.c[i].n && b.c[j].n) r.c[i + j] = add(r.c[i + j], mul(a.c[i], b.c[j]));
  return r;
}
// integral over [-1,1]
constexpr Rat integral(const Poly& p) {
  Rat s = mk(0);
  for (int i = 0; i < kPolyLen; i += 2) s = add(s, mul(p.c[i], mk(2, i + 1)));
  return s;
}
// p(x + t) for an integer shift t
constexpr Poly shift(const Poly& p, long long t) {
  Poly r{};
  for (int i = 0; i < kPolyLen; ++i) {
    if (!p.c[i].n) continue;
    // (x + t)^i = sum_k C(i,k) t^(i-k) x^k
    long long binom = 1;
    for (int k = 0; k <= i; ++k) {
      long long tp = 1;
      for (int e = 0; e < i - k; ++e) tp *= t;
      r.c[k] = add(r.c[k], mul(p.c[i], mk(binom * tp)));
      binom = binom * (i - k) / (k + 1);
    }
  }
  return r;
}
constexpr Rat leg_at(int a, int x) {  // P_a(x) for x = +-1
  Poly p = legendre(a);
  Rat s = mk(0);
  long long xp = 1;
  for (int i = 0; i < kPolyLen; ++i) {
    s = add(s, mul(p.c[i], mk(xp)));
    xp *= x;
  }
  return s;
}

// ---------------------------------------------------------------------------
// Gauss-Legendre rules
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;
constexpr double ccos(double x) {
  while (x > kPi) x -= 2 * kPi;
  while (x < -kPi) x += 2 * kPi;
  double term = 1, sum = 1;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
template <int Q>
struct Gauss {
  double x[Q] = {}, w[Q] = {};
};
template <int Q>
constexpr Gauss<Q> make_gauss() {
  Gauss<Q> g{};
  for (int i = 0; i < Q; ++i) {
    double x = ccos(kPi * (i + 0.75) / (Q + 0.5));
    double dp = 1;
    for (int it = 0; it < 60; ++it) {
      double p0 = 1, p1 = x;
      for (int k = 2; k <= Q; ++k) {
        double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = Q * (x * p1 - p0) / (x * x - 1);
      x -= p1 / dp;
    }
    double p0 = 1, p1 = x;
    for (int k = 2; k <= Q; ++k) {
      double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = Q * (x * p1 - p0) / (x * x - 1);
    g.x[Q - 1 - i] = x;  // ascending
    g.w[Q - 1 - i] = 2 / ((1 - x * x) * dp * dp);
  }
  return g;
}
constexpr double horner(const Poly& p, double x) {
  double s = 0;
  for (int i = kPolyLen - 1; i >= 0; --i) s = s * x + to_d(p.c[i]);
  return s;
}

// ---------------------------------------------------------------------------
// Node tables for degree P and Q points: L[a][q] = P_a(x_q), D[a][q] = P_a'(x_q)
// ---------------------------------------------------------------------------
template <int P, int Q>
struct NodeTab {
  static constexpr int N = P + 1;
  double L[N][Q] = {}, D[N][Q] = {}, w[Q] = {}, x[Q] = {};
};
template <int P, int Q>
constexpr NodeTab<P, Q> make_nodes() {
  NodeTab<P, Q> t{};
  Gauss<Q> g = make_gauss<Q>();
  for (int q = 0; q < Q; ++q) {
    t.w[q] = g.w[q];
    t.x[q] = g.x[q];
    for (int a = 0; a <= P; ++a) {
      const Poly la = legendre(a);
      t.L[a][q] = horner(la, g.x[q]);
      t.D[a][q] = horner(deriv(la, 1), g.x[q]);
    }
  }
  return t;
}

// ---------------------------------------------------------------------------
// Degree tables
//   mhat[a] = int P_a^2 = 2/(2a+1), minv[a] = 1/mhat[a]
//   S[a][b] = int P_a' P_b'   (the 1D stiffness of the dissipative term)
//   G[k][a][b] = int P_a^(k) P_b^(k)
//   T[s][a][b]: P_a(xi - 2 s) = sum_b T[s][a][b] P_b(xi), s = 0: side -1
//               (left/bottom neighbour, xi + 2), s = 1: side +1 (xi - 2)
//   sgn[a] = P_a(-1) = (-1)^a
// ---------------------------------------------------------------------------
template <int P>
struct DegTab {
  static constexpr int N = P + 1;
  double mhat[N] = {}, minv[N] = {}, sgn[N] = {};
  double S[N][N] = {};
  double G[P + 1][N][N] = {};
  double T[2][N][N] = {};
};
template <int P>
constexpr DegTab<P> make_deg() {
  DegTab<P> t{};
  constexpr int N = P + 1;
  Poly leg[N] = {}, dl[P + 1][N] = {};
  for (int a = 0; a < N; ++a) {
    leg[a] = legendre(a);
    for (int k = 0; k <= P; ++k) dl[k][a] = deriv(leg[a], k);
  }
  for (int a = 0; a < N; ++a) {
    t.mhat[a] = to_d(mk(2, 2 * a + 1));
    t.minv[a] = to_d(mk(2 * a + 1, 2));
    t.sgn[a] = to_d(leg_at(a, -1));
    for (int b = 0; b < N; ++b) {
      t.S[a][b] = to_d(integral(pmul(dl[1][a], dl[1][b])));
      for (int k = 0; k <= P; ++k) t.G[k][a][b] = to_d(integral(pmul(dl[k][a], dl[k][b])));
    }
    for (int s = 0; s < 2; ++s) {
      Poly sh = shift(leg[a], s == 0 ? 2 : -2);
      for (int b = 0; b < N; ++b) t.T[s][a][b] = to_d(mul(mk(2 * b + 1, 2), integral(pmul(sh, leg[b]))));
    }
  }
  return t;
}

// Sensor quadratic form: ||v||_e^2 = c^T B c for v = sum_j c_j phi_j, i.e.
// sum over 1 <= |k| <= p of 2^{2|k| - d} int_{[-1,1]^d} (D^k v)^2 (the scaled
// Sobolev semi-norm, h-independent on the reference cell).
template <int DIM, int P>
struct SenTab {
  static constexpr int N = P + 1;
  static constexpr int NL = DIM == 1 ? N : N * N;
  double B[NL][NL] = {};
};
template <int DIM, int P>
constexpr SenTab<DIM, P> make_sen() {
  SenTab<DIM, P> t{};
  constexpr int N = P + 1;
  // exact Gram matrices of derivatives
  Rat G[P + 1][N][N] = {};
  Poly dl[P + 1][N] = {};
  for (int a = 0; a < N; ++a)
    for (int k = 0; k <= P; ++k) dl[k][a] = deriv(legendre(a), k);
  for (int k = 0; k <= P; ++k)
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) G[k][a][b] = integral(pmul(dl[k][a], dl[k][b]));
  if constexpr (DIM == 1) {
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) {
        Rat s = mk(0);
        for (int k = 1; k <= P; ++k) s = add(s, mul(mk(1LL << (2 * k - 1)), G[k][a][b]));
        t.B[a][b] = to_d(s);
      }
  } else {
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b)
        for (int a2 = 0; a2 < N; ++a2)
          for (int b2 = 0; b2 < N; ++b2) {
            Rat s = mk(0);
            for (int k1 = 0; k1 <= P; ++k1)
              for (int k2 = 0; k1 + k2 <= P; ++k2) {
                if (k1 + k2 < 1) continue;
                s = add(s, mul(mk(1LL << (2 * (k1 + k2) - 2)), mul(G[k1][a][a2], G[k2][b][b2])));
              }
            t.B[a + N * b][a2 + N * b2] = to_d(s);
          }
  }
  return t;
}

// Gauss points per axis used for volume and face quadrature: exact for the
// polynomial part of the integrands.  Linear flux: degree 2p+1 -> p+1 points.
// Burgers: 1D degree 3p-1 -> ceil(3p/2); 2D degree 3p -> ceil((3p+1)/2).
// KPP (sin and cos of u_h: no exact rule): p+2.
constexpr int quad_points(int dim, int p, int flux) {
  if (flux == 0) return p + 1;
  if (flux == 2 || flux == 3) return p + 2;  // KPP, Euler: rational or transcendental fluxes
  return dim == 1 ? (3 * p + 1) / 2 : (3 * p + 2) / 2;
}

template <int DIM, int P, int FLUX>
struct Tables {
  static constexpr int N = P + 1;
  static constexpr int NL = DIM == 1 ? N : N * N;
  static constexpr int Q = quad_points(DIM, P, FLUX);
  static constexpr NodeTab<P, Q> nd = make_nodes<P, Q>();
  static constexpr DegTab<P> dg = make_deg<P>();
  static constexpr SenTab<DIM, P> sn = make_sen<DIM, P>();
};

}  // namespace dgk
