"""Brute-force evaluation of the paper's integrals on tiny meshes.

An implementation independent of the oracle: numpy Legendre series
(numpy.polynomial.legendre), integrals in *physical* coordinates with
high-order Gauss rules, one Python loop iteration per cell and per face.  It
evaluates, for every cell K_e:

* R_i = int_K grad(phi_i) . F(u_h) dx - int_dK phi_i H_LLF ds   (Sec. 2, eq. weak2)
* lambda_e, nu_e = lambda_e h / (2p), s_i = gamma nu int grad(phi_i).grad(u_h)  (Sec. 3)
* the scaled Sobolev semi-norm sum_k h^{2|k|-d} int_K |D^k v|^2 dx and the
  sensor gamma_e built from the continued neighbour polynomials (Sec. 4)
* dU/dt = M^{-1}(R - s)

Integrands that are not polynomials (the Burgers LLF wave speed, lambda_e,
every integrand of the KPP flux) use the same Gauss point counts as the
method, taken from numpy.  The LLF wave speed s+ is the maximum of |F'.n|
along the segment between the two states, found by sampling the segment and
refining the best sample by ternary search.
"""

import math

import numpy as np
from numpy.polynomial import legendre as L

HIGH = 24  # points per axis for polynomial integrands


def _gauss(n):
    return L.leggauss(n)


class Brute:
    def __init__(self, w, exterior=None):
        """w: an inputs.Workload-like object (fields only); exterior(x, y):
        the state outside non-periodic faces (default: the constant
        bc_value)."""
        self.w = w
        self.exterior = exterior
        self.d = w.dim
        self.p = w.p
        self.n1 = w.p + 1
        self.h = (w.x1 - w.x0) / w.nx
        self.ny = w.ny if w.dim == 2 else 1

    # -- geometry --------------------------------------------------------
    def centre(self, e):
        ix, iy = e % self.w.nx, e // self.w.nx
        xc = self.w.x0 + (ix + 0.5) * self.h
        yc = self.w.y0 + (iy + 0.5) * self.h
        return xc, yc

    def neighbour(self, e, axis, side):
        """(index, geometric centre) of the face neighbour, or None."""
        w = self.w
        ix, iy = e % w.nx, e // w.nx
        jx, jy = (ix + side, iy) if axis == 0 else (ix, iy + side)
        n = w.nx if axis == 0 else self.ny
        j = jx if axis == 0 else jy
        per = w.periodic_x if axis == 0 else w.periodic_y
        if not (0 <= j < n):
            if not per:
                return None
            jx, jy = jx % w.nx, jy % self.ny
        xc, yc = self.centre(e)
        if axis == 0:
            xc += side * self.h
        else:
            yc += side * self.h
        return jx + w.nx * jy, (xc, yc)

    # -- polynomials in physical coordinates ------------------------------
    def coef(self, c):
        c = np.asarray(c, dtype=np.float64)
        if self.d == 1:
            return c
        return c.reshape(self.n1, self.n1).T      # C[a, b], j = a + n1 b

    def value(self, c, centre, x, y=None, k=(0, 0)):
        """D^k of sum_j c_j phi_j((x - centre)/(h/2)) at physical points."""
        C = self.coef(c)
        s = 2.0 / self.h
        if self.d == 1:
            return L.legval((x - centre[0]) * s, L.legder(C, k[0]) if k[0] else C) * s ** k[0]
        D = C
        if k[0]:
            D = L.legder(D, k[0], axis=0)
        if k[1]:
            D = L.legder(D, k[1], axis=1)
        return L.legval2d((x - centre[0]) * s, (y - centre[1]) * s, D) * s ** (k[0] + k[1])

    def unit(self, j):
        c = np.zeros(self.n1 ** self.d)
        c[j] = 1.0
        return c

    def cell_rule(self, e, n=HIGH):
        t, wt = _gauss(n)
        xc, yc = self.centre(e)
        x = xc + 0.5 * self.h * t
        if self.d == 1:
            return x, None, 0.5 * self.h * wt
        y = yc + 0.5 * self.h * t
        X, Y = np.meshgrid(x, y, indexing="xy")
        W = np.outer(wt, wt) * (0.5 * self.h) ** 2
        return X.ravel(), Y.ravel(), W.ravel()

    # -- flux -------------------------------------------------------------
    def vel(self, x, y):
        w = self.w
        if self.d == 1:
            return np.full_like(x, w.vx), None
        return w.vx - w.omega * (y - w.cy), w.vy + w.omega * (x - w.cx)

    def F(self, u, x, y):
        w = self.w
        if w.flux == 2:
            return (np.sin(u), np.cos(u))
        if w.flux == 0:
            vx, vy = self.vel(x, y)
            return (vx * u,) if self.d == 1 else (vx * u, vy * u)
        return (w.vx * u * u / 2,) if self.d == 1 else (w.vx * u * u / 2, w.vy * u * u / 2)

    def dF(self, u, x, y):
        w = self.w
        if w.flux == 2:
            return (np.cos(u), -np.sin(u))
        if w.flux == 0:
            vx, vy = self.vel(x, y)
            return (vx + 0 * u,) if self.d == 1 else (vx + 0 * u, vy + 0 * u)
        return (w.vx * u,) if self.d == 1 else (w.vx * u, w.vy * u)

    # -- the operator -----------------------------------------------------
    def mass(self, e):
        x, y, W = self.cell_rule(e)
        c = self.centre(e)
        n = self.n1 ** self.d
        Phi = np.stack([self.value(self.unit(j), c, x, y) for j in range(n)])
        return (Phi * W) @ Phi.T

    def residual(self, U, e, qv, qf):
        w = self.w
        c = self.centre(e)
        n = self.n1 ** self.d
        R = np.zeros(n)
        # volume (polynomial integrand: high-order rule; KPP: the method's rule)
        x, y, W = self.cell_rule(e, qv if w.flux == 2 else HIGH)
        u = self.value(U[e], c, x, y)
        Fx = self.F(u, x, y)
        for j in range(n):
            for ax in range(self.d):
                k = (1, 0) if ax == 0 else (0, 1)
                R[j] += np.sum(W * Fx[ax] * self.value(self.unit(j), c, x, y, k))
        # faces
        for ax in range(self.d):
            for side in (-1, 1):
                if self.d == 1:
                    xf = np.array([c[0] + side * self.h / 2])
                    yf = None
                    wf = np.array([1.0])
                else:
                    nq = qf if w.flux in (1, 2) else HIGH
                    t, wt = _gauss(nq)
                    if ax == 0:
                        xf = np.full(nq, c[0] + side * self.h / 2)
                        yf = c[1] + 0.5 * self.h * t
                    else:
                        yf = np.full(nq, c[1] + side * self.h / 2)
                        xf = c[0] + 0.5 * self.h * t
                    wf = 0.5 * self.h * wt
                um = self.value(U[e], c, xf, yf)
                nb = self.neighbour(e, ax, side)
                if nb is None:
                    up = (np.full_like(um, w.bc_value) if self.exterior is None
                          else np.asarray(self.exterior(xf, yf), dtype=np.float64))
                else:
                    up = self.value(U[nb[0]], nb[1], xf, yf)
                Fm = self.F(um, xf, yf)[ax] * side
                Fp = self.F(up, xf, yf)[ax] * side
                # s+ = max over the segment between the states of |F'.n|
                wgrid = np.linspace(0.0, 1.0, 2001)[:, None]
                seg = wgrid * um[None, :] + (1 - wgrid) * up[None, :]
                xs = np.broadcast_to(xf, seg.shape)
                ys = None if yf is None else np.broadcast_to(yf, seg.shape)
                sp = np.max(np.abs(self.dF(seg, xs, ys)[ax] * side), axis=0)
                best = np.argmax(np.abs(self.dF(seg, xs, ys)[ax] * side), axis=0)
                for q in range(um.shape[0]):
                    def f(t, q=q):
                        s_ = np.array([t * um[q] + (1 - t) * up[q]])
                        xq = np.array([xf[q]])
                        yq = None if yf is None else np.array([yf[q]])
                        return float(np.abs(self.dF(s_, xq, yq)[ax] * side)[0])
                    a_, b_ = max(0.0, wgrid[max(best[q] - 1, 0), 0]), min(1.0, wgrid[min(best[q] + 1, 2000), 0])
                    for _ in range(100):
                        m1, m2 = a_ + (b_ - a_) / 3, b_ - (b_ - a_) / 3
                        if f(m1) < f(m2):
                            a_ = m1
                        else:
                            b_ = m2
                    sp[q] = max(sp[q], f(0.5 * (a_ + b_)))
                H = 0.5 * (Fm + Fp) - 0.5 * sp * (up - um)
                for j in range(n):
                    R[j] -= np.sum(wf * H * self.value(self.unit(j), c, xf, yf))
        return R

    def seminorm2(self, coeffs, e):
        """sum_{1<=|k|<=p} h^{2|k|-d} int_K |D^k v|^2 dx, physical coordinates."""
        c = self.centre(e)
        x, y, W = self.cell_rule(e, HIGH)
        tot = 0.0
        ks = ([(k, 0) for k in range(1, self.p + 1)] if self.d == 1 else
              [(a, b) for a in range(self.p + 1) for b in range(self.p + 1) if 1 <= a + b <= self.p])
        for k in ks:
            v = self.value(coeffs, c, x, y, k)
            tot += self.h ** (2 * (k[0] + k[1]) - self.d) * np.sum(W * v * v)
        return tot

    def candidates(self, U, e):
        """Own polynomial and each existing face neighbour's polynomial continued
        into K_e, L2-projected onto V_p(K_e), mean replaced by the own mean."""
        c = self.centre(e)
        n = self.n1 ** self.d
        x, y, W = self.cell_rule(e, HIGH)
        Phi = np.stack([self.value(self.unit(j), c, x, y) for j in range(n)])
        M = (Phi * W) @ Phi.T
        own_mean = np.sum(W * self.value(U[e], c, x, y)) / np.sum(W)
        out = [np.array(U[e], dtype=np.float64)]
        for ax in range(self.d):
            for side in (-1, 1):
                nb = self.neighbour(e, ax, side)
                if nb is None:
                    continue
                v = self.value(U[nb[0]], nb[1], x, y)
                cl = np.linalg.solve(M, (Phi * W) @ v)
                # replace the mean: shift the constant mode
                mean = np.sum(W * self.value(cl, c, x, y)) / np.sum(W)
                cl[0] += own_mean - mean
                out.append(cl)
        return out

    def gamma(self, U, e):
        w = self.w
        if w.mode == 0:
            return 0.0
        if w.mode == 1:
            return 1.0
        cands = self.candidates(U, e)
        m = len(cands) - 1
        lin = [1.0 - m * w.w_nb] + [w.w_nb] * m
        beta = [self.seminorm2(cl, e) for cl in cands]
        alpha = np.array([lin[l] / (w.eps + beta[l]) ** w.r for l in range(m + 1)])
        om = alpha / alpha.sum()
        ustar = sum(om[l] * cands[l] for l in range(m + 1))
        num = math.sqrt(self.seminorm2(np.asarray(U[e]) - ustar, e))
        den = math.sqrt(beta[0])
        if num == 0.0:
            ratio = 0.0
        elif den == 0.0:
            ratio = math.inf
        else:
            ratio = num / den
        if ratio < w.b:
            return 0.0
        return min(1.0, ratio) ** w.q

    def lam(self, U, e, qv):
        w = self.w
        if w.lambda_override > 0:
            return w.lambda_override
        t, _ = _gauss(qv)
        c = self.centre(e)
        x = c[0] + 0.5 * self.h * t
        if self.d == 1:
            return float(np.max(np.abs(self.dF(self.value(U[e], c, x), x, None)[0])))
        X, Y = np.meshgrid(x, c[1] + 0.5 * self.h * t, indexing="xy")
        X, Y = X.ravel(), Y.ravel()
        g = self.dF(self.value(U[e], c, X, Y), X, Y)
        return float(np.max(np.hypot(g[0], g[1])))

    def rhs(self, U, qv, qf):
        """dU/dt for every cell, plus gamma and lambda per cell."""
        U = np.asarray(U, dtype=np.float64)
        out = np.zeros_like(U)
        gam = np.zeros(U.shape[0])
        lam = np.zeros(U.shape[0])
        n = self.n1 ** self.d
        for e in range(U.shape[0]):
            R = self.residual(U, e, qv, qf)
            g = self.gamma(U, e)
            lm = self.lam(U, e, qv)
            nu = lm * self.h / (2 * self.p)
            c = self.centre(e)
            x, y, W = self.cell_rule(e, HIGH)
            s = np.zeros(n)
            if g > 0:
                for i in range(n):
                    for ax in range(self.d):
                        k = (1, 0) if ax == 0 else (0, 1)
                        s[i] += np.sum(W * self.value(self.unit(i), c, x, y, k)
                                       * self.value(U[e], c, x, y, k))
                s *= g * nu
            out[e] = np.linalg.solve(self.mass(e), R - s)
            gam[e], lam[e] = g, lm
        return out, gam, lam
