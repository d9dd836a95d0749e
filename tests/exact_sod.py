"""The exact solution of Sod's shock tube (test side): the star state of the
Riemann problem from the pressure function of the two waves (a rarefaction to
the left, a shock to the right), solved by bisection, and the density at
(x, t) sampled through the fan, the contact and the shock.  Its jump
conditions are checked in test_oracle_euler.py."""
import math

import numpy as np

GAMMA = 1.4   # the heat capacity ratio of Sec. 5.6


def _star(g=GAMMA):
    rl, pl, rr, pr = 1.0, 1.0, 0.125, 0.1
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def fk(p, rk, pk, ck):
        if p > pk:
            A, B = 2 / ((g + 1) * rk), (g - 1) / (g + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        return 2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)

    lo, hi = 1e-8, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if fk(mid, rl, pl, cl) + fk(mid, rr, pr, cr) < 0 else (lo, mid)
    ps = 0.5 * (lo + hi)
    us = 0.5 * (fk(ps, rr, pr, cr) - fk(ps, rl, pl, cl))
    rls = rl * (ps / pl) ** (1 / g)
    q = ps / pr
    rrs = rr * (q + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * q + 1)
    S = cr * math.sqrt((g + 1) / (2 * g) * q + (g - 1) / (2 * g))
    return dict(ps=ps, us=us, rls=rls, rrs=rrs, S=S, cl=cl, cls=cl * (ps / pl) ** ((g - 1) / (2 * g)))


def sod_density(x, t, g=GAMMA):
    s = _star(g)
    xi = (np.asarray(x) - 0.5) / t
    cl = s["cl"]
    fan_c = 2 / (g + 1) * (cl - (g - 1) / 2 * xi)
    fan = 1.0 * (np.maximum(fan_c, 1e-300) / cl) ** (2 / (g - 1))
    return np.select([xi < -cl, xi < s["us"] - s["cls"], xi < s["us"], xi < s["S"]],
                     [1.0, fan, s["rls"], s["rrs"]], 0.125)
