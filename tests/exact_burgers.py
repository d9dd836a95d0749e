"""The exact solution of the 1D Burgers problem of Sec. 5.2 before the shock
(test side): u = u0(x - u t) for u0 = sin(2 pi x), solved by Newton's method."""
import numpy as np


def burgers_exact(x, t):
    """u = u0(x - u t) for u0 = sin(2 pi x), solved by Newton's method."""
    u = np.sin(2 * np.pi * x)
    for _ in range(60):
        a = 2 * np.pi * (x - u * t)
        u = u - (u - np.sin(a)) / (1 + 2 * np.pi * t * np.cos(a))
    return u
