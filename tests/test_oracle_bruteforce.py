"""The oracle's operator against brute-force evaluation of the paper's integrals
(tests/bruteforce.py: numpy Legendre series, physical coordinates) on tiny meshes."""
import numpy as np
import pytest
import torch

from bruteforce import Brute
from helpers import oracle_for
from paper_2309_12019_amd import inputs


def _random_state(w, seed, smooth=False):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((w.ncells, w.nloc))
    if smooth:
        U[:, 1:] *= 0.05
    return U


CASES = []
for p in (1, 2, 3):
    for mode in (inputs.MODE_DG, inputs.MODE_LO, inputs.MODE_WENO):
        CASES.append(("adv1d", p, mode))
        CASES.append(("burgers1d", p, mode))
for p in (1, 2, 3):
    CASES.append(("rot2d", p, inputs.MODE_WENO))
    CASES.append(("burgers2d", p, inputs.MODE_WENO))
CASES += [("rot2d", 2, inputs.MODE_LO), ("burgers2d", 2, inputs.MODE_DG),
          ("adv2d", 2, inputs.MODE_WENO), ("rot2d_per", 2, inputs.MODE_WENO),
          ("kpp2d", 1, inputs.MODE_WENO), ("kpp2d", 2, inputs.MODE_DG), ("kpp2d", 2, inputs.MODE_WENO),
          ("kpp2d_per", 3, inputs.MODE_LO)]


def _workload(kind, p, mode):
    if kind == "adv1d":
        w = inputs.adv1d(5, p, mode=mode)
        w.vx = -0.7
    elif kind == "burgers1d":
        w = inputs.burgers1d(5, p, mode=mode)
    elif kind == "rot2d":
        w = inputs.rot2d(4, p, mode=mode, ny=2)
        w.cy = 0.25
    elif kind == "rot2d_per":
        w = inputs.rot2d(4, p, mode=mode)
        w.periodic_x = w.periodic_y = True
        w.vx, w.vy = 0.25, -0.25   # v.n changes sign only on grid lines
    elif kind == "adv2d":
        w = inputs.rot2d(3, p, mode=mode)
        w.omega, w.vx, w.vy = 0.0, 0.6, -1.1
        w.periodic_x, w.bc_value = True, 0.4
    elif kind.startswith("kpp2d"):
        w = inputs.kpp2d(3, p, mode=mode, steps=1, lam=0.0)
        if kind == "kpp2d_per":
            w.periodic_x = w.periodic_y = True
    else:
        w = inputs.burgers2d(3, p, steps=1)
        w.mode = mode
        w.vx, w.vy = 1.0, 0.5
    return w


@pytest.mark.parametrize("kind,p,mode", CASES)
def test_rhs_matches_bruteforce(kind, p, mode):
    w = _workload(kind, p, mode)
    O = oracle_for(w)
    for seed, smooth in ((1, False), (2, True)):
        U = _random_state(w, seed, smooth)
        if kind.startswith("kpp2d"):
            U = 3.0 * U   # states several pi apart: s+ peaks inside the segments
        L, gam = O.rhs(torch.from_numpy(U), with_gamma=True)
        lam = O.max_speed(torch.from_numpy(U))
        Lb, gb, lb = Brute(w).rhs(U, O.P.qv(), O.P.qf())
        scale = np.abs(Lb).max()
        assert np.abs(L.numpy() - Lb).max() <= 1e-12 * scale
        assert np.allclose(gam.numpy(), gb, rtol=1e-11, atol=1e-13)
        assert np.allclose(lam.numpy(), lb, rtol=1e-14, atol=1e-15)
        if mode == inputs.MODE_WENO and smooth:
            assert (gb < 1).any()


@pytest.mark.parametrize("dim,p", [(1, 2), (1, 4), (2, 2), (2, 3)])
def test_seminorm_matches_bruteforce(dim, p):
    w = inputs.adv1d(3, p) if dim == 1 else inputs.rot2d(3, p)
    O = oracle_for(w)
    U = _random_state(w, 7)
    sn = O.seminorm2(torch.from_numpy(U)).numpy()
    bf = Brute(w)
    ref = np.array([bf.seminorm2(U[e], e) for e in range(w.ncells)])
    assert np.allclose(sn, ref, rtol=1e-13)


def test_sensor_weights_match_bruteforce():
    """beta_l and omega_l of the HWENO reconstruction (2D, non-periodic corner
    cells have fewer candidates)."""
    w = inputs.rot2d(3, 2)
    O = oracle_for(w)
    U = _random_state(w, 3)
    _, det = O.sensor(torch.from_numpy(U), details=True)
    bf = Brute(w)
    for e in range(w.ncells):
        cands = bf.candidates(U, e)
        ex = det["exists"][e].numpy()
        assert ex[1:].sum() == len(cands) - 1
        got = det["cands"][e][ex].numpy()
        assert np.allclose(got, np.array(cands), rtol=1e-12, atol=1e-12)
        beta = np.array([bf.seminorm2(c, e) for c in cands])
        assert np.allclose(det["beta"][e][ex].numpy(), beta, rtol=1e-12)
