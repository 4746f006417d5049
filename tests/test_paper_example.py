"""The oracle at the paper's example parameters (tests/golden/paper_example.json).

The cold start makes every link the identity, so D is diagonal in momentum
space and D^dag D = M(p)^2 + 4 kappa^2 sum sin^2 p on each plane wave (a
closed form derived by hand, independent of the oracle's code).  The solve
of D^dag D x = b at eps_CG is then checked against that closed form.
"""

import json
import os

import numpy as np

import oracle as O
import qcdgen

HERE = os.path.dirname(os.path.abspath(__file__))
BC = (1, 1, 1, -1)


def test_paper_example_cold_solve():
    cfg = json.load(open(os.path.join(HERE, "golden", "paper_example.json")))
    L = tuple(cfg["lattice"])
    kappa, eps = cfg["kappa"], cfg["eps_CG"]
    U = qcdgen.links_unit(L)
    b = qcdgen.gaussian_spinor(L, qcdgen.rng(123))
    x, info = O.solve_DdagD(U, b, kappa, BC, eo=False, tol=eps)
    assert info["converged"] and info["true_resid"] <= eps
    # closed form: FFT with the antiperiodic phase, divide by the scalar symbol
    Lx, Ly, Lz, Lt = L
    t = np.arange(Lt)
    tw = np.exp(-1j * np.pi * t / Lt)[:, None, None, None, None, None]   # removes the half-integer t momentum
    bh = np.fft.fftn(b * tw, axes=(0, 1, 2, 3))
    k = [2 * np.pi * np.fft.fftfreq(n) for n in (Lt, Lz, Ly, Lx)]
    pt, pz, py, px = np.meshgrid(*k, indexing="ij")
    pt = pt + np.pi / Lt
    ps = (px, py, pz, pt)
    M = 1 - 2 * kappa * sum(np.cos(p) for p in ps)
    lam = M ** 2 + 4 * kappa ** 2 * sum(np.sin(p) ** 2 for p in ps)
    xe = np.fft.ifftn(bh / lam[..., None, None], axes=(0, 1, 2, 3)) / tw
    cond = lam.max() / lam.min()
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) <= 4 * cond * eps
