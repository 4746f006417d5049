"""GPU pseudofermion heatbath, action, force and momentum update against the
oracle, plus finite differences of the GPU action against the GPU force."""

import numpy as np
import pytest

import oracle as O
import qcdgen

pytestmark = pytest.mark.gpu

BC = (1, 1, 1, -1)


def _torch():
    import torch
    return torch


def _W():
    from paper_2409_03030_amd import wdirac
    return wdirac


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def _lattice(L, U, recon=12):
    W = _W()
    lat = W.Lattice(L, BC)
    Ud = _dev(U)
    for prec in ("f64", "f32", "f16"):
        lat.set_gauge(Ud, prec, recon)
    return lat


def _random_su3_algebra(g):
    A = g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3))
    T = 0.5 * (A - A.conj().T)
    return T - np.trace(T) / 3 * np.eye(3)


def _expm_antihermitian(T):
    w, V = np.linalg.eigh(-1j * T)
    return (V * np.exp(1j * w)) @ V.conj().T


@pytest.mark.parametrize("L,inner,recon", [((4, 4, 4, 4), "f64", 18), ((6, 4, 4, 6), "f64", 12),
                                           ((6, 4, 4, 6), "f32", 12)])
def test_force_and_action_match_oracle(L, inner, recon):
    W = _W()
    g = qcdgen.rng(81)
    U = qcdgen.links_exp(L, 0.4, g)
    eta = qcdgen.gaussian_spinor(L, g)
    kappa = 0.12
    lat = _lattice(L, U, recon)
    p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0, tol=1e-12)
    F, S, st = lat.fermion_force(_dev(eta), kappa, params=p)
    assert st[0]["status"] == 0 and st[1]["status"] == 0
    F_ref, S_ref, info = O.fermion_force(U, eta, kappa, BC, tol=1e-13)
    assert info["converged"]
    Fh = _host(F)
    assert np.linalg.norm(Fh - F_ref) / np.linalg.norm(F_ref) <= 1e-8
    assert S == pytest.approx(S_ref, rel=1e-10)
    # the action alone skips the second solve and gives the same value
    F2, S2, st2 = lat.fermion_force(_dev(eta), kappa, params=p, force=False)
    assert F2 is None and S2 == S and st2[1]["iters"] == 0


def test_heatbath_identity_and_momentum_update():
    W = _W()
    L = (4, 4, 2, 6)
    g = qcdgen.rng(82)
    U = qcdgen.links_haar(L, g)
    xi = qcdgen.gaussian_spinor(L, g)
    kappa = 0.13
    lat = _lattice(L, U)
    eta = lat.pseudofermion(_dev(xi), kappa)
    eta_h = _host(eta)
    ref = O.pseudofermion_heatbath(U, xi, kappa, BC)
    assert np.linalg.norm(eta_h - ref) / np.linalg.norm(ref) <= 1e-13
    p = W.default_params(tol=1e-12)
    F, S, _ = lat.fermion_force(eta, kappa, params=p)
    assert S == pytest.approx(float(np.vdot(xi.ravel(), xi.ravel()).real), rel=1e-9)
    # p += factor TA(F)
    mom = g.standard_normal((4,) + qcdgen.site_shape(L) + (3, 3)) * 1j
    mom = O.traceless_antihermitian(mom + g.standard_normal(mom.shape))
    pd = _dev(mom)
    lat.ta_add(pd, -0.05, F)
    expect = O.momentum_update(mom, -0.05, _host(F))
    assert np.allclose(_host(pd), expect, rtol=0, atol=1e-14)


def test_gpu_force_matches_gpu_action_differences():
    """Central differences of the GPU action along random su(3) directions at
    single links, against Re tr[T F] of the GPU force."""
    W = _W()
    L = (4, 4, 4, 6)
    g = qcdgen.rng(83)
    U = qcdgen.links_exp(L, 0.4, g)
    eta = _dev(qcdgen.gaussian_spinor(L, g))
    kappa = 0.125
    p = W.default_params(tol=1e-14)
    lat = _lattice(L, U)
    F, S, _ = lat.fermion_force(eta, kappa, params=p)
    Fh = _host(F)
    eps = 1e-4
    for mu, t, z, y, x in [(0, 0, 1, 2, 3), (3, 5, 0, 1, 1), (2, 2, 3, 3, 0)]:
        T = _random_su3_algebra(g)
        vals = []
        for sgn in (+1, -1):
            U2 = U.copy()
            U2[mu, t, z, y, x] = _expm_antihermitian(sgn * eps * T) @ U[mu, t, z, y, x]
            lat2 = _lattice(L, U2)
            _, S2, _ = lat2.fermion_force(eta, kappa, params=p, force=False)
            vals.append(S2)
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = float(np.real(np.trace(T @ Fh[mu, t, z, y, x])))
        assert abs(fd - an) <= 1e-4 * max(1.0, abs(an)), (mu, t, z, y, x, fd, an)


def test_full_size_force_from_gpu_solutions():
    """16^3x32 (the benchmark field), kappa 0.1365, eta = D^dag xi: the GPU force
    against the oracle's force formula evaluated on the GPU's own solutions
    X and Y (from wd_solve_D with the same parameters), and the action against
    xi^dag xi."""
    W = _W()
    L = (16, 16, 16, 32)
    U = qcdgen.links_exp(L, 0.3, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 1))
    lat = _lattice(L, U)
    kappa = 0.1365
    xi = qcdgen.gaussian_spinor(L, qcdgen.rng(84))
    eta = lat.pseudofermion(_dev(xi), kappa)
    p = W.default_params(inner="f32", delta=1e-2)
    F, S, st = lat.fermion_force(eta, kappa, params=p)
    assert st[0]["status"] == 0 and st[1]["status"] == 0
    Y, _ = lat.solve_D(eta, kappa, params=p, dagger=True)
    X, _ = lat.solve_D(Y, kappa, params=p)
    F_ref = O.force_from_solutions(U, _host(X), _host(Y), kappa, BC)
    Fh = _host(F)
    assert np.linalg.norm(Fh - F_ref) / np.linalg.norm(F_ref) <= 1e-12
    xx = float(np.vdot(xi.ravel(), xi.ravel()).real)
    assert S == pytest.approx(xx, rel=1e-8)
