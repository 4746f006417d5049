"""Pins of the oracle's pseudofermion action, force and momentum update.

* The force against central finite differences of the action along random
  su(3) directions at single links (including links that cross the
  antiperiodic time boundary).  This pins every factor of the force
  formula (2 kappa, the projector signs, which site's fields enter, the
  boundary sign) through the action alone.
* The heatbath identity of the paper's HMC listing: for eta = D^dag xi the
  action equals xi^dag xi (its Sfold = dot(xi, xi)).
* Gauge covariance F^Om_mu(x) = Om(x) F_mu(x) Om(x)^dag, kappa = 0, and the
  traceless antihermitian projection.
"""

import numpy as np
import pytest

import oracle as O
import qcdgen

BC_AP = (1, 1, 1, -1)


def _random_su3_algebra(g):
    """A random traceless antihermitian 3x3 matrix."""
    A = g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3))
    T = 0.5 * (A - A.conj().T)
    return T - np.trace(T) / 3 * np.eye(3)


def _expm_antihermitian(T):
    """exp(T) for antihermitian T via the eigen-decomposition of the Hermitian -iT."""
    w, V = np.linalg.eigh(-1j * T)
    return (V * np.exp(1j * w)) @ V.conj().T


def _transform_links(U, Om):
    out = np.empty_like(U)
    for mu in range(4):
        Omf = O.shift_forward(Om, mu)
        out[mu] = np.einsum("...ab,...bc,...dc->...ad", Om, U[mu], np.conj(Omf))
    return out


@pytest.fixture(scope="module")
def setup():
    L = (4, 4, 4, 4)
    g = qcdgen.rng(71)
    U = qcdgen.links_exp(L, 0.4, g)
    eta = qcdgen.gaussian_spinor(L, g)
    kappa = 0.12
    F, S, info = O.fermion_force(U, eta, kappa, BC_AP, tol=1e-14)
    assert info["converged"]
    return L, U, eta, kappa, F, S


def test_force_matches_finite_differences(setup):
    L, U, eta, kappa, F, S = setup
    g = qcdgen.rng(72)
    # (mu, t, z, y, x): interior links and links across every boundary
    links = [(0, 1, 2, 3, 1), (1, 0, 1, 3, 2), (2, 3, 3, 0, 0), (3, 3, 1, 2, 1), (3, 0, 0, 0, 0)]
    eps = 1e-4
    for mu, t, z, y, x in links:
        T = _random_su3_algebra(g)
        vals = []
        for sgn in (+1, -1):
            U2 = U.copy()
            U2[mu, t, z, y, x] = _expm_antihermitian(sgn * eps * T) @ U[mu, t, z, y, x]
            S2, info = O.fermion_action(U2, eta, kappa, BC_AP, tol=1e-14)
            assert info["converged"]
            vals.append(S2)
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = np.real(np.trace(T @ F[mu, t, z, y, x]))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (mu, t, z, y, x, fd, an)
        assert abs(an) > 1e-3  # a nontrivial direction


def test_heatbath_identity():
    L = (4, 4, 2, 4)
    g = qcdgen.rng(73)
    U = qcdgen.links_haar(L, g)
    xi = qcdgen.gaussian_spinor(L, g)
    kappa = 0.13
    eta = O.pseudofermion_heatbath(U, xi, kappa, BC_AP)
    S, info = O.fermion_action(U, eta, kappa, BC_AP, tol=1e-13)
    assert info["converged"]
    xx = float(np.vdot(xi.ravel(), xi.ravel()).real)
    assert S == pytest.approx(xx, rel=1e-10)


def test_force_gauge_covariant(setup):
    L, U, eta, kappa, F, S = setup
    Om = qcdgen.random_gauge_transform(L, qcdgen.rng(74))
    eta2 = np.einsum("...ab,...sb->...sa", Om, eta)
    F2, S2, _ = O.fermion_force(_transform_links(U, Om), eta2, kappa, BC_AP, tol=1e-14)
    assert S2 == pytest.approx(S, rel=1e-11)
    F_rot = np.einsum("...ab,m...bc,...dc->m...ad", Om, F, np.conj(Om))
    assert np.linalg.norm(F2 - F_rot) / np.linalg.norm(F) < 1e-10


def test_kappa_zero_and_projection():
    L = (2, 2, 2, 4)
    g = qcdgen.rng(75)
    U = qcdgen.links_haar(L, g)
    eta = qcdgen.gaussian_spinor(L, g)
    F, S, _ = O.fermion_force(U, eta, 0.0, BC_AP)
    assert np.all(F == 0)
    assert S == pytest.approx(float(np.vdot(eta.ravel(), eta.ravel()).real), rel=1e-14)
    M = g.standard_normal((5, 3, 3)) + 1j * g.standard_normal((5, 3, 3))
    TA = O.traceless_antihermitian(M)
    assert np.allclose(TA, -np.conj(np.swapaxes(TA, -1, -2)), atol=1e-15)
    assert np.allclose(np.trace(TA, axis1=-2, axis2=-1), 0, atol=1e-15)
    for k in range(5):
        T = _random_su3_algebra(g)
        assert np.real(np.trace(T @ M[k])) == pytest.approx(np.real(np.trace(T @ TA[k])), rel=1e-12)
    p = g.standard_normal((5, 3, 3)) * 1j
    assert np.allclose(O.momentum_update(p, -0.1, M), p - 0.1 * TA)
