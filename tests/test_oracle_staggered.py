"""Pins of the staggered-operator oracle.

* Free field in closed form: with the staggered phases the hopping terms of
  different directions anticommute and each squares to -sin^2 p_mu on a plane
  wave, so D^dag D e^{ipx} c = (m^2 + sum_mu sin^2 p_mu) e^{ipx} c for every
  momentum allowed by the boundary signs.  A wrong phase, a missing 1/2 or a
  wrong boundary sign breaks it.
* The point propagator at U = 1 against the closed form of the test helpers
  (their own phases and shifts), the pion correlator's time reflection there,
  the heavy-quark limit and gauge invariance.
* The phases at hard-coded sites, anti-Hermiticity of the hopping part,
  gauge covariance, the even/odd structure, the dense solve and the spectrum
  (real part m) on a 2^4 lattice.
"""

import itertools

import numpy as np
import pytest

import oracle as O
import qcdgen
from closed_forms import free_staggered_point_propagator
from oracle import staggered as S

BC_AP = (1, 1, 1, -1)


def _sshape(L):
    return qcdgen.site_shape(L) + (3,)


def _gauss(L, g):
    return g.standard_normal(_sshape(L)) + 1j * g.standard_normal(_sshape(L))


def test_phase_table():
    L = (4, 4, 4, 4)
    # (x, y, z, t) -> expected eta_1..eta_4
    cases = {(0, 0, 0, 0): (1, 1, 1, 1), (1, 0, 0, 0): (1, -1, -1, -1), (0, 1, 0, 0): (1, 1, -1, -1),
             (1, 1, 0, 0): (1, -1, 1, 1), (0, 0, 1, 0): (1, 1, 1, -1), (3, 2, 1, 3): (1, -1, -1, 1)}
    for (x, y, z, t), want in cases.items():
        got = tuple(int(S.staggered_phase(L, mu)[t, z, y, x]) for mu in range(4))
        assert got == want, ((x, y, z, t), got)


def test_free_field_normal_operator_closed_form():
    L = (4, 4, 4, 6)
    U = qcdgen.links_unit(L)
    m = 0.1
    Lt, Lz, Ly, Lx = qcdgen.site_shape(L)
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    g = qcdgen.rng(91)
    for n in [(0, 0, 0, 0), (1, 2, 3, 5), (3, 1, 0, 2)] + [tuple(int(v) for v in g.integers(0, L)) for _ in range(3)]:
        p = [2 * np.pi * (n[mu] + (0.5 if BC_AP[mu] == -1 else 0.0)) / L[mu] for mu in range(4)]
        c = g.standard_normal(3) + 1j * g.standard_normal(3)
        wave = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None] * c
        lhs = S.apply_staggered_dag(U, S.apply_staggered(U, wave, m, BC_AP), m, BC_AP)
        lam = m * m + sum(np.sin(pm) ** 2 for pm in p)
        assert np.linalg.norm(lhs - lam * wave) <= 1e-12 * np.linalg.norm(wave), n


def test_hopping_anti_hermitian_and_parity():
    L = (4, 4, 2, 6)
    g = qcdgen.rng(92)
    U = qcdgen.links_exp(L, 0.4, g)
    a, b = _gauss(L, g), _gauss(L, g)
    Ha = S.hopping_staggered(U, a, BC_AP)
    Hb = S.hopping_staggered(U, b, BC_AP)
    assert abs(np.vdot(b, Ha) + np.vdot(Hb, a)) <= 1e-12 * np.linalg.norm(a) * np.linalg.norm(b)
    # D^dag is the adjoint of D
    m = 0.3
    lhs = np.vdot(b, S.apply_staggered(U, a, m, BC_AP))
    rhs = np.vdot(S.apply_staggered_dag(U, b, m, BC_AP), a)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the hopping part connects even and odd sites only
    ev = (O.parity(L) == 0)[..., None]
    He = S.hopping_staggered(U, a * ev, BC_AP)
    assert np.all(He[np.broadcast_to(ev, He.shape)] == 0)


def test_gauge_covariance():
    L = (4, 4, 4, 4)
    g = qcdgen.rng(93)
    U = qcdgen.links_exp(L, 0.4, g)
    Om = qcdgen.random_gauge_transform(L, g)
    chi = _gauss(L, g)
    UO = np.empty_like(U)
    for mu in range(4):
        UO[mu] = np.einsum("...ab,...bc,...dc->...ad", Om, U[mu], np.conj(O.shift_forward(Om, mu)))
    lhs = S.apply_staggered(UO, np.einsum("...ab,...b->...a", Om, chi), 0.2, BC_AP)
    rhs = np.einsum("...ab,...b->...a", Om, S.apply_staggered(U, chi, 0.2, BC_AP))
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)


def test_dense_solve_and_spectrum():
    L = (2, 2, 2, 2)
    g = qcdgen.rng(94)
    U = qcdgen.links_haar(L, g)
    m = 0.15
    shape = _sshape(L)
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = S.apply_staggered(U, e.reshape(shape), m, BC_AP).ravel()
    ev = np.linalg.eigvals(M)
    assert np.allclose(ev.real, m, atol=1e-12)
    Md = np.zeros_like(M)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        Md[:, j] = S.apply_staggered_dag(U, e.reshape(shape), m, BC_AP).ravel()
    assert np.allclose(Md, M.conj().T, atol=1e-14)
    b = _gauss(L, g)
    x_ref = np.linalg.solve(M, b.ravel()).reshape(shape)
    x, info = S.solve_staggered(U, b, m, BC_AP, tol=1e-13)
    assert info["converged"]
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-10
    assert S.residual_staggered(U, x, b, m, BC_AP) < 1e-11


def test_staggered_free_propagator_and_pion():
    """At U = 1 the point propagator is the closed form (m - H) G with the scalar
    G(x) = (1/V) sum_p e^{ipx} / (m^2 + sum sin^2 p) (an inverse FFT, with the
    antiperiodic twist in t), written in the test helpers with their own phases
    and shifts; on a second lattice every direction but y is antiperiodic."""
    m = 0.2
    for L, bc in (((4, 4, 4, 6), BC_AP), ((4, 2, 6, 4), (-1, 1, -1, -1))):
        U = qcdgen.links_unit(L)
        G, infos = S.staggered_point_propagator(U, m, bc, S.point_sources_staggered(L), tol=1e-13)
        assert all(i["converged"] for i in infos)
        ref = free_staggered_point_propagator(L, m, bc)
        assert np.linalg.norm(G - ref) / np.linalg.norm(ref) < 1e-10, bc
    L = (4, 4, 4, 6)
    U = qcdgen.links_unit(L)
    Lt = L[3]
    src = S.point_sources_staggered(L)
    G, infos = S.staggered_point_propagator(U, m, BC_AP, src, tol=1e-13)
    C = S.staggered_pion_correlator(G)
    assert np.all(C > 0)
    for t in range(1, Lt):
        assert C[t] == pytest.approx(C[Lt - t], rel=1e-10)
    # a heavy quark: G ~ delta / m, C(0) ~ 3 / m^2
    Gh, _ = S.staggered_point_propagator(U, 50.0, BC_AP, src)
    assert S.staggered_pion_correlator(Gh)[0] == pytest.approx(3 / 50.0 ** 2, rel=1e-3)


def test_staggered_pion_gauge_invariant():
    L = (4, 4, 4, 4)
    g = qcdgen.rng(95)
    U = qcdgen.links_exp(L, 0.4, g)
    Om = qcdgen.random_gauge_transform(L, g)
    UO = np.empty_like(U)
    for mu in range(4):
        UO[mu] = np.einsum("...ab,...bc,...dc->...ad", Om, U[mu], np.conj(O.shift_forward(Om, mu)))
    src = S.point_sources_staggered(L)
    G1, _ = S.staggered_point_propagator(U, 0.2, BC_AP, src, tol=1e-13)
    G2, _ = S.staggered_point_propagator(UO, 0.2, BC_AP, src, tol=1e-13)
    assert np.allclose(S.staggered_pion_correlator(G1), S.staggered_pion_correlator(G2), rtol=1e-9, atol=0)
