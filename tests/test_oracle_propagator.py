"""Pins of the oracle's D x = b solve, point propagator and pion correlator.

Each pin is a fact the oracle does not compute itself: a dense linear solve,
the free-field propagator in closed form (momentum space, inverted 4x4 by 4x4
and Fourier transformed), gauge invariance, time-reflection symmetry of the
free correlator, and the kappa = 0 limit.  A wrong adjoint in the normal
equations, a transposed propagator index, a missing modulus square or a
shifted time origin fails at least one of them.
"""

import numpy as np
import pytest

import oracle as O
import qcdgen
from closed_forms import free_point_propagator as _free_propagator

BC_AP = (1, 1, 1, -1)


def _dense(apply, sites_shape):
    shape = sites_shape + (4, 3)
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = apply(e.reshape(shape)).ravel()
    return M


def _transform_links(U, Om):
    out = np.empty_like(U)
    for mu in range(4):
        Omf = O.shift_forward(Om, mu)
        out[mu] = np.einsum("...ab,...bc,...dc->...ad", Om, U[mu], np.conj(Omf))
    return out


@pytest.mark.parametrize("dagger", [False, True])
def test_solve_D_matches_dense_solve(dagger):
    L = (2, 2, 2, 2)
    g = qcdgen.rng(41)
    U = qcdgen.links_haar(L, g)
    b = qcdgen.gaussian_spinor(L, g)
    kappa = 0.13
    op = O.apply_Ddag if dagger else O.apply_D
    M = _dense(lambda v: op(U, v, kappa, BC_AP), qcdgen.site_shape(L))
    x_ref = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    x, info = O.solve_D(U, b, kappa, BC_AP, dagger=dagger, tol=1e-13)
    assert info["converged"]
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-10
    assert O.residual_D(U, x, b, kappa, BC_AP, dagger) < 1e-11


def test_free_propagator_and_correlator_closed_form():
    L = (4, 4, 4, 6)
    kappa = 0.11
    U = qcdgen.links_unit(L)
    S_ref = _free_propagator(L, kappa, BC_AP)
    # the closed form does solve D S = point sources
    src = qcdgen.point_sources(L)
    for k in (0, 5, 11):
        assert np.linalg.norm(O.apply_D(U, S_ref[k], kappa, BC_AP) - src[k]) < 1e-12
    S, infos = O.point_propagator(U, kappa, BC_AP, src, tol=1e-13)
    assert all(i["converged"] for i in infos)
    assert np.linalg.norm(S - S_ref) / np.linalg.norm(S_ref) < 1e-10
    C = O.pion_correlator(S)
    C_ref = 3 * np.sum(np.abs(_free_propagator(L, kappa, BC_AP)[0::3, ..., 0]) ** 2, axis=(0, 2, 3, 4, 5))
    assert np.allclose(C, C_ref, rtol=1e-10, atol=0)
    # time-reflection symmetry of the free correlator
    Lt = L[3]
    for t in range(1, Lt):
        assert C[t] == pytest.approx(C[Lt - t], rel=1e-10)
    assert np.all(C > 0)


def test_pion_correlator_gauge_invariant():
    L = (4, 4, 4, 4)
    g = qcdgen.rng(43)
    U = qcdgen.links_exp(L, 0.4, g)
    Om = qcdgen.random_gauge_transform(L, g)
    kappa = 0.12
    src = qcdgen.point_sources(L)
    S, _ = O.point_propagator(U, kappa, BC_AP, src, tol=1e-13)
    S2, _ = O.point_propagator(_transform_links(U, Om), kappa, BC_AP, src, tol=1e-13)
    C, C2 = O.pion_correlator(S), O.pion_correlator(S2)
    assert np.allclose(C, C2, rtol=1e-9, atol=0)
    # and the propagator itself rotates: S^Om(x) = Om(x) S(x) Om(0)^dag
    Sx = np.einsum("...ab,k...sb->k...sa", Om, S)
    Om0 = Om[0, 0, 0, 0]
    S_rot = np.empty_like(S)
    for alpha in range(4):
        for a in range(3):
            S_rot[3 * alpha + a] = sum(Sx[3 * alpha + b] * np.conj(Om0[a, b]) for b in range(3))
    assert np.linalg.norm(S2 - S_rot) / np.linalg.norm(S2) < 1e-9


def test_kappa_zero_and_time_origin():
    L = (2, 2, 2, 4)
    U = qcdgen.links_haar(L, qcdgen.rng(44))
    src = qcdgen.point_sources(L)
    S, _ = O.point_propagator(U, 0.0, BC_AP, src)
    assert np.array_equal(S, src)
    C = O.pion_correlator(S)
    assert list(C) == [12.0, 0.0, 0.0, 0.0]
    # t counts from the source time slice
    src2 = qcdgen.point_sources(L, origin=(0, 0, 0, 2))
    S2, _ = O.point_propagator(U, 0.0, BC_AP, src2)
    assert list(O.pion_correlator(S2, t0=2)) == [12.0, 0.0, 0.0, 0.0]
