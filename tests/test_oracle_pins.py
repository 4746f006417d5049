"""Pins of the CPU oracle against facts it does not compute itself.

The paper prints no numeric outputs for the Dirac operator or its solver
(its listings print values without showing them, App. C), so every pin here
is a closed form, an algebraic invariant, a special case or a brute-force
dense computation.  Each is chosen so that a plausible slip in the oracle (a
wrong projector sign, a transposed link, a shift in the wrong direction, a
missing boundary sign, a wrong even-odd factor) fails at least one of them.
"""

import itertools

import numpy as np
import pytest

import oracle as O
import qcdgen

BC_AP = (1, 1, 1, -1)


def _plane_wave(L, p, chi):
    """e^{i p.x} chi on every site."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None, None] * chi[None, None, None, None]


def _momenta(L, bc):
    """All momenta compatible with the boundary signs."""
    out = []
    ranges = [range(L[mu]) for mu in range(4)]
    for n in itertools.product(*ranges):
        p = []
        for mu in range(4):
            shift = 0.5 if bc[mu] == -1 else 0.0
            p.append(2 * np.pi * (n[mu] + shift) / L[mu])
        out.append(np.array(p))
    return out


def _Dp(p, kappa):
    """Free Wilson operator on e^{ipx}chi: D(p) = 1 - 2 kappa sum cos p + 2i kappa sum gamma sin p."""
    M = 1 - 2 * kappa * np.sum(np.cos(p))
    return M * np.eye(4) + 2j * kappa * sum(O.GAMMA[mu] * np.sin(p[mu]) for mu in range(4))


def _dense(apply, n_sites_shape):
    """Dense matrix of a linear map on spinor fields, column by column."""
    shape = n_sites_shape + (4, 3)
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = apply(e.reshape(shape)).ravel()
    return M


def _sorted_spectrum(ev):
    """Eigenvalues ordered by rounded (real, imag), robust to rounding ties."""
    key = np.lexsort((np.round(ev.imag, 8), np.round(ev.real, 8)))
    return ev[key]


# ---------------------------------------------------------------------------
# P-1: gamma matrices
# ---------------------------------------------------------------------------
def test_gamma_table_chiral_basis():
    # gamma_4 = [[0,1],[1,0]] blocks; gamma_1 = [[0,-i sigma_1],[i sigma_1,0]]
    g4 = np.zeros((4, 4), complex)
    g4[0, 2] = g4[1, 3] = g4[2, 0] = g4[3, 1] = 1
    assert np.array_equal(O.GAMMA[3], g4)
    g1 = np.zeros((4, 4), complex)
    g1[0, 3] = g1[1, 2] = -1j
    g1[2, 1] = g1[3, 0] = 1j
    assert np.array_equal(O.GAMMA[0], g1)
    assert np.allclose(O.GAMMA5, np.diag([1, 1, -1, -1]))


def test_clifford_algebra():
    for mu in range(4):
        assert np.allclose(O.GAMMA[mu], O.GAMMA[mu].conj().T)
        assert np.allclose(O.GAMMA5 @ O.GAMMA[mu] + O.GAMMA[mu] @ O.GAMMA5, 0)
        for nu in range(4):
            anti = O.GAMMA[mu] @ O.GAMMA[nu] + O.GAMMA[nu] @ O.GAMMA[mu]
            assert np.allclose(anti, 2 * np.eye(4) * (mu == nu))
    assert np.allclose(O.GAMMA5 @ O.GAMMA5, np.eye(4))


# ---------------------------------------------------------------------------
# P-2: free field, plane waves and spectrum
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_free_field_plane_waves(L):
    kappa = 0.137
    U = qcdgen.links_unit(L)
    g = qcdgen.rng(5)
    moms = _momenta(L, BC_AP)
    for k in g.choice(len(moms), 12, replace=False):
        p = moms[k]
        chi = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        psi = _plane_wave(L, p, chi)
        got = O.apply_D(U, psi, kappa, BC_AP)
        want = _plane_wave(L, p, _Dp(p, kappa) @ chi)
        assert np.abs(got - want).max() < 1e-13


def test_free_field_DdagD_scalar():
    kappa = 0.13
    for p in _momenta((2, 2, 2, 4), BC_AP):
        Dp = _Dp(p, kappa)
        M = 1 - 2 * kappa * np.sum(np.cos(p))
        lam = M * M + 4 * kappa * kappa * np.sum(np.sin(p) ** 2)
        assert np.allclose(Dp.conj().T @ Dp, lam * np.eye(4), atol=1e-14)


def test_free_field_spectrum_dense():
    L = (2, 2, 2, 4)
    kappa = 0.141139  # the paper's example hopping parameter (App. C)
    U = qcdgen.links_unit(L)
    D = _dense(lambda v: O.apply_D(U, v, kappa, BC_AP), qcdgen.site_shape(L))
    ev = _sorted_spectrum(np.linalg.eigvals(D))
    want = []
    for p in _momenta(L, BC_AP):
        M = 1 - 2 * kappa * np.sum(np.cos(p))
        w = 2 * kappa * np.sqrt(np.sum(np.sin(p) ** 2))
        want += [M + 1j * w] * 6 + [M - 1j * w] * 6
    want = _sorted_spectrum(np.array(want))
    assert np.abs(ev - want).max() < 1e-9


# ---------------------------------------------------------------------------
# P-3: free field, even-odd Schur complement
# ---------------------------------------------------------------------------
def test_free_field_eo_eigen():
    L = (4, 4, 2, 6)
    kappa = 0.1365
    U = qcdgen.links_unit(L)
    e = O.even_mask(L)
    g = qcdgen.rng(7)
    moms = _momenta(L, BC_AP)
    for k in g.choice(len(moms), 10, replace=False):
        p = moms[k]
        chi = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        psi = _plane_wave(L, p, chi) * e
        A = 2 * np.sum(np.cos(p))
        s2 = 4 * np.sum(np.sin(p) ** 2)
        lam = (1 - kappa ** 2 * (A * A - s2)) ** 2 + 4 * kappa ** 4 * A * A * s2
        got = O.apply_Ahat(U, psi, kappa, BC_AP)
        assert np.abs(got - lam * psi).max() < 1e-12 * max(1.0, lam)


# ---------------------------------------------------------------------------
# P-4: CG finite termination on a few plane waves
# ---------------------------------------------------------------------------
def test_cg_finite_termination():
    L = (4, 4, 4, 4)
    kappa = 0.12
    U = qcdgen.links_unit(L)
    e = O.even_mask(L)
    g = qcdgen.rng(11)
    moms = _momenta(L, BC_AP)
    picks, lams = [], []
    for k in g.permutation(len(moms)):
        p = moms[k]
        A = 2 * np.sum(np.cos(p))
        s2 = 4 * np.sum(np.sin(p) ** 2)
        lam = (1 - kappa ** 2 * (A * A - s2)) ** 2 + 4 * kappa ** 4 * A * A * s2
        if all(abs(lam - l0) > 1e-3 for l0 in lams):
            picks.append(p)
            lams.append(lam)
        if len(picks) == 3:
            break
    b = np.zeros(qcdgen.site_shape(L) + (4, 3), complex)
    x_exact = np.zeros_like(b)
    for p, lam in zip(picks, lams):
        chi = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        w = _plane_wave(L, p, chi) * e
        b += w
        x_exact += w / lam
    x, info = O.solve_DdagD(U, b, kappa, BC_AP, eo=True, tol=1e-12)
    assert info["converged"]
    assert info["iters"] <= 4
    assert np.abs(x - x_exact).max() < 1e-10 * np.abs(x_exact).max()
    # a single plane wave needs exactly one iteration
    x1, info1 = O.solve_DdagD(U, _plane_wave(L, picks[0], np.ones((4, 3))) * e, kappa, BC_AP, eo=True)
    assert info1["iters"] == 1


# ---------------------------------------------------------------------------
# P-5: gamma5-hermiticity and the literal adjoint
# ---------------------------------------------------------------------------
def test_gamma5_hermiticity_and_adjoint():
    L = (4, 4, 4, 4)
    g = qcdgen.rng(13)
    U = qcdgen.links_haar(L, g)
    x = qcdgen.gaussian_spinor(L, g)
    y = qcdgen.gaussian_spinor(L, g)
    kappa = 0.12
    Dx = O.apply_D(U, x, kappa, BC_AP)
    Dy = O.apply_D(U, y, kappa, BC_AP)
    # gamma5 D is Hermitian: <x, g5 D y> = conj(<y, g5 D x>)
    lhs = O.vdot(x, O.gamma5(Dy))
    rhs = np.conj(O.vdot(y, O.gamma5(Dx)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the literal adjoint is the adjoint: <y, D x> = <D^dag y, x>
    assert abs(O.vdot(y, Dx) - O.vdot(O.apply_Ddag(U, y, kappa, BC_AP), x)) < 1e-12 * abs(O.vdot(y, Dx))
    # and equals the gamma5 sandwich element by element
    sand = O.gamma5(O.apply_D(U, O.gamma5(x), kappa, BC_AP))
    assert np.abs(O.apply_Ddag(U, x, kappa, BC_AP) - sand).max() < 1e-14 * 10
    # the same for the Schur complement
    e = O.even_mask(L)
    sand_hat = O.gamma5(O.apply_Dhat(U, O.gamma5(x * e), kappa, BC_AP))
    assert np.abs(O.apply_Dhat_dag(U, x * e, kappa, BC_AP) - sand_hat).max() < 1e-13


# ---------------------------------------------------------------------------
# P-6 / P-7: gauge covariance, pure gauge
# ---------------------------------------------------------------------------
def _transform_links(U, Om):
    """U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        Omf = O.shift_forward(Om, mu)
        out[mu] = np.einsum("...ab,...bc,...dc->...ad", Om, U[mu], np.conj(Omf))
    return out


def _transform_spinor(psi, Om):
    return np.einsum("...ab,...sb->...sa", Om, psi)


def test_gauge_covariance():
    L = (4, 4, 2, 6)
    g = qcdgen.rng(17)
    U = qcdgen.links_exp(L, 0.4, g)
    Om = qcdgen.random_gauge_transform(L, g)
    psi = qcdgen.gaussian_spinor(L, g)
    kappa = 0.13
    UO = _transform_links(U, Om)
    lhs = O.apply_D(UO, _transform_spinor(psi, Om), kappa, BC_AP)
    rhs = _transform_spinor(O.apply_D(U, psi, kappa, BC_AP), Om)
    assert np.abs(lhs - rhs).max() < 1e-13
    # and for the even-odd normal operator's solution
    b = psi * O.even_mask(L)
    x, info = O.solve_DdagD(U, b, kappa, BC_AP, eo=True)
    xO, infoO = O.solve_DdagD(UO, _transform_spinor(b, Om), kappa, BC_AP, eo=True)
    assert info["converged"] and infoO["converged"]
    assert np.abs(xO - _transform_spinor(x, Om)).max() < 1e-7 * np.abs(x).max()


def test_pure_gauge_is_rotated_free_field():
    L = (4, 2, 4, 4)
    g = qcdgen.rng(19)
    Om = qcdgen.random_gauge_transform(L, g)
    U = _transform_links(qcdgen.links_unit(L), Om)   # Omega(x) Omega(x+mu)^dag
    kappa = 0.125
    for p in [_momenta(L, BC_AP)[k] for k in (3, 17, 40)]:
        chi = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        psi = _transform_spinor(_plane_wave(L, p, chi), Om)
        got = O.apply_D(U, psi, kappa, BC_AP)
        want = _transform_spinor(_plane_wave(L, p, _Dp(p, kappa) @ chi), Om)
        assert np.abs(got - want).max() < 1e-13


# ---------------------------------------------------------------------------
# P-8: Schur identity through the full operator
# ---------------------------------------------------------------------------
def test_schur_identity():
    L = (4, 4, 4, 2)
    g = qcdgen.rng(23)
    U = qcdgen.links_haar(L, g)
    kappa = 0.13
    e, o = O.even_mask(L), O.odd_mask(L)
    xe = qcdgen.gaussian_spinor(L, g) * e
    xo = kappa * O.hopping(U, xe, BC_AP) * o
    Dx = O.apply_D(U, xe + xo, kappa, BC_AP)
    assert np.abs(Dx * o).max() < 1e-13
    assert np.abs(Dx * e - O.apply_Dhat(U, xe, kappa, BC_AP)).max() < 1e-13


def test_det_D_equals_det_Dhat():
    L = (2, 2, 2, 2)
    g = qcdgen.rng(29)
    U = qcdgen.links_haar(L, g)
    kappa = 0.15
    sh = qcdgen.site_shape(L)
    D = _dense(lambda v: O.apply_D(U, v, kappa, BC_AP), sh)
    Dh = _dense(lambda v: O.apply_Dhat(U, v, kappa, BC_AP), sh)
    ev = O.even_mask(L)[..., 0, 0]
    sel = np.repeat(ev.ravel(), 12)
    Dh_e = Dh[np.ix_(sel, sel)]
    s1, ld1 = np.linalg.slogdet(D)
    s2, ld2 = np.linalg.slogdet(Dh_e)
    assert abs(ld1 - ld2) < 1e-10 and abs(s1 - s2) < 1e-10


# ---------------------------------------------------------------------------
# P-9: kappa = 0
# ---------------------------------------------------------------------------
def test_kappa_zero_is_identity():
    L = (4, 4, 4, 4)
    g = qcdgen.rng(31)
    U = qcdgen.links_haar(L, g)
    b = qcdgen.gaussian_spinor(L, g)
    assert np.array_equal(O.apply_D(U, b, 0.0, BC_AP), b)
    for eo in (False, True):
        x, info = O.solve_DdagD(U, b, 0.0, BC_AP, eo=eo)
        assert info["iters"] == 1
        want = b * O.even_mask(L) if eo else b
        assert np.abs(x - want).max() < 1e-15


# ---------------------------------------------------------------------------
# P-10: brute force on a 2^4 lattice
# ---------------------------------------------------------------------------
def test_brute_force_dense():
    L = (2, 2, 2, 2)
    g = qcdgen.rng(37)
    U = qcdgen.links_haar(L, g)
    kappa = 0.14
    sh = qcdgen.site_shape(L)
    D = _dense(lambda v: O.apply_D(U, v, kappa, BC_AP), sh)
    Dd = _dense(lambda v: O.apply_Ddag(U, v, kappa, BC_AP), sh)
    assert np.abs(Dd - D.conj().T).max() < 1e-15
    A = _dense(lambda v: O.apply_DdagD(U, v, kappa, BC_AP), sh)
    assert np.abs(A - A.conj().T).max() < 1e-14
    assert np.linalg.eigvalsh(A).min() > 0
    b = qcdgen.gaussian_spinor(L, g)
    x, info = O.solve_DdagD(U, b, kappa, BC_AP, eo=False)
    xd = np.linalg.solve(A, b.ravel()).reshape(b.shape)
    cond = np.linalg.cond(A)
    assert info["converged"]
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 10 * cond * 1e-10
    # dense gamma5 D is Hermitian
    G5 = np.kron(np.eye(int(np.prod(sh))), np.kron(O.GAMMA5, np.eye(3)))
    assert np.abs(G5 @ D - (G5 @ D).conj().T).max() < 1e-15


def test_lanczos_bounds_bracket_spectrum():
    L = (2, 2, 2, 2)
    g = qcdgen.rng(41)
    U = qcdgen.links_haar(L, g)
    kappa = 0.12
    sh = qcdgen.site_shape(L)
    A = _dense(lambda v: O.apply_DdagD(U, v, kappa, BC_AP), sh)
    w = np.linalg.eigvalsh(A)
    b = qcdgen.gaussian_spinor(L, g)
    x, info = O.solve_DdagD(U, b, kappa, BC_AP, eo=False, tol=1e-13)
    lo, hi = O.lanczos_extremes(info["alphas"], info["betas"])
    assert w[0] - 1e-8 <= lo <= hi <= w[-1] + 1e-8
    assert hi > 0.9 * w[-1]


# ---------------------------------------------------------------------------
# site-wise evaluation agrees with the whole-field one
# ---------------------------------------------------------------------------
def test_sitewise_matches_field():
    L = (4, 6, 2, 8)
    g = qcdgen.rng(43)
    U = qcdgen.links_exp(L, 0.3, g)
    psi = qcdgen.gaussian_spinor(L, g)
    kappa = 0.1365
    y = O.apply_D(U, psi, kappa, BC_AP)
    sites = [(0, 0, 0, 0), (3, 5, 1, 7), (1, 2, 0, 0), (2, 0, 1, 7), (3, 3, 1, 4)]
    ys = O.apply_D_sites(U, psi, kappa, BC_AP, sites)
    for i, s in enumerate(sites):
        assert np.abs(ys[i] - y[s[3], s[2], s[1], s[0]]).max() < 1e-14


# ---------------------------------------------------------------------------
# generators: SU(3) and the reconstruction identity the GPU relies on
# ---------------------------------------------------------------------------
def test_generators_su3_and_row3_identity():
    g = qcdgen.rng(47)
    for U in (qcdgen.haar_su3(500, g), qcdgen.exp_i_hermitian_su3(500, 0.4, g)):
        I = np.einsum("nab,ncb->nac", U, U.conj())
        assert np.abs(I - np.eye(3)).max() < 1e-13
        assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
        row3 = np.conj(np.cross(U[:, 0, :], U[:, 1, :]))
        assert np.abs(row3 - U[:, 2, :]).max() < 1e-13
    H = qcdgen.random_hermitian_traceless(20000, g)
    assert np.abs(H - np.conj(np.swapaxes(H, -1, -2))).max() == 0
    assert np.abs(np.trace(H, axis1=1, axis2=2)).max() < 1e-13
    # unit variance of the off-diagonal entries
    assert abs(np.mean(np.abs(H[:, 0, 1]) ** 2) - 1.0) < 0.05


def test_haar_first_moments():
    # Haar on SU(3): E[U_ij] = 0 and E|U_ij|^2 = 1/3
    g = qcdgen.rng(53)
    U = qcdgen.haar_su3(40000, g)
    assert np.abs(U.mean(axis=0)).max() < 0.02
    assert np.abs((np.abs(U) ** 2).mean(axis=0) - 1 / 3).max() < 0.01
    # E[tr U] = 0, E|tr U|^2 = 1 for Haar SU(3)
    tr = np.trace(U, axis1=1, axis2=2)
    assert abs(tr.mean()) < 0.02
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 0.03


def test_point_sources():
    L = (4, 4, 4, 4)
    P = qcdgen.point_sources(L)
    assert P.shape == (12, 4, 4, 4, 4, 4, 3)
    assert P.sum() == 12
    for k in range(12):
        assert P[k, 0, 0, 0, 0, k // 3, k % 3] == 1
