"""GPU parity of the stencil operators against the CPU oracle (through the C ABI).

Tolerances (norm-wise relative, ||y_gpu - y_oracle|| / ||y_oracle||):
FP64 1e-12, FP32 1e-5, FP16 (per-site scaled spinors, half links) 3e-3.
"""

import numpy as np
import pytest

import oracle as O
import qcdgen

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 3e-3}
BC = (1, 1, 1, -1)


def _torch():
    import torch
    return torch


def _W():
    from paper_2409_03030_amd import wdirac
    return wdirac


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _lattice(L, U, precs=(("f64", 18),), bc=BC):
    W = _W()
    lat = W.Lattice(L, bc)
    Ud = _dev(U)
    for prec, recon in precs:
        lat.set_gauge(Ud, prec, recon)
    return lat


LATTICES = [(4, 4, 4, 4), (8, 8, 8, 8), (4, 6, 8, 10), (2, 2, 2, 2), (6, 2, 4, 2)]


@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("prec,recon", [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12), ("f16", 12), ("f16", 18)])
def test_apply_D_full(L, prec, recon):
    g = qcdgen.rng(101)
    U = qcdgen.links_haar(L, g)
    psi = qcdgen.gaussian_spinor(L, g)
    kappa = 0.12
    lat = _lattice(L, U, [(prec, recon)])
    y = _host(lat.apply_D(_dev(psi), kappa, dagger=False, precond=0, prec=prec))
    ref = O.apply_D(U, psi, kappa, BC)
    assert _rel(y, ref) < TOL[prec]
    yd = _host(lat.apply_D(_dev(psi), kappa, dagger=True, precond=0, prec=prec))
    refd = O.apply_Ddag(U, psi, kappa, BC)
    assert _rel(yd, refd) < TOL[prec]


@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("prec,recon", [("f64", 18), ("f32", 12), ("f16", 12)])
def test_apply_Dhat_eo(L, prec, recon):
    g = qcdgen.rng(103)
    U = qcdgen.links_exp(L, 0.4, g)
    psi = qcdgen.gaussian_spinor(L, g)
    kappa = 0.137
    lat = _lattice(L, U, [(prec, recon)])
    e = O.even_mask(L)
    y = _host(lat.apply_D(_dev(psi), kappa, dagger=False, precond=1, prec=prec))
    ref = O.apply_Dhat(U, psi * e, kappa, BC)
    assert np.abs(y * O.odd_mask(L)).max() == 0.0
    assert _rel(y, ref) < TOL[prec]
    yd = _host(lat.apply_D(_dev(psi), kappa, dagger=True, precond=1, prec=prec))
    assert _rel(yd, O.apply_Dhat_dag(U, psi * e, kappa, BC)) < TOL[prec]
    yn = _host(lat.apply_DdagD(_dev(psi), kappa, precond=1, prec=prec))
    assert _rel(yn, O.apply_Ahat(U, psi * e, kappa, BC)) < 2 * TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_apply_DdagD_full(prec):
    L = (4, 4, 4, 8)
    g = qcdgen.rng(107)
    U = qcdgen.links_haar(L, g)
    psi = qcdgen.gaussian_spinor(L, g)
    lat = _lattice(L, U, [(prec, 18)])
    y = _host(lat.apply_DdagD(_dev(psi), 0.13, precond=0, prec=prec))
    assert _rel(y, O.apply_DdagD(U, psi, 0.13, BC)) < 2 * TOL[prec]


@pytest.mark.parametrize("nrhs", [3, 12])
def test_multi_rhs_matches_single(nrhs):
    L = (4, 4, 6, 8)
    g = qcdgen.rng(109)
    U = qcdgen.links_exp(L, 0.3, g)
    psi = qcdgen.gaussian_spinor(L, g, nrhs)
    lat = _lattice(L, U, [("f64", 18), ("f32", 12)])
    for prec in ("f64", "f32"):
        y = _host(lat.apply_D(_dev(psi), 0.1365, precond=1, prec=prec))
        for r in range(nrhs):
            ys = _host(lat.apply_D(_dev(psi[r]), 0.1365, precond=1, prec=prec))
            # identical arithmetic per site and rhs: bitwise equal
            assert np.array_equal(y[r], ys)
            assert _rel(y[r], O.apply_Dhat(U, psi[r] * O.even_mask(L), 0.1365, BC)) < TOL[prec]


def test_recon12_equals_recon18_fp64():
    L = (4, 4, 4, 4)
    g = qcdgen.rng(113)
    U = qcdgen.links_haar(L, g)
    psi = qcdgen.gaussian_spinor(L, g)
    W = _W()
    l18 = _lattice(L, U, [("f64", 18)])
    l12 = _lattice(L, U, [("f64", 12)])
    a = _host(l18.apply_D(_dev(psi), 0.12, prec="f64"))
    b = _host(l12.apply_D(_dev(psi), 0.12, prec="f64"))
    assert _rel(a, b) < 1e-14


def test_free_field_and_gamma5_hermiticity_on_gpu():
    L = (4, 4, 4, 8)
    U = qcdgen.links_unit(L)
    lat = _lattice(L, U, [("f64", 18)])
    kappa = 0.137
    # plane wave: D e^{ipx} chi = e^{ipx} D(p) chi
    p = np.array([2 * np.pi / 4, 0.0, 2 * np.pi * 3 / 4, np.pi * 3 / 8])
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    g = qcdgen.rng(127)
    chi = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
    psi = ph[..., None, None] * chi
    Dp = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4) + 2j * kappa * sum(
        O.GAMMA[m] * np.sin(p[m]) for m in range(4))
    got = _host(lat.apply_D(_dev(psi), kappa, prec="f64"))
    assert np.abs(got - ph[..., None, None] * (Dp @ chi)).max() < 1e-13
    # gamma5-hermiticity through the GPU on random links
    Uh = qcdgen.links_haar(L, g)
    lat2 = _lattice(L, Uh, [("f64", 18)])
    a = qcdgen.gaussian_spinor(L, g)
    b = qcdgen.gaussian_spinor(L, g)
    Da = _host(lat2.apply_D(_dev(a), kappa, prec="f64"))
    Db = _host(lat2.apply_D(_dev(b), kappa, prec="f64"))
    lhs = O.vdot(a, O.gamma5(Db))
    rhs = np.conj(O.vdot(b, O.gamma5(Da)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gauge_covariance_on_gpu():
    L = (4, 4, 2, 6)
    g = qcdgen.rng(131)
    U = qcdgen.links_exp(L, 0.4, g)
    Om = qcdgen.random_gauge_transform(L, g)
    psi = qcdgen.gaussian_spinor(L, g)
    UO = np.empty_like(U)
    for mu in range(4):
        UO[mu] = np.einsum("...ab,...bc,...dc->...ad", Om, U[mu], np.conj(O.shift_forward(Om, mu)))
    rot = lambda v: np.einsum("...ab,...sb->...sa", Om, v)
    a = _host(_lattice(L, UO).apply_D(_dev(rot(psi)), 0.13, prec="f64"))
    b = rot(_host(_lattice(L, U).apply_D(_dev(psi), 0.13, prec="f64")))
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("L,width,kappa", [((16, 16, 16, 32), 0.3, 0.1365), ((24, 24, 24, 48), 0.4, 0.137)])
def test_full_size_sampled_sites(L, width, kappa):
    """Full configuration sizes: 128 sampled output sites against the site-wise oracle."""
    g = qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 2)
    U = qcdgen.links_exp(L, width, g)
    psi = qcdgen.gaussian_spinor(L, g)
    lat = _lattice(L, U, [("f64", 18), ("f32", 12)])
    y64 = _host(lat.apply_D(_dev(psi), kappa, prec="f64"))
    y32 = _host(lat.apply_D(_dev(psi), kappa, prec="f32"))
    gs = qcdgen.rng(7)
    sites = [tuple(int(gs.integers(0, L[m])) for m in range(4)) for _ in range(120)]
    # include the corners where every boundary sign is taken
    sites += [(0, 0, 0, 0), (L[0] - 1, L[1] - 1, L[2] - 1, L[3] - 1), (0, L[1] - 1, 0, L[3] - 1),
              (L[0] - 1, 0, L[2] - 1, 0), (1, 0, 0, L[3] - 1), (0, 1, L[2] - 1, 0), (L[0] - 1, 1, 1, 1),
              (2, L[1] - 1, 3, 0)]
    ref = O.apply_D_sites(U, psi, kappa, BC, sites)
    got64 = np.array([y64[s[3], s[2], s[1], s[0]] for s in sites])
    got32 = np.array([y32[s[3], s[2], s[1], s[0]] for s in sites])
    assert _rel(got64, ref) < 1e-12
    assert _rel(got32, ref) < 1e-5


def test_streamed_fp32_links_sampled_sites():
    """24^3x56 with FP32 recon-18 links: the link field (223 MB) exceeds three
    quarters of the Infinity Cache, so the FP32 Wilson and staggered stencils
    take the kernels that read the links with non-temporal loads (smaller
    FP32 link fields never do).  Wilson D at 128 sampled sites against the
    site-wise oracle, and the staggered D against the oracle's full apply, both
    within the FP32 tolerance."""
    from oracle import staggered as S
    L = (24, 24, 24, 56)
    g = qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 3)
    U = qcdgen.links_exp(L, 0.4, g)
    psi = qcdgen.gaussian_spinor(L, g)
    lat = _lattice(L, U, [("f32", 18)])
    y32 = _host(lat.apply_D(_dev(psi), 0.137, prec="f32"))
    gs = qcdgen.rng(11)
    sites = [tuple(int(gs.integers(0, L[m])) for m in range(4)) for _ in range(124)]
    sites += [(0, 0, 0, 0), (L[0] - 1, L[1] - 1, L[2] - 1, L[3] - 1), (0, L[1] - 1, 0, L[3] - 1),
              (L[0] - 1, 0, L[2] - 1, 0)]
    ref = O.apply_D_sites(U, psi, 0.137, BC, sites)
    got = np.array([y32[s[3], s[2], s[1], s[0]] for s in sites])
    assert _rel(got, ref) < TOL["f32"]
    del y32, psi
    shape = qcdgen.site_shape(L) + (3,)
    chi = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    ys = _host(lat.stag_apply(_dev(chi), 0.1, prec="f32"))
    assert _rel(ys, S.apply_staggered(U, chi, 0.1, BC)) < TOL["f32"]


@pytest.mark.parametrize("nrhs", [1, 4])
@pytest.mark.parametrize("split,sblk,swz", [(1, 64, 0), (1, 256, 1), (2, 64, 1), (2, 128, 0), (4, 64, 1), (8, 64, 1)])
def test_launch_shapes_match_oracle(nrhs, split, sblk, swz):
    """Every stencil launch shape (hop split, block size, XCD order) gives the oracle's D_hat."""
    W = _W()
    L = (8, 4, 6, 8)   # dims used by no other test: the tuning table is process-wide
    sb = sblk if nrhs == 1 else max(16, sblk // 4)
    if split * sb * nrhs > (512 if split == 8 else 256):
        pytest.skip("block too large")
    g = qcdgen.rng(137)
    U = qcdgen.links_exp(L, 0.4, g)
    psi = qcdgen.gaussian_spinor(L, g, nrhs)
    lat = _lattice(L, U, [("f64", 18), ("f32", 12), ("f16", 12)])
    # the 8-way split exists below FP64 only: FP64 keeps a 4-way split there
    lines = "".join(f"{L[0]} {L[1]} {L[2]} {L[3]} {p} {r} {nrhs} {sb} {swz} {split if (split < 8 or p) else 4}\n"
                    for p, r in ((0, 18), (1, 12), (2, 12)))
    W.tune_import(lines)
    e = O.even_mask(L)
    for prec in ("f64", "f32", "f16"):
        y = _host(lat.apply_D(_dev(psi), 0.1365, precond=1, prec=prec))
        yd = _host(lat.apply_DdagD(_dev(psi), 0.1365, precond=1, prec=prec))
        for r in range(nrhs):
            assert _rel(y[r], O.apply_Dhat(U, psi[r] * e, 0.1365, BC)) < TOL[prec]
            assert _rel(yd[r], O.apply_Ahat(U, psi[r] * e, 0.1365, BC)) < 2 * TOL[prec]
    # and solves through the same shapes (every reducing epilogue: the norms
    # of the CG at each inner precision and of the FP64 reliable updates)
    b = np.ascontiguousarray(psi[0])
    for inner in ("f64", "f32", "f16"):
        x, st = lat.solve(_dev(b), 0.1365, W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0))
        assert st[0]["status"] == 0, inner
        assert O.residual_DdagD(U, _host(x), b, 0.1365, BC, True) <= 1e-10, inner


def test_time_hop_modes():
    """The stencil timer runs every timed epilogue, and the four stencils of a CG
    iteration in order, on scratch data and rejects other modes."""
    W = _W()
    L = (8, 8, 8, 8)
    lat = _lattice(L, qcdgen.links_unit(L), [("f64", 12), ("f16", 12)])
    for prec in ("f64", "f16"):
        for mode in (0, 1, 2, 4):
            ms = lat.time_hop(prec, 1, n=5, mode=mode)
            assert 0.0 < ms < 10.0
    for mode in (3, 5):
        with pytest.raises(W.WDError) as e:
            lat.time_hop("f64", 1, n=5, mode=mode)
        assert e.value.status == W.WD_EINVAL


def test_autotune_shapes_and_solve():
    """The autotuner returns a valid launch shape for every precision and for
    1 and 4 fields, records it in the exported tuning table, and the stencil
    and a solve through the tuned shapes still meet the oracle."""
    W = _W()
    L = (10, 4, 8, 6)   # dims used by no other test: the tuning table is process-wide
    g = qcdgen.rng(139)
    U = qcdgen.links_exp(L, 0.4, g)
    lat = _lattice(L, U, [("f64", 12), ("f32", 12), ("f16", 12)])
    for prec, p in (("f64", 0), ("f32", 1), ("f16", 2)):
        for nrhs in (1, 4):
            sb, sw, sp = lat.autotune(prec, nrhs)
            assert sb > 0 and sb & (sb - 1) == 0 and sw in (0, 1) and sp in (1, 2, 4, 8), (prec, nrhs)
            assert sp * sb * nrhs <= (512 if sp == 8 else 256) and not (prec == "f64" and sp == 8)
            rows = [r.split() for r in W.tune_export().splitlines()]
            want = [str(v) for v in (*L, p, 12, nrhs, sb, sw, sp)]
            assert want in rows, (prec, nrhs, want)
    psi = qcdgen.gaussian_spinor(L, g, 4)
    e = O.even_mask(L)
    for prec in ("f64", "f32", "f16"):
        y = _host(lat.apply_DdagD(_dev(psi), 0.1365, precond=1, prec=prec))
        for r in range(4):
            assert _rel(y[r], O.apply_Ahat(U, psi[r] * e, 0.1365, BC)) < 2 * TOL[prec], (prec, r)
    for inner in ("f64", "f32", "f16"):
        x, st = lat.solve(_dev(psi), 0.1365, W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0))
        xh = _host(x)
        for r in range(4):
            assert st[r]["status"] == 0, (inner, r)
            assert O.residual_DdagD(U, xh[r], psi[r], 0.1365, BC, True) <= 1e-10, (inner, r)


@pytest.mark.parametrize("nrhs", [1, 4])
@pytest.mark.parametrize("split", [1, 2, 4])
def test_tslice_block_order(nrhs, split):
    """The XCD order that visits each XCD's t-slices innermost (swz 2) gives the
    oracle's D_hat, bitwise the same as the plain XCD order with the same split,
    and solves through it meet the oracle's residual.  8x4x8x16 at 64 sites per
    block has 2 blocks per t-slice and 2 slices per XCD range, so the order
    really differs from swz 1."""
    W = _W()
    L = (8, 4, 8, 16)   # dims used by no other test: the tuning table is process-wide
    sb = 64 // nrhs
    g = qcdgen.rng(141)
    U = qcdgen.links_exp(L, 0.4, g)
    psi = qcdgen.gaussian_spinor(L, g, nrhs)
    lat = _lattice(L, U, [("f64", 12), ("f32", 12), ("f16", 12)])
    e = O.even_mask(L)
    out = {}
    for swz in (1, 2):
        lines = "".join(f"{L[0]} {L[1]} {L[2]} {L[3]} {p} 12 {nrhs} {sb} {swz} {split}\n" for p in (0, 1, 2))
        W.tune_import(lines)
        for prec in ("f64", "f32", "f16"):
            y = _host(lat.apply_D(_dev(psi), 0.1365, precond=1, prec=prec))
            out[(swz, prec)] = y
            for r in range(nrhs):
                assert _rel(y[r], O.apply_Dhat(U, psi[r] * e, 0.1365, BC)) < TOL[prec]
    for prec in ("f64", "f32", "f16"):
        assert np.array_equal(out[(1, prec)], out[(2, prec)]), prec
    b = np.ascontiguousarray(psi[0])
    for inner in ("f64", "f16"):
        x, st = lat.solve(_dev(b), 0.1365, W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0))
        assert st[0]["status"] == 0, inner
        assert O.residual_DdagD(U, _host(x), b, 0.1365, BC, True) <= 1e-10, inner
    if nrhs != 4:
        return
    # 8 sources as 2 groups of 4 in the same launches (interleaved slots): the
    # t-slice order then spans both groups' blocks
    b8 = qcdgen.gaussian_spinor(L, g, 8)
    xs = {}
    for swz in (1, 2):
        W.tune_import("".join(f"{L[0]} {L[1]} {L[2]} {L[3]} {p} 12 4 {sb} {swz} {split}\n" for p in (0, 1)))
        par = W.default_params(inner="f32", delta=1e-2)
        par.rhs_group = 4
        x, st = lat.solve(_dev(b8), 0.1365, par)
        assert all(s["status"] == 0 for s in st), swz
        xs[swz] = _host(x)
    assert np.array_equal(xs[1], xs[2])
    for r in range(8):
        assert O.residual_DdagD(U, xs[2][r], b8[r], 0.1365, BC, True) <= 1e-10, r
