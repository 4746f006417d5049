"""GPU staggered operator against the oracle: D and D^dag at FP64/FP32 with
both link formats and several lattices, and the even-odd solve of D x = b
(FP64 and mixed FP32 inner iterations), checked by the oracle's FP64
residual of D x = b, against its own solution, against the free-field closed
form and at the full benchmark size; the 3 colour point-source propagators
and the Goldstone pion correlator against the oracle and the free-field
closed form."""

import numpy as np
import pytest

import qcdgen
from closed_forms import free_staggered_point_propagator
from oracle import staggered as S

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


def _field(L, g, n=None):
    shape = qcdgen.site_shape(L) + (3,)
    if n is not None:
        shape = (n,) + shape
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _lattice(L, U, recon=12, bc=BC):
    W = _W()
    lat = W.Lattice(L, bc)
    Ud = _dev(U)
    for prec in ("f64", "f32"):
        lat.set_gauge(Ud, prec, recon)
    return lat


@pytest.mark.parametrize("L,bc,recon,nrhs", [((4, 4, 4, 4), BC, 18, 1), ((6, 4, 4, 6), BC, 12, 3),
                                             ((2, 2, 2, 2), (-1, 1, -1, 1), 12, 1), ((4, 6, 8, 10), BC, 18, 2)])
def test_apply_matches_oracle(L, bc, recon, nrhs):
    g = qcdgen.rng(101)
    U = qcdgen.links_exp(L, 0.4, g)
    x = _field(L, g, nrhs)
    lat = _lattice(L, U, recon, bc)
    m = 0.2
    for prec, tol in (("f64", 1e-13), ("f32", 2e-6)):
        for dagger in (False, True):
            y = _host(lat.stag_apply(_dev(x), m, dagger=dagger, prec=prec))
            op = S.apply_staggered_dag if dagger else S.apply_staggered
            for r in range(nrhs):
                ref = op(U, x[r], m, bc)
                assert np.linalg.norm(y[r] - ref) / np.linalg.norm(ref) <= tol, (prec, dagger, r)


@pytest.mark.parametrize("inner,dagger", [("f64", False), ("f64", True), ("f32", False)])
def test_solve_matches_oracle(inner, dagger):
    W = _W()
    L = (6, 4, 4, 6)
    g = qcdgen.rng(102)
    U = qcdgen.links_exp(L, 0.3, g)
    b = _field(L, g, 2)
    masses = [0.1, 0.25]
    lat = _lattice(L, U)
    p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0, tol=1e-12)
    x, st = lat.stag_solve(_dev(b), masses, params=p, dagger=dagger)
    x = _host(x)
    op = S.apply_staggered_dag if dagger else S.apply_staggered
    for r in range(2):
        assert st[r]["status"] == 0
        res = np.linalg.norm(b[r] - op(U, x[r], masses[r], BC)) / np.linalg.norm(b[r])
        assert res <= 1e-10, (r, res)
        if not dagger:
            xr, info = S.solve_staggered(U, b[r], masses[r], BC, tol=1e-13)
            assert info["converged"]
            assert np.linalg.norm(x[r] - xr) / np.linalg.norm(xr) <= 1e-9


def test_free_field_plane_wave():
    W = _W()
    L = (4, 4, 4, 6)
    U = qcdgen.links_unit(L)
    lat = _lattice(L, U)
    m = 0.1
    Lt, Lz, Ly, Lx = qcdgen.site_shape(L)
    t, z, y, x = np.indices((Lt, Lz, Ly, Lx))
    n = (1, 2, 3, 4)
    p = [2 * np.pi * (n[mu] + (0.5 if BC[mu] == -1 else 0.0)) / L[mu] for mu in range(4)]
    c = np.array([1.0, 0.5j, -0.25])
    b = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None] * c
    lam = m * m + sum(np.sin(pm) ** 2 for pm in p)
    # D D^dag = D^dag D = m^2 - H^2 is the scalar lam on this wave, so D^-1 b = D^dag b / lam
    x_ref = S.apply_staggered_dag(U, b, m, BC) / lam
    xs, st = lat.stag_solve(_dev(b), m, params=W.default_params(tol=1e-13))
    assert st[0]["status"] == 0
    assert np.linalg.norm(_host(xs) - x_ref) / np.linalg.norm(x_ref) <= 1e-11


def test_full_size_solve():
    """16^3x32 (the benchmark field), mass 0.1: the oracle's FP64 residual of D x = b."""
    W = _W()
    L = (16, 16, 16, 32)
    U = qcdgen.links_exp(L, 0.3, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 1))
    lat = _lattice(L, U)
    b = _field(L, qcdgen.rng(103))
    for inner in ("f64", "f32"):
        p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0)
        x, st = lat.stag_solve(_dev(b), 0.1, params=p)
        assert st[0]["status"] == 0, inner
        res = np.linalg.norm(b - S.apply_staggered(U, _host(x), 0.1, BC)) / np.linalg.norm(b)
        # the CG tolerance 1e-10 applies to M_e x_e = b'_e; |r_D| = |r_M| / m and |b'| <= 3 |b|
        assert res <= 5e-9, (inner, res)


def test_streamed_link_kernels_solve():
    """24^3x28 with recon-18 FP64 links, mass 0.1: the link field (223 MB)
    exceeds three quarters of the Infinity Cache, so the FP64 staggered
    stencils take the kernels that read the links with non-temporal loads,
    which the smaller lattices of the other tests never reach.  Plain FP64 and
    FP32 inner (FP64 reliable updates) both meet the oracle's FP64 residual of
    D x = b."""
    W = _W()
    L = (24, 24, 24, 28)
    U = qcdgen.links_exp(L, 0.3, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 1))
    lat = _lattice(L, U, recon=18)
    b = _field(L, qcdgen.rng(104))
    for inner in ("f64", "f32"):
        p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0)
        x, st = lat.stag_solve(_dev(b), 0.1, params=p)
        assert st[0]["status"] == 0, inner
        res = np.linalg.norm(b - S.apply_staggered(U, _host(x), 0.1, BC)) / np.linalg.norm(b)
        assert res <= 5e-9, (inner, res)


def test_autotune_then_solve():
    """The staggered autotuner's shapes give the same stencil output; a solve
    with the tuned shapes still meets the oracle's residual."""
    W = _W()
    L = (8, 4, 6, 8)
    g = qcdgen.rng(104)
    U = qcdgen.links_exp(L, 0.3, g)
    lat = _lattice(L, U)
    b = _field(L, g)
    y0 = _host(lat.stag_apply(_dev(b), 0.2))
    for prec in ("f64", "f32"):
        sb, sw, sp = lat.stag_autotune(prec, 1)
        assert 128 <= sb * sp <= 256 and sw in (0, 1) and sp in (1, 2, 4)
    y1 = _host(lat.stag_apply(_dev(b), 0.2))
    assert np.array_equal(y0, y1) or np.linalg.norm(y1 - y0) <= 1e-14 * np.linalg.norm(y0)
    x, st = lat.stag_solve(_dev(b), 0.2, params=W.default_params(inner="f32", delta=1e-2))
    assert st[0]["status"] == 0
    res = np.linalg.norm(b - S.apply_staggered(U, _host(x), 0.2, BC)) / np.linalg.norm(b)
    assert res <= 1e-9


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_propagator_and_pion_match_oracle(inner):
    """Point propagator at a site of slice 3 against the oracle's solution, the
    correlator against the oracle's contraction of the same GPU columns (only
    the summation order differs) and against the oracle's whole pipeline."""
    W = _W()
    L = (4, 4, 4, 6)
    origin, t0, m = (1, 2, 0, 3), 3, 0.15
    U = qcdgen.links_exp(L, 0.3, qcdgen.rng(105))
    lat = _lattice(L, U)
    p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0, tol=1e-12)
    G, st = lat.stag_propagator(m, params=p, origin=origin)
    assert all(s["status"] == 0 for s in st)
    Gh = _host(G)
    Gref, infos = S.staggered_point_propagator(U, m, BC, S.point_sources_staggered(L, origin), tol=1e-13)
    assert all(i["converged"] for i in infos)
    assert np.linalg.norm(Gh - Gref) / np.linalg.norm(Gref) <= 1e-9
    C = lat.stag_pion_correlator(G, t0)
    assert C.shape == (L[3],)
    np.testing.assert_allclose(C, S.staggered_pion_correlator(Gh, t0), rtol=1e-12, atol=0)
    np.testing.assert_allclose(C, S.staggered_pion_correlator(Gref, t0), rtol=1e-8, atol=0)
    # a single column: the correlator is additive over columns
    C0 = lat.stag_pion_correlator(G[:1].contiguous(), t0)
    np.testing.assert_allclose(C0, S.staggered_pion_correlator(Gh[:1], t0), rtol=1e-12, atol=0)


def test_free_propagator_and_pion():
    """U = 1: the propagator equals the closed form (m - H) G of the test
    helpers, and the correlator is symmetric under t -> Lt - t."""
    W = _W()
    L = (4, 4, 4, 8)
    m = 0.2
    lat = _lattice(L, qcdgen.links_unit(L))
    G, st = lat.stag_propagator(m, params=W.default_params(tol=1e-13))
    assert all(s["status"] == 0 for s in st)
    ref = free_staggered_point_propagator(L, m, BC)
    assert np.linalg.norm(_host(G) - ref) / np.linalg.norm(ref) <= 1e-10
    C = lat.stag_pion_correlator(G)
    assert np.all(C > 0)
    for t in range(1, L[3]):
        assert C[t] == pytest.approx(C[L[3] - t], rel=1e-9)


def test_full_size_propagator_and_pion():
    """16^3x32, 3 colour columns at mass 0.1 with FP32 inner iterations (with
    three fields each CG reduction has more block partials than the fold
    limit, so this covers the finalize-kernel path): the oracle's FP64 residual
    of every column and the oracle's contraction of the GPU columns."""
    W = _W()
    L = (16, 16, 16, 32)
    U = qcdgen.links_exp(L, 0.3, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 1))
    lat = _lattice(L, U)
    origin = (3, 5, 7, 11)
    G, st = lat.stag_propagator(0.1, params=W.default_params(inner="f32", delta=1e-2), origin=origin)
    assert all(s["status"] == 0 for s in st)
    Gh = _host(G)
    src = S.point_sources_staggered(L, origin)
    for a in range(3):
        res = np.linalg.norm(src[a] - S.apply_staggered(U, Gh[a], 0.1, BC)) / np.linalg.norm(src[a])
        assert res <= 5e-9, (a, res)
    C = lat.stag_pion_correlator(G, origin[3])
    np.testing.assert_allclose(C, S.staggered_pion_correlator(Gh, origin[3]), rtol=1e-12, atol=0)


@pytest.mark.parametrize("split,sblk,swz", [(1, 128, 0), (2, 64, 1), (2, 128, 0), (4, 32, 1), (4, 64, 0)])
def test_launch_shapes_match_oracle(split, sblk, swz):
    """Every staggered launch shape (hops split over 1, 2 or 4 threads, block
    size, XCD order) gives the oracle's D and D^dag, with 1 and 2 fields, and
    solves through the same shape (FP64 and FP32 inner) meet the oracle's
    residual."""
    W = _W()
    L = (8, 6, 4, 10)   # dims used by no other staggered test: shapes are kept per lattice
    g = qcdgen.rng(106)
    U = qcdgen.links_exp(L, 0.4, g)
    lat = _lattice(L, U)
    m = 0.15
    for nrhs in (1, 2):
        sb = sblk if nrhs == 1 else sblk // 2
        for prec in ("f64", "f32"):
            lat.stag_set_shape(prec, nrhs, sb, swz, split)
        x = _field(L, g, nrhs)
        for prec, tol in (("f64", 1e-13), ("f32", 2e-6)):
            for dagger in (False, True):
                y = _host(lat.stag_apply(_dev(x), m, dagger=dagger, prec=prec))
                op = S.apply_staggered_dag if dagger else S.apply_staggered
                for r in range(nrhs):
                    ref = op(U, x[r], m, BC)
                    assert np.linalg.norm(y[r] - ref) / np.linalg.norm(ref) <= tol, (prec, dagger, r)
        for inner in ("f64", "f32"):
            p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0, tol=1e-12)
            xs, st = lat.stag_solve(_dev(x), m, params=p)
            xs = _host(xs)
            for r in range(nrhs):
                assert st[r]["status"] == 0, (inner, r)
                res = np.linalg.norm(x[r] - S.apply_staggered(U, xs[r], m, BC)) / np.linalg.norm(x[r])
                assert res <= 1e-10, (inner, r, res)
