"""GPU CG on D^dag D against the oracle: every solution must have an FP64 true
residual ||b - A x|| / ||b|| <= 1e-10 recomputed by the oracle (the CG's
contract), and is compared with the oracle's own CG solution within the
bound cond(A) * 1e-10 that two correct solvers can differ by."""

import numpy as np
import pytest

import oracle as O
import qcdgen

pytestmark = pytest.mark.gpu

BC = (1, 1, 1, -1)
TOL = 1e-10


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


def _lattice(L, U, precs):
    W = _W()
    lat = W.Lattice(L, BC)
    Ud = _dev(U)
    for prec, recon in precs:
        lat.set_gauge(Ud, prec, recon)
    return lat


def _oracle_resid(U, x, b, kappa, eo):
    return O.residual_DdagD(U, x, b, kappa, BC, eo)


def test_config1_full_fp64_cg():
    """4^4 Haar links, kappa 0.12, unpreconditioned, plain FP64 CG to 1e-10."""
    L = (4, 4, 4, 4)
    g = qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 0)
    U = qcdgen.links_haar(L, g)
    b = qcdgen.gaussian_spinor(L, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 100))
    W = _W()
    lat = _lattice(L, U, [("f64", 18)])
    # D once
    y = _host(lat.apply_D(_dev(b), 0.12, prec="f64"))
    ref = O.apply_D(U, b, 0.12, BC)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-12
    x, st = lat.solve(_dev(b), 0.12, W.default_params(precond=W.FULL))
    x = _host(x)
    assert st[0]["status"] == 0
    assert st[0]["true_resid"] <= TOL
    r = _oracle_resid(U, x, b, 0.12, eo=False)
    assert r <= TOL
    xo, info = O.solve_DdagD(U, b, 0.12, BC, eo=False)
    lo, hi = O.lanczos_extremes(info["alphas"], info["betas"])
    cond = hi / lo
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 4 * cond * TOL
    # iteration counts agree closely with the oracle's (same algorithm, other rounding)
    assert abs(st[0]["iters"] - info["iters"]) <= max(3, info["iters"] // 10)


@pytest.mark.parametrize("inner,recon", [("f64", 18), ("f64", 12), ("f32", 12), ("f32", 18), ("f16", 12)])
def test_eo_solve_precisions(inner, recon):
    L = (8, 8, 8, 8)
    g = qcdgen.rng(201)
    U = qcdgen.links_exp(L, 0.3, g)
    b = qcdgen.gaussian_spinor(L, g)
    kappa = 0.1365
    W = _W()
    precs = [("f64", 18 if inner != "f64" else recon)]
    if inner != "f64":
        precs.append((inner, recon))
    lat = _lattice(L, U, precs)
    p = W.default_params(precond=W.EO, inner=inner, delta=(0.0 if inner == "f64" else 1e-2))
    x, st = lat.solve(_dev(b), kappa, p)
    x = _host(x)
    assert st[0]["status"] == 0, st
    assert st[0]["true_resid"] <= TOL
    assert _oracle_resid(U, x, b, kappa, eo=True) <= TOL
    assert np.abs(x * O.odd_mask(L)).max() == 0.0
    if inner != "f64":
        assert st[0]["reliable_updates"] >= 2


def test_mixed_matches_plain_solution():
    L = (8, 8, 8, 8)
    g = qcdgen.rng(203)
    U = qcdgen.links_exp(L, 0.4, g)
    b = qcdgen.gaussian_spinor(L, g)
    kappa = 0.13
    W = _W()
    lat = _lattice(L, U, [("f64", 12), ("f32", 12), ("f16", 12)])
    x64, s64 = lat.solve(_dev(b), kappa, W.default_params())
    x64 = _host(x64)
    xo, info = O.solve_DdagD(U, b, kappa, BC, eo=True)
    lo, hi = O.lanczos_extremes(info["alphas"], info["betas"])
    bound = 4 * hi / lo * TOL
    assert np.linalg.norm(x64 - xo) / np.linalg.norm(xo) <= bound
    for inner in ("f32", "f16"):
        x, s = lat.solve(_dev(b), kappa, W.default_params(inner=inner, delta=1e-2))
        x = _host(x)
        assert s[0]["status"] == 0
        assert _oracle_resid(U, x, b, kappa, eo=True) <= TOL
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= bound


def test_solve_is_deterministic():
    L = (8, 8, 4, 8)
    g = qcdgen.rng(205)
    U = qcdgen.links_exp(L, 0.3, g)
    b = qcdgen.gaussian_spinor(L, g)
    W = _W()
    lat = _lattice(L, U, [("f64", 18), ("f32", 12)])
    for inner in ("f64", "f32"):
        p = W.default_params(inner=inner, delta=0.0 if inner == "f64" else 1e-2)
        x1, s1 = lat.solve(_dev(b), 0.135, p)
        x2, s2 = lat.solve(_dev(b), 0.135, p)
        assert np.array_equal(_host(x1), _host(x2))
        assert s1[0]["iters"] == s2[0]["iters"]
    # graphs on and off run the same launches
    p = W.default_params(use_graph=0)
    x3, _ = lat.solve(_dev(b), 0.135, p)
    x4, _ = lat.solve(_dev(b), 0.135, W.default_params())
    assert np.array_equal(_host(x3), _host(x4))


def test_twelve_point_sources_batched():
    """12 spin-colour point sources in one launch; each rhs equals its alone solve."""
    L = (8, 8, 8, 8)
    g = qcdgen.rng(207)
    U = qcdgen.links_exp(L, 0.3, g)
    B = qcdgen.point_sources(L)
    W = _W()
    lat = _lattice(L, U, [("f64", 18), ("f32", 12)])
    kappas = [0.130, 0.134, 0.1365] * 4
    p = W.default_params(inner="f32", delta=1e-2)
    X, st = lat.solve(_dev(B), kappas, p)
    X = _host(X)
    for r in range(12):
        assert st[r]["status"] == 0
        assert _oracle_resid(U, X[r], B[r], kappas[r], eo=True) <= TOL
        xa, sa = lat.solve(_dev(B[r]), kappas[r], p)
        xa = _host(xa)
        assert np.linalg.norm(X[r] - xa) / np.linalg.norm(xa) < 1e-8


def test_batch_of_uneven_lattices():
    W = _W()
    reqs, host = [], []
    for i, (L, w, k) in enumerate([((4, 4, 4, 4), 0.3, 0.12), ((8, 8, 8, 8), 0.4, 0.13), ((4, 6, 8, 10), 0.2, 0.125)]):
        g = qcdgen.rng(300 + i)
        U = qcdgen.links_exp(L, w, g)
        b = qcdgen.gaussian_spinor(L, g)
        lat = _lattice(L, U, [("f64", 18), ("f32", 12)])
        reqs.append((lat, _dev(b), [k]))
        host.append((U, b, k, lat))
    p = W.default_params(inner="f32", delta=1e-2)
    res = W.solve_batch(reqs, p)
    for (x, st), (U, b, k, lat) in zip(res, host):
        x = _host(x)
        assert st[0]["status"] == 0
        assert _oracle_resid(U, x, b, k, eo=True) <= TOL
        xa, _ = lat.solve(_dev(b), k, p)
        # same per-slot arithmetic alone and in the batch
        assert np.array_equal(x, _host(xa))


def test_failure_paths():
    W = _W()
    L = (4, 4, 4, 4)
    g = qcdgen.rng(401)
    U = qcdgen.links_haar(L, g)
    lat = _lattice(L, U, [("f64", 18)])
    b = qcdgen.gaussian_spinor(L, g)
    # too few iterations: not converged, stats filled, x holds the last iterate
    x, st = lat.solve(_dev(b), 0.12, W.default_params(maxiter=3), check=False)
    assert st[0]["status"] == W.WD_ENOTCONVERGED
    assert st[0]["iters"] >= 3 and st[0]["true_resid"] > TOL
    # non-finite source
    bn = b.copy()
    bn[0, 0, 0, 0, 0, 0] = np.nan
    x, st = lat.solve(_dev(bn), 0.12, W.default_params(), check=False)
    assert st[0]["status"] == W.WD_ENONFINITE
    # zero source: x = 0 immediately
    x, st = lat.solve(_dev(np.zeros_like(b)), 0.12, W.default_params())
    assert st[0]["status"] == 0 and np.abs(_host(x)).max() == 0.0
    # missing inner store
    with pytest.raises(W.WDError) as e:
        lat.solve(_dev(b), 0.12, W.default_params(inner="f32"))
    assert e.value.status == W.WD_ENOGAUGE


def test_kappa_zero_one_iteration():
    W = _W()
    L = (4, 4, 4, 4)
    g = qcdgen.rng(403)
    U = qcdgen.links_haar(L, g)
    b = qcdgen.gaussian_spinor(L, g)
    lat = _lattice(L, U, [("f64", 18)])
    x, st = lat.solve(_dev(b), 0.0, W.default_params(precond=W.FULL))
    assert st[0]["iters"] == 1
    assert np.abs(_host(x) - b).max() < 1e-15


def test_config2_full_size_fp64_cg():
    """16^3x32, exp(0.3 i H) links, kappa 0.1365, even-odd, plain FP64 CG to 1e-10."""
    L = (16, 16, 16, 32)
    g = qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 1)
    U = qcdgen.links_exp(L, 0.3, g)
    b = qcdgen.gaussian_spinor(L, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 101))
    W = _W()
    lat = _lattice(L, U, [("f64", 18), ("f32", 12), ("f16", 12)])
    x, st = lat.solve(_dev(b), 0.1365, W.default_params())
    x = _host(x)
    assert st[0]["status"] == 0 and st[0]["true_resid"] <= TOL
    assert _oracle_resid(U, x, b, 0.1365, eo=True) <= TOL
    for inner in ("f32", "f16"):
        xm, sm = lat.solve(_dev(b), 0.1365, W.default_params(inner=inner, delta=1e-2))
        xm = _host(xm)
        assert sm[0]["status"] == 0
        assert _oracle_resid(U, xm, b, 0.1365, eo=True) <= TOL


def test_streamed_link_kernels_solve():
    """24^3x28 (193536 sites per parity), exp(0.4 i H) links, kappa 0.137,
    even-odd, FP64 recon-18 links: the link field (223 MB) exceeds three
    quarters of the Infinity Cache, so the FP64 stencils take the kernels that
    read the links with non-temporal loads, which the smaller lattices of the
    other tests never reach.  The plain FP64 CG and the FP16-inner CG, whose
    reliable updates run the FP64 true-residual stencil, both reach the
    oracle's 1e-10."""
    L = (24, 24, 24, 28)
    g = qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 2)
    U = qcdgen.links_exp(L, 0.4, g)
    b = qcdgen.gaussian_spinor(L, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 102))
    W = _W()
    lat = _lattice(L, U, [("f64", 18), ("f16", 12)])
    for inner in ("f64", "f16"):
        p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0)
        x, st = lat.solve(_dev(b), 0.137, p)
        x = _host(x)
        assert st[0]["status"] == 0 and st[0]["true_resid"] <= TOL, inner
        assert _oracle_resid(U, x, b, 0.137, eo=True) <= TOL, inner


def test_batch_mixed_nrhs_and_many_items():
    """More items than slots per launch, and items with different nrhs in one batch."""
    W = _W()
    p = W.default_params(inner="f32", delta=1e-2)
    reqs, host = [], []
    for i in range(11):
        L = [(4, 4, 4, 4), (4, 4, 2, 6), (6, 4, 4, 4)][i % 3]
        g = qcdgen.rng(500 + i)
        U = qcdgen.links_exp(L, 0.3, g)
        nrhs = 1 if i % 4 else 3
        b = qcdgen.gaussian_spinor(L, g, nrhs) if nrhs > 1 else qcdgen.gaussian_spinor(L, g)
        kap = [0.12 + 0.001 * i] * nrhs
        lat = _lattice(L, U, [("f64", 18), ("f32", 12)])
        reqs.append((lat, _dev(b), kap))
        host.append((U, b, kap))
    res = W.solve_batch(reqs, p)
    for (x, st), (U, b, kap) in zip(res, host):
        x = _host(x)
        if b.ndim == 6:
            assert st[0]["status"] == 0
            assert _oracle_resid(U, x, b, kap[0], eo=True) <= TOL
        else:
            for r in range(b.shape[0]):
                assert st[r]["status"] == 0
                assert _oracle_resid(U, x[r], b[r], kap[r], eo=True) <= TOL


@pytest.mark.parametrize("inner", ["f32", "f16"])
def test_full_mode_mixed_precision(inner):
    L = (4, 4, 4, 8)
    g = qcdgen.rng(601)
    U = qcdgen.links_haar(L, g)
    b = qcdgen.gaussian_spinor(L, g)
    W = _W()
    lat = _lattice(L, U, [("f64", 18), (inner, 12)])
    x, st = lat.solve(_dev(b), 0.12, W.default_params(precond=W.FULL, inner=inner, delta=1e-2))
    assert st[0]["status"] == 0
    assert _oracle_resid(U, _host(x), b, 0.12, eo=False) <= TOL


def test_server_multi_rhs_requests():
    W = _W()
    L = (8, 8, 4, 8)
    g = qcdgen.rng(701)
    U = qcdgen.links_exp(L, 0.3, g)
    lat = _lattice(L, U, [("f64", 18), ("f32", 12)])
    p = W.default_params(inner="f32", delta=1e-2)
    srv = W.Server(1 << 30, max_slots=4, params=p)
    B = qcdgen.point_sources(L)
    b1 = qcdgen.gaussian_spinor(L, g)
    t12 = srv.submit(lat, _dev(B), [0.13] * 12)
    t1 = srv.submit(lat, _dev(b1), 0.125)
    X, st12 = srv.wait(t12, 60000)
    x1, st1 = srv.wait(t1, 60000)
    srv.close()
    X, x1 = _host(X), _host(x1)
    for r in range(12):
        assert st12[r]["status"] == 0
        assert _oracle_resid(U, X[r], B[r], 0.13, eo=True) <= TOL
    assert st1[0]["status"] == 0 and _oracle_resid(U, x1, b1, 0.125, eo=True) <= TOL


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_batch_mixes_link_recons(inner):
    """Lattices whose FP64 (and inner) stores hold different recons share one
    batch: each launch takes only slots of one recon, so every result meets
    the oracle's residual and equals its solve alone bit for bit."""
    W = _W()
    cases = [((4, 4, 4, 4), 0.3, 0.12, 18, 12), ((8, 8, 8, 8), 0.4, 0.13, 12, 18),
             ((4, 6, 8, 10), 0.2, 0.125, 18, 18), ((6, 4, 4, 4), 0.35, 0.128, 12, 12)]
    reqs, host = [], []
    for i, (L, w, k, r64, rin) in enumerate(cases):
        g = qcdgen.rng(800 + i)
        U = qcdgen.links_exp(L, w, g)
        b = qcdgen.gaussian_spinor(L, g)
        stores = [("f64", r64)] + ([("f32", rin)] if inner == "f32" else [])
        lat = _lattice(L, U, stores)
        reqs.append((lat, _dev(b), [k]))
        host.append((U, b, k, lat))
    p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0)
    res = W.solve_batch(reqs, p)
    for (x, st), (U, b, k, lat) in zip(res, host):
        x = _host(x)
        assert st[0]["status"] == 0
        assert _oracle_resid(U, x, b, k, eo=True) <= TOL
        xa, sa = lat.solve(_dev(b), k, p)
        assert np.array_equal(x, _host(xa))
        assert st[0]["iters"] == sa[0]["iters"]


@pytest.mark.parametrize("inner", ["f64", "f16"])
def test_timed_solve_stats(inner):
    """A solve with per-launch timing returns bitwise the solution of the untimed
    solve, and its stencil figures are consistent: the per-mode launches add up
    to the launches counted, every counted launch carries its mode's algorithmic
    bytes (8 links, input spinor, epilogue vectors per output site), and the
    launches left out as skipped are few beside them."""
    L = (8, 8, 8, 16)
    g = qcdgen.rng(177)
    U = qcdgen.links_exp(L, 0.3, g)
    b = qcdgen.gaussian_spinor(L, g)
    W = _W()
    lat = _lattice(L, U, [("f64", 12), ("f16", 12)])
    p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0)
    x0, st0 = lat.solve(_dev(b), 0.1365, p)
    pt = W.SolveParams.from_buffer_copy(p)
    pt.timing = 1
    x1, st1 = lat.solve(_dev(b), 0.1365, pt)
    assert np.array_equal(_host(x0), _host(x1))
    s = st1[0]
    assert s["status"] == 0 and s["iters"] == st0[0]["iters"]
    assert sum(s["hop_mode_launches"]) == s["hop_launches"] > 0
    assert 0 <= s["hop_skipped"] <= s["hop_launches"]
    half = L[0] * L[1] * L[2] * L[3] // 2
    link = {"f64": 96, "f16": 24}
    sp = {"f64": 192, "f16": 52}
    acc = {"f64": 192, "f16": 96}
    for m in range(4):
        n = s["hop_mode_launches"][m]
        if n == 0:
            continue
        per = s["hop_mode_bytes"][m] / n
        # inner-precision launches and FP64 reliable-update launches mix in
        # a mixed solve: their bytes per launch lie between the two formats'
        lo = min(8 * link[q] + sp[q] + (sp[q], 2 * sp[q], sp[q] + 2 * acc[q], sp[q] + 2 * 192)[m]
                 for q in {inner, "f64"}) * half
        hi = max(8 * link[q] + sp[q] + (sp[q], 2 * sp[q], sp[q] + 2 * acc[q], sp[q] + 2 * 192)[m]
                 for q in {inner, "f64"}) * half
        assert lo - 1 <= per <= hi + 1, (m, per, lo, hi)
        assert s["hop_mode_ms"][m] > 0.0
