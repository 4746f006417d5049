"""The measured workloads at their own sizes, checked against the oracle.

* 24^3x48, links exp(0.4 i H), kappa 0.137, FP64 recon-12 links: the even-odd
  D_hat applied once and compared element by element with the oracle; the
  plain FP64 CG and the FP32- and FP16-inner CG (recon-12 inner links, FP64
  reliable updates at 1e-2), each in the launch shapes the autotuner picks
  and the plain FP64 CG also with 4 threads per site (the non-temporal
  recon-12 stencil), each to the oracle's FP64 true residual of 1e-10.
* 32^3x64 with FP32 recon-12 (402 MB) and FP16 recon-12 and recon-18 links (201 and
  302 MB), all streamed: D at sampled sites.
* 16^3x32, links exp(0.3 i H): 12 spin-colour point sources per kappa in
  {0.130, 0.134, 0.1365} in one batched solve (FP32 inner), and all 36 in
  one solve with per-rhs kappa; every column to the oracle's 1e-10.
* A served mix that holds 8^4, 12^3x24, 16^3x32 and 24^3x48 requests at once:
  each result meets the oracle's residual and equals its solve alone.

The oracle's residuals at these sizes take seconds each on the host; they
are evaluated in a thread pool (numpy releases the interpreter lock in its
array operations), which changes nothing in the oracle's arithmetic.
"""

from concurrent.futures import ThreadPoolExecutor

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


def _residuals(U, xs, bs, kappas):
    """Oracle FP64 true residuals ||b - A_hat x|| / ||b|| of several solutions."""
    def one(i):
        return O.residual_DdagD(U, xs[i], bs[i], kappas[i], BC, True)
    with ThreadPoolExecutor(min(8, len(xs))) as ex:
        return list(ex.map(one, range(len(xs))))


def _residuals_each(cases):
    """Oracle residuals of (U, x, b, kappa) cases on different lattices."""
    with ThreadPoolExecutor(len(cases)) as ex:
        return list(ex.map(lambda c: O.residual_DdagD(c[0], c[1], c[2], c[3], BC, True), cases))


@pytest.fixture(scope="module")
def cfg3():
    """24^3x48 workload with the seeds of the benchmark."""
    L = (24, 24, 24, 48)
    U = qcdgen.links_exp(L, 0.4, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 2))
    b = qcdgen.gaussian_spinor(L, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 102))
    W = _W()
    lat = W.Lattice(L, BC)
    Ud = _dev(U)
    shapes = {}
    for prec in ("f64", "f32", "f16"):
        lat.set_gauge(Ud, prec, 12)
        shapes[prec] = lat.autotune(prec, 1)
    del Ud
    _torch().cuda.empty_cache()
    yield L, U, b, lat, shapes
    lat.close()


def test_cfg3_dhat_apply_fp64_recon12(cfg3):
    L, U, b, lat, _ = cfg3
    W = _W()
    y = _host(lat.apply_D(_dev(b), 0.137, precond=W.EO, prec="f64"))
    ref = O.apply_Dhat(U, b * O.even_mask(L), 0.137, BC)
    assert np.abs(y * O.odd_mask(L)).max() == 0.0
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert err < 1e-12, err
    # element by element: no site deviates beyond rounding of its own size
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def _tune_line(L, prec, recon, nrhs, sblk, swz, split):
    return f"{L[0]} {L[1]} {L[2]} {L[3]} {prec} {recon} {nrhs} {sblk} {swz} {split}"


@pytest.mark.parametrize("inner", ["f64", "f32", "f16"])
def test_cfg3_solve(cfg3, inner):
    L, U, b, lat, shapes = cfg3
    W = _W()
    p = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0)
    xs, sts = [], []
    x, st = lat.solve(_dev(b), 0.137, p)
    xs.append(_host(x))
    sts.append(st[0])
    if inner == "f64":
        # the FP64 stencil with 4 threads per site (one direction each), the
        # shape of the 24^3x48 profile, whatever the autotuner picked above
        saved = W.tune_export()
        W.tune_import(_tune_line(L, 0, 12, 1, 64, 1, 4))
        try:
            x4, st4 = lat.solve(_dev(b), 0.137, p)
        finally:
            W.tune_import(saved)
        xs.append(_host(x4))
        sts.append(st4[0])
    for s in sts:
        assert s["status"] == 0 and s["true_resid"] <= TOL, s
    res = _residuals(U, xs, [b] * len(xs), [0.137] * len(xs))
    assert max(res) <= TOL, res
    if inner != "f64":
        assert sts[0]["reliable_updates"] >= 2


@pytest.fixture(scope="module")
def big():
    L = (32, 32, 32, 64)
    U = qcdgen.links_exp(L, 0.4, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 2))
    b = qcdgen.gaussian_spinor(L, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 103))
    g = qcdgen.rng(11)
    sites = [(0, 0, 0, 0), (L[0] - 1, L[1] - 1, L[2] - 1, L[3] - 1), (0, L[1] - 1, 0, L[3] - 1),
             (L[0] - 1, 0, L[2] - 1, 0)]
    sites += [tuple(int(g.integers(0, L[m])) for m in range(4)) for _ in range(124)]
    ref = O.apply_D_sites(U, b, 0.137, BC, sites)
    return L, U, b, sites, ref


@pytest.mark.parametrize("prec,recon,tol", [("f32", 12, 1e-5), ("f16", 12, 3e-3), ("f16", 18, 3e-3)])
def test_streamed_links_sampled_sites(big, prec, recon, tol):
    """32^3x64 with link fields beyond three quarters of the Infinity Cache
    (FP32 recon-12 402 MB, FP16 recon-12 201 MB, FP16 recon-18 302 MB): the
    streamed stencils at 128 sampled sites, corners included, against the
    oracle's site-wise D."""
    L, U, b, sites, ref = big
    W = _W()
    lat = W.Lattice(L, BC)
    Ud = _dev(U)
    assert lat.gauge_bytes(prec, recon) > 192e6
    lat.set_gauge(Ud, prec, recon)
    del Ud
    y = _host(lat.apply_D(_dev(b), 0.137, precond=W.FULL, prec=prec))
    got = np.stack([y[t, z, yy, x] for (x, yy, z, t) in sites])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < tol, err
    lat.close()


@pytest.fixture(scope="module")
def cfg4():
    L = (16, 16, 16, 32)
    U = qcdgen.links_exp(L, 0.3, qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 1))
    B = qcdgen.point_sources(L)
    W = _W()
    lat = W.Lattice(L, BC)
    Ud = _dev(U)
    for prec, recon in (("f64", 18), ("f32", 12)):
        lat.set_gauge(Ud, prec, recon)
        for nrhs in (1, 4):
            lat.autotune(prec, nrhs)
    yield L, U, B, lat
    lat.close()


@pytest.mark.parametrize("kappa", [0.130, 0.134, 0.1365])
def test_cfg4_twelve_point_sources(cfg4, kappa):
    L, U, B, lat = cfg4
    W = _W()
    p = W.default_params(inner="f32", delta=1e-2)
    X, st = lat.solve(_dev(B), [kappa] * 12, p)
    X = _host(X)
    assert all(s["status"] == 0 for s in st), st
    res = _residuals(U, list(X), list(B), [kappa] * 12)
    assert max(res) <= TOL, res


def test_cfg4_thirty_six_sources_mixed_kappa(cfg4):
    """36 sources in one request: their FP32-inner vectors (1.1 GB) exceed the
    cache-blocking budget, so the request runs as waves of 12 sources, each
    bitwise the same as that 12-source request solved alone."""
    L, U, B, lat = cfg4
    W = _W()
    p = W.default_params(inner="f32", delta=1e-2)
    ks = [0.130] * 12 + [0.134] * 12 + [0.1365] * 12
    B36 = np.concatenate([B, B, B], 0)
    X, st = lat.solve(_dev(B36), ks, p)
    X = _host(X)
    assert all(s["status"] == 0 for s in st), st
    res = _residuals(U, list(X), list(B36), ks)
    assert max(res) <= TOL, res
    # iterations grow with kappa (the operator's condition number does)
    its = [st[12 * k]["iters"] for k in range(3)]
    assert its[0] < its[1] < its[2], its
    for k in range(3):
        Xk, stk = lat.solve(_dev(B), ks[12 * k: 12 * k + 12], p)
        assert np.array_equal(_host(Xk), X[12 * k: 12 * k + 12]), k
        assert [s["iters"] for s in stk] == [s["iters"] for s in st[12 * k: 12 * k + 12]], k


@pytest.mark.parametrize("inner", ["f16", "f64"])
def test_served_mix_of_full_sizes(inner):
    """One request per lattice size of the served stream, 24^3x48 included,
    submitted together: each result meets the oracle's 1e-10 and equals the
    same request solved alone (1e-12, same iteration count)."""
    W = _W()
    g = qcdgen.rng(qcdgen.CONFIG_SEED_BASE + 4)
    params = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0)
    reqs = []
    for i, L in enumerate([(8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32), (24, 24, 24, 48)]):
        w = float(g.uniform(0.2, 0.5))
        U = qcdgen.links_exp(L, w, g)
        lat = W.Lattice(L, BC)
        Ud = _dev(U)
        for prec, recon in (("f64", 18), ("f32", 12), ("f16", 12)):
            lat.set_gauge(Ud, prec, recon)
        del Ud
        b = qcdgen.gaussian_spinor(L, g)
        kappa = float(g.uniform(0.12, 0.136))
        reqs.append((lat, U, b, kappa))
    free, _ = _torch().cuda.mem_get_info()
    srv = W.Server(int(min(8 << 30, free // 2)), max_slots=8, params=params)
    tickets = [srv.submit(lat, _dev(b), kappa) for lat, U, b, kappa in reqs]
    outs = [srv.wait(t, timeout_ms=60000) for t in tickets]
    srv.close()
    assert all(o is not None for o in outs)
    xs = [_host(o[0]) for o in outs]
    for (x, st) in outs:
        assert st[0]["status"] == 0, st
    res = _residuals_each([(U, x, b, k) for (lat, U, b, k), x in zip(reqs, xs)])
    assert max(res) <= TOL, res
    for (lat, U, b, kappa), x, (xo, st) in zip(reqs, xs, outs):
        xa, sa = lat.solve(_dev(b), kappa, params)
        xa = _host(xa)
        assert np.linalg.norm(x - xa) / np.linalg.norm(xa) <= 1e-12
        assert st[0]["iters"] == sa[0]["iters"]
    for lat, *_ in reqs:
        lat.close()
