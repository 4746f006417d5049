"""Continuous-batching server: every result equals its alone solve, requests of
uneven lattices run together, admission respects the pool footprint."""

import time

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


def _field(L, w, seed):
    W = _W()
    g = qcdgen.rng(seed)
    U = qcdgen.links_exp(L, w, g)
    lat = W.Lattice(L, BC)
    Ud = _dev(U)
    for prec, recon in (("f64", 18), ("f32", 12), ("f16", 12)):
        lat.set_gauge(Ud, prec, recon)
    return lat, U


@pytest.mark.parametrize("inner", ["f16", "f64"])
def test_served_equals_alone(inner):
    W = _W()
    fields = [_field((4, 4, 4, 4), 0.3, 1), _field((8, 8, 8, 8), 0.4, 2), _field((6, 4, 8, 4), 0.25, 3)]
    g = qcdgen.rng(77)
    params = W.default_params(inner=inner, delta=1e-2 if inner != "f64" else 0.0)
    srv = W.Server(1 << 30, max_slots=4, params=params)
    reqs = []
    for i in range(9):
        lat, U = fields[i % 3]
        b = qcdgen.gaussian_spinor(lat.L, g)
        kappa = float(g.uniform(0.12, 0.136))
        reqs.append((lat, U, b, kappa, srv.submit(lat, _dev(b), kappa)))
        time.sleep(0.002 * (i % 2))   # arrivals while others run
    results = {}
    t0 = time.time()
    while len(results) < len(reqs) and time.time() - t0 < 60:
        for lat, U, b, kappa, t in reqs:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.001)
    srv.close()
    assert len(results) == len(reqs)
    for lat, U, b, kappa, t in reqs:
        x, st = results[t]
        x = _host(x)
        assert st[0]["status"] == 0
        assert O.residual_DdagD(U, x, b, kappa, BC, True) <= 1e-10
        xa, sa = lat.solve(_dev(b), kappa, params)
        xa = _host(xa)
        # same per-request arithmetic alone and in the mix
        assert np.linalg.norm(x - xa) / np.linalg.norm(xa) <= 1e-12
        assert st[0]["iters"] == sa[0]["iters"]
        assert st[0]["seconds"] > 0


def test_admission_by_footprint():
    W = _W()
    lat, U = _field((8, 8, 8, 8), 0.3, 5)
    params = W.default_params(inner="f32", delta=1e-2)
    probe = W.Server(64 << 20, max_slots=2, params=params)
    need = probe.footprint(lat)
    probe.close()
    # a pool that fits one request at a time: requests queue FIFO and all finish
    srv = W.Server(need + 2 * 16 * 128 + 4096, max_slots=2, params=params)
    g = qcdgen.rng(9)
    bs = [qcdgen.gaussian_spinor(lat.L, g) for _ in range(3)]
    ts = [srv.submit(lat, _dev(b), 0.13) for b in bs]
    outs = [srv.wait(t, timeout_ms=30000) for t in ts]
    assert all(o is not None for o in outs)
    for (x, st), b in zip(outs, bs):
        assert st[0]["status"] == 0
        assert O.residual_DdagD(U, _host(x), b, 0.13, BC, True) <= 1e-10
    # a request that can never fit is refused at submit
    big, _ = _field((16, 8, 8, 8), 0.3, 6)
    with pytest.raises(W.WDError) as e:
        srv.submit(big, _dev(qcdgen.gaussian_spinor(big.L, g)), 0.13)
    assert e.value.status == W.WD_EBUSY
    srv.close()
