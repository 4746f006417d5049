"""The allocation-free entry point wd_apply_D_noalloc against wd_apply_D.

Both run the same kernels in the same launch shapes, so the outputs must be
bitwise equal; the first is also checked against the oracle.  Two calls in a
row, the second on a smaller lattice (the shared scratch array keeps the
first call's contents), then a call too large for the array."""

import numpy as np
import pytest

import oracle as O
import qcdgen

pytestmark = pytest.mark.gpu

BC = (1, 1, 1, -1)


def _W():
    from paper_2409_03030_amd import wdirac
    return wdirac


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _case(L, seed, precs, nrhs=None):
    W = _W()
    g = qcdgen.rng(seed)
    U = qcdgen.links_exp(L, 0.4, g)
    psi = qcdgen.gaussian_spinor(L, g, nrhs)
    lat = W.Lattice(L, BC)
    Ud = _dev(U)
    for prec, recon in precs:
        lat.set_gauge(Ud, prec, recon)
    return lat, U, psi


def test_noalloc_apply_matches_apply_twice():
    W = _W()
    # first call: 16^3x16 (65536 sites), the largest FP64 even-odd D_hat that fits
    L1 = (16, 16, 16, 16)
    lat1, U1, psi1 = _case(L1, 901, [("f64", 12), ("f32", 12)])
    y1n = _host(lat1.apply_D_noalloc(_dev(psi1), 0.137, precond=W.EO, prec="f64"))
    y1 = _host(lat1.apply_D(_dev(psi1), 0.137, precond=W.EO, prec="f64"))
    assert np.array_equal(y1n, y1)
    ref = O.apply_Dhat(U1, psi1 * O.even_mask(L1), 0.137, BC)
    assert np.linalg.norm(y1n - ref) / np.linalg.norm(ref) < 1e-12
    # second call: smaller, full lattice, D^dag, 3 fields, FP32
    L2 = (4, 6, 4, 8)
    lat2, U2, psi2 = _case(L2, 902, [("f64", 18), ("f32", 18)], nrhs=3)
    y2n = _host(lat2.apply_D_noalloc(_dev(psi2), 0.125, dagger=True, precond=W.FULL, prec="f32"))
    y2 = _host(lat2.apply_D(_dev(psi2), 0.125, dagger=True, precond=W.FULL, prec="f32"))
    assert np.array_equal(y2n, y2)
    for r in range(3):
        ref = O.apply_Ddag(U2, psi2[r], 0.125, BC)
        assert np.linalg.norm(y2n[r] - ref) / np.linalg.norm(ref) < 1e-5
    # and the first lattice again after the smaller call
    y1b = _host(lat1.apply_D_noalloc(_dev(psi1), 0.137, precond=W.EO, prec="f64"))
    assert np.array_equal(y1b, y1)
    lat1.close()
    lat2.close()


def test_noalloc_apply_rejects_what_does_not_fit():
    W = _W()
    L = (16, 16, 16, 32)
    lat, U, psi = _case(L, 903, [("f64", 12)])
    assert W.lib().wd_apply_workspace_bytes(lat.handle, W.F64, 1) > W.NOALLOC_SCRATCH_BYTES
    with pytest.raises(W.WDError) as e:
        lat.apply_D_noalloc(_dev(psi), 0.137, precond=W.EO, prec="f64")
    assert e.value.status == W.WD_EBUFSIZE
    lat.close()
