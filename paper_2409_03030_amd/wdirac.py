"""ctypes binding of ``libwdirac.so`` (argument marshalling only).

Every computation happens in the HIP library; this module only passes device
pointers of PyTorch tensors, sizes and the current HIP stream through the
C ABI declared in ``include/wdirac.h``, allocating outputs, gauge stores and
workspaces as torch tensors.  If the library is missing the import fails:
there is no fallback.

Fields use the boundary layout of the C ABI: complex128 spinors
``[Lt, Lz, Ly, Lx, 4, 3]`` (or ``[nrhs, Lt, Lz, Ly, Lx, 4, 3]``) and links
``[4, Lt, Lz, Ly, Lx, 3, 3]``.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwdirac.so")

WD_OK, WD_EINVAL, WD_EBUFSIZE, WD_ENOGAUGE, WD_ENOTCONVERGED, WD_ENONFINITE, WD_EDEVICE, WD_EBUSY, WD_ENOTFOUND = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
F64, F32, F16 = 0, 1, 2
FULL, EO = 0, 1
# size of the allocation-free call's scratch array (WD_NOALLOC_SCRATCH_BYTES in wdirac.h)
NOALLOC_SCRATCH_BYTES = 64 << 20
PREC = {"f64": F64, "f32": F32, "f16": F16, F64: F64, F32: F32, F16: F16}


class WDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class SolveParams(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("maxiter", C.c_int32),
        ("inner", C.c_int32),
        ("recon", C.c_int32),
        ("delta", C.c_double),
        ("precond", C.c_int32),
        ("poll_every", C.c_int32),
        ("use_graph", C.c_int32),
        ("timing", C.c_int32),
        ("rhs_group", C.c_int32),
    ]


class SolveStats(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("iters", C.c_int32),
        ("reliable_updates", C.c_int32),
        ("hop_skipped", C.c_int32),
        ("true_resid", C.c_double),
        ("iter_resid", C.c_double),
        ("seconds", C.c_double),
        ("hop_ms", C.c_double),
        ("hop_launches", C.c_int64),
        ("hop_site_updates", C.c_int64),
        ("hop_bytes", C.c_double),
        ("hop_mode_ms", C.c_double * 4),
        ("hop_mode_launches", C.c_int64 * 4),
        ("hop_mode_bytes", C.c_double * 4),
        ("hop_inner_mode_ms", C.c_double * 4),
        ("hop_inner_mode_launches", C.c_int64 * 4),
        ("hop_inner_mode_bytes", C.c_double * 4),
    ]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if hasattr(v, "__len__") else v
        return d


class SolveRequest(C.Structure):
    _fields_ = [
        ("lat", C.c_void_p),
        ("x", C.c_void_p),
        ("b", C.c_void_p),
        ("nrhs", C.c_int32),
        ("pad", C.c_int32),
        ("kappa", C.POINTER(C.c_double)),
    ]


# exported symbols and their signatures (name, restype, argtypes)
_P = C.c_void_p
_SIGS = [
    ("wd_lattice_create", C.c_int32, [C.POINTER(C.c_void_p), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("wd_lattice_destroy", C.c_int32, [_P]),
    ("wd_gauge_bytes", C.c_size_t, [_P, C.c_int32, C.c_int32]),
    ("wd_set_gauge", C.c_int32, [_P, _P, _P, C.c_size_t, C.c_int32, C.c_int32, _P]),
    ("wd_apply_workspace_bytes", C.c_size_t, [_P, C.c_int32, C.c_int32]),
    ("wd_apply_D", C.c_int32, [_P, _P, _P, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_int32, _P, C.c_size_t, _P]),
    ("wd_apply_DdagD", C.c_int32, [_P, _P, _P, C.c_int32, C.c_double, C.c_int32, C.c_int32, _P, C.c_size_t, _P]),
    ("wd_apply_D_noalloc", C.c_int32, [_P, _P, _P, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_int32, _P]),
    ("wd_solver_workspace_bytes", C.c_size_t, [_P, C.POINTER(SolveParams), C.c_int32]),
    ("wd_solve_params_default", None, [C.POINTER(SolveParams)]),
    ("wd_solve_DdagD", C.c_int32, [_P, _P, _P, C.c_int32, C.POINTER(C.c_double), C.POINTER(SolveParams), _P,
                                   C.c_size_t, C.POINTER(SolveStats), _P]),
    ("wd_solve_D_workspace_bytes", C.c_size_t, [_P, C.POINTER(SolveParams), C.c_int32]),
    ("wd_solve_D", C.c_int32, [_P, _P, _P, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.POINTER(SolveParams), _P,
                               C.c_size_t, C.POINTER(SolveStats), _P]),
    ("wd_pion_workspace_bytes", C.c_size_t, [_P]),
    ("wd_pion_correlator", C.c_int32, [_P, C.POINTER(C.c_double), _P, C.c_int32, C.c_int32, _P, C.c_size_t, _P]),
    ("wd_stag_pion_correlator", C.c_int32, [_P, C.POINTER(C.c_double), _P, C.c_int32, C.c_int32, _P, C.c_size_t,
                                            _P]),
    ("wd_pseudofermion_heatbath", C.c_int32, [_P, _P, _P, C.c_double, _P, C.c_size_t, _P]),
    ("wd_fermion_force_workspace_bytes", C.c_size_t, [_P, C.POINTER(SolveParams)]),
    ("wd_fermion_force", C.c_int32, [_P, _P, C.POINTER(C.c_double), _P, C.c_double, C.POINTER(SolveParams), _P,
                                     C.c_size_t, C.POINTER(SolveStats), _P]),
    ("wd_ta_add", C.c_int32, [_P, _P, C.c_double, _P, _P]),
    ("wd_stag_apply_workspace_bytes", C.c_size_t, [_P, C.c_int32, C.c_int32]),
    ("wd_stag_apply", C.c_int32, [_P, _P, _P, C.c_int32, C.c_double, C.c_int32, C.c_int32, _P, C.c_size_t, _P]),
    ("wd_stag_set_shape", C.c_int32, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    ("wd_stag_autotune", C.c_int32, [_P, C.c_int32, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P]),
    ("wd_stag_solve_workspace_bytes", C.c_size_t, [_P, C.POINTER(SolveParams), C.c_int32]),
    ("wd_stag_solve", C.c_int32, [_P, _P, _P, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.POINTER(SolveParams),
                                  _P, C.c_size_t, C.POINTER(SolveStats), _P]),
    ("wd_batch_workspace_bytes", C.c_size_t, [C.c_int32, C.POINTER(SolveRequest), C.POINTER(SolveParams)]),
    ("wd_solve_batch", C.c_int32, [C.c_int32, C.POINTER(SolveRequest), C.POINTER(SolveParams), _P, C.c_size_t,
                                   C.POINTER(SolveStats), _P]),
    ("wd_time_hop", C.c_int32, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.c_size_t,
                                C.POINTER(C.c_double), _P]),
    ("wd_time_read", C.c_int32, [_P, C.c_size_t, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_double), _P]),
    ("wd_autotune", C.c_int32, [_P, C.c_int32, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P]),
    ("wd_tune_export", C.c_size_t, [C.c_char_p, C.c_size_t]),
    ("wd_tune_import", C.c_int32, [C.c_char_p]),
    ("wd_server_create", C.c_int32, [C.POINTER(C.c_void_p), _P, C.c_size_t, C.c_int32, C.POINTER(SolveParams), _P]),
    ("wd_server_destroy", C.c_int32, [_P]),
    ("wd_server_footprint", C.c_size_t, [_P, _P, C.c_int32]),
    ("wd_server_submit", C.c_int32, [_P, _P, _P, _P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    ("wd_server_poll", C.c_int32, [_P, C.c_uint64, C.POINTER(SolveStats)]),
    ("wd_server_wait", C.c_int32, [_P, C.c_uint64, C.POINTER(SolveStats), C.c_int32]),
    ("wd_status_string", C.c_char_p, [C.c_int32]),
    ("wd_last_error", C.c_char_p, []),
    ("wd_version", C.c_char_p, []),
]
SYMBOLS = [s[0] for s in _SIGS]

_lib = None


def lib():
    """The loaded library (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_03030_amd.build`")
        # torch first: its wheel carries its own HIP runtime, and the library
        # must bind to that one.  Loaded the other way round, the process holds
        # two HIP runtimes and a kernel launched through one is unknown to the
        # other ("invalid device function").
        _torch()
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, what=""):
    if status != WD_OK:
        msg = lib().wd_last_error().decode()
        raise WDError(status, f"{what}: {msg}" if what else msg)


def default_params(**kw) -> SolveParams:
    p = SolveParams()
    lib().wd_solve_params_default(C.byref(p))
    for k, v in kw.items():
        if k in ("inner",):
            v = PREC[v]
        if k == "precond" and isinstance(v, str):
            v = EO if v.lower() == "eo" else FULL
        setattr(p, k, v)
    return p


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _check_field(t, shape, name):
    torch = _torch()
    if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Lattice:
    """A lattice with boundary signs and its registered gauge stores."""

    def __init__(self, L, bc=(1, 1, 1, -1)):
        self.L = tuple(int(v) for v in L)
        self.bc = tuple(int(v) for v in bc)
        h = C.c_void_p()
        Ls = (C.c_int32 * 4)(*self.L)
        bcs = (C.c_int32 * 4)(*self.bc)
        _check(lib().wd_lattice_create(C.byref(h), Ls, bcs), "wd_lattice_create")
        self.handle = h
        self.stores = {}
        self._ws = {}

    def close(self):
        if self.handle:
            lib().wd_lattice_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def site_shape(self):
        Lx, Ly, Lz, Lt = self.L
        return (Lt, Lz, Ly, Lx)

    @property
    def volume(self):
        v = 1
        for x in self.L:
            v *= x
        return v

    def gauge_bytes(self, prec, recon=18):
        return int(lib().wd_gauge_bytes(self.handle, PREC[prec], recon))

    def set_gauge(self, U, prec="f64", recon=18, stream=None):
        """Convert the complex128 device field U into a new store of (prec, recon)."""
        torch = _torch()
        _check_field(U, (4,) + self.site_shape + (3, 3), "U")
        nb = self.gauge_bytes(prec, recon)
        if nb == 0:
            raise ValueError("bad precision or recon")
        store = torch.empty(nb, dtype=torch.uint8, device=U.device)
        _check(lib().wd_set_gauge(self.handle, _ptr(U), _ptr(store), nb, PREC[prec], recon, _stream(stream)),
               "wd_set_gauge")
        self.stores[PREC[prec]] = store
        return store

    def _workspace(self, nbytes, device, key):
        torch = _torch()
        w = self._ws.get(key)
        if w is None or w.numel() < nbytes:
            w = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            self._ws[key] = w
        return w

    def _field_shape(self, nrhs):
        base = self.site_shape + (4, 3)
        return base if nrhs is None else (nrhs,) + base

    def apply_D(self, x, kappa, dagger=False, precond=FULL, prec="f64", out=None, stream=None):
        torch = _torch()
        nrhs = None if x.dim() == 6 else x.shape[0]
        _check_field(x, self._field_shape(nrhs), "x")
        n = 1 if nrhs is None else nrhs
        y = torch.empty_like(x) if out is None else out
        nb = int(lib().wd_apply_workspace_bytes(self.handle, PREC[prec], n))
        ws = self._workspace(nb, x.device, ("apply", PREC[prec], n))
        _check(lib().wd_apply_D(self.handle, _ptr(y), _ptr(x), n, float(kappa), int(bool(dagger)), int(precond),
                                PREC[prec], _ptr(ws), ws.numel(), _stream(stream)), "wd_apply_D")
        return y

    def apply_D_noalloc(self, x, kappa, dagger=False, precond=FULL, prec="f64", out=None, stream=None):
        """apply_D through the allocation-free entry point (no workspace; see wdirac.h)."""
        torch = _torch()
        nrhs = None if x.dim() == 6 else x.shape[0]
        _check_field(x, self._field_shape(nrhs), "x")
        n = 1 if nrhs is None else nrhs
        y = torch.empty_like(x) if out is None else out
        _check(lib().wd_apply_D_noalloc(self.handle, _ptr(y), _ptr(x), n, float(kappa), int(bool(dagger)),
                                        int(precond), PREC[prec], _stream(stream)), "wd_apply_D_noalloc")
        return y

    def apply_DdagD(self, x, kappa, precond=FULL, prec="f64", out=None, stream=None):
        torch = _torch()
        nrhs = None if x.dim() == 6 else x.shape[0]
        _check_field(x, self._field_shape(nrhs), "x")
        n = 1 if nrhs is None else nrhs
        y = torch.empty_like(x) if out is None else out
        nb = int(lib().wd_apply_workspace_bytes(self.handle, PREC[prec], n))
        ws = self._workspace(nb, x.device, ("apply", PREC[prec], n))
        _check(lib().wd_apply_DdagD(self.handle, _ptr(y), _ptr(x), n, float(kappa), int(precond), PREC[prec],
                                    _ptr(ws), ws.numel(), _stream(stream)), "wd_apply_DdagD")
        return y

    def solve(self, b, kappa, params=None, out=None, stream=None, check=True):
        """x = (D^dag D)^{-1} b (or the even-odd system); returns (x, [stats dict per rhs])."""
        torch = _torch()
        params = params or default_params()
        nrhs = None if b.dim() == 6 else b.shape[0]
        _check_field(b, self._field_shape(nrhs), "b")
        n = 1 if nrhs is None else nrhs
        kap = [float(kappa)] * n if not hasattr(kappa, "__len__") else [float(k) for k in kappa]
        if len(kap) != n:
            raise ValueError("need one kappa per rhs")
        x = torch.empty_like(b) if out is None else out
        nb = int(lib().wd_solver_workspace_bytes(self.handle, C.byref(params), n))
        ws = self._workspace(nb, b.device, ("solve", params.inner, params.precond, n))
        stats = (SolveStats * n)()
        ka = (C.c_double * n)(*kap)
        st = lib().wd_solve_DdagD(self.handle, _ptr(x), _ptr(b), n, ka, C.byref(params), _ptr(ws), ws.numel(),
                                  stats, _stream(stream))
        if check and st not in (WD_OK,):
            _check(st, "wd_solve_DdagD")
        return x, [s.as_dict() for s in stats]

    def solve_D(self, b, kappa, params=None, dagger=False, out=None, stream=None, check=True):
        """x with D x = b (or D^dag x = b); every site of b and x is used.
        Returns (x, [stats dict per rhs]) with the stats of the normal-equation CG."""
        torch = _torch()
        params = params or default_params()
        nrhs = None if b.dim() == 6 else b.shape[0]
        _check_field(b, self._field_shape(nrhs), "b")
        n = 1 if nrhs is None else nrhs
        kap = [float(kappa)] * n if not hasattr(kappa, "__len__") else [float(k) for k in kappa]
        if len(kap) != n:
            raise ValueError("need one kappa per rhs")
        x = torch.empty_like(b) if out is None else out
        nb = int(lib().wd_solve_D_workspace_bytes(self.handle, C.byref(params), n))
        ws = self._workspace(nb, b.device, ("solve_D", params.inner, params.precond, n))
        stats = (SolveStats * n)()
        ka = (C.c_double * n)(*kap)
        st = lib().wd_solve_D(self.handle, _ptr(x), _ptr(b), n, ka, int(bool(dagger)), C.byref(params), _ptr(ws),
                              ws.numel(), stats, _stream(stream))
        if check and st not in (WD_OK,):
            _check(st, "wd_solve_D")
        return x, [s.as_dict() for s in stats]

    def propagator(self, kappa, params=None, origin=(0, 0, 0, 0), stream=None, device="cuda"):
        """The 12 point-source solutions S[3*alpha + a] of D S = delta_{x,origin} e_alpha e_a."""
        torch = _torch()
        src = torch.zeros((12,) + self._field_shape(None), dtype=torch.complex128, device=device)
        x, y, z, t = origin
        for alpha in range(4):
            for a in range(3):
                src[3 * alpha + a, t, z, y, x, alpha, a] = 1.0
        return self.solve_D(src, kappa, params=params, stream=stream)

    def pion_correlator(self, S, t0=0, stream=None):
        """C(t) = sum over the spatial sites of slice (t0 + t) mod Lt, the columns of S,
        spin and colour of |S|^2, for t = 0 .. Lt-1 (numpy array)."""
        import numpy as np
        if S.dim() != 7 or tuple(S.shape[1:]) != self._field_shape(None):
            raise ValueError(f"S must be [nsrc, {self._field_shape(None)}]")
        _check_field(S, tuple(S.shape), "S")
        nb = int(lib().wd_pion_workspace_bytes(self.handle))
        ws = self._workspace(nb, S.device, ("pion",))
        Lt = self.L[3]
        out = (C.c_double * Lt)()
        _check(lib().wd_pion_correlator(self.handle, out, _ptr(S), int(S.shape[0]), int(t0), _ptr(ws), ws.numel(),
                                        _stream(stream)), "wd_pion_correlator")
        return np.array(out[:], dtype=np.float64)

    def stag_propagator(self, mass, params=None, origin=(0, 0, 0, 0), stream=None, device="cuda"):
        """The 3 colour point-source solutions G[a] of D G = delta_{x,origin} e_a
        (staggered); returns (G, [stats dict per colour])."""
        torch = _torch()
        src = torch.zeros((3,) + self._stag_shape(None), dtype=torch.complex128, device=device)
        x, y, z, t = origin
        for a in range(3):
            src[a, t, z, y, x, a] = 1.0
        return self.stag_solve(src, mass, params=params, stream=stream)

    def stag_pion_correlator(self, G, t0=0, stream=None):
        """Goldstone pion correlator of staggered propagator columns G
        [nsrc, Lt, Lz, Ly, Lx, 3]: C(t) = sum of |G|^2 over slice (t0 + t) mod Lt."""
        import numpy as np
        if G.dim() != 6 or tuple(G.shape[1:]) != self._stag_shape(None):
            raise ValueError(f"G must be [nsrc, {self._stag_shape(None)}]")
        _check_field(G, tuple(G.shape), "G")
        nb = int(lib().wd_pion_workspace_bytes(self.handle))
        ws = self._workspace(nb, G.device, ("pion",))
        Lt = self.L[3]
        out = (C.c_double * Lt)()
        _check(lib().wd_stag_pion_correlator(self.handle, out, _ptr(G), int(G.shape[0]), int(t0), _ptr(ws),
                                             ws.numel(), _stream(stream)), "wd_stag_pion_correlator")
        return np.array(out[:], dtype=np.float64)

    def pseudofermion(self, xi, kappa, out=None, stream=None):
        """eta = D^dag xi (pseudofermion heatbath from a Gaussian xi)."""
        torch = _torch()
        _check_field(xi, self._field_shape(None), "xi")
        eta = torch.empty_like(xi) if out is None else out
        nb = int(lib().wd_apply_workspace_bytes(self.handle, PREC["f64"], 1))
        ws = self._workspace(nb, xi.device, ("apply", PREC["f64"], 1))
        _check(lib().wd_pseudofermion_heatbath(self.handle, _ptr(eta), _ptr(xi), float(kappa), _ptr(ws), ws.numel(),
                                               _stream(stream)), "wd_pseudofermion_heatbath")
        return eta

    def fermion_force(self, eta, kappa, params=None, force=True, stream=None, check=True):
        """(F, S_f, [stats of the two solves]): F_mu(x) = U dS_f/dU as a
        [4, Lt, Lz, Ly, Lx, 3, 3] complex128 tensor (None when force=False) and
        S_f = eta^dag (D^dag D)^{-1} eta."""
        torch = _torch()
        params = params or default_params()
        _check_field(eta, self._field_shape(None), "eta")
        F = torch.empty((4,) + self.site_shape + (3, 3), dtype=torch.complex128, device=eta.device) if force else None
        nb = int(lib().wd_fermion_force_workspace_bytes(self.handle, C.byref(params)))
        ws = self._workspace(nb, eta.device, ("force", params.inner, params.precond))
        stats = (SolveStats * 2)()
        act = C.c_double()
        st = lib().wd_fermion_force(self.handle, _ptr(F) if force else None, C.byref(act), _ptr(eta), float(kappa),
                                    C.byref(params), _ptr(ws), ws.numel(), stats, _stream(stream))
        if check and st != WD_OK:
            _check(st, "wd_fermion_force")
        return F, act.value, [s.as_dict() for s in stats]

    def ta_add(self, p, factor, F, stream=None):
        """p += factor * TA(F) in place (momentum update); returns p."""
        shape = (4,) + self.site_shape + (3, 3)
        for t, name in ((p, "p"), (F, "F")):
            torch = _torch()
            if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
                raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape {shape}")
        _check(lib().wd_ta_add(self.handle, _ptr(p), float(factor), _ptr(F), _stream(stream)), "wd_ta_add")
        return p

    def _stag_shape(self, nrhs):
        base = self.site_shape + (3,)
        return base if nrhs is None else (nrhs,) + base

    def stag_apply(self, x, mass, dagger=False, prec="f64", out=None, stream=None):
        """y = D x (or D^dag x) for the staggered operator; x is [(nrhs,) Lt, Lz, Ly, Lx, 3]."""
        torch = _torch()
        nrhs = None if x.dim() == 5 else x.shape[0]
        _check_field(x, self._stag_shape(nrhs), "x")
        n = 1 if nrhs is None else nrhs
        y = torch.empty_like(x) if out is None else out
        nb = int(lib().wd_stag_apply_workspace_bytes(self.handle, PREC[prec], n))
        ws = self._workspace(nb, x.device, ("stag_apply", PREC[prec], n))
        _check(lib().wd_stag_apply(self.handle, _ptr(y), _ptr(x), n, float(mass), int(bool(dagger)), PREC[prec],
                                   _ptr(ws), ws.numel(), _stream(stream)), "wd_stag_apply")
        return y

    def stag_autotune(self, prec="f64", nrhs=1, stream=None):
        """Tune the staggered stencil's launch shape; returns (sites per block, swizzle, split)."""
        nb = int(lib().wd_stag_apply_workspace_bytes(self.handle, PREC[prec], nrhs))
        dev = next(iter(self.stores.values())).device
        ws = self._workspace(nb, dev, ("stag_apply", PREC[prec], nrhs))
        sb, sw, sp = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().wd_stag_autotune(self.handle, PREC[prec], nrhs, _ptr(ws), ws.numel(), C.byref(sb), C.byref(sw),
                                      C.byref(sp), _stream(stream)), "wd_stag_autotune")
        return sb.value, sw.value, sp.value

    def stag_set_shape(self, prec, nrhs, sites_per_block, swizzle, split):
        """Force the staggered stencil's launch shape for (prec, nrhs)."""
        _check(lib().wd_stag_set_shape(self.handle, PREC[prec], int(nrhs), int(sites_per_block), int(swizzle),
                                       int(split)), "wd_stag_set_shape")

    def stag_solve(self, b, mass, params=None, dagger=False, out=None, stream=None, check=True):
        """x with D x = b (or D^dag x = b) for the staggered operator, even-odd CG.
        Returns (x, [stats dict per rhs])."""
        torch = _torch()
        params = params or default_params()
        nrhs = None if b.dim() == 5 else b.shape[0]
        _check_field(b, self._stag_shape(nrhs), "b")
        n = 1 if nrhs is None else nrhs
        ms = [float(mass)] * n if not hasattr(mass, "__len__") else [float(m) for m in mass]
        if len(ms) != n:
            raise ValueError("need one mass per rhs")
        x = torch.empty_like(b) if out is None else out
        nb = int(lib().wd_stag_solve_workspace_bytes(self.handle, C.byref(params), n))
        ws = self._workspace(nb, b.device, ("stag_solve", params.inner, n))
        stats = (SolveStats * n)()
        st = lib().wd_stag_solve(self.handle, _ptr(x), _ptr(b), n, (C.c_double * n)(*ms), int(bool(dagger)),
                                 C.byref(params), _ptr(ws), ws.numel(), stats, _stream(stream))
        if check and st != WD_OK:
            _check(st, "wd_stag_solve")
        return x, [s.as_dict() for s in stats]

    def time_hop(self, prec="f64", nrhs=1, n=50, mode=0, stream=None):
        """Mean duration (ms) of n back-to-back stencil launches; mode 0 plain,
        1 with the aux - c H epilogue and reduction, 2 the fused CG residual update;
        mode 4 the four stencil launches of one CG iteration in order (ms per four)."""
        nb = int(lib().wd_apply_workspace_bytes(self.handle, PREC[prec], nrhs))
        dev = next(iter(self.stores.values())).device
        ws = self._workspace(nb, dev, ("apply", PREC[prec], nrhs))
        ms = C.c_double()
        _check(lib().wd_time_hop(self.handle, PREC[prec], nrhs, int(mode), n, _ptr(ws), ws.numel(), C.byref(ms),
                                 _stream(stream)), "wd_time_hop")
        return ms.value

    def autotune(self, prec="f64", nrhs=1, stream=None):
        nb = int(lib().wd_apply_workspace_bytes(self.handle, PREC[prec], nrhs))
        dev = next(iter(self.stores.values())).device
        ws = self._workspace(nb, dev, ("apply", PREC[prec], nrhs))
        sb, sw, sp = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().wd_autotune(self.handle, PREC[prec], nrhs, _ptr(ws), ws.numel(), C.byref(sb), C.byref(sw),
                                 C.byref(sp), _stream(stream)), "wd_autotune")
        return sb.value, sw.value, sp.value


def time_read(nbytes, n=20, device="cuda", stream=None):
    """Mean duration (ms) of a plain streaming read of a device buffer of nbytes."""
    torch = _torch()
    buf = torch.zeros(nbytes, dtype=torch.uint8, device=device)
    out = torch.empty(2048, dtype=torch.float64, device=device)
    ms = C.c_double()
    _check(lib().wd_time_read(_ptr(buf), nbytes, n, _ptr(out), out.numel() * 8, C.byref(ms), _stream(stream)),
           "wd_time_read")
    return ms.value


def tune_import(text: str):
    """Load tuning lines "Lx Ly Lz Lt prec recon nrhs sblk swz split"."""
    _check(lib().wd_tune_import(text.encode()), "wd_tune_import")


def tune_export() -> str:
    n = lib().wd_tune_export(None, 0)
    buf = C.create_string_buffer(n)
    lib().wd_tune_export(buf, n)
    return buf.value.decode()


def solve_batch(requests, params=None, stream=None, check=True):
    """requests: list of (Lattice, b, kappa_list).  Returns list of (x, stats)."""
    torch = _torch()
    params = params or default_params()
    n = len(requests)
    reqs = (SolveRequest * n)()
    keep = []
    total = 0
    for i, (lat, b, kap) in enumerate(requests):
        nrhs = None if b.dim() == 6 else b.shape[0]
        _check_field(b, lat._field_shape(nrhs), "b")
        m = 1 if nrhs is None else nrhs
        kap = [float(kap)] * m if not hasattr(kap, "__len__") else [float(k) for k in kap]
        x = torch.empty_like(b)
        ka = (C.c_double * m)(*kap)
        keep.append((x, ka, m))
        reqs[i].lat = lat.handle
        reqs[i].x = x.data_ptr()
        reqs[i].b = b.data_ptr()
        reqs[i].nrhs = m
        reqs[i].kappa = C.cast(ka, C.POINTER(C.c_double))
        total += m
    nb = int(lib().wd_batch_workspace_bytes(n, reqs, C.byref(params)))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=requests[0][1].device)
    stats = (SolveStats * total)()
    st = lib().wd_solve_batch(n, reqs, C.byref(params), _ptr(ws), nb, stats, _stream(stream))
    if check and st != WD_OK:
        _check(st, "wd_solve_batch")
    out, k = [], 0
    for x, _, m in keep:
        out.append((x, [stats[k + j].as_dict() for j in range(m)]))
        k += m
    return out


class Server:
    """Continuous-batching solve server over a device pool of pool_bytes."""

    def __init__(self, pool_bytes, max_slots=16, params=None, device="cuda", stream=None):
        torch = _torch()
        self.params = params or default_params()
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        self.stream = stream or torch.cuda.Stream(device=device)
        h = C.c_void_p()
        _check(lib().wd_server_create(C.byref(h), _ptr(self.pool), self.pool.numel(), int(max_slots),
                                      C.byref(self.params), C.c_void_p(self.stream.cuda_stream)),
               "wd_server_create")
        self.handle = h
        self._live = {}

    def footprint(self, lat, nrhs=1):
        return int(lib().wd_server_footprint(self.handle, lat.handle, nrhs))

    def submit(self, lat, b, kappa, out=None):
        torch = _torch()
        nrhs = None if b.dim() == 6 else b.shape[0]
        _check_field(b, lat._field_shape(nrhs), "b")
        m = 1 if nrhs is None else nrhs
        kap = [float(kappa)] * m if not hasattr(kappa, "__len__") else [float(k) for k in kappa]
        x = torch.empty_like(b) if out is None else out
        # the server's stream must see b (and x) fully written before use
        self.stream.wait_stream(torch.cuda.current_stream())
        t = C.c_uint64()
        ka = (C.c_double * m)(*kap)
        _check(lib().wd_server_submit(self.handle, lat.handle, _ptr(x), _ptr(b), m, ka, C.byref(t)),
               "wd_server_submit")
        self._live[t.value] = (x, b, m)
        return t.value

    def poll(self, ticket):
        x, b, m = self._live[ticket]
        stats = (SolveStats * m)()
        r = lib().wd_server_poll(self.handle, C.c_uint64(ticket), stats)
        if r < 0:
            _check(r, "wd_server_poll")
        if r == 1:
            del self._live[ticket]
            return x, [s.as_dict() for s in stats]
        return None

    def wait(self, ticket, timeout_ms=-1):
        x, b, m = self._live[ticket]
        stats = (SolveStats * m)()
        r = lib().wd_server_wait(self.handle, C.c_uint64(ticket), stats, int(timeout_ms))
        if r < 0:
            _check(r, "wd_server_wait")
        if r == 1:
            del self._live[ticket]
            return x, [s.as_dict() for s in stats]
        return None

    def close(self):
        if self.handle:
            lib().wd_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
