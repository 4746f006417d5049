"""Seeded synthetic inputs for the Wilson-Dirac solver.

This module only *draws* inputs: SU(3) link fields, Gaussian and point-source
spinors, random gauge transformations.  It holds none of the operator's
arithmetic, so both the CPU oracle and the GPU library can be fed from it
without sharing any code of the method.

Array conventions (the library's boundary layout, colour index fastest as in
the paper's pseudo-fermion element ``x[ic,ix,iy,iz,it,ialpha]``, App. C
"Definition of pseudo-fermion fields"):

* lattice extents are given as ``L = (Lx, Ly, Lz, Lt)``;
* a spinor field is complex128 ``[Lt, Lz, Ly, Lx, 4, 3]`` (spin, colour);
  a batch of ``n`` spinors is ``[n, Lt, Lz, Ly, Lx, 4, 3]``;
* a link field is complex128 ``[4, Lt, Lz, Ly, Lx, 3, 3]`` with direction
  order x, y, z, t (the paper's ``U[mu]``, App. B "Hybrid Monte Carlo") and
  (row, column) colour indices.

Random streams: ``numpy.random.Generator(PCG64(seed))``.  Link and source
draws take separate generators so that changing one does not move the other.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "volume",
    "site_shape",
    "gaussian_spinor",
    "point_sources",
    "haar_su3",
    "exp_i_hermitian_su3",
    "random_hermitian_traceless",
    "links_unit",
    "links_haar",
    "links_exp",
    "random_gauge_transform",
    "CONFIG_SEED_BASE",
]

# Seeds are a base of 123 (the paper seeds its examples with Random.seed!(123),
# App. B "Hybrid Monte Carlo") plus a per-workload offset.
CONFIG_SEED_BASE = 123


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def volume(L) -> int:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return Lx * Ly * Lz * Lt


def site_shape(L) -> tuple:
    """Lattice axes in storage order: (Lt, Lz, Ly, Lx)."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return (Lt, Lz, Ly, Lx)


def _complex_gaussian(g: np.random.Generator, shape, var_per_part: float = 1.0):
    s = np.sqrt(var_per_part)
    return s * g.standard_normal(shape) + 1j * (s * g.standard_normal(shape))


def gaussian_spinor(L, g: np.random.Generator, n: int | None = None) -> np.ndarray:
    """Gaussian spinor(s): real and imaginary parts i.i.d. N(0, 1)."""
    shape = site_shape(L) + (4, 3)
    if n is not None:
        shape = (int(n),) + shape
    return _complex_gaussian(g, shape)


def point_sources(L, origin=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 point sources b^(alpha,a)(x) = delta_{x,origin} e_alpha (x) e_a.

    Returned as ``[12, Lt, Lz, Ly, Lx, 4, 3]`` with source index
    ``3*alpha + a`` (spin-major, colour fastest).
    """
    out = np.zeros((12,) + site_shape(L) + (4, 3), dtype=np.complex128)
    x, y, z, t = origin
    for alpha in range(4):
        for a in range(3):
            out[3 * alpha + a, t, z, y, x, alpha, a] = 1.0
    return out


def haar_su3(n: int, g: np.random.Generator) -> np.ndarray:
    """``n`` Haar-random SU(3) matrices.

    QR of a complex Ginibre matrix with the phases of R's diagonal moved into
    Q (Mezzadri's recipe for Haar measure on U(3)), then divided by a cube
    root of the determinant.  Multiplying a Haar U(3) element by a function of
    its determinant that lands in SU(3) leaves the SU(3) part Haar distributed
    because SU(3)'s centre acts freely on the choice of cube root.
    """
    z = _complex_gaussian(g, (n, 3, 3), 0.5)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    q = q * ph[:, None, :]
    det = np.linalg.det(q)
    phi = np.angle(det)
    q = q * np.exp(-1j * phi / 3.0)[:, None, None]
    return q


def random_hermitian_traceless(n: int, g: np.random.Generator) -> np.ndarray:
    """H = (G + G^dagger)/2 - tr/3, G entries complex Gaussian with N(0,1) parts.

    Every entry of (G + G^dagger)/2 then has E|H_ij|^2 = 1 (unit variance).
    """
    gm = _complex_gaussian(g, (n, 3, 3))
    h = 0.5 * (gm + np.conj(np.swapaxes(gm, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real
    h = h - (tr / 3.0)[:, None, None] * np.eye(3)[None]
    return h


def exp_i_hermitian_su3(n: int, width: float, g: np.random.Generator) -> np.ndarray:
    """U = exp(i * width * H), H random traceless Hermitian (see above).

    Computed through the eigen-decomposition H = V diag(w) V^dagger, so U is
    unitary to rounding and det U = exp(i*width*tr H) = 1 to rounding.
    """
    h = random_hermitian_traceless(n, g)
    w, v = np.linalg.eigh(h)
    e = np.exp(1j * width * w)
    return np.einsum("nij,nj,nkj->nik", v, e, np.conj(v))


def links_unit(L) -> np.ndarray:
    """Cold start: every link the identity (free field)."""
    out = np.zeros((4,) + site_shape(L) + (3, 3), dtype=np.complex128)
    out[..., 0, 0] = 1.0
    out[..., 1, 1] = 1.0
    out[..., 2, 2] = 1.0
    return out


def links_haar(L, g: np.random.Generator) -> np.ndarray:
    n = 4 * volume(L)
    return haar_su3(n, g).reshape((4,) + site_shape(L) + (3, 3))


def links_exp(L, width: float, g: np.random.Generator, chunk: int = 1 << 20) -> np.ndarray:
    """Links exp(i*width*H) drawn site by site (chunked to bound memory)."""
    n = 4 * volume(L)
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        out[s:e] = exp_i_hermitian_su3(e - s, width, g)
    return out.reshape((4,) + site_shape(L) + (3, 3))


def random_gauge_transform(L, g: np.random.Generator) -> np.ndarray:
    """Omega(x): one Haar SU(3) matrix per site, ``[Lt, Lz, Ly, Lx, 3, 3]``."""
    return haar_su3(volume(L), g).reshape(site_shape(L) + (3, 3))
