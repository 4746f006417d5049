"""Plain FP64 CPU oracle for the staggered Dirac operator and its solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests use it.  It shares no code with the HIP
library.

The paper's second fermion discretisation (App. C, "Definition of Dirac
operators": the staggered operator with a mass parameter, applied with
``mul!`` and inverted with ``solve_DinvX!``) is not printed either.  The
oracle takes the textbook Kogut-Susskind form, one colour vector per site:

    (D chi)(x) = m chi(x) + 1/2 sum_mu eta_mu(x) [ s+ U_mu(x) chi(x+mu)
                                                 - s- U_mu(x-mu)^dag chi(x-mu) ]

with the staggered phases eta_1 = 1, eta_2 = (-1)^x1, eta_3 = (-1)^(x1+x2),
eta_4 = (-1)^(x1+x2+x3) (x1..x4 = x, y, z, t) and the boundary signs s+/s- of
``wilson.py`` (a hop across the boundary of direction mu picks up bc[mu]).
The hopping part is anti-Hermitian, so D^dag = m - (hopping part).

The solve of D x = b is CG on the normal equations D^dag D x = D^dag b over
the whole lattice (no even-odd algebra, which the GPU path uses).  The pion
correlator of staggered quarks (listed with the Wilson one among the paper's
measurements, Sec. 2 and App. D) is the Goldstone channel from the 3 colour
point sources.

Fields use the boundary layout ``[Lt, Lz, Ly, Lx, 3]`` (complex128); links
``[4, Lt, Lz, Ly, Lx, 3, 3]``.
"""

from __future__ import annotations

import numpy as np

from .wilson import cg, coordinate, eta_backward, eta_forward, norm, shift_backward, shift_forward


def staggered_phase(L, mu: int) -> np.ndarray:
    """eta_mu(x) = (-1)^(x_1 + ... + x_{mu-1}) at every site, shape (Lt, Lz, Ly, Lx)."""
    s = np.zeros(tuple(reversed(L)), dtype=np.int64)
    for nu in range(mu):
        s = s + coordinate(L, nu)
    return np.where(s % 2 == 0, 1.0, -1.0)


def _lattice(chi):
    Lt, Lz, Ly, Lx = chi.shape[:4]
    return (Lx, Ly, Lz, Lt)


def hopping_staggered(U, chi, bc):
    """1/2 sum_mu eta_mu(x) [s+ U_mu(x) chi(x+mu) - s- U_mu(x-mu)^dag chi(x-mu)]."""
    L = _lattice(chi)
    out = np.zeros_like(chi)
    for mu in range(4):
        eta = staggered_phase(L, mu)[..., None]
        fwd = np.einsum("...ab,...b->...a", U[mu], shift_forward(chi, mu))
        Ub = shift_backward(U[mu], mu)
        bwd = np.einsum("...ba,...b->...a", np.conj(Ub), shift_backward(chi, mu))
        sp = eta_forward(L, bc, mu)[..., None]
        sm = eta_backward(L, bc, mu)[..., None]
        out += 0.5 * eta * (sp * fwd - sm * bwd)
    return out


def apply_staggered(U, chi, mass, bc):
    """y = D chi = m chi + hopping."""
    return mass * chi + hopping_staggered(U, chi, bc)


def apply_staggered_dag(U, chi, mass, bc):
    """y = D^dag chi = m chi - hopping (the hopping part is anti-Hermitian)."""
    return mass * chi - hopping_staggered(U, chi, bc)


def solve_staggered(U, b, mass, bc, tol: float = 1e-12, maxiter: int = 100000):
    """x with D x = b, from CG on D^dag D x = D^dag b over the whole lattice."""
    rhs = apply_staggered_dag(U, b, mass, bc)
    return cg(lambda v: apply_staggered_dag(U, apply_staggered(U, v, mass, bc), mass, bc), rhs, tol=tol,
              maxiter=maxiter)


def residual_staggered(U, x, b, mass, bc) -> float:
    """||b - D x|| / ||b|| in FP64."""
    return norm(b - apply_staggered(U, x, mass, bc)) / norm(b)


def point_sources_staggered(L, origin=(0, 0, 0, 0)):
    """The 3 colour point sources delta_{x,origin} e_a, ``[3, Lt, Lz, Ly, Lx, 3]``."""
    Lx, Ly, Lz, Lt = L
    out = np.zeros((3, Lt, Lz, Ly, Lx, 3), dtype=np.complex128)
    x, y, z, t = origin
    for a in range(3):
        out[a, t, z, y, x, a] = 1.0
    return out


def staggered_point_propagator(U, mass, bc, sources, tol: float = 1e-12):
    """G[k] = D^{-1} sources[k] (the columns G(x, origin) of the staggered propagator)."""
    out = np.empty_like(sources)
    infos = []
    for k in range(sources.shape[0]):
        out[k], info = solve_staggered(U, sources[k], mass, bc, tol=tol)
        infos.append(info)
    return out, infos


def staggered_pion_correlator(G, t0: int = 0) -> np.ndarray:
    """Goldstone pion correlator: C(t) = sum over the spatial sites of time slice
    (t0 + t) mod Lt, over the source and sink colours, of |G|^2.  The staggered
    analogue of gamma5-hermiticity, G(0, x) = eps(0) eps(x) G(x, 0)^dag with
    eps(x) = (-1)^(x+y+z+t), turns the pion contraction into this sum of squared
    moduli."""
    Lt = G.shape[1]
    per_slice = np.sum(np.abs(G) ** 2, axis=(0, 2, 3, 4, 5))
    return np.array([per_slice[(t0 + t) % Lt] for t in range(Lt)])
