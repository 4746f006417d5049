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
the whole lattice (no even-odd algebra, which the GPU path uses).

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
