"""Plain FP64 CPU oracle for solving D x = b and for the Wilson pion correlator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library.

What it computes:

* ``solve_D``: the solution of D x = b, or of D^dag x = b, the paper's
  ``solve_DinvX!(y, D, x)`` and ``solve_DinvX!(y, D', x)`` (App. C, the
  LatticeDiracOperators.jl listings).  The solution of a linear system has a
  plain definition, x = D^{-1} b; the oracle reaches it by CG on the normal
  equations of the full lattice, D^dag D x = D^dag b (or D D^dag x = D b for
  the adjoint), with the literal adjoint of ``wilson.py``.  It does not use
  the even-odd decomposition, so it pins the GPU's Schur-complement path
  without sharing its algebra.
* ``point_propagator``: the 12 solutions of D x = b for the point sources
  b = delta_{x, origin} e_alpha (x) e_a, i.e. the columns S(x, origin) of the
  quark propagator.
* ``pion_correlator``: the zero-momentum pion two-point function of Wilson
  quarks (the paper lists the momentum-projected Wilson pion correlator among
  its measurements in Sec. 2 and in App. D, QCDMeasurements.jl, and checks it
  against published results in App. E).  With gamma5-hermiticity,
  S(origin, x) = gamma5 S(x, origin)^dag gamma5, the pion contraction
  tr[gamma5 S(x,0) gamma5 gamma5 S(0,x) gamma5] becomes tr[S(x,0) S(x,0)^dag],
  so C(t) = sum over spatial x and all spin and colour indices of
  |S(x, t)_{alpha a, beta b}|^2, with t counted from the source time slice.
  This normalisation (no minus sign, no volume factor) is a reading: the paper
  prints neither.

Fields use the boundary layout of ``qcdgen``: spinors ``[Lt, Lz, Ly, Lx, 4, 3]``,
propagators ``[12, Lt, Lz, Ly, Lx, 4, 3]`` with source index 3*alpha + a.
"""

from __future__ import annotations

import numpy as np

from .wilson import apply_D, apply_Ddag, apply_DdagD, cg, norm


def solve_D(U, b, kappa, bc, dagger: bool = False, tol: float = 1e-12, maxiter: int = 100000):
    """x with D x = b (dagger False) or D^dag x = b (dagger True).

    CG on D^dag D x = D^dag b, or on D D^dag x = D b for the adjoint system.
    Returns (x, info) with the CG info of the normal equations.
    """
    if not dagger:
        rhs = apply_Ddag(U, b, kappa, bc)
        return cg(lambda v: apply_DdagD(U, v, kappa, bc), rhs, tol=tol, maxiter=maxiter)
    rhs = apply_D(U, b, kappa, bc)
    return cg(lambda v: apply_D(U, apply_Ddag(U, v, kappa, bc), kappa, bc), rhs, tol=tol, maxiter=maxiter)


def residual_D(U, x, b, kappa, bc, dagger: bool = False) -> float:
    """||b - D x|| / ||b|| (or with D^dag), in FP64."""
    op = apply_Ddag if dagger else apply_D
    return norm(b - op(U, x, kappa, bc)) / norm(b)


def point_propagator(U, kappa, bc, sources, tol: float = 1e-12):
    """S[k] = D^{-1} sources[k] for each of the given sources (usually the 12
    point sources); returns (S, list of CG infos)."""
    out = np.empty_like(sources)
    infos = []
    for k in range(sources.shape[0]):
        out[k], info = solve_D(U, sources[k], kappa, bc, tol=tol)
        infos.append(info)
    return out, infos


def pion_correlator(S, t0: int = 0) -> np.ndarray:
    """C(t) = sum over spatial sites of time slice (t0 + t) mod Lt, over the
    sources and over spin and colour, of |S|^2; t = 0 .. Lt-1."""
    Lt = S.shape[1]
    per_slice = np.sum(np.abs(S) ** 2, axis=(0, 2, 3, 4, 5, 6))
    return np.array([per_slice[(t0 + t) % Lt] for t in range(Lt)])
