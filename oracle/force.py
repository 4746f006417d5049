"""Plain FP64 CPU oracle for the Wilson pseudofermion action and its force.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests use it.  It shares no code with the HIP
library.

The paper's fermion action (App. C, "Definition of fermion actions" and its
HMC listing) is used through three calls: ``sample_pseudofermions!`` draws
eta = D^dag xi from a Gaussian xi, ``evaluate_FermiAction`` returns
S_f = eta^dag (D^dag D)^{-1} eta, and ``calc_UdSfdU`` returns "U dS_f/dU" per
direction, whose traceless antihermitian part updates the momenta
(``Traceless_antihermitian_add!``).  The paper prints none of the formulas;
the ones below are derived from the definition of D in ``wilson.py``:

* with X = (D^dag D)^{-1} eta and Y = D X, a change dU of the links changes
  the action by dS_f = -X^dag d(D^dag D) X = -2 Re[Y^dag dD X], and
  dD = -kappa dH;
* collecting the two hops that use the link U_mu(x) (the forward hop out of
  x and the backward hop out of x+mu), for dU_mu(x) = eps T U_mu(x) with T
  traceless antihermitian, dS_f = eps Re tr[T F_mu(x)] with

      F_mu(x) = 2 kappa s_mu(x) U_mu(x) [ M_mu(x) + N_mu(x)^dag ],
      M_mu(x) = sum_s ((1 - g_mu) X(x+mu))_s  Y(x)_s^dag,
      N_mu(x) = sum_s ((1 + g_mu) X(x))_s  Y(x+mu)_s^dag,

  colour outer products summed over the four spins, s_mu(x) the boundary
  sign of the link.  F is the "U dS_f/dU" of the paper's call.
* TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6, so Re tr[T M] = Re tr[T TA(M)]
  for every traceless antihermitian T.

Fields use the boundary layout of ``qcdgen``; forces and momenta are
``[4, Lt, Lz, Ly, Lx, 3, 3]`` like the links.
"""

from __future__ import annotations

import numpy as np

from .wilson import GAMMA, ONE4, apply_D, apply_Ddag, apply_DdagD, cg, eta_forward, lattice_extents, \
    shift_forward, vdot


def pseudofermion_heatbath(U, xi, kappa, bc):
    """eta = D^dag xi (the paper's sample_pseudofermions! from Gaussian xi)."""
    return apply_Ddag(U, xi, kappa, bc)


def fermion_action(U, eta, kappa, bc, tol: float = 1e-12):
    """S_f = eta^dag (D^dag D)^{-1} eta, from CG on D^dag D."""
    X, info = cg(lambda v: apply_DdagD(U, v, kappa, bc), eta, tol=tol)
    return float(vdot(eta, X).real), info


def _spin(P, psi):
    return np.einsum("st,...ta->...sa", P, psi)


def fermion_force(U, eta, kappa, bc, tol: float = 1e-12):
    """F_mu(x) = U dS_f/dU for S_f = eta^dag (D^dag D)^{-1} eta (formula above).

    Returns (F, S_f, CG info)."""
    X, info = cg(lambda v: apply_DdagD(U, v, kappa, bc), eta, tol=tol)
    Y = apply_D(U, X, kappa, bc)
    return force_from_solutions(U, X, Y, kappa, bc), float(vdot(eta, X).real), info


def force_from_solutions(U, X, Y, kappa, bc):
    """The force formula above for given X and Y = D X."""
    L = lattice_extents(X.shape)
    F = np.empty_like(U)
    for mu in range(4):
        Xf = shift_forward(X, mu)
        Yf = shift_forward(Y, mu)
        PmXf = _spin(ONE4 - GAMMA[mu], Xf)
        PpX = _spin(ONE4 + GAMMA[mu], X)
        M = np.einsum("...sb,...sa->...ba", PmXf, np.conj(Y))
        N = np.einsum("...sb,...sa->...ba", PpX, np.conj(Yf))
        sgn = eta_forward(L, bc, mu)[..., None, None]
        F[mu] = 2.0 * kappa * sgn * (U[mu] @ (M + np.conj(np.swapaxes(N, -1, -2))))
    return F


def traceless_antihermitian(M):
    """TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6 * 1, on the last two axes."""
    A = 0.5 * (M - np.conj(np.swapaxes(M, -1, -2)))
    tr = np.trace(A, axis1=-2, axis2=-1)
    return A - (tr / 3.0)[..., None, None] * np.eye(3)


def momentum_update(p, factor, F):
    """p + factor * TA(F) (the paper's Traceless_antihermitian_add!)."""
    return p + factor * traceless_antihermitian(F)
