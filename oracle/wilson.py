"""Plain FP64 CPU oracle for the Wilson-Dirac operator and CG on D^dagger D.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; the two meet
only in the seeded input generators (``qcdgen``), which hold none of the
operator's arithmetic.

What it computes follows the paper's statement of the problem (App. C,
"Definition of Dirac operators"): a Wilson Dirac operator ``D`` parametrised
by the hopping parameter kappa, its adjoint ``D'``, the normal operator
``D'D`` (``DdagD_operator``) and an iterative solve of ``D'D x = b``
(``solve_DinvX!`` with tolerance ``eps_CG``).  The paper does not print the
operator's formula (it cites Wilson's lattice formulation, Sec. 1), so the
definitions below are the textbook ones, with the conventions it leaves open
fixed as follows:

* hopping-parameter form with Wilson parameter r = 1::

      (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) eta+_mu(x) psi(x+mu)
                                          + (1 + gamma_mu) U_mu(x-mu)^dag eta-_mu(x) psi(x-mu) ]

* Euclidean chiral gamma basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
  (k = 1, 2, 3), gamma_4 = [[0, 1], [1, 0]], gamma_5 = gamma_1 gamma_2
  gamma_3 gamma_4 = diag(1, 1, -1, -1);
* per-direction boundary signs ``bc[mu]`` in {+1, -1}: a hop that crosses
  the boundary of direction mu picks up bc[mu] (antiperiodic time is
  ``bc = (1, 1, 1, -1)``);
* even-odd: parity of x is (x1+x2+x3+x4) mod 2; the Schur complement on the
  even sites is D_hat = 1 - kappa^2 H_eo H_oe where D = 1 - kappa H;
* the solve is CG (Hestenes and Stiefel) on A = D^dag D (full lattice) or
  A_hat = D_hat^dag D_hat (even sites), from x0 = 0, stopped when the true
  residual ||b - A x|| / ||b|| is at most ``tol``.

Fields use the boundary layout of ``qcdgen``: spinors ``[Lt, Lz, Ly, Lx, 4, 3]``,
links ``[4, Lt, Lz, Ly, Lx, 3, 3]``.  Every array here is complex128.
Nothing is blocked, fused or reordered: each function is its definition.
"""

from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# gamma matrices (chiral basis, written from the definition above)
# ---------------------------------------------------------------------------
_SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)

GAMMA = tuple(
    [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in _SIGMA]
    + [np.block([[_Z2, _I2], [_I2, _Z2]])]
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=np.complex128)

# numpy axis of direction mu inside a site array [Lt, Lz, Ly, Lx, ...]
_AXIS = (3, 2, 1, 0)


def lattice_extents(field_sites_shape) -> tuple:
    """(Lx, Ly, Lz, Lt) from a site shape (Lt, Lz, Ly, Lx)."""
    Lt, Lz, Ly, Lx = field_sites_shape[:4]
    return (Lx, Ly, Lz, Lt)


def shift_forward(f: np.ndarray, mu: int) -> np.ndarray:
    """g(x) = f(x + mu_hat), periodic in the index."""
    return np.roll(f, -1, axis=_AXIS[mu])


def shift_backward(f: np.ndarray, mu: int) -> np.ndarray:
    """g(x) = f(x - mu_hat), periodic in the index."""
    return np.roll(f, +1, axis=_AXIS[mu])


def coordinate(L, mu: int) -> np.ndarray:
    """x_mu at every site, shape (Lt, Lz, Ly, Lx)."""
    Lx, Ly, Lz, Lt = L
    shape = (Lt, Lz, Ly, Lx)
    idx = np.indices(shape)
    return idx[_AXIS[mu]]


def eta_forward(L, bc, mu: int) -> np.ndarray:
    """Sign of the hop x -> x+mu: bc[mu] where x_mu = L_mu - 1, else 1."""
    c = coordinate(L, mu)
    return np.where(c == L[mu] - 1, float(bc[mu]), 1.0)


def eta_backward(L, bc, mu: int) -> np.ndarray:
    """Sign of the hop x -> x-mu: bc[mu] where x_mu = 0, else 1."""
    c = coordinate(L, mu)
    return np.where(c == 0, float(bc[mu]), 1.0)


def parity(L) -> np.ndarray:
    """(x+y+z+t) mod 2 at every site."""
    return sum(coordinate(L, mu) for mu in range(4)) % 2


def even_mask(L) -> np.ndarray:
    return (parity(L) == 0)[..., None, None]


def odd_mask(L) -> np.ndarray:
    return (parity(L) == 1)[..., None, None]


def _spin(P: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(P psi)(x)_{s a} = sum_t P_{st} psi(x)_{t a}."""
    return np.einsum("st,...ta->...sa", P, psi)


def _colour(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)(x)_{s a} = sum_b U(x)_{ab} psi(x)_{s b}."""
    return np.einsum("...ab,...sb->...sa", U, psi)


def _dagger(U: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(U, -1, -2))


def gamma5(psi: np.ndarray) -> np.ndarray:
    return _spin(GAMMA5, psi)


# ---------------------------------------------------------------------------
# the operator
# ---------------------------------------------------------------------------
def hopping(U: np.ndarray, psi: np.ndarray, bc) -> np.ndarray:
    """H psi with D = 1 - kappa H (hopping term of the definition above)."""
    L = lattice_extents(psi.shape)
    out = np.zeros_like(psi)
    for mu in range(4):
        fwd = shift_forward(psi, mu) * eta_forward(L, bc, mu)[..., None, None]
        out += _spin(ONE4 - GAMMA[mu], _colour(U[mu], fwd))
        Ub = shift_backward(U[mu], mu)
        bwd = shift_backward(psi, mu) * eta_backward(L, bc, mu)[..., None, None]
        out += _spin(ONE4 + GAMMA[mu], _colour(_dagger(Ub), bwd))
    return out


def hopping_adjoint(U: np.ndarray, psi: np.ndarray, bc) -> np.ndarray:
    """H^dag psi, the conjugate transpose of ``hopping`` written out.

    The forward matrix element of H from x to x+mu is (1-gamma_mu) U_mu(x)
    eta+(x); its transpose-conjugate is a backward element at x+mu with
    projector (1-gamma_mu) (gamma_mu is Hermitian) and link U_mu(x)^dag.  Likewise
    the backward element turns into a forward one with (1+gamma_mu).  The
    boundary sign is real and shared by both ends of a link.
    """
    L = lattice_extents(psi.shape)
    out = np.zeros_like(psi)
    for mu in range(4):
        fwd = shift_forward(psi, mu) * eta_forward(L, bc, mu)[..., None, None]
        out += _spin(ONE4 + GAMMA[mu], _colour(U[mu], fwd))
        Ub = shift_backward(U[mu], mu)
        bwd = shift_backward(psi, mu) * eta_backward(L, bc, mu)[..., None, None]
        out += _spin(ONE4 - GAMMA[mu], _colour(_dagger(Ub), bwd))
    return out


def apply_D(U, psi, kappa, bc):
    """y = D psi on the full lattice."""
    return psi - kappa * hopping(U, psi, bc)


def apply_Ddag(U, psi, kappa, bc):
    """y = D^dag psi (literal adjoint, not the gamma5 sandwich)."""
    return psi - kappa * hopping_adjoint(U, psi, bc)


def apply_DdagD(U, psi, kappa, bc):
    return apply_Ddag(U, apply_D(U, psi, kappa, bc), kappa, bc)


def apply_Dhat(U, psi, kappa, bc):
    """Even-odd Schur complement D_hat = 1 - kappa^2 H_eo H_oe on the even sites.

    ``psi`` is a full-lattice array whose odd sites are ignored; the result is
    zero on the odd sites.
    """
    L = lattice_extents(psi.shape)
    e, o = even_mask(L), odd_mask(L)
    pe = psi * e
    t = hopping(U, pe, bc) * o          # H_oe psi_e
    return (pe - kappa * kappa * hopping(U, t, bc)) * e


def apply_Dhat_dag(U, psi, kappa, bc):
    """D_hat^dag = 1 - kappa^2 (H_oe)^dag (H_eo)^dag, from the literal H^dag."""
    L = lattice_extents(psi.shape)
    e, o = even_mask(L), odd_mask(L)
    pe = psi * e
    t = hopping_adjoint(U, pe, bc) * o
    return (pe - kappa * kappa * hopping_adjoint(U, t, bc)) * e


def apply_Ahat(U, psi, kappa, bc):
    """A_hat = D_hat^dag D_hat (even sites)."""
    return apply_Dhat_dag(U, apply_Dhat(U, psi, kappa, bc), kappa, bc)


def apply_D_sites(U, psi, kappa, bc, sites):
    """(D psi)(x) at the listed sites only, one site at a time.

    ``sites`` is a sequence of (x, y, z, t).  Written with explicit neighbour
    coordinates so that single outputs of a large lattice can be checked
    without applying the whole operator.  Returns ``[len(sites), 4, 3]``.
    """
    L = lattice_extents(psi.shape)
    res = []
    for s in sites:
        x = [int(v) for v in s]
        acc = np.zeros((4, 3), dtype=np.complex128)
        for mu in range(4):
            xp = list(x)
            xp[mu] = (x[mu] + 1) % L[mu]
            sgn_p = float(bc[mu]) if x[mu] == L[mu] - 1 else 1.0
            xm = list(x)
            xm[mu] = (x[mu] - 1) % L[mu]
            sgn_m = float(bc[mu]) if x[mu] == 0 else 1.0
            u_here = U[mu, x[3], x[2], x[1], x[0]]
            u_back = U[mu, xm[3], xm[2], xm[1], xm[0]]
            p_fwd = psi[xp[3], xp[2], xp[1], xp[0]]
            p_bwd = psi[xm[3], xm[2], xm[1], xm[0]]
            acc += sgn_p * (ONE4 - GAMMA[mu]) @ (p_fwd @ u_here.T)
            acc += sgn_m * (ONE4 + GAMMA[mu]) @ (p_bwd @ np.conj(u_back))
        res.append(psi[x[3], x[2], x[1], x[0]] - kappa * acc)
    return np.array(res)


# ---------------------------------------------------------------------------
# inner products and CG
# ---------------------------------------------------------------------------
def vdot(a, b) -> complex:
    """<a, b> = sum conj(a) b over every site and component."""
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm(a) -> float:
    return float(np.sqrt(np.vdot(a.ravel(), a.ravel()).real))


def true_residual(apply_A, x, b) -> float:
    """||b - A x|| / ||b|| in FP64."""
    return norm(b - apply_A(x)) / norm(b)


def cg(apply_A, b, tol=1e-10, maxiter=100000, x0=None):
    """Conjugate gradient on a Hermitian positive-definite A (Hestenes-Stiefel).

    When the iterated residual reaches ``tol * ||b||`` the true residual
    b - A x is recomputed; if it is still above, CG restarts from it.  Also
    returns the CG coefficients, which define the Lanczos tridiagonal of A
    (used to bound the solution error from the residual).

    Returns (x, info) with info = dict(iters, true_resid, converged, alphas,
    betas, restarts).
    """
    bn = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    if bn == 0.0:
        return x, dict(iters=0, true_resid=0.0, converged=True, alphas=[], betas=[], restarts=0)
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = r.copy()
    rho = vdot(r, r).real
    alphas, betas = [], []
    it = 0
    restarts = 0
    converged = False
    while it < maxiter:
        q = apply_A(p)
        alpha = rho / vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rho_new = vdot(r, r).real
        it += 1
        alphas.append(alpha)
        if np.sqrt(rho_new) <= tol * bn:
            r_true = b - apply_A(x)
            if norm(r_true) <= tol * bn:
                converged = True
                break
            r = r_true
            p = r.copy()
            rho = vdot(r, r).real
            restarts += 1
            continue
        beta = rho_new / rho
        betas.append(beta)
        p = r + beta * p
        rho = rho_new
    tr = true_residual(apply_A, x, b)
    return x, dict(iters=it, true_resid=tr, converged=converged and tr <= tol,
                   alphas=alphas, betas=betas, restarts=restarts)


def lanczos_extremes(alphas, betas):
    """Extreme Ritz values of A from the CG coefficients.

    The Lanczos tridiagonal built from CG has diagonal 1/alpha_k +
    beta_{k-1}/alpha_{k-1} and off-diagonal sqrt(beta_k)/alpha_k.
    """
    m = len(alphas)
    if m == 0:
        return (np.nan, np.nan)
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 and k - 1 < len(betas) else 0.0)
        if k + 1 < m and k < len(betas):
            T[k, k + 1] = T[k + 1, k] = np.sqrt(betas[k]) / alphas[k]
    w = np.linalg.eigvalsh(T)
    return (float(w[0]), float(w[-1]))


def solve_DdagD(U, b, kappa, bc, eo: bool, tol=1e-10, maxiter=100000):
    """x = (D^dag D)^{-1} b (full) or x_e = A_hat^{-1} b_e (even-odd)."""
    if eo:
        L = lattice_extents(b.shape)
        be = b * even_mask(L)
        return cg(lambda v: apply_Ahat(U, v, kappa, bc), be, tol=tol, maxiter=maxiter)
    return cg(lambda v: apply_DdagD(U, v, kappa, bc), b, tol=tol, maxiter=maxiter)


def residual_DdagD(U, x, b, kappa, bc, eo: bool) -> float:
    """True relative residual of a returned solution, in FP64."""
    if eo:
        L = lattice_extents(b.shape)
        e = even_mask(L)
        return true_residual(lambda v: apply_Ahat(U, v, kappa, bc), x * e, b * e)
    return true_residual(lambda v: apply_DdagD(U, v, kappa, bc), x, b)
