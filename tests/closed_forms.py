"""Closed forms that pin the oracle and the GPU path (test helpers only).

Written from the definitions, sharing no arithmetic with the oracle's
position-space operator or with the HIP library.
"""

import numpy as np

import oracle as O


def free_point_propagator(L, kappa, bc):
    """Point propagator at U = 1 in closed form.

    For a plane wave e^{ipx} chi the free operator is the 4x4 matrix
    D(p) = (1 - 2 kappa sum_mu cos p_mu) + 2i kappa sum_mu gamma_mu sin p_mu,
    with p_mu = (2 pi n + pi [bc_mu = -1]) / L_mu.  The point source at the
    origin is (1/V) sum_p e^{ipx}, so S(x)_{alpha a, beta b} =
    delta_ab (1/V) sum_p e^{ipx} [D(p)^{-1}]_{alpha beta}: an inverse FFT of
    D(p)^{-1} times the twist e^{i pi x_mu / L_mu} of antiperiodic directions.
    Returned as [12, Lt, Lz, Ly, Lx, 4, 3] with source index 3*beta + b.
    """
    Lx, Ly, Lz, Lt = L
    shift = [0.5 if bc[mu] == -1 else 0.0 for mu in range(4)]
    n = np.indices((Lt, Lz, Ly, Lx))
    # momentum component mu lives on array axis 3 - mu
    p = [2 * np.pi * (n[3 - mu] + shift[mu]) / L[mu] for mu in range(4)]
    G = np.array([np.asarray(g) for g in O.GAMMA])
    D = (1 - 2 * kappa * sum(np.cos(p[mu]) for mu in range(4)))[..., None, None] * np.eye(4)
    D = D + 2j * kappa * sum(np.sin(p[mu])[..., None, None] * G[mu] for mu in range(4))
    M = np.linalg.inv(D)                                   # [Lt, Lz, Ly, Lx, 4, 4]
    Sx = np.fft.ifftn(M, axes=(0, 1, 2, 3))                # (1/V) sum_n e^{+2 pi i n.x / L}
    x = np.indices((Lt, Lz, Ly, Lx))
    twist = np.exp(1j * np.pi * sum(shift[mu] * 2 * x[3 - mu] / L[mu] for mu in range(4)))
    Sx = Sx * twist[..., None, None]
    S = np.zeros((12, Lt, Lz, Ly, Lx, 4, 3), dtype=np.complex128)
    for beta in range(4):
        for b in range(3):
            S[3 * beta + b, ..., :, b] = Sx[..., :, beta]
    return S


def free_staggered_point_propagator(L, mass, bc):
    """Staggered point propagator at U = 1 in closed form, [3, Lt, Lz, Ly, Lx, 3].

    At U = 1 the hopping part H obeys H^2 = -sum_mu sin^2 p_mu on every plane
    wave (the phases make different directions anticommute), and D = m + H
    with H anti-Hermitian, so D^-1 = (m - H) / (m^2 - H^2).  The scalar
    G(x) = (1/V) sum_p e^{ipx} / (m^2 + sum_mu sin^2 p_mu) is an inverse FFT
    (times the antiperiodic twist); (m - H) G is written out here with the
    phases eta_mu(x) = (-1)^(x_1 + .. + x_{mu-1}) taken from the coordinates
    and the boundary signs applied to the wrapped slices of np.roll.
    Colour is a spectator: column a carries G in colour a.
    """
    Lx, Ly, Lz, Lt = L
    shift = [0.5 if bc[mu] == -1 else 0.0 for mu in range(4)]
    n = np.indices((Lt, Lz, Ly, Lx))
    p = [2 * np.pi * (n[3 - mu] + shift[mu]) / L[mu] for mu in range(4)]
    lam = mass * mass + sum(np.sin(pm) ** 2 for pm in p)
    G = np.fft.ifftn(1.0 / lam, axes=(0, 1, 2, 3))
    G = G * np.exp(1j * np.pi * sum(shift[mu] * 2 * n[3 - mu] / L[mu] for mu in range(4)))
    HG = np.zeros_like(G)
    for mu in range(4):
        ax = 3 - mu
        eta = (-1.0) ** sum(n[3 - nu] for nu in range(mu))
        fwd = np.roll(G, -1, axis=ax)              # G(x + mu)
        bwd = np.roll(G, 1, axis=ax)               # G(x - mu)
        last = [slice(None)] * 4
        last[ax] = L[mu] - 1
        first = [slice(None)] * 4
        first[ax] = 0
        fwd[tuple(last)] *= bc[mu]
        bwd[tuple(first)] *= bc[mu]
        HG += 0.5 * eta * (fwd - bwd)
    Gm = mass * G - HG
    out = np.zeros((3, Lt, Lz, Ly, Lx, 3), dtype=np.complex128)
    for a in range(3):
        out[a, ..., a] = Gm
    return out
