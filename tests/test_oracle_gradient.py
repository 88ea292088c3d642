"""Pins for the oracle's permittivity sensitivity (adjoint method).

Against central finite differences of exact (dense LU) solves on a tiny
grid: the gradient of the scattered intensity on the observation row and of
the mean squared residual, with respect to single absorber voxels (real and
imaginary parts), and of the residual loss with respect to the field.
"""

import numpy as np

from oracle import psfd_ref as R
from psfd_synth import base_config, eps_absorber_default, random_field, rect_layout


def _setup(seed=2):
    rng = np.random.default_rng(seed)
    cfg = base_config(4, 4, 4, 7.5, theta_deg=6.0, phi_deg=20.0, pol=1)
    a = rect_layout(4, 4, rng, wmin=1, wmax=2)
    eps = R.eps_from_fill(cfg, R.smooth_layout(cfg, a), eps_absorber_default())
    return cfg, eps


def _intensity(cfg, eps):
    P = R.Problem(cfg, eps)
    A = R.dense_by_columns(P)
    E = np.linalg.solve(A, R.rhs(P).ravel()).reshape(P.g.shape)
    return float(np.sum(np.abs(E[:, P.g.j_obs]) ** 2)), P, A, E


def test_intensity_gradient_matches_finite_differences():
    cfg, eps = _setup()
    J0, P, A, E = _intensity(cfg, eps)
    g = np.zeros_like(E)
    g[:, P.g.j_obs] = 2 * E[:, P.g.j_obs]         # dJ/dRe E + i dJ/dIm E
    mu = np.linalg.solve(A.conj().T, g.ravel()).reshape(E.shape)
    grad = R.eps_gradient(P, E, mu, P.g.k0 ** 2)
    h = 1e-6
    for v in [(0, 1, 2), (3, 0, 0), (2, 3, 1)]:
        fd = []
        for step in (h, 1j * h):
            ep, em = eps.copy(), eps.copy()
            ep[v] += step
            em[v] -= step
            fd.append((_intensity(cfg, ep)[0] - _intensity(cfg, em)[0]) / (2 * h))
        fd = complex(fd[0], fd[1])
        assert abs(grad[v] - fd) <= 1e-6 * abs(fd) + 1e-12, (v, grad[v], fd)


def test_residual_loss_gradients_match_finite_differences():
    cfg, eps = _setup(5)
    rng = np.random.default_rng(3)
    P = R.Problem(cfg, eps)
    E = 0.1 * random_field(P.g.shape, rng)
    N = P.g.nx * P.g.ny * P.g.nz
    r = R.rhs(P) - R.apply_A(P, E)
    grad_eps = R.eps_gradient(P, E, r, 2 * P.g.k0 ** 2 / N)
    grad_E = -(2.0 / N) * R.apply_AH(P, r)
    h = 1e-6
    v = (1, 2, 3)
    fd = []
    for step in (h, 1j * h):
        ep, em = eps.copy(), eps.copy()
        ep[v] += step
        em[v] -= step
        fd.append((R.residual_loss(R.Problem(cfg, ep), E) - R.residual_loss(R.Problem(cfg, em), E)) / (2 * h))
    fd = complex(fd[0], fd[1])
    assert abs(grad_eps[v] - fd) <= 1e-6 * abs(fd)
    w = (2, 5, 1, 3)
    fd = []
    for step in (h, 1j * h):
        Ep, Em = E.copy(), E.copy()
        Ep[w] += step
        Em[w] -= step
        fd.append((R.residual_loss(P, Ep) - R.residual_loss(P, Em)) / (2 * h))
    fd = complex(fd[0], fd[1])
    assert abs(grad_E[w] - fd) <= 1e-6 * abs(fd)
