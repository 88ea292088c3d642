"""Pins for the oracle's physics loss with the high-frequency penalty (paper,
section 2.2, equation loss and its weight w(nu) = w0 + eta_hf |nu|).

* lambda = 0 is the mean-squared residual; eta = 0 (constant weight) gives
  by Parseval the closed form J = (1/N)||r||^2 + lambda w0^2 ||r||^2;
* a residual that is one DFT bin: the penalty is lambda N |a|^2 w(nu)^2 with
  nu computed by hand from the bin's signed indices, the Bloch shift and the
  grid steps (checks the bin-to-frequency map, axis order, Nyquist bin);
* gradients against central differences of J in random complex directions,
  for the field and for the absorber permittivity (J is quadratic in both,
  so the differences are exact up to rounding);
* at the exact solution (dense LU, tiny grid) J and both gradients vanish.
"""

import numpy as np
import pytest

from oracle import psfd_ref as R
from psfd_synth import random_field

from conftest import small_cfg


def _problem(pol=0, seed=0):
    cfg = small_cfg(pol=pol)
    rng = np.random.default_rng(seed)
    eps = 1.0 + rng.uniform(0.1, 0.5, (cfg["nz_abs"], cfg["ny"], cfg["nx"])) \
        + 1j * rng.uniform(0.0, 0.1, (cfg["nz_abs"], cfg["ny"], cfg["nx"]))
    return cfg, R.Problem(cfg, eps)


def test_special_cases():
    cfg, P = _problem()
    E = random_field(P.g.shape, np.random.default_rng(1))
    J, t1, t2 = R.pino_loss(P, E, 0.7, 3.0, 0.0)
    assert t2 == 0.0 and J == t1
    assert abs(t1 - R.residual_loss(P, E)) < 1e-14 * t1
    r = R.apply_A(P, E) - R.rhs(P)
    rr = float(np.vdot(r, r).real)
    n = P.g.nx * P.g.ny * P.g.nz
    J, t1, t2 = R.pino_loss(P, E, 0.7, 0.0, 0.25)
    assert abs(t2 - 0.25 * 0.49 * rr) < 1e-12 * t2
    assert abs(J - (rr / n + 0.25 * 0.49 * rr)) < 1e-12 * J


@pytest.mark.parametrize("bin_", [(0, 0, 0), (3, 1, 2), (-5, -2, 3), (-16, 3, -2)])
def test_single_bin_weight(bin_):
    cfg, P = _problem()
    g = P.g
    p, n, m = bin_          # z, y, x signed indices
    nz, ny, nx = g.nz, g.ny, g.nx
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    a = 0.3 - 0.2j
    field = a * np.exp(2j * np.pi * (p * z / nz + n * y / ny + m * x / nx))
    r = np.stack([field, 0 * field, 0 * field])
    # by hand: bin (p, n, m) carries physical frequencies kx0/2pi + m/(nx dx), ...
    nu_x = g.kx0 / (2 * np.pi) + ((m + nx // 2) % nx - nx // 2) / (nx * cfg["dx"])
    nu_y = g.ky0 / (2 * np.pi) + ((n + ny // 2) % ny - ny // 2) / (ny * cfg["dy"])
    nu_z = ((p + nz // 2) % nz - nz // 2) / (nz * cfg["dz"])
    w = 0.4 + 2.5 * np.sqrt(nu_x ** 2 + nu_y ** 2 + nu_z ** 2)
    N = nx * ny * nz
    want = 0.3 * N * abs(a) ** 2 * w ** 2
    got = R.hf_penalty(P, r, 0.4, 2.5, 0.3)
    assert abs(got - want) < 1e-11 * want


@pytest.mark.parametrize("pol", [0, 1])
def test_gradients_match_finite_differences(pol):
    cfg, P = _problem(pol, seed=pol)
    rng = np.random.default_rng(7 + pol)
    E = random_field(P.g.shape, rng)
    w0, eta, lam = 0.8, 4.0, 0.05
    gE, geps = R.pino_loss_grad(P, E, w0, eta, lam)
    # J is quadratic in E and in eps (the residual is affine in both), so central
    # differences are exact up to rounding for any step
    h = 0.1
    for _ in range(3):
        d = random_field(P.g.shape, rng)
        fd = (R.pino_loss(P, E + h * d, w0, eta, lam)[0]
              - R.pino_loss(P, E - h * d, w0, eta, lam)[0]) / (2 * h)
        an = float(np.vdot(gE, d).real)
        assert abs(fd - an) < 1e-8 * max(abs(an), 1e-3), (fd, an)
    eps0 = P.deps + cfg["eps_bg"]
    for _ in range(2):
        de = rng.standard_normal(eps0.shape) + 1j * rng.standard_normal(eps0.shape)
        Jp = R.pino_loss(R.Problem(cfg, eps0 + h * de), E, w0, eta, lam)[0]
        Jm = R.pino_loss(R.Problem(cfg, eps0 - h * de), E, w0, eta, lam)[0]
        fd = (Jp - Jm) / (2 * h)
        an = float(np.vdot(geps, de).real)
        assert abs(fd - an) < 1e-8 * max(abs(an), 1e-3), (fd, an)


def test_exact_solution_zeroes_loss_and_gradients():
    cfg = small_cfg(nx=4, ny=4, nz_abs=2, nz_pml=3, nz_gap=1)
    P = R.Problem(cfg, np.full((2, 4, 4), 1.3 + 0.05j))
    A = R.dense_by_columns(P)
    E = np.linalg.solve(A, R.rhs(P).ravel()).reshape(P.g.shape)
    J, _, _ = R.pino_loss(P, E, 1.0, 5.0, 0.1)
    gE, geps = R.pino_loss_grad(P, E, 1.0, 5.0, 0.1)
    scale = np.abs(R.rhs(P)).max()
    assert J < 1e-24 * scale ** 2
    assert np.abs(gE).max() < 1e-10 * scale and np.abs(geps).max() < 1e-10 * scale
