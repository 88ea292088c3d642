"""Physics pins of the oracle's whole chain (operator + source + R_ml + PML).

* a laterally uniform absorber slab: the 3-D solve equals a 1-D dense solve
  of the (0, 0) mode, and the reflected field converges, monotonically under
  axial refinement, to the transfer-matrix reflection of
  [vacuum | slab | multilayer | substrate];
* eps = eps_bg gives a zero source and a zero scattered field;
* lossless stacks conserve energy (reflected + multilayer-transmitted flux
  equals the incident flux, within the PML/discretisation error, which
  decreases under refinement);
* at normal incidence on a square grid the TM field of a layout equals the
  TE field of the transposed layout with x and y exchanged.
"""

import numpy as np
import pytest

from oracle import psfd_ref as R
from psfd_synth import base_config, eps_absorber_default, multilayer_stack, rect_layout

EPS_ABS = eps_absorber_default()


def _dense_solve(P):
    A = R.dense_by_columns(P)
    b = R.rhs(P)
    return np.linalg.solve(A, b.ravel()).reshape(P.g.shape)


def _slab_problem(nx, nabs, theta, pol, t_abs=30.0, f=1):
    cfg = base_config(nx, nx, nabs, t_abs, theta_deg=theta, pol=pol, nz_pml=6 * f, nz_gap=2 * f)
    return cfg, R.Problem(cfg, np.full((nabs, nx, nx), EPS_ABS, np.complex128))


@pytest.mark.parametrize("pol", [0, 1])
def test_uniform_slab_3d_equals_1d(pol):
    cfg, P = _slab_problem(4, 8, 6.0, pol, t_abs=15.0)
    E3 = _dense_solve(P)
    A1 = R.slab_1d_matrix(P)
    b = R.rhs(P)
    b1 = np.concatenate([b[c, :, 0, 0] for c in range(3)])
    E1 = np.linalg.solve(A1, b1).reshape(3, -1)
    scale = np.abs(E1).max()
    assert np.abs(E3 - E1[:, :, None, None]).max() <= 1e-12 * scale


def _slab_reflection_error(nabs, theta, pol, t_abs=30.0):
    f = nabs // 16
    cfg, P = _slab_problem(1, nabs, theta, pol, t_abs, f)
    g, bs = P.g, P.basis
    A1 = R.slab_1d_matrix(P)
    b = R.rhs(P)
    E1 = np.linalg.solve(A1, np.concatenate([b[c, :, 0, 0] for c in range(3)])).reshape(3, -1)
    E = np.zeros(g.shape, np.complex128)
    E[:, :, 0, 0] = E1
    up = R.reflected_obs(P, E)[:, 0, 0]
    back = np.exp(-1j * g.kz0 * g.z[g.j_obs])
    if pol == 0:
        val = (bs.sx[0, 0] * up[0] + bs.sy[0, 0] * up[1]) * back
    else:
        val = (bs.tx[0, 0] * up[0] + bs.ty[0, 0] * up[1]) * back / np.cos(g.theta)
    kt2 = np.array(g.kx0 ** 2 + g.ky0 ** 2)
    r = R.tmm_reflection(g.k0, kt2, 1.0, [EPS_ABS] + cfg["ml_eps"], [t_abs] + cfg["ml_thick"],
                         cfg["eps_sub"], pol)
    r_top = r if pol == 0 else -r
    return abs(val - r_top * np.exp(-2j * g.kz0 * t_abs))


@pytest.mark.parametrize("pol,theta", [(0, 0.0), (0, 6.0), (1, 0.0), (1, 6.0)])
def test_uniform_slab_converges_to_tmm(pol, theta):
    errs = [_slab_reflection_error(n, theta, pol) for n in (16, 32, 64, 128)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4, errs
    assert errs[0] < 5e-3, errs


def test_zero_contrast_gives_zero_field():
    cfg = base_config(8, 8, 4, 8.0)
    P = R.Problem(cfg, np.full((4, 8, 8), 1.0 + 0j))
    b = R.rhs(P)
    assert np.all(b == 0)
    E, info = R.solve(P, tol=1e-10)
    assert info["iters"] == 0 and np.all(E == 0)


def test_bare_multilayer_background_is_tmm():
    cfg = base_config(4, 4, 4, 8.0, theta_deg=6.0, pol=0)
    g = R.Grid(cfg)
    bg = R.background_field(g, cfg, [g.j_obs])[:, 0]
    e_in, _ = R.incident_vectors(g, 0)
    refl = bg - e_in * np.exp(-1j * g.kz0 * g.z[g.j_obs])
    ml_eps, ml_d, eps_s = multilayer_stack()
    r = R.tmm_reflection(g.k0, np.array((g.k0 * np.sin(g.theta)) ** 2), 1.0, ml_eps, ml_d, eps_s, 0)
    np.testing.assert_allclose(refl, r * e_in * np.exp(1j * g.kz0 * g.z[g.j_obs]), atol=1e-14)


def _lossless_cfg(nabs, pol):
    f = nabs // 16
    cfg = base_config(16, 1, nabs, 30.0, dx=4.0, theta_deg=6.0, phi_deg=20.0, pol=pol,
                      nz_pml=6 * f, nz_gap=2 * f)
    cfg["ml_eps"] = [complex(e.real, 0.0) for e in cfg["ml_eps"]]
    cfg["eps_sub"] = complex(cfg["eps_sub"].real, 0.0)
    return cfg


@pytest.mark.parametrize("pol", [0, 1])
def test_energy_balance_lossless(pol):
    a = np.zeros((1, 16))
    a[0, 3:9] = 1.0
    devs = []
    for nabs in (16, 32):
        cfg = _lossless_cfg(nabs, pol)
        P = R.Problem(cfg, R.eps_from_fill(cfg, R.smooth_layout(cfg, a), 0.88 + 0j))
        E = _dense_solve(P)
        devs.append(abs(R.flux_balance(P, E) - 1.0))
    assert devs[1] < devs[0] < 2e-3, devs


def test_energy_balance_detects_loss():
    """With the lossy absorber the balance falls well below one."""
    a = np.zeros((1, 16))
    a[0, 3:9] = 1.0
    cfg = base_config(16, 1, 16, 30.0, dx=4.0, theta_deg=6.0, pol=0)
    P = R.Problem(cfg, R.eps_from_fill(cfg, R.smooth_layout(cfg, a), EPS_ABS))
    assert R.flux_balance(P, _dense_solve(P)) < 0.95


def test_tm_equals_transposed_te_at_normal_incidence():
    rng = np.random.default_rng(7)
    n = 6
    a = rect_layout(n, n, rng, wmin=1, wmax=3)
    cfg_tm = base_config(n, n, 4, 7.5, theta_deg=0.0, pol=1)
    cfg_te = base_config(n, n, 4, 7.5, theta_deg=0.0, pol=0)
    P_tm = R.Problem(cfg_tm, R.eps_from_fill(cfg_tm, R.smooth_layout(cfg_tm, a), EPS_ABS))
    P_te = R.Problem(cfg_te, R.eps_from_fill(cfg_te, R.smooth_layout(cfg_te, a.T), EPS_ABS))
    E_tm = _dense_solve(P_tm)
    E_te = _dense_solve(P_te)
    swapped = np.stack([E_te[1], E_te[0], E_te[2]]).transpose(0, 1, 3, 2)
    assert np.abs(E_tm - swapped).max() <= 1e-12 * np.abs(E_tm).max()
