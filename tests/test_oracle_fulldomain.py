"""Pins for the oracle's standard full-domain PSFD pieces (paper, Results,
"Background-decomposition" paragraph and its first figure, panels c and d).

* the stack discretisation (row means of eps) against the exact integral,
  layer-aligned grids and brute-force sub-sampling;
* the specular reflection read-out against a synthetic upgoing plane wave
  of known amplitude (TE and TM) and, for the background-decomposed bare
  multilayer, against the transfer matrix of the stack under a vacuum layer;
* a single discretised slab converging to the Airy formula under axial
  refinement;
* the 40-bilayer Mo/Si stack discretised at 1, 0.5 and 0.25 nm: the
  reflection deviates from the transfer-matrix value and the deviation
  shrinks under refinement at each of the four incidence angles the
  paper's 150 nm cell represents (the discretisation-leak effect);
* the 3-D full-domain solve of a laterally uniform stack equals the 1-D
  solve of its (0, 0) mode.
"""

import numpy as np
import pytest

from oracle import psfd_ref as R
from psfd_synth import (FULL_DOMAIN_THETAS_DEG, full_domain_config, full_domain_stack,
                        multilayer_stack)

K0 = 2 * np.pi / 13.5


def _solve_1d(P):
    A1 = R.slab_1d_matrix(P)
    b = R.rhs(P)
    E1 = np.linalg.solve(A1, np.concatenate([b[c, :, 0, 0] for c in range(3)])).reshape(3, -1)
    E = np.zeros(P.g.shape, np.complex128)
    E[:, :, 0, 0] = E1
    return E


def _full_domain_problem(dz, theta, pol, n_bilayers=40, nx=1, nz=None):
    cfg = full_domain_config(dz, theta, pol, nx=nx, n_bilayers=n_bilayers, nz=nz)
    eps_l, d_l = full_domain_stack(n_bilayers)
    rows = R.layered_eps_rows(cfg["nz_abs"], dz, eps_l, d_l, cfg["eps_bg"])
    return cfg, R.Problem(cfg, np.broadcast_to(rows[:, None, None], (cfg["nz_abs"], nx, nx)).copy())


# ------------------------------------------------------------ stack sampling


def test_layered_rows_integral_and_alignment():
    eps_l, d_l, _ = multilayer_stack(3)
    # integral: sum_j eps_j dz = sum_i eps_i d_i + eps_bg * (height - stack)
    for dz in (1.0, 0.7, 0.25):
        n = int(np.ceil(sum(d_l) / dz)) + 3
        rows = R.layered_eps_rows(n, dz, eps_l, d_l, 1.0)
        exact = sum(e * d for e, d in zip(eps_l, d_l)) + 1.0 * (n * dz - sum(d_l))
        assert abs(rows.sum() * dz - exact) < 1e-12
    # grid aligned with every interface (thicknesses 2.8 and 4.2 are multiples of 0.7 and 1.4):
    # every row is one material
    rows = R.layered_eps_rows(30, 1.4, eps_l, d_l, 1.0)
    top = rows[::-1]
    want = []
    for e, d in zip(eps_l, d_l):
        want += [e] * int(round(d / 1.4))
    want += [1.0] * (30 - len(want))
    assert np.allclose(top, want, rtol=0, atol=1e-14)


def test_layered_rows_brute_force_sampling():
    eps_l, d_l = [2.0 + 0.1j, 0.5, 1.5 - 0.2j], [0.37, 1.9, 0.63]
    dz, n, sub = 0.3, 12, 4000
    rows = R.layered_eps_rows(n, dz, eps_l, d_l, 1.0)
    top = n * dz
    bounds = top - np.cumsum([0.0] + d_l)
    for j in range(n):
        z = (j + (np.arange(sub) + 0.5) / sub) * dz
        val = np.ones(sub, np.complex128)
        for e, hi, lo in zip(eps_l, bounds[:-1], bounds[1:]):
            val[(z >= lo) & (z < hi)] = e
        assert abs(val.mean() - rows[j]) < 2e-3


# ------------------------------------------------------- specular read-out


@pytest.mark.parametrize("pol,theta,phi", [(0, 0.0, 0.0), (0, 9.0, 30.0), (1, 9.0, 30.0),
                                           (1, 0.0, 20.0)])
def test_specular_reads_a_synthetic_upgoing_wave(pol, theta, phi):
    cfg = full_domain_config(1.0, theta, pol, nx=4, n_bilayers=2, nz=48)
    cfg["phi"] = np.radians(phi)
    P = R.Problem(cfg, np.ones((cfg["nz_abs"], 4, 4), np.complex128))
    g = P.g
    r0 = 0.3 - 0.55j
    z_t = g.nz_abs * g.dz
    th, ph = g.theta, g.phi
    if pol == 0:
        e_up, amp = np.array([-np.sin(ph), np.cos(ph), 0.0]), r0
    else:  # upgoing TM wave whose magnetic field reflects with r0
        e_up, amp = np.array([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)]), -r0
    E = np.zeros(g.shape, np.complex128)
    for j in range(g.nz):
        E[:, j] = (amp * e_up * np.exp(1j * g.kz0 * (g.z[j] - 2 * z_t)))[:, None, None]
    assert abs(R.specular_reflection(P, E) - r0) < 1e-13


@pytest.mark.parametrize("pol", [0, 1])
def test_bare_multilayer_background_specular_is_tmm_under_vacuum(pol):
    from psfd_synth import base_config
    cfg = base_config(4, 4, 6, 9.0, theta_deg=7.0, phi_deg=15.0, pol=pol)
    P = R.Problem(cfg, np.ones((6, 4, 4), np.complex128))        # no absorber: E_scat = 0
    g = P.g
    E = np.zeros(g.shape, np.complex128)
    kt2 = np.array(g.kx0 ** 2 + g.ky0 ** 2)
    want = R.tmm_reflection(g.k0, kt2, 1.0, [1.0] + cfg["ml_eps"], [9.0] + cfg["ml_thick"],
                            cfg["eps_sub"], pol)
    assert abs(R.specular_reflection(P, E) - complex(want)) < 1e-12


# ------------------------------------------------------- physics under refinement


def _airy(kt2, eps_slab, d, pol):
    """Single slab in vacuum from the two Fresnel coefficients (no transfer matrices)."""
    kz0 = np.sqrt(K0 * K0 - kt2 + 0j)
    kz1 = R.principal_sqrt(K0 * K0 * eps_slab - kt2)
    q0, q1 = (kz0, kz1) if pol == 0 else (kz0, kz1 / eps_slab)
    r01 = (q0 - q1) / (q0 + q1)
    r10 = -r01
    ph = np.exp(2j * kz1 * d)
    return (r01 + r10 * ph) / (1 + r01 * r10 * ph)


@pytest.mark.parametrize("theta", [0.0, 10.37])
def test_discretised_slab_converges_to_airy(theta):
    eps_s, d = (0.921 + 0.0064j) ** 2, 11.3    # 11.3 nm never falls on a row boundary
    errs = []
    for dz, nz in ((1.0, 48), (0.5, 96), (0.25, 192)):
        cfg = full_domain_config(dz, theta, 0, n_bilayers=1, nz=nz, pml_nm=6.0)
        n = int(np.ceil(d / dz))
        cfg["nz_abs"] = n
        cfg["nz_gap_top"] = nz - n - 2 * cfg["nz_pml"] - cfg["nz_gap_bot"]
        rows = R.layered_eps_rows(n, dz, [eps_s], [d], 1.0)
        P = R.Problem(cfg, rows[:, None, None].copy())
        r = R.specular_reflection(P, _solve_1d(P))
        # the slab hangs from the face; the row below it is partly vacuum
        errs.append(abs(r - _airy(P.g.kx0 ** 2, eps_s, d, 0)))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 2e-3, errs


@pytest.mark.parametrize("theta", FULL_DOMAIN_THETAS_DEG)
def test_full_domain_multilayer_leak_shrinks_under_refinement(theta):
    eps_l, d_l = full_domain_stack()
    errs, r_tmm = [], None
    for dz in (1.0, 0.5, 0.25):
        cfg, P = _full_domain_problem(dz, theta, 0)
        r = R.specular_reflection(P, _solve_1d(P))
        g = P.g
        r_tmm = complex(R.tmm_reflection(g.k0, np.array(g.kx0 ** 2), 1.0, eps_l, d_l, 1.0, 0))
        errs.append(abs(r - r_tmm))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[0] > 5e-3, errs          # the 1 nm grid visibly leaks
    assert errs[2] < 1e-3, errs          # and the error converges under refinement
    assert 0.05 < abs(r_tmm) ** 2 < 0.8


def test_full_domain_3d_equals_1d():
    cfg, P = _full_domain_problem(1.0, 6.0, 0, n_bilayers=2, nx=2, nz=48)
    A = R.dense_by_columns(P)
    E3 = np.linalg.solve(A, R.rhs(P).ravel()).reshape(P.g.shape)
    E1 = _solve_1d(P)[:, :, 0, 0]
    assert np.abs(E3 - E1[:, :, None, None]).max() < 1e-12 * np.abs(E1).max()


def _golden_angles():
    vals = {}
    path = __file__.rsplit("/", 1)[0] + "/golden/representable_angles.txt"
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                vals[line[0]] = [float(v) for v in line[1:]]
    return vals


@pytest.mark.parametrize("dx", [1.0, 0.5])
def test_grid_represents_the_printed_incidence_angles(dx):
    """The lateral wavenumbers of a 150 nm cell give exactly the incidence
    angles the paper prints for its bare-multilayer comparison, and the
    oracle's Bloch shift puts each of them on a grid order."""
    gold = _golden_angles()
    assert dx in gold["dx_nm"]
    lam, (lo, hi), printed = gold["lambda_nm"][0], gold["range_deg"], gold["theta_deg"]
    nx = int(round(150.0 / dx))
    g = R.Grid(full_domain_config(dx, 0.0, 0, nx=nx))
    assert abs(g.k0 - 2 * np.pi / lam) < 1e-15
    kx = np.sort(g.kx[(g.kx >= 0) & (g.kx <= g.k0 * np.sin(np.radians(hi)))])
    got = np.degrees(np.arcsin(kx / g.k0))
    assert got[0] >= lo and len(got) == len(printed)
    assert np.all(np.abs(np.round(got, 2) - printed) < 1e-9), (got, printed)
    dk = 2 * np.pi / (nx * dx)
    for m, th in enumerate(printed):
        gt = R.Grid(full_domain_config(dx, th, 0, nx=nx))
        # the printed two decimals put k0 sin(theta) within 2e-3 of order m
        assert abs(gt.kx0 / dk - m) < 2e-3
        assert abs(gt.kx[0] - gt.kx0) == 0.0 and abs(gt.ky0) == 0.0
    assert np.allclose(FULL_DOMAIN_THETAS_DEG, printed, atol=5e-3)
