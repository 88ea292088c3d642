"""Pins for the oracle's transfer-matrix reflection (multilayer operator step (iii)).

Checked against closed forms (Fresnel, single-slab Airy formula), invariants
(zero-thickness and split layers, energy conservation of lossless stacks,
TE/TM degeneracy at normal incidence) and an independent algorithm (Parratt's
bottom-up recursion), which shares no step with the Abeles product.
"""

import numpy as np
import pytest

from oracle import psfd_ref as R
from psfd_synth import multilayer_stack

K0 = 2 * np.pi / 13.5


def _q(eps, kt2, pol):
    kz = R.principal_sqrt(K0 * K0 * eps - kt2)
    return kz, (kz if pol == 0 else kz / eps)


def parratt(kt2, eps_top, layers_eps, layers_d, eps_sub, pol):
    """Bottom-up recursion of interface reflections (independent of the Abeles product)."""
    eps_all = [eps_top] + list(layers_eps) + [eps_sub]
    d_all = [0.0] + list(layers_d) + [0.0]
    kz = [_q(e, kt2, pol)[0] for e in eps_all]
    q = [_q(e, kt2, pol)[1] for e in eps_all]
    n = len(eps_all)
    Rn = (q[n - 2] - q[n - 1]) / (q[n - 2] + q[n - 1])
    for j in range(n - 3, -1, -1):
        rj = (q[j] - q[j + 1]) / (q[j] + q[j + 1])
        ph = np.exp(2j * kz[j + 1] * d_all[j + 1])
        Rn = (rj + Rn * ph) / (1 + rj * Rn * ph)
    return Rn


KT2 = np.array([0.0, (K0 * np.sin(0.1)) ** 2, (0.9 * K0) ** 2, (1.3 * K0) ** 2, (3.0 * K0) ** 2])


@pytest.mark.parametrize("pol", [0, 1])
def test_no_layers_is_fresnel(pol):
    eps_s = 0.93 + 0.01j
    r = R.tmm_reflection(K0, KT2, 1.0, [], [], eps_s, pol)
    _, q0 = _q(1.0, KT2, pol)
    _, qs = _q(eps_s, KT2, pol)
    np.testing.assert_allclose(r, (q0 - qs) / (q0 + qs), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("pol", [0, 1])
def test_single_slab_airy(pol):
    eps1, eps_s, d = 0.88 + 0.075j, 0.998 + 0.004j, 23.0
    r = R.tmm_reflection(K0, KT2, 1.0, [eps1], [d], eps_s, pol)
    kz1, q1 = _q(eps1, KT2, pol)
    _, q0 = _q(1.0, KT2, pol)
    _, qs = _q(eps_s, KT2, pol)
    r01 = (q0 - q1) / (q0 + q1)
    r12 = (q1 - qs) / (q1 + qs)
    ph = np.exp(2j * kz1 * d)
    np.testing.assert_allclose(r, (r01 + r12 * ph) / (1 + r01 * r12 * ph), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("pol", [0, 1])
def test_zero_thickness_and_split_layers(pol):
    ml_eps, ml_d, eps_s = multilayer_stack(5)
    r = R.tmm_reflection(K0, KT2, 1.0, ml_eps, ml_d, eps_s, pol)
    # a zero-thickness layer of any material changes nothing
    r0 = R.tmm_reflection(K0, KT2, 1.0, [3.0 + 1j] + ml_eps, [0.0] + ml_d, eps_s, pol)
    np.testing.assert_allclose(r0, r, rtol=1e-13, atol=1e-15)
    # splitting a layer into two of the same material changes nothing
    sp_eps = ml_eps[:3] + [ml_eps[3]] + ml_eps[3:]
    sp_d = ml_d[:3] + [0.3 * ml_d[3], 0.7 * ml_d[3]] + ml_d[4:]
    r1 = R.tmm_reflection(K0, KT2, 1.0, sp_eps, sp_d, eps_s, pol)
    np.testing.assert_allclose(r1, r, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("pol", [0, 1])
def test_matches_parratt_full_multilayer(pol):
    ml_eps, ml_d, eps_s = multilayer_stack()
    kt2 = np.linspace(0.0, (4.0 * K0) ** 2, 97)
    r = R.tmm_reflection(K0, kt2, 1.0, ml_eps, ml_d, eps_s, pol)
    rp = parratt(kt2, 1.0, ml_eps, ml_d, eps_s, pol)
    np.testing.assert_allclose(r, rp, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("pol", [0, 1])
def test_lossless_energy_conservation(pol):
    ml_eps, ml_d, eps_s = multilayer_stack(12)
    ml_eps = [complex(e.real, 0.0) for e in ml_eps]
    eps_s = 1.3 + 0j  # denser substrate: transmission is propagating
    kt2 = (K0 * np.sin(np.radians(np.array([0.0, 6.0, 20.0, 45.0])))) ** 2
    r = R.tmm_reflection(K0, kt2, 1.0, ml_eps, ml_d, eps_s, pol)
    # transmission from the Abeles matrix, written out here
    kz0, q0 = _q(1.0, kt2, pol)
    kzs, qs = _q(eps_s, kt2, pol)
    M = np.stack([np.eye(2, dtype=complex)] * len(kt2))
    for e, d in zip(ml_eps, ml_d):
        kz, q = _q(e, kt2, pol)
        dl = kz * d
        Mj = np.empty_like(M)
        Mj[:, 0, 0] = np.cos(dl)
        Mj[:, 0, 1] = -1j * np.sin(dl) / q
        Mj[:, 1, 0] = -1j * q * np.sin(dl)
        Mj[:, 1, 1] = np.cos(dl)
        M = M @ Mj
    den = q0 * M[:, 0, 0] + q0 * qs * M[:, 0, 1] + M[:, 1, 0] + qs * M[:, 1, 1]
    t = 2 * q0 / den
    T = (qs.real / q0.real) * np.abs(t) ** 2
    np.testing.assert_allclose(np.abs(r) ** 2 + T, 1.0, rtol=0, atol=1e-13)


def test_normal_incidence_te_tm_degenerate():
    ml_eps, ml_d, eps_s = multilayer_stack()
    r_te = R.tmm_reflection(K0, np.array([0.0]), 1.0, ml_eps, ml_d, eps_s, 0)
    r_tm_h = R.tmm_reflection(K0, np.array([0.0]), 1.0, ml_eps, ml_d, eps_s, 1)
    np.testing.assert_allclose(-r_tm_h, r_te, rtol=1e-13)


def test_mo_si_reflectance_plausible():
    """40 Mo/Si bilayers near 13.5 nm reflect roughly 70 % at normal incidence."""
    ml_eps, ml_d, eps_s = multilayer_stack()
    r = R.tmm_reflection(K0, np.array([0.0]), 1.0, ml_eps, ml_d, eps_s, 0)
    assert 0.6 < abs(r[0]) ** 2 < 0.8
