"""Pins for the oracle's discrete operator A, its adjoint, the multilayer
reflection chain and the preconditioner.

* closed form of curl curl on a single 3-D Fourier mode;
* curl curl annihilates gradients built with an explicit D_z matrix (PML on);
* hermiticity of A when PML, loss and multilayer are off;
* matrix-free A equals A assembled from explicit DFT matrices;
* the discrete R_ml applied to the sampled incident wave equals the analytic
  reflected background;
* <u, A v> = <A^H u, v>;
* the damping multiplier reduces to min(1, k_bg^2/k^2) with the baseline
  parameters, and M = I when m_min = 1.
"""

import numpy as np
import pytest

from oracle import psfd_ref as R
from psfd_synth import random_field

from conftest import small_cfg


def _uniform_problem(nx, ny, nz, eps_val, theta=9.0, phi=35.0):
    cfg = small_cfg(nx=nx, ny=ny, nz_abs=nz, t_abs=nz * 1.5, theta_deg=theta, phi_deg=phi,
                    pml=False, ml=False, nz_pml=0, nz_gap=0)
    return R.Problem(cfg, np.full((nz, ny, nx), eps_val, np.complex128))


def test_single_mode_closed_form(rng):
    """Paper, equation vector_helmholtz_operator: on e exp(i k.r) the operator
    is (|k|^2 I - k k^T - k0^2 eps) e."""
    nx, ny, nz = 6, 5, 8
    eps_val = 0.9 + 0.07j
    P = _uniform_problem(nx, ny, nz, eps_val)
    g = P.g
    for (l, n, m) in [(1, 2, 3), (7, 4, 5), (4, 0, 0), (3, 3, 1)]:  # fftfreq indices
        e = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        jz, jy, jx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        wave = np.exp(2j * np.pi * (l * jz / nz + n * jy / ny + m * jx / nx))
        x = e[:, None, None, None] * wave[None]
        k = np.array([g.kx[m], g.ky[n], g.kz[l]])
        Mk = (k @ k) * np.eye(3) - np.outer(k, k) - g.k0 ** 2 * eps_val * np.eye(3)
        expect = (Mk @ e)[:, None, None, None] * wave[None]
        y = R.apply_A(P, x)
        scale = np.abs(Mk).max() * np.abs(e).max()
        assert np.abs(y - expect).max() <= 1e-13 * scale


def _explicit_dz(g):
    nz = g.nz
    j = np.arange(nz)
    F = np.exp(-2j * np.pi * np.outer(j, j) / nz)
    return np.diag(1 / g.s) @ (np.conj(F).T / nz) @ np.diag(1j * g.kz) @ F


def test_curlcurl_annihilates_gradients(rng):
    """curl curl grad phi = 0 with PML-stretched axial derivatives."""
    cfg = small_cfg(nx=6, ny=4, nz_abs=4, ml=False)
    P = R.Problem(cfg, np.full((4, 4, 6), 1.0 + 0j))   # eps = eps_bg: A = curl curl - kbg^2
    g = P.g
    phi = random_field((g.nz, g.ny, g.nx), rng)
    Ph = np.fft.fft2(phi)
    Dz = _explicit_dz(g)
    gx = np.fft.ifft2(1j * g.kx[None, None, :] * Ph)
    gy = np.fft.ifft2(1j * g.ky[None, :, None] * Ph)
    gz = np.einsum("ij,jkl->ikl", Dz, phi)
    grad = np.stack([gx, gy, gz])
    y = R.apply_A(P, grad) + g.kbg ** 2 * grad
    kmax2 = (np.abs(g.kx).max() ** 2 + np.abs(g.ky).max() ** 2 + np.abs(g.kz).max() ** 2)
    assert np.linalg.norm(y) <= 1e-12 * kmax2 * np.linalg.norm(grad)


def test_hermitian_without_pml_loss_multilayer(rng):
    cfg = small_cfg(nx=4, ny=3, nz_abs=3, pml=False, ml=False, theta_deg=11.0)
    a = rng.uniform(0, 1, (3, 4))
    eps = R.eps_from_fill(cfg, a, 0.8 + 0j)
    P = R.Problem(cfg, eps)
    A = R.dense_by_columns(P)
    assert np.abs(A - A.conj().T).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("pol", [0, 1])
def test_matrix_free_equals_kronecker(rng, pol):
    cfg = small_cfg(nx=4, ny=3, nz_abs=3, pol=pol)
    eps = 1.0 + rng.uniform(-0.2, 0.1, (3, 3, 4)) + 1j * rng.uniform(0, 0.1, (3, 3, 4))
    P = R.Problem(cfg, eps)
    A1 = R.dense_by_columns(P)
    A2 = R.dense_kronecker(P)
    assert np.abs(A1 - A2).max() <= 1e-12 * np.abs(A2).max()


@pytest.mark.parametrize("pol", [0, 1])
def test_discrete_ml_chain_matches_analytic_background(pol):
    """R_ml applied to the grid-sampled incident wave (an exactly representable
    single lateral mode) gives the analytic reflected background."""
    cfg = small_cfg(nx=6, ny=4, nz_abs=5, pol=pol, theta_deg=8.0, phi_deg=30.0)
    P = R.Problem(cfg, np.full((5, 4, 6), 0.9 + 0.05j))
    g = P.g
    e_in, _ = R.incident_vectors(g, pol)
    inc = e_in[:, None] * np.exp(-1j * g.kz0 * g.z)[None, :]
    x = np.broadcast_to(inc[:, :, None, None], g.shape).astype(np.complex128)
    V = R.ml_field_hat(g, P.basis, P.r_te, P.r_pe, R.fft2(x)[:, g.j_ev], g.abs_rows)
    e_ml = R.ifft2(V)
    expect = R.background_field(g, cfg, g.abs_rows) - inc[:, g.abs_rows]
    np.testing.assert_allclose(e_ml, np.broadcast_to(expect[:, :, None, None], e_ml.shape),
                               rtol=0, atol=1e-13)


@pytest.mark.parametrize("pol", [0, 1])
def test_adjoint_inner_product(rng, pol):
    cfg = small_cfg(nx=6, ny=4, nz_abs=4, pol=pol)
    eps = 0.9 + rng.uniform(-0.1, 0.1, (4, 4, 6)) + 1j * rng.uniform(0, 0.08, (4, 4, 6))
    P = R.Problem(cfg, eps)
    u = random_field(P.g.shape, rng)
    v = random_field(P.g.shape, rng)
    lhs = np.vdot(u, R.apply_A(P, v))
    rhs = np.vdot(R.apply_AH(P, u), v)
    scale = np.linalg.norm(u) * np.linalg.norm(R.apply_A(P, v))
    assert abs(lhs - rhs) <= 1e-13 * scale


def test_adjoint_dense_is_conjugate_transpose(rng):
    cfg = small_cfg(nx=3, ny=2, nz_abs=2, pol=1)
    eps = 0.9 + 1j * rng.uniform(0, 0.1, (2, 2, 3))
    P = R.Problem(cfg, eps)
    A = R.dense_by_columns(P)
    AH = R.dense_by_columns(P, lambda u: R.apply_AH(P, u))
    assert np.abs(AH - A.conj().T).max() <= 1e-12 * np.abs(A).max()


def test_damping_baseline_reduces_to_min():
    """Paper: m_min = 0, gamma = 1, reg -> 0, k_ref = k_bg gives min(1, k_bg^2/k^2)."""
    kbg = 2 * np.pi / 13.5
    k2 = np.linspace(0, 40 * kbg * kbg, 1001)
    m = R.damping_multiplier(k2, kbg, 0.0, 1.0, 0.0)
    with np.errstate(divide="ignore"):
        ref = np.minimum(1.0, kbg * kbg / k2)
    np.testing.assert_allclose(m, ref, rtol=1e-15, atol=0)


def test_damping_floor_and_exponent():
    kref = 0.5
    k2 = np.array([0.0, 0.25, 1.0, 4.0])
    m = R.damping_multiplier(k2, kref, 0.1, 2.0, 0.0)
    np.testing.assert_allclose(m, [1.0, 1.0, 0.1 + 0.9 * (0.25 / 1.0) ** 2, 0.1 + 0.9 * (0.25 / 4.0) ** 2])
    assert np.all(R.damping_multiplier(k2, kref, 1.0, 3.0, 0.0) == 1.0)


def test_preconditioner_identity_and_single_mode(rng):
    cfg = small_cfg(nx=6, ny=4, nz_abs=4)
    P = R.Problem(cfg, np.full((4, 4, 6), 0.9 + 0.05j))
    g = P.g
    x = random_field(g.shape, rng)
    cfg1 = dict(cfg, pc_mmin=1.0)
    np.testing.assert_allclose(R.apply_M(R.Problem(cfg1, np.full((4, 4, 6), 1.0 + 0j)), x), x,
                               rtol=0, atol=1e-14 * np.abs(x).max())
    l, n, m = 5, 3, 2
    jz, jy, jx = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    wave = np.exp(2j * np.pi * (l * jz / g.nz + n * jy / g.ny + m * jx / g.nx))
    k2 = g.kx[m] ** 2 + g.ky[n] ** 2 + g.kz[l] ** 2
    mk = min(1.0, g.kbg ** 2 / k2)
    y = R.apply_M(P, np.stack([wave, 2 * wave, -wave]))
    np.testing.assert_allclose(y, mk * np.stack([wave, 2 * wave, -wave]), rtol=0, atol=1e-14)


def test_smoothing_single_mode_and_constant():
    cfg = small_cfg(nx=16, ny=8)
    jy, jx = np.meshgrid(np.arange(8), np.arange(16), indexing="ij")
    a = 0.5 + 0.4 * np.cos(2 * np.pi * 3 * jx / 16)
    kx = 2 * np.pi * 3 / (16 * cfg["dx"])
    sig = cfg["smooth_sigma"] * cfg["dx"]
    expect = 0.5 + 0.4 * np.exp(-0.5 * sig * sig * kx * kx) * np.cos(2 * np.pi * 3 * jx / 16)
    np.testing.assert_allclose(R.smooth_layout(cfg, a), expect, atol=1e-15)
    np.testing.assert_allclose(R.smooth_layout(cfg, np.ones((8, 16))), 1.0, atol=1e-15)


def test_grazing_cutoff_zeroes_only_grazing_modes(rng):
    """With ml_kz_min the multilayer response of modes with |kz| < ml_kz_min k0
    vanishes and every other mode keeps it unchanged."""
    cfg = small_cfg(nx=16, ny=8, nz_abs=4, dx=4.0, theta_deg=6.0)
    eps = np.full((4, 8, 16), 0.9 + 0.05j)
    P0 = R.Problem(cfg, eps)
    P1 = R.Problem(dict(cfg, ml_kz_min=0.5), eps)
    g = P0.g
    cut = np.abs(P0.basis.kzb) < 0.5 * g.k0
    assert cut.any() and (~cut).any()
    Xt = random_field((3, g.ny, g.nx), rng)
    V0 = R.ml_field_hat(g, P0.basis, P0.r_te, P0.r_pe, Xt, g.abs_rows)
    V1 = R.ml_field_hat(g, P1.basis, P1.r_te, P1.r_pe, Xt, g.abs_rows)
    assert np.all(V1[:, :, cut] == 0)
    np.testing.assert_array_equal(V1[:, :, ~cut], V0[:, :, ~cut])
    assert np.abs(V0[:, :, cut]).max() > 0


def _downgoing_wave_rows(g, b, a_s, a_p, rows):
    """Lateral coefficients of the downgoing wave sum_k [a_s s_hat + a_p (t_hat +
    (kt/kz) z_hat)] exp(-i kz z), written out from the plane-wave relations."""
    out = np.zeros((3, len(rows), g.ny, g.nx), np.complex128)
    for i, j in enumerate(rows):
        ph = np.exp(-1j * b.kzb * g.z[j])
        out[0, i] = (a_s * b.sx + a_p * b.tx) * ph
        out[1, i] = (a_s * b.sy + a_p * b.ty) * ph
        out[2, i] = a_p * b.kt / b.kzb * ph
    return out


@pytest.mark.parametrize("pol", [0, 1])
def test_downgoing_amplitudes_of_plane_waves(rng, pol):
    """Every lateral order (propagating and evanescent) of a pure downgoing TE + TM
    wave returns its own amplitudes at z_ml, and R_ml returns r times them."""
    cfg = small_cfg(nx=16, ny=12, nz_abs=3, dx=4.0, theta_deg=7.0, phi_deg=25.0, pol=pol)
    P = R.Problem(cfg, np.full((3, 12, 16), 0.9 + 0.05j))
    g, b = P.g, P.basis
    assert (b.kzb.imag > 0).any() and (b.kzb.imag == 0).any()
    a_s = random_field((g.ny, g.nx), rng)
    a_p = random_field((g.ny, g.nx), rng)
    X = _downgoing_wave_rows(g, b, a_s, a_p, [g.j_ev])[:, 0]
    d_s, d_p = R.downgoing_amplitudes(g, b, X)
    np.testing.assert_allclose(d_s, a_s, rtol=0, atol=1e-12 * np.abs(a_s).max())
    np.testing.assert_allclose(d_p, a_p, rtol=0, atol=1e-12 * np.abs(a_p).max())
    V = R.ml_field_hat(g, b, P.r_te, P.r_pe, X, [g.j_obs])[:, 0]
    ph = np.exp(1j * b.kzb * g.z[g.j_obs])
    up_s = P.r_te * a_s * ph
    up_p = P.r_pe * a_p * ph
    expect = np.stack([up_s * b.sx + up_p * b.tx, up_s * b.sy + up_p * b.ty, -up_p * b.kt / b.kzb])
    np.testing.assert_allclose(V, expect, rtol=0, atol=1e-11 * np.abs(expect).max())


def test_tm_reading_ignores_content_orthogonal_to_tm_polarisation(rng):
    """The TM amplitude is the least-squares fit of the downgoing TM polarisation
    (1, kt/kz) in (t_hat . E_t, E_z): content along (-conj(kt/kz), 1) reads as zero,
    and TE-polarised tangential content does not enter it."""
    cfg = small_cfg(nx=16, ny=12, nz_abs=3, dx=4.0, theta_deg=7.0, phi_deg=25.0)
    P = R.Problem(cfg, np.full((3, 12, 16), 0.9 + 0.05j))
    g, b = P.g, P.basis
    c = random_field((g.ny, g.nx), rng)
    q = b.kt / b.kzb
    X = np.stack([-np.conj(q) * c * b.tx, -np.conj(q) * c * b.ty, c])
    d_s, d_p = R.downgoing_amplitudes(g, b, X)
    assert np.abs(d_p).max() <= 1e-13 * np.abs(c).max() * (1 + np.abs(q).max())
    assert np.abs(d_s).max() <= 1e-13 * np.abs(c).max() * (1 + np.abs(q).max())
    X2 = np.stack([c * b.sx, c * b.sy, np.zeros_like(c)])
    _, d_p2 = R.downgoing_amplitudes(g, b, X2)
    assert np.abs(d_p2).max() <= 1e-14 * np.abs(c).max()


@pytest.mark.parametrize("kt_over_k0", [0.99, 0.995, 0.999, 0.9995])
def test_near_grazing_tm_block_stays_passive(kt_over_k0):
    """The 1-D operator of a near-grazing lateral order (the incidence order of a
    laterally uniform slab at theta = asin(kt/k0)), with the lossy mean contrast of
    a 45 % absorber fill and the multilayer on, keeps every eigenvalue in the lower
    half plane (exp(-i omega t): loss gives Im < 0) up to 1e-2 k0^2.  Reading the
    TM amplitude from E_t alone puts eigenvalues up to +0.6 k0^2 there, which stalls
    BiCGSTAB on layouts that scatter into such orders."""
    from psfd_synth import base_config, eps_absorber_default
    theta = float(np.degrees(np.arcsin(kt_over_k0)))
    cfg = base_config(1, 1, 32, 60.0, theta_deg=theta, pol=1)
    eps = np.full((32, 1, 1), 1.0 + 0.45 * (eps_absorber_default() - 1.0))
    P = R.Problem(cfg, eps)
    w = np.linalg.eigvals(R.slab_1d_matrix(P)) / P.g.k0 ** 2
    assert w.imag.max() < 1e-2, w.imag.max()
