"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Element-by-element comparisons on seeded inputs at sizes the oracle handles
in seconds (several FFT tiles, radix-3 sizes, non-square grids, both
polarisations, oblique incidence out of the x-z plane), plus the edge cases
of the method (normal incidence, no multilayer, no PML, zero contrast).
Tolerances: FP64 operator pieces 1e-12 relative (max-norm); complex64
kernels 3e-5; solves: field relative L2 1e-10 (FP64) / 1e-6 (mixed),
intensity 1e-5 absolute.
"""

import numpy as np
import pytest
import torch

from oracle import psfd_ref as R
from psfd_synth import base_config, config_c1, eps_absorber_default, random_field, rect_layout

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
EPS_ABS = eps_absorber_default()


@pytest.fixture(scope="module")
def psfd():
    import paper_2607_25330_amd as m
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def case(cfg, seed=0, wmax=12):
    rng = np.random.default_rng(seed)
    a = rect_layout(cfg["nx"], cfg["ny"], rng, wmin=2, wmax=wmax)
    eps = R.eps_from_fill(cfg, R.smooth_layout(cfg, a), EPS_ABS)
    return a, eps


def _cfg(nx, ny, nabs, t_abs, **kw):
    return base_config(nx, ny, nabs, t_abs, **kw)


APPLY_CASES = {
    "c1": config_c1(0),
    "c1_tm": config_c1(1),
    "nonsq_tm_phi": _cfg(64, 32, 32, 60.0, dy=2.5, theta_deg=8.0, phi_deg=30.0, pol=1),
    "radix3_lateral": _cfg(192, 16, 8, 15.0, theta_deg=5.0, phi_deg=-20.0),
    "nz24_normal": _cfg(32, 64, 8, 15.0, theta_deg=0.0),
    "nz96": _cfg(16, 32, 80, 100.0, theta_deg=6.0, pol=1),
    "nz128": _cfg(16, 16, 112, 140.0, theta_deg=3.0),
    "no_ml_no_pml": dict(_cfg(32, 32, 16, 30.0, multilayer=False), pml_sigma0=0.0),
    "grazing_cut": dict(_cfg(64, 64, 32, 60.0, theta_deg=6.0, pol=1), ml_kz_min=0.3),
    "nz64": _cfg(32, 16, 48, 70.0, theta_deg=6.0, phi_deg=15.0),
    "wide_512": _cfg(512, 16, 8, 15.0, theta_deg=4.0, phi_deg=10.0, pol=1),
    "wide_1024": _cfg(1024, 16, 8, 15.0, theta_deg=4.0, phi_deg=10.0),
    "tall_1024": _cfg(16, 1024, 8, 15.0, theta_deg=7.0, phi_deg=-35.0, pol=1),
}


@pytest.mark.parametrize("name", list(APPLY_CASES))
def test_operator_pieces(psfd, name):
    cfg = APPLY_CASES[name]
    a, eps = case(cfg, seed=sum(map(ord, name)))
    P = R.Problem(cfg, eps)
    plan = psfd.Plan(cfg, dev(eps))
    rng = np.random.default_rng(5)
    x = random_field(P.g.shape, rng)
    xd = dev(x)
    assert relmax(host(plan.apply(xd)), R.apply_A(P, x)) < 1e-12
    assert relmax(host(plan.adjoint(xd)), R.apply_AH(P, x)) < 1e-12
    assert relmax(host(plan.precond(xd)), R.apply_M(P, x)) < 1e-12
    assert relmax(host(plan.rhs()), R.rhs(P)) < 1e-12
    rte, rpe = plan.ml_reflection()
    assert relmax(host(rte), P.r_te) < 1e-12
    assert relmax(host(rpe), P.r_pe) < 1e-12
    plan.close()


@pytest.mark.parametrize("name", ["c1", "nonsq_tm_phi", "radix3_lateral", "nz64", "wide_1024",
                                  "tall_1024"])
def test_operator_pieces_c64(psfd, name):
    cfg = APPLY_CASES[name]
    a, eps = case(cfg, seed=3)
    P = R.Problem(cfg, eps)
    plan = psfd.Plan(cfg, dev(eps), prec=psfd.PSFD_C64_REFINE64)
    x = random_field(P.g.shape, np.random.default_rng(9))
    xd = dev(x).to(torch.complex64)
    assert relmax(host(plan.apply_c64(xd)).astype(np.complex128), R.apply_A(P, x)) < 3e-5
    assert relmax(host(plan.adjoint_c64(xd)).astype(np.complex128), R.apply_AH(P, x)) < 3e-5
    assert relmax(host(plan.precond_c64(xd)).astype(np.complex128), R.apply_M(P, x)) < 3e-5
    plan.close()


# every value of every schedule knob (others at their default), against the oracle
SCHEDULES = [(v, 0, 0, 0) for v in (1, 2, 3)] + [(0, v, 0, 0) for v in (1, 2, 3)] + \
    [(0, 0, v, 0) for v in (1, 2, 3)] + [(0, 0, 0, v) for v in (1, 2, 3)]


@pytest.mark.parametrize("name", ["c1", "nonsq_tm_phi", "radix3_lateral", "tall_1024", "wide_512"])
def test_operator_all_schedules(psfd, name):
    cfg = APPLY_CASES[name]
    a, eps = case(cfg, seed=7)
    P = R.Problem(cfg, eps)
    x = random_field(P.g.shape, np.random.default_rng(12))
    refA, refM = R.apply_A(P, x), R.apply_M(P, x)
    p64 = psfd.Plan(cfg, dev(eps))
    p32 = psfd.Plan(cfg, dev(eps), prec=psfd.PSFD_C64_REFINE64)
    xd = dev(x)
    x32 = xd.to(torch.complex64)
    for sc in SCHEDULES:
        for p in (p64, p32):
            p.set_schedule(sc)
            assert p.schedule() == sc
        assert relmax(host(p64.apply(xd)), refA) < 1e-12, sc
        assert relmax(host(p64.precond(xd)), refM) < 1e-12, sc
        assert relmax(host(p32.apply_c64(x32)).astype(np.complex128), refA) < 3e-5, sc
    p64.close()
    p32.close()


def test_tuned_solve_matches_oracle(psfd, small_ref):
    """psfd_tune picks schedules by timing; the solve with them still meets the bar."""
    cfg, eps, P, E_ref = small_ref[1]
    for prec, tol, bound in ((psfd.PSFD_C128, 1e-12, 1e-10), (psfd.PSFD_C64_REFINE64, 1e-9, 1e-6)):
        plan = psfd.Plan(cfg, dev(eps), prec=prec)
        sc = plan.tune()
        assert len(sc) == 4 and plan.schedule() == sc
        E, info = plan.solve(tol=tol)
        assert np.linalg.norm(host(E) - E_ref) / np.linalg.norm(E_ref) <= bound
        plan.close()
    with pytest.raises(psfd.PsfdError):
        plan = psfd.Plan(cfg, dev(eps))
        try:
            plan.set_schedule((0, 0, 0, 4))
        finally:
            plan.close()


@pytest.mark.parametrize("nx,ny", [(32, 32), (64, 16), (192, 16)])
def test_layout_eps(psfd, nx, ny):
    cfg = _cfg(nx, ny, 4, 8.0, dy=1.5)
    rng = np.random.default_rng(nx + ny)
    a = rect_layout(nx, ny, rng)
    ref = R.eps_from_fill(cfg, R.smooth_layout(cfg, a), EPS_ABS)
    got = host(psfd.psfd_layout_eps(cfg, dev(a), EPS_ABS))
    assert np.abs(got - ref).max() < 1e-13


def _small_solve_case(pol=0, seed=11):
    cfg = _cfg(16, 16, 8, 15.0, theta_deg=6.0, phi_deg=12.0, pol=pol)
    return (cfg,) + case(cfg, seed=seed, wmax=6)


@pytest.fixture(scope="module")
def small_ref():
    out = {}
    for pol in (0, 1):
        cfg, a, eps = _small_solve_case(pol)
        P = R.Problem(cfg, eps)
        E, info = R.solve(P, tol=1e-13)
        out[pol] = (cfg, eps, P, E)
    return out


@pytest.mark.parametrize("pol", [0, 1])
def test_solve_fp64_matches_oracle(psfd, small_ref, pol):
    cfg, eps, P, E_ref = small_ref[pol]
    plan = psfd.Plan(cfg, dev(eps))
    E, info = plan.solve(tol=1e-12)
    E = host(E)
    assert info["rrel"] <= 1e-12
    assert np.linalg.norm(E - E_ref) / np.linalg.norm(E_ref) <= 1e-10
    assert np.abs(R.intensity_obs(P, E) - R.intensity_obs(P, E_ref)).max() <= 1e-5
    r = np.linalg.norm(R.rhs(P) - R.apply_A(P, E)) / np.linalg.norm(R.rhs(P))
    assert r <= 1.01e-12
    plan.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_solve_mixed_matches_oracle(psfd, small_ref, prec):
    cfg, eps, P, E_ref = small_ref[0]
    plan = psfd.Plan(cfg, dev(eps), prec=prec)
    E, info = plan.solve(tol=1e-9)
    E = host(E)
    assert info["rrel"] <= 1e-9
    assert np.linalg.norm(E - E_ref) / np.linalg.norm(E_ref) <= 1e-6
    assert np.abs(R.intensity_obs(P, E) - R.intensity_obs(P, E_ref)).max() <= 1e-5
    plan.close()


def test_mixed_reliable_updates_and_restart_form_agree(psfd, small_ref, monkeypatch):
    """The mixed solve with reliable updates (default) and with plain restarts
    (PSFD_RELIABLE=0) both reach the FP64 oracle field within the mixed bar,
    for a tolerance that needs several residual replacements."""
    cfg, eps, P, E_ref = small_ref[1]
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("PSFD_RELIABLE", mode)
        plan = psfd.Plan(cfg, dev(eps), prec=psfd.PSFD_C64_REFINE64)
        E, info = plan.solve(tol=1e-10)
        plan.close()
        assert info["status"] == "OK" and info["rrel"] <= 1e-10
        out[mode] = host(E)
        assert np.linalg.norm(out[mode] - E_ref) / np.linalg.norm(E_ref) <= 1e-7
    assert np.linalg.norm(out["1"] - out["0"]) / np.linalg.norm(E_ref) <= 2e-7


def test_solve_unpreconditioned_and_warm_start(psfd, small_ref):
    cfg, eps, P, E_ref = small_ref[0]
    plan0 = psfd.Plan(dict(cfg, precond=0), dev(eps))
    E0, i0 = plan0.solve(tol=1e-12)
    assert np.linalg.norm(host(E0) - E_ref) / np.linalg.norm(E_ref) <= 1e-10
    plan = psfd.Plan(cfg, dev(eps))
    # x0 = zeros behaves as x0 = NULL (same iterations, same field)
    Ea, ia = plan.solve(tol=1e-8)
    Eb, ib = plan.solve(tol=1e-8, x0=torch.zeros_like(Ea))
    assert ia["iters"] == ib["iters"]
    assert relmax(host(Eb), host(Ea)) < 1e-12
    # the exact solution as warm start needs no iteration
    Ec, ic = plan.solve(tol=1e-10, x0=dev(E_ref))
    assert ic["iters"] == 0
    # a perturbed warm start reaches the same field
    x0 = E_ref + 0.01 * np.abs(E_ref).max() * random_field(E_ref.shape, np.random.default_rng(2))
    Ed, idd = plan.solve(tol=1e-12, x0=dev(x0))
    assert np.linalg.norm(host(Ed) - E_ref) / np.linalg.norm(E_ref) <= 1e-10
    plan.close()
    plan0.close()


def test_adjoint_solve(psfd, small_ref):
    cfg, eps, P, _ = small_ref[1]
    g = random_field(P.g.shape, np.random.default_rng(4))
    lam_ref, _ = R.solve(P, b=g, tol=1e-13, adjoint=True)
    plan = psfd.Plan(cfg, dev(eps))
    lam, info = plan.solve(b=dev(g), tol=1e-12, adjoint=True)
    assert np.linalg.norm(host(lam) - lam_ref) / np.linalg.norm(lam_ref) <= 1e-10
    plan.close()


def test_zero_contrast_returns_zero(psfd):
    cfg = _cfg(16, 16, 8, 15.0)
    eps = np.ones((8, 16, 16), np.complex128)
    plan = psfd.Plan(cfg, dev(eps))
    E, info = plan.solve(tol=1e-10)
    assert info["iters"] == 0 and torch.count_nonzero(E).item() == 0
    plan.close()


def test_bad_arguments_rejected(psfd):
    cfg = _cfg(16, 16, 8, 15.0)
    eps = dev(np.ones((8, 16, 16), np.complex128))
    with pytest.raises(psfd.PsfdError):  # unsupported lateral size, caught by the library
        psfd.Plan(dict(cfg, nx=20), dev(np.ones((8, 16, 20), np.complex128)))
    with pytest.raises(ValueError):  # shape mismatch, caught by the binding
        psfd.Plan(dict(cfg, nx=32), eps)
    with pytest.raises(psfd.PsfdError):
        psfd.Plan(dict(cfg, nz_gap_bot=0, nz_gap_top=4), eps)
    plan = psfd.Plan(cfg, eps)
    x = torch.zeros(plan.shape, dtype=torch.complex128, device=DEV)
    with pytest.raises(psfd.PsfdError):
        plan.apply(x, out=x)
    with pytest.raises(psfd.PsfdError):
        plan.apply_c64(x.to(torch.complex64))  # complex64 needs a mixed plan
    plan.close()
