"""GPU: the solver never returns a field worse than its start, and a mixed plan
whose complex64 Krylov run fails finishes the solve in FP64.

Workload: a seeded rectangle layout, 128 x 128 lateral at 1 nm, 50 nm absorber,
TE normal incidence, no grazing cutoff (the lateral order m = 9 travels almost
parallel to the multilayer, which makes the system hard: the FP64 solve needs
about 10^4 iterations and a complex64 run stalls).  Before the fold guard the
mixed solve ran to its iteration limit and returned a diverged field.
"""

import numpy as np
import pytest
import torch

from psfd_synth import base_config, eps_absorber_default, rect_layout

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def psfd():
    import paper_2607_25330_amd as m
    m.lib()
    return m


def test_mixed_solve_of_a_hard_system_matches_fp64(psfd):
    print("robust: 128x128x96, 1 nm, no grazing cutoff", flush=True)
    a = torch.from_numpy(rect_layout(128, 128, np.random.default_rng(700), wmin=8, wmax=48)).to(DEV)
    cfg = base_config(128, 128, 50, 50.0, dx=1.0, theta_deg=0.0, pol=0, nz_pml=12, nz_gap=11)
    eps = psfd.psfd_layout_eps(cfg, a, eps_absorber_default())
    ref = psfd.Plan(cfg, eps, psfd.PSFD_C128)
    E_ref, i_ref = ref.solve(tol=1e-8, maxit=30000)
    print(f"  fp64: {i_ref['iters']} iterations", flush=True)
    mixed = psfd.Plan(cfg, eps, psfd.PSFD_C64_REFINE64)
    E, info = mixed.solve(tol=1e-6, maxit=30000)
    print(f"  mixed: {info['iters']} iterations, restarts {info['restarts']}", flush=True)
    assert info["rrel"] <= 1e-6
    err = float(torch.linalg.vector_norm(E - E_ref) / torch.linalg.vector_norm(E_ref))
    assert err < 1e-2, err
    # a budget far too small: the solve stops NOT_CONVERGED but its field is
    # no worse than the zero start
    E2, i2 = mixed.solve(tol=1e-12, maxit=64, check=False)
    assert i2["status"] != "OK"
    assert np.isfinite(i2["rrel"]) and i2["rrel"] <= 1.0
    ref.close()
    mixed.close()


def test_plans_reuse_cached_device_memory(psfd):
    """Blocks of destroyed plans are reused by later plans (and freed by trim_cache):
    repeated solves on recycled memory give bit-identical fields."""
    print("robust: memory cache reuse", flush=True)
    cfg_a = base_config(32, 32, 16, 30.0)
    cfg_b = base_config(64, 32, 8, 15.0, pol=1)
    a = torch.from_numpy(rect_layout(32, 32, np.random.default_rng(3), wmin=2, wmax=8)).to(DEV)
    b = torch.from_numpy(rect_layout(64, 32, np.random.default_rng(4), wmin=2, wmax=8)).to(DEV)
    eps_a = psfd.psfd_layout_eps(cfg_a, a, eps_absorber_default())
    eps_b = psfd.psfd_layout_eps(cfg_b, b, eps_absorber_default())

    def solve(cfg, eps, prec):
        p = psfd.Plan(cfg, eps, prec)
        E, _ = p.solve(tol=1e-8)
        p.close()
        return E.clone()

    ref = {prec: solve(cfg_a, eps_a, prec) for prec in (psfd.PSFD_C128, psfd.PSFD_C64_REFINE64)}
    for _ in range(2):
        solve(cfg_b, eps_b, psfd.PSFD_C64_REFINE64)
        for prec, E0 in ref.items():
            assert torch.equal(solve(cfg_a, eps_a, prec), E0)
    psfd.trim_cache()
    assert torch.equal(solve(cfg_a, eps_a, psfd.PSFD_C128), ref[psfd.PSFD_C128])
