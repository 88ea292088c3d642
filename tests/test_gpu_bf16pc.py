"""GPU: the bfloat16 preconditioner trial (PSFD_C64_BF16PC_REFINE64).

* its complex64 M apply differs from the oracle's M only by the bfloat16 rounding of
  the damped spectrum (a relative error of order 2^-9, and not zero: the rounding
  really happens), on the register and on the LDS axial kernels;
* the operator A is that of the complex64 plans;
* solves reach the oracle's field within the mixed-precision bar (rel. L2 1e-6,
  intensity 1e-5), TE and TM.
"""

import numpy as np
import pytest
import torch

from oracle import psfd_ref as R
from psfd_synth import base_config, eps_absorber_default, random_field, rect_layout

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
EPS_ABS = eps_absorber_default()


@pytest.fixture(scope="module")
def psfd():
    import paper_2607_25330_amd as m
    m.lib()
    return m


def _case(pol, n=32, nabs=16, t=30.0, seed=5):
    cfg = base_config(n, n, nabs, t, theta_deg=6.0, phi_deg=10.0, pol=pol)
    a = rect_layout(n, n, np.random.default_rng(seed), wmin=2, wmax=8)
    eps = R.eps_from_fill(cfg, R.smooth_layout(cfg, a), EPS_ABS)
    return cfg, eps, R.Problem(cfg, eps)


@pytest.mark.parametrize("sched_ax", [0, 2], ids=["register", "lds"])
def test_bf16_preconditioner_is_m_rounded(psfd, sched_ax):
    cfg, eps, P = _case(0)
    plan = psfd.Plan(cfg, torch.from_numpy(eps).to(DEV), prec=psfd.PSFD_C64_BF16PC_REFINE64)
    sched = list(plan.schedule())
    sched[3] = sched_ax
    plan.set_schedule(sched)
    x = random_field(P.g.shape, np.random.default_rng(9))
    Mx = R.apply_M(P, x)
    got = plan.precond_c64(torch.from_numpy(x).to(DEV).to(torch.complex64)).cpu().numpy()
    err = np.abs(got - Mx).max() / np.abs(Mx).max()
    assert 1e-5 < err < 8e-3, err
    Ax = R.apply_A(P, x)
    gotA = plan.apply_c64(torch.from_numpy(x).to(DEV).to(torch.complex64)).cpu().numpy()
    assert np.abs(gotA - Ax).max() / np.abs(Ax).max() < 3e-5
    plan.close()


@pytest.mark.parametrize("pol", [0, 1], ids=["TE", "TM"])
def test_bf16_preconditioned_solve_matches_oracle(psfd, pol):
    cfg, eps, P = _case(pol, seed=6 + pol)
    E_ref, _ = R.solve(P, tol=1e-13)
    plan = psfd.Plan(cfg, torch.from_numpy(eps).to(DEV), prec=psfd.PSFD_C64_BF16PC_REFINE64)
    E, info = plan.solve(tol=1e-9)
    plan.close()
    assert info["status"] == "OK"
    E = E.cpu().numpy()
    ferr = np.linalg.norm(E - E_ref) / np.linalg.norm(E_ref)
    ierr = np.abs(R.intensity_obs(P, E) - R.intensity_obs(P, E_ref)).max()
    assert ferr <= 1e-6, ferr
    assert ierr <= 1e-5, ierr
