"""GPU parity of the standard full-domain PSFD comparison (paper, Results,
"Background-decomposition" paragraph and its first figure, panels c and d):
the bare Mo/Si stack discretised in the absorber rows of a tall grid, no
multilayer operator, solved by the same HIP kernels (the LDS-staged axial
kernel for columns of 324 and 648 rows).

* the stack discretisation (psfd_layered_eps) against the oracle's row means;
* operator, adjoint, preconditioner (FP64 and complex64) on the tall grids
  against the oracle, element by element;
* the specular read-out (psfd_specular) against the oracle on one seeded
  field, for the full-domain plan and for a background-decomposed plan with
  a multilayer;
* the full-domain solve of the bare stack at 1 and 0.5 nm and the four
  incidence angles the paper's 150 nm cell represents: the (0, 0)-mode
  field profile and the reflection coefficient against the oracle's dense
  1-D solve (the stack is laterally uniform, so the 16 x 16 GPU grid and the
  1 x 1 oracle grid carry the same single mode).
Tolerances: FP64 operator pieces 1e-12 relative (max-norm), complex64 3e-5;
row means 1e-14; read-out 1e-12; solves at tol 1e-10: field 1e-8 relative,
reflection 1e-8 absolute (FP64) and 1e-6 (mixed).
"""

import numpy as np
import pytest
import torch

from oracle import psfd_ref as R
from psfd_synth import (FULL_DOMAIN_THETAS_DEG, base_config, full_domain_config,
                        full_domain_stack, random_field)

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


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


def _rows(cfg, n_bilayers=40):
    eps_l, d_l = full_domain_stack(n_bilayers)
    return R.layered_eps_rows(cfg["nz_abs"], cfg["dz"], eps_l, d_l, cfg["eps_bg"])


def _gpu_eps(psfd, cfg, n_bilayers=40):
    eps_l, d_l = full_domain_stack(n_bilayers)
    return psfd.psfd_layered_eps(cfg, eps_l, d_l, DEV)


@pytest.mark.parametrize("dz,nz,nb", [(1.0, 324, 40), (0.5, 648, 40), (0.7, 96, 4), (1.3, 48, 3)])
def test_layered_eps_matches_oracle(psfd, dz, nz, nb):
    print(f"layered eps dz={dz} nz={nz} bilayers={nb}", flush=True)
    cfg = full_domain_config(dz, 0.0, 0, nx=16, n_bilayers=nb, nz=nz)
    e = host(_gpu_eps(psfd, cfg, nb))
    want = _rows(cfg, nb)
    assert e.shape == (cfg["nz_abs"], 16, 16)
    assert np.abs(e - want[:, None, None]).max() < 1e-14


@pytest.mark.parametrize("dz,theta,pol", [(1.0, 5.16, 0), (0.5, 10.37, 1)])
def test_full_domain_operator_pieces(psfd, dz, theta, pol):
    print(f"full-domain operator dz={dz} theta={theta} pol={pol}", flush=True)
    cfg = full_domain_config(dz, theta, pol, nx=16)
    cfg["phi"] = np.radians(20.0)
    eps = _gpu_eps(psfd, cfg)
    P = R.Problem(cfg, np.broadcast_to(_rows(cfg)[:, None, None], (cfg["nz_abs"], 16, 16)).copy())
    x = random_field(P.g.shape, np.random.default_rng(11))
    for prec in (psfd.PSFD_C128, psfd.PSFD_C64_REFINE64):
        plan = psfd.Plan(cfg, eps, prec)
        if prec == psfd.PSFD_C128:
            assert relmax(host(plan.apply(dev(x))), R.apply_A(P, x)) < 1e-12
            assert relmax(host(plan.adjoint(dev(x))), R.apply_AH(P, x)) < 1e-12
            assert relmax(host(plan.precond(dev(x))), R.apply_M(P, x)) < 1e-12
            assert relmax(host(plan.rhs()), R.rhs(P)) < 1e-12
        else:
            x32 = dev(x.astype(np.complex64))
            assert relmax(host(plan.apply_c64(x32)), R.apply_A(P, x)) < 3e-5
            assert relmax(host(plan.precond_c64(x32)), R.apply_M(P, x)) < 3e-5
        plan.close()


def test_specular_readout_matches_oracle(psfd):
    rng = np.random.default_rng(5)
    cfgs = [full_domain_config(1.0, 10.37, 0, nx=16, n_bilayers=4, nz=64),
            base_config(16, 32, 8, 15.0, theta_deg=7.0, phi_deg=25.0, pol=0),
            base_config(32, 16, 8, 15.0, theta_deg=7.0, phi_deg=-15.0, pol=1),
            base_config(16, 16, 8, 15.0, theta_deg=0.0, phi_deg=0.0, pol=1)]
    for cfg in cfgs:
        eps = np.full((cfg["nz_abs"], cfg["ny"], cfg["nx"]), 1.3 + 0.1j)
        P = R.Problem(cfg, eps)
        E = random_field(P.g.shape, rng)
        plan = psfd.Plan(cfg, dev(eps))
        r = plan.specular(dev(E))
        plan.close()
        assert abs(r - R.specular_reflection(P, E)) < 1e-12 * max(1.0, np.abs(E).max())


def _oracle_1d(cfg):
    c1 = dict(cfg, nx=1, ny=1)
    P = R.Problem(c1, _rows(c1)[:, None, None].copy())
    A1 = R.slab_1d_matrix(P)
    b = R.rhs(P)
    E1 = np.linalg.solve(A1, np.concatenate([b[c, :, 0, 0] for c in range(3)])).reshape(3, -1)
    E = np.zeros(P.g.shape, np.complex128)
    E[:, :, 0, 0] = E1
    return E1, R.specular_reflection(P, E)


@pytest.mark.parametrize("dz", [1.0, 0.5])
@pytest.mark.parametrize("theta", FULL_DOMAIN_THETAS_DEG)
def test_full_domain_bare_stack_solve(psfd, dz, theta):
    print(f"full-domain solve dz={dz} theta={theta:.2f}", flush=True)
    cfg = full_domain_config(dz, theta, 0, nx=16)
    E1, r_ref = _oracle_1d(cfg)
    eps = _gpu_eps(psfd, cfg)
    for prec, tol_f, tol_r in ((psfd.PSFD_C128, 1e-8, 1e-8), (psfd.PSFD_C64_REFINE64, 1e-6, 1e-6)):
        plan = psfd.Plan(cfg, eps, prec)
        E, info = plan.solve(tol=1e-10, maxit=5000)
        print(f"  prec {prec}: {info['iters']} iterations, r_rel {info['rrel']:.2e}", flush=True)
        assert info["rrel"] <= 1e-10, info
        r = plan.specular(E)
        plan.close()
        Eh = host(E)
        mode = Eh.mean(axis=(2, 3))
        # every other lateral mode stays empty
        assert np.abs(Eh - mode[:, :, None, None]).max() < 1e-9 * np.abs(mode).max()
        assert np.linalg.norm(mode - E1) / np.linalg.norm(E1) < tol_f
        assert abs(r - r_ref) < tol_r, (r, r_ref)
