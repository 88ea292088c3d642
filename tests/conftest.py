import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture
def rng():
    return np.random.default_rng(1234)


def small_cfg(nx=6, ny=4, nz_abs=4, t_abs=8.0, dx=2.0, theta_deg=7.0, phi_deg=25.0, pol=0,
              pml=True, ml=True, nz_pml=6, nz_gap=2, precond=1):
    """A tiny but fully general problem: non-square lateral grid, oblique
    incidence out of the x-z plane, PML, multilayer."""
    from psfd_synth import base_config
    cfg = base_config(nx, ny, nz_abs, t_abs, dx=dx, dy=dx * 1.25, theta_deg=theta_deg,
                      phi_deg=phi_deg, pol=pol, precond=precond, nz_pml=nz_pml, nz_gap=nz_gap,
                      multilayer=ml)
    if not pml:
        cfg["pml_sigma0"] = 0.0
    return cfg
