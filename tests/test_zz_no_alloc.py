"""The allocation-free layout entry point (psfd_layout_eps_noalloc) against the
allocating one (psfd_layout_eps): same permittivity on two calls in a row, the
second on a smaller layout (the fixed workspace keeps the first call's data),
and a clear error beyond its 512 x 512 workspace."""

import numpy as np
import pytest
import torch

from psfd_synth import base_config, eps_absorber_default, line_space, rect_layout

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def psfd():
    import paper_2607_25330_amd as m
    m.lib()
    return m


def _case(n_x, n_y, gen, seed):
    cfg = base_config(n_x, n_y, 6, 12.0, dx=2.0)
    a = gen(n_x, n_y, np.random.default_rng(seed))
    return cfg, torch.from_numpy(a).to(DEV)


def test_noalloc_layout_matches_allocating_entry_point(psfd):
    eps_abs = eps_absorber_default()
    cases = [_case(512, 512, lambda nx, ny, r: rect_layout(nx, ny, r), 11),
             _case(192, 64, lambda nx, ny, r: line_space(nx, ny, 2.0, r), 12)]
    for cfg, a in cases:
        print(f"no-alloc layout {cfg['nx']}x{cfg['ny']}", flush=True)
        ref = psfd.psfd_layout_eps(cfg, a, eps_abs)
        got = psfd.psfd_layout_eps_noalloc(cfg, a, eps_abs)
        torch.cuda.synchronize()
        err = (got - ref).abs().max().item()
        assert err <= 1e-13, err
        assert (ref - 1.0).abs().max().item() > 0.05   # a real layout, not a constant


def test_noalloc_layout_rejects_oversize(psfd):
    cfg, a = _case(1024, 512, lambda nx, ny, r: rect_layout(nx, ny, r), 13)
    with pytest.raises(psfd.PsfdError) as ei:
        psfd.psfd_layout_eps_noalloc(cfg, a, eps_absorber_default())
    assert "512" in str(ei.value)
