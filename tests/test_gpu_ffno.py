"""GPU parity of the factorised Fourier neural operator forward pass (paper,
section 2.1) against the oracle, with seeded random weights (no trained
weights exist here) shared by both sides as FP32 values.

* grids with non-power-of-two and unequal sizes, all three (d_v, d_h) pairs,
  one to four layers, asymmetric mode counts, ragged row blocks and odd nz,
  kx_max above 15 on rows taken by the scalar and by the 16-byte x kernels;
* output E (complex128, the solver's layout) within 2e-5 of max |E| (FP32
  hidden state and transforms, FP64 oracle);
* the prediction serves as the solver's warm start: a solve from it reaches
  the same field as a solve from zero.
"""

import numpy as np
import pytest
import torch

from oracle import ffno_ref as F
from psfd_synth import base_config, eps_absorber_default, ffno_desc, ffno_weights, rect_layout

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def psfd():
    import paper_2607_25330_amd as m
    m.lib()
    return m


def smooth_input(nz, ny, nx, seed):
    rng = np.random.default_rng(seed)
    a = np.zeros((nz, ny, nx))
    a[nz // 4: nz // 4 + max(1, nz // 3)] = (rng.random((ny, nx)) > 0.5)
    k = np.exp(-0.5 * (np.fft.fftfreq(ny)[:, None] ** 2 + np.fft.fftfreq(nx)[None, :] ** 2) * 40.0)
    return np.clip(np.fft.ifft2(np.fft.fft2(a, axes=(1, 2)) * k, axes=(1, 2)).real, 0, 1)


CASES = [
    dict(nx=24, ny=20, nz=16, d_v=8, d_h=16, n_layers=2, kx_max=3, ky_max=4, kz_max=3),
    dict(nx=64, ny=48, nz=32, d_v=16, d_h=32, n_layers=3, kx_max=8, ky_max=6, kz_max=5),
    dict(nx=80, ny=72, nz=48, d_v=32, d_h=64, n_layers=4, kx_max=12, ky_max=12, kz_max=8),
    dict(nx=40, ny=36, nz=100, d_v=32, d_h=64, n_layers=1, kx_max=5, ky_max=7, kz_max=15),
    # row counts (d_v nz ny) that leave ragged x-pass blocks, odd nz (the axial passes take
    # four z rows at a time), kx_max > 15 (the wider x kernels)
    dict(nx=30, ny=18, nz=11, d_v=8, d_h=16, n_layers=2, kx_max=4, ky_max=3, kz_max=2),
    dict(nx=70, ny=22, nz=13, d_v=16, d_h=32, n_layers=1, kx_max=20, ky_max=5, kz_max=6),
    # rows whose length is a multiple of 4 but not of 64 with kx_max > 15: the 16-byte
    # load / store x kernels with the wider mode count
    dict(nx=72, ny=20, nz=12, d_v=16, d_h=32, n_layers=2, kx_max=20, ky_max=5, kz_max=4),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_forward_matches_oracle(psfd, case):
    d = ffno_desc(**CASES[case])
    print(f"ffno forward {d}", flush=True)
    w = ffno_weights(d, 11 + case)
    a = smooth_input(d["nz"], d["ny"], d["nx"], 3 + case).astype(np.float32)
    net = psfd.Ffno(d, torch.from_numpy(w).to(DEV))
    E = net(torch.from_numpy(a).to(DEV))
    torch.cuda.synchronize()
    want = F.forward(d, w.astype(np.float64), a.astype(np.float64))
    err = float(np.abs(E.cpu().numpy() - want).max() / np.abs(want).max())
    print(f"  rel err {err:.2e}", flush=True)
    assert err < 2e-5, err


def test_prediction_is_a_warm_start(psfd):
    cfg = base_config(32, 32, 16, 30.0)
    nz = cfg["nz_abs"] + 16
    d = ffno_desc(32, 32, nz, d_v=8, d_h=16, n_layers=2, kx_max=6, ky_max=6, kz_max=6)
    rng = np.random.default_rng(2)
    a_bin = torch.from_numpy(rect_layout(32, 32, rng, wmin=2, wmax=10)).to(DEV)
    eps = psfd.psfd_layout_eps(cfg, a_bin, eps_absorber_default())
    a = torch.zeros((nz, 32, 32), dtype=torch.float32, device=DEV)
    j0 = cfg["nz_pml"] + cfg["nz_gap_bot"]
    fill = (eps[0].real - 1.0) / (eps_absorber_default().real - 1.0)
    a[j0:j0 + cfg["nz_abs"]] = fill.to(torch.float32)
    net = psfd.Ffno(d, torch.from_numpy(0.01 * ffno_weights(d, 5)).to(DEV))
    x0 = net(a)
    plan = psfd.Plan(cfg, eps)
    E0, _ = plan.solve(tol=1e-10)
    E1, info = plan.solve(x0=x0, tol=1e-10)
    plan.close()
    err = float(torch.linalg.vector_norm(E1 - E0) / torch.linalg.vector_norm(E0))
    assert err < 1e-8, err
