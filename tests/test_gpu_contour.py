"""GPU parity of the threshold-contour width metric (paper, Results,
"Practical assessment of scattered-field convergence" paragraph, equation
logistic_sigmoid) against the oracle, on seeded smooth complex fields whose
intensity crosses the threshold many times per line.

* segment counts bit-exact (the above/below decision is exact on both
  sides), starts and widths within 1e-12 nm;
* deviation per reference segment within 1e-12 nm, unresolved slots at the
  same places, statistics within 1e-9 relative;
* sizes: square and non-square planes, more scan lines than rows, the
  largest line (1024), several planes in one launch taken as strided views
  of a stacked field, a plane that never crosses.
"""

import math

import numpy as np
import pytest
import torch

from oracle import contour_ref as C

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def psfd():
    import paper_2607_25330_amd as m
    m.lib()
    return m


def smooth_field(ny, nx, seed, sigma=4.0, level=0.15):
    """Seeded complex Gaussian noise, low-passed, scaled so that the mean intensity is ~2 level."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    f = np.fft.ifft2(np.fft.fft2(z) * np.exp(-2 * (math.pi * sigma) ** 2 * (kx ** 2 + ky ** 2)))
    return f * math.sqrt(2 * level / np.mean(np.abs(f) ** 2))


def gpu_segments(psfd, planes, dx, dy, nlines):
    seg, nseg = psfd.contour_segments(planes, dx, dy, nlines=nlines)
    torch.cuda.synchronize()
    return seg, nseg


def check_segments(seg, nseg, oracle_lines):
    seg = seg.cpu().numpy()
    nseg = nseg.cpu().numpy()
    for li, segs in enumerate(oracle_lines):
        assert nseg[li] == len(segs), li
        if segs:
            ref = np.array(segs)
            assert np.abs(seg[li, :len(segs)] - ref).max() < 1e-12, li


@pytest.mark.parametrize("ny,nx,dx,dy,nlines", [(64, 64, 2.0, 2.0, 100), (96, 160, 1.0, 1.5, 37),
                                                (1024, 256, 1.0, 1.0, 100)])
def test_segments_match_oracle(psfd, ny, nx, dx, dy, nlines):
    print(f"contour segments {ny}x{nx} lines {nlines}", flush=True)
    E = smooth_field(ny, nx, seed=ny + nx)
    seg, nseg = gpu_segments(psfd, torch.from_numpy(E).to(DEV), dx, dy, nlines)
    lines, _ = C.plane_segments(E, dx, dy, nlines)
    assert int(nseg.sum()) > 2 * nlines   # the fields really cross the threshold
    check_segments(seg[0], nseg[0], lines)


def test_strided_batch_and_degenerate_plane(psfd):
    ny, nx, nz = 128, 64, 6
    F = np.zeros((3, 3, nz, ny, nx), np.complex128)
    for b in range(3):
        F[b, 1, 4] = smooth_field(ny, nx, seed=40 + b)
    F[2, 1, 4] = 0.1   # below threshold everywhere: no segments
    Fd = torch.from_numpy(F).to(DEV)
    planes = Fd[:, 1, 4]
    assert planes.stride(0) == 3 * nz * ny * nx
    seg, nseg = gpu_segments(psfd, planes, 2.0, 2.0, 50)
    for b in range(3):
        lines, _ = C.plane_segments(F[b, 1, 4], 2.0, 2.0, 50)
        check_segments(seg[b], nseg[b], lines)
    assert int(nseg[2].sum()) == 0


@pytest.mark.parametrize("ny,nx", [(128, 128), (256, 192)])
def test_deviation_matches_oracle(psfd, ny, nx):
    print(f"contour deviation {ny}x{nx}", flush=True)
    dx, dy, nl = 2.0, 2.0, 100
    refs, others = [], []
    for b in range(2):
        E0 = smooth_field(ny, nx, seed=100 + b)
        E1 = E0 + 0.08 * smooth_field(ny, nx, seed=200 + b, sigma=6.0)
        refs.append(E0)
        others.append(E1)
    R_ = gpu_segments(psfd, torch.from_numpy(np.stack(refs)).to(DEV), dx, dy, nl)
    K_ = gpu_segments(psfd, torch.from_numpy(np.stack(others)).to(DEV), dx, dy, nl)
    delta, stats = psfd.contour_deviation(R_, K_, nx, ny, dx, dy, demag=4.0, thr=0.25)
    delta = delta.cpu().numpy()
    want_stats = np.zeros(5)
    for b in range(2):
        lr, L = C.plane_segments(refs[b], dx, dy, nl)
        lk, _ = C.plane_segments(others[b], dx, dy, nl)
        dev = C.width_deviation(lr, lk, L)
        want_stats += np.array(C.deviation_stats(dev, thr=0.25), dtype=np.float64)
        for li, row in enumerate(dev):
            for q, v in enumerate(row):
                got = delta[b, li, q]
                if v is None:
                    assert np.isnan(got), (b, li, q)
                else:
                    assert abs(got - v) < 1e-12, (b, li, q, got, v)
            assert np.all(delta[b, li, len(row):] == 0.0)
    got = np.array([stats["sum_abs"], stats["sum_sq"], stats["resolved"], stats["unresolved"],
                    stats["above_thr"]], dtype=np.float64)
    assert np.all(got[2:] == want_stats[2:])
    assert np.allclose(got[:2], want_stats[:2], rtol=1e-9, atol=1e-12)
    assert stats["resolved"] > 100 and stats["unresolved"] >= 0
