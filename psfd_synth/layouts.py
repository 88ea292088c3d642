"""Seeded synthetic mask layouts and random fields.

Layouts are binary absorber indicators ``a_bin[ny, nx]`` in {0, 1} (1 =
absorber), extruded through the absorber rows.  They stand in for the
LithoBench Manhattan masks the paper trains and evaluates on, which are not
available here; no item of that library is reproduced.  Every generator
takes a ``numpy.random.Generator`` so that runs are reproducible.
"""

import numpy as np
from scipy import ndimage


def rect_layout(nx, ny, rng, fill_range=(0.30, 0.60), wmin=2, wmax=12):
    """Random axis-aligned rectangles (periodic wrap) OR-ed until a target fill."""
    target = rng.uniform(*fill_range)
    a = np.zeros((ny, nx), dtype=np.float64)
    wmax_x = max(wmin, min(wmax, nx - 1))
    wmax_y = max(wmin, min(wmax, ny - 1))
    while a.mean() < target:
        w = int(rng.integers(wmin, wmax_x + 1))
        h = int(rng.integers(wmin, wmax_y + 1))
        x0 = int(rng.integers(0, nx))
        y0 = int(rng.integers(0, ny))
        ys = (y0 + np.arange(h)) % ny
        xs = (x0 + np.arange(w)) % nx
        a[np.ix_(ys, xs)] = 1.0
    return a


def line_space(nx, ny, dx, rng):
    """Lines and spaces: CD and space drawn from 16..40 nm (2 nm steps)."""
    orient = int(rng.integers(0, 2))  # 0: lines along y (vary in x), 1: along x
    n = nx if orient == 0 else ny
    length_nm = n * dx
    profile = np.zeros(n)
    pos = 0.0
    while True:
        cd = float(rng.choice(np.arange(16, 42, 2)))
        space = float(rng.choice(np.arange(16, 42, 2)))
        if pos + cd + space > length_nm:
            break
        i0, i1 = int(round(pos / dx)), int(round((pos + cd) / dx))
        profile[i0:i1] = 1.0
        pos += cd + space
    if orient == 0:
        return np.tile(profile[None, :], (ny, 1))
    return np.tile(profile[:, None], (1, nx))


def contact_holes(nx, ny, dx, rng):
    """Absorber-free rectangles (holes) on a jittered grid; CD 16..40 nm."""
    a = np.ones((ny, nx), dtype=np.float64)
    cd = float(rng.choice(np.arange(16, 42, 2)))
    pitch = rng.uniform(2.0 * cd, 3.0 * cd)
    cdc = max(1, int(round(cd / dx)))
    pc = max(cdc + 1, int(round(pitch / dx)))
    for gy in range(0, ny, pc):
        for gx in range(0, nx, pc):
            jx = int(rng.integers(-(pc - cdc) // 4, (pc - cdc) // 4 + 1))
            jy = int(rng.integers(-(pc - cdc) // 4, (pc - cdc) // 4 + 1))
            w = cdc + int(rng.integers(0, 2))
            h = cdc + int(rng.integers(0, 2))
            ys = (gy + jy + np.arange(h)) % ny
            xs = (gx + jx + np.arange(w)) % nx
            a[np.ix_(ys, xs)] = 0.0
    return a


def curvilinear(nx, ny, rng, sigma_cells=12.0):
    """White noise, periodic Gaussian filter, thresholded at a seeded quantile."""
    f = rng.uniform(0.3, 0.6)
    noise = rng.standard_normal((ny, nx))
    sm = ndimage.gaussian_filter(noise, sigma=sigma_cells, mode="wrap")
    thr = np.quantile(sm, 1.0 - f)
    return (sm > thr).astype(np.float64)


def random_field(shape, rng):
    """Complex standard-normal field (test vectors for operator applies)."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def smooth_perturbation(shape, rng, sigma_cells=8.0):
    """Smooth complex noise over the last two axes (warm-start perturbation)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    sig = [0.0] * (len(shape) - 2) + [sigma_cells, sigma_cells]
    re = ndimage.gaussian_filter(re, sigma=sig, mode="wrap")
    im = ndimage.gaussian_filter(im, sigma=sig, mode="wrap")
    return re + 1j * im
