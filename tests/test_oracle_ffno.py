"""Pins for the oracle's factorised Fourier neural operator (paper, section
2.1: lateral and axial Fourier layers, pointwise MLP with residual, lifting
and decoding).

* the lateral and axial branches against explicit double / single sums of
  the truncated DFT and its half-spectrum inverse (no FFT routine);
* a retained lateral frequency passes an identity kernel unchanged, a
  truncated one is removed;
* with zero spectral kernels a layer is the pointwise MLP, checked voxel by
  voxel by hand;
* with no coordinate channels the network commutes with periodic shifts in
  x, y and z;
* gelu at 0 and +-1 (the standard normal distribution function).
"""

import math

import numpy as np
import pytest

from oracle import ffno_ref as F
from psfd_synth import ffno_desc, ffno_weights


def _desc(**kw):
    base = dict(nx=7, ny=6, nz=5, d_v=2, d_h=3, n_layers=2, kx_max=2, ky_max=1, kz_max=1)
    base.update(kw)
    return ffno_desc(**base)


def test_gelu_values():
    g = F.gelu(np.array([0.0, 1.0, -1.0]))
    assert g[0] == 0.0
    assert abs(g[1] - 0.8413447460685429) < 1e-15
    assert abs(g[2] + 0.15865525393145707) < 1e-15


def test_branches_against_explicit_sums():
    d = _desc()
    rng = np.random.default_rng(0)
    dv, nz, ny, nx = 2, 5, 6, 7
    v = rng.standard_normal((dv, nz, ny, nx))
    my, mx = 2 * d["ky_max"] + 1, d["kx_max"] + 1
    Kxy = rng.standard_normal((dv, dv, my, mx, 2))
    K = Kxy[..., 0] + 1j * Kxy[..., 1]
    got = F.lateral_branch(d, v, Kxy)
    want = np.zeros_like(v)
    for z in range(nz):
        V = np.zeros((dv, my, mx), complex)
        for i in range(dv):
            for m in range(my):
                ky = m - d["ky_max"]
                for kx in range(mx):
                    s = 0j
                    for y in range(ny):
                        for x in range(nx):
                            s += v[i, z, y, x] * np.exp(-2j * np.pi * (ky * y / ny + kx * x / nx))
                    V[i, m, kx] = s
        U = np.einsum("oimk,imk->omk", K, V)
        for o in range(dv):
            for y in range(ny):
                for x in range(nx):
                    acc = 0.0
                    for m in range(my):
                        ky = m - d["ky_max"]
                        for kx in range(mx):
                            term = (U[o, m, kx] * np.exp(2j * np.pi * (ky * y / ny + kx * x / nx))).real
                            acc += term if kx == 0 else 2 * term
                    want[o, z, y, x] = acc / (nx * ny)
    assert np.abs(got - want).max() < 1e-12
    Kz = rng.standard_normal((dv, dv, d["kz_max"] + 1, 2))
    Kc = Kz[..., 0] + 1j * Kz[..., 1]
    got = F.axial_branch(d, v, Kz)
    want = np.zeros_like(v)
    for y in range(ny):
        for x in range(nx):
            W = np.array([[sum(v[i, z, y, x] * np.exp(-2j * np.pi * kz * z / nz) for z in range(nz))
                           for kz in range(d["kz_max"] + 1)] for i in range(dv)])
            Z = np.einsum("oik,ik->ok", Kc, W)
            for o in range(dv):
                for z in range(nz):
                    acc = 0.0
                    for kz in range(d["kz_max"] + 1):
                        term = (Z[o, kz] * np.exp(2j * np.pi * kz * z / nz)).real
                        acc += term if kz == 0 else 2 * term
                    want[o, z, y, x] = acc / nz
    assert np.abs(got - want).max() < 1e-12


def test_identity_kernel_keeps_retained_and_drops_truncated_modes():
    d = _desc(d_v=1, nx=16, ny=12, nz=4, kx_max=3, ky_max=2)
    Kxy = np.zeros((1, 1, 5, 4, 2))
    Kxy[..., 0] = 1.0
    y = np.arange(12)[:, None]
    x = np.arange(16)[None, :]
    keep = np.cos(2 * np.pi * (2 * x / 16 - 1 * y / 12))
    drop = np.cos(2 * np.pi * (5 * x / 16 + 1 * y / 12))
    v = np.broadcast_to(keep + drop, (1, 4, 12, 16)).copy()
    u = F.lateral_branch(d, v, Kxy)
    assert np.abs(u - keep[None, None]).max() < 1e-12


def test_zero_spectral_kernels_leave_the_pointwise_mlp():
    d = _desc()
    w = ffno_weights(d, 3).astype(np.float64)
    wts = F.unpack(d, w)
    lw = dict(wts["layers"][0])
    lw["Kxy"] = np.zeros_like(lw["Kxy"])
    lw["Kz"] = np.zeros_like(lw["Kz"])
    rng = np.random.default_rng(4)
    v = rng.standard_normal((2, 5, 6, 7))
    out = F.layer(d, lw, v, last=False)
    for (z, y, x) in [(0, 0, 0), (3, 5, 2), (4, 1, 6)]:
        h = [0.5 * b * (1 + math.erf(b / math.sqrt(2))) for b in lw["b1"]]
        for o in range(2):
            t = lw["b2"][o] + sum(lw["W2"][o, j] * h[j] for j in range(3))
            g = 0.5 * t * (1 + math.erf(t / math.sqrt(2)))
            assert abs(out[o, z, y, x] - (v[o, z, y, x] + g)) < 1e-13


@pytest.mark.parametrize("axis,shift", [(0, 2), (1, 3), (2, 4)])
def test_shift_equivariance_without_coordinates(axis, shift):
    d = _desc(nx=10, ny=8, nz=6, d_v=3, d_h=4, kx_max=3, ky_max=2, kz_max=2)
    w = ffno_weights(d, 5).astype(np.float64)
    w[: 3 * 4].reshape(3, 4)[:, 1:] = 0.0      # P[:, x, y, z] = 0
    rng = np.random.default_rng(6)
    a = rng.random((6, 8, 10))
    E = F.forward(d, w, a)
    Es = F.forward(d, w, np.roll(a, shift, axis=axis))
    assert np.abs(Es - np.roll(E, shift, axis=axis + 1)).max() < 1e-11 * np.abs(E).max()


def test_lift_channel_order_by_hand():
    """Lifting P [a, x/nx, y/ny, z/nz] + p at single voxels of a non-square grid,
    with distinct weights on every input channel."""
    d = _desc(nx=7, ny=6, nz=5, d_v=2)
    wts = {"P": np.array([[1.5, 2.0, -3.0, 5.0], [-0.5, 7.0, 11.0, -13.0]]),
           "p": np.array([0.25, -0.75])}
    rng = np.random.default_rng(9)
    a = rng.random((5, 6, 7))
    v = F.lift(d, wts, a)
    for (z, y, x) in [(0, 0, 0), (3, 5, 2), (4, 1, 6), (2, 3, 1)]:
        for c in range(2):
            P = wts["P"][c]
            want = P[0] * a[z, y, x] + P[1] * x / 7 + P[2] * y / 6 + P[3] * z / 5 + wts["p"][c]
            assert abs(v[c, z, y, x] - want) < 1e-14


def _inert_layers(wts):
    """Zero spectral kernels and zero second MLP layer: every layer leaves v unchanged
    (gelu(0) = 0 and the residual keeps v)."""
    for lw in wts["layers"]:
        for k in ("Kxy", "Kz", "W2", "b2"):
            lw[k][...] = 0.0


def test_decode_interleave_by_hand():
    """With layers that leave the hidden state unchanged, E_c = (Q v + q)[2c] + i (Q v + q)[2c+1]
    at each voxel, v the lifted input."""
    d = _desc(nx=7, ny=6, nz=5, d_v=2, d_h=3, n_layers=2)
    w = ffno_weights(d, 8).astype(np.float64)
    wts = F.unpack(d, w)
    _inert_layers(wts)
    flat = np.concatenate([wts["P"].ravel(), wts["p"]]
                          + [np.concatenate([lw[k].ravel() for k in ("Kxy", "Kz", "W1", "b1", "W2", "b2")])
                             for lw in wts["layers"]]
                          + [wts["Q"].ravel(), wts["q"]])
    rng = np.random.default_rng(10)
    a = rng.random((5, 6, 7))
    E = F.forward(d, flat, a)
    assert E.shape == (3, 5, 6, 7)
    Q, q, P, p = wts["Q"], wts["q"], wts["P"], wts["p"]
    for (z, y, x) in [(0, 0, 0), (3, 5, 2), (4, 1, 6)]:
        feats = [a[z, y, x], x / 7, y / 6, z / 5]
        v = [sum(P[c, k] * feats[k] for k in range(4)) + p[c] for c in range(2)]
        for comp in range(3):
            re = sum(Q[2 * comp, c] * v[c] for c in range(2)) + q[2 * comp]
            im = sum(Q[2 * comp + 1, c] * v[c] for c in range(2)) + q[2 * comp + 1]
            assert abs(E[comp, z, y, x] - complex(re, im)) < 1e-13


def test_layer_on_uniform_state_by_hand():
    """A spatially uniform hidden state only meets the (0, 0) lateral and the 0 axial
    mode: u_xy = Re K_xy(0,0) v, u_z = Re K_z(0) u_xy, and the layer output is
    v + gelu(W2 gelu(W1 (u_xy + u_z) + b1) + b2), all written out as sums."""
    d = _desc(nx=7, ny=6, nz=5, d_v=2, d_h=3, kx_max=2, ky_max=1, kz_max=1)
    w = ffno_weights(d, 11).astype(np.float64)
    lw = F.unpack(d, w)["layers"][0]
    lw["Kxy"] = 20.0 * lw["Kxy"]                      # spectral outputs of order one
    lw["Kz"] = 20.0 * lw["Kz"]
    v0 = np.array([0.7, -1.3])
    v = np.broadcast_to(v0[:, None, None, None], (2, 5, 6, 7)).copy()
    out = F.layer(d, lw, v, last=False)
    kxy = lw["Kxy"][:, :, d["ky_max"], 0, 0]          # Re K_xy at kx = ky = 0
    kz = lw["Kz"][:, :, 0, 0]                          # Re K_z at kz = 0
    uxy = [sum(kxy[o, i] * v0[i] for i in range(2)) for o in range(2)]
    uz = [sum(kz[o, i] * uxy[i] for i in range(2)) for o in range(2)]
    s = [uxy[i] + uz[i] for i in range(2)]
    gel = lambda t: 0.5 * t * (1 + math.erf(t / math.sqrt(2)))
    h = [gel(sum(lw["W1"][j, i] * s[i] for i in range(2)) + lw["b1"][j]) for j in range(3)]
    for o in range(2):
        t = sum(lw["W2"][o, j] * h[j] for j in range(3)) + lw["b2"][o]
        want = v0[o] + gel(t)
        assert np.abs(out[o] - want).max() < 1e-13
    assert abs(s[0]) > 0.05 and abs(s[1]) > 0.05      # the W1 input is not zero
