"""Plain FP64 CPU reference (the oracle) for the factorised Fourier neural
operator of the paper's PINO (section 2.1, the lateral and axial Fourier
layers, the pointwise MLP with its residual connection, the lifting and
decoding layers).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP library.

Forward pass on a grid nz x ny x nx (hidden state v: d_v real channels):

  v0 = P [a, x/nx, y/ny, z/nz] + p                      (lifting, pointwise)
  for each layer l:
    u_xy = F2^-1 [ K_xy(kx, ky) . F2 v ]                (each z slice; modes
            kx = 0..kx_max of the real-input half spectrum, |ky| <= ky_max)
    u_z  = F1^-1 [ K_z(kz) . F1 u_xy ]                  (along z, kz = 0..kz_max)
    v   <- v + act( W2 gelu( W1 (u_xy + u_z) + b1 ) + b2 ),
           act = gelu except in the last layer (identity)
  E = Q v + q                                           (decoding: 6 reals = 3 complex)

where "K . X" mixes channels, (K . X)_o = sum_i K_oi X_i, for each retained
mode.  F2 / F1 are the real-input DFTs and their inverses the half-spectrum
inverses (the imaginary part of the zero-frequency term is dropped), as in
the reference FNO implementations; the paper does not spell out these
conventions, nor d_v, d_h, the layer count or the retained modes, which are
therefore parameters.  gelu is the exact (erf) form.

Weights: one flat float array, blocks in this order (row-major):
  P [d_v][4], p [d_v];
  per layer: K_xy [d_v][d_v][2 ky_max + 1][kx_max + 1][2] (re, im; ky index
  m = ky + ky_max), K_z [d_v][d_v][kz_max + 1][2], W1 [d_h][d_v], b1 [d_h],
  W2 [d_v][d_h], b2 [d_v];
  Q [6][d_v], q [6]  (outputs Ex.re, Ex.im, Ey.re, Ey.im, Ez.re, Ez.im).
"""

from math import sqrt

import numpy as np
from scipy.special import erf


def block_sizes(desc):
    dv, dh, L = desc["d_v"], desc["d_h"], desc["n_layers"]
    my, mx, mz = 2 * desc["ky_max"] + 1, desc["kx_max"] + 1, desc["kz_max"] + 1
    head = [("P", (dv, 4)), ("p", (dv,))]
    layer = [("Kxy", (dv, dv, my, mx, 2)), ("Kz", (dv, dv, mz, 2)), ("W1", (dh, dv)),
             ("b1", (dh,)), ("W2", (dv, dh)), ("b2", (dv,))]
    tail = [("Q", (6, dv)), ("q", (6,))]
    return head, layer, tail, L


def unpack(desc, w):
    w = np.asarray(w, dtype=np.float64)
    head, layer, tail, L = block_sizes(desc)
    pos = 0
    out = {"layers": []}

    def take(shape):
        nonlocal pos
        n = int(np.prod(shape))
        blk = w[pos:pos + n].reshape(shape)
        pos += n
        return blk

    for name, shape in head:
        out[name] = take(shape)
    for _ in range(L):
        out["layers"].append({name: take(shape) for name, shape in layer})
    for name, shape in tail:
        out[name] = take(shape)
    assert pos == w.size, (pos, w.size)
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / sqrt(2.0)))


def _cplx(K):
    return K[..., 0] + 1j * K[..., 1]


def lateral_branch(desc, v, Kxy):
    """F2^-1 [K_xy . F2 v] on every z slice; v: (d_v, nz, ny, nx) real."""
    ny, nx = v.shape[2], v.shape[3]
    ky, kxm = desc["ky_max"], desc["kx_max"]
    V = np.fft.rfft2(v, axes=(2, 3))                       # (c, z, ny, nx//2+1)
    rows = [m % ny for m in range(-ky, ky + 1)]            # ky = -ky_max..ky_max
    Vs = V[:, :, rows, :kxm + 1]                           # (i, z, my, mx)
    Us = np.einsum("oiyx,izyx->ozyx", _cplx(Kxy), Vs)
    U = np.zeros_like(V)
    U[:, :, rows, :kxm + 1] = Us
    return np.fft.irfft2(U, s=(ny, nx), axes=(2, 3))


def axial_branch(desc, u, Kz):
    """F1^-1 [K_z . F1 u] along z; u: (d_v, nz, ny, nx) real."""
    nz = u.shape[1]
    mz = desc["kz_max"] + 1
    W = np.fft.rfft(u, axis=1)                             # (c, nz//2+1, ny, nx)
    Z = np.zeros_like(W)
    Z[:, :mz] = np.einsum("oik,ikyx->okyx", _cplx(Kz), W[:, :mz])
    return np.fft.irfft(Z, n=nz, axis=1)


def lift(desc, wts, a):
    nz, ny, nx = a.shape
    z = np.broadcast_to((np.arange(nz) / nz)[:, None, None], a.shape)
    y = np.broadcast_to((np.arange(ny) / ny)[None, :, None], a.shape)
    x = np.broadcast_to((np.arange(nx) / nx)[None, None, :], a.shape)
    feats = np.stack([a, x, y, z])                         # (4, nz, ny, nx)
    return np.einsum("ck,kzyx->czyx", wts["P"], feats) + wts["p"][:, None, None, None]


def layer(desc, lw, v, last):
    uxy = lateral_branch(desc, v, lw["Kxy"])
    uz = axial_branch(desc, uxy, lw["Kz"])
    s = uxy + uz
    h = gelu(np.einsum("ji,izyx->jzyx", lw["W1"], s) + lw["b1"][:, None, None, None])
    o = np.einsum("oj,jzyx->ozyx", lw["W2"], h) + lw["b2"][:, None, None, None]
    return v + (o if last else gelu(o))


def forward(desc, w, a):
    """E (3, nz, ny, nx) complex128 predicted from the input field a (nz, ny, nx)."""
    wts = unpack(desc, w)
    a = np.asarray(a, dtype=np.float64)
    v = lift(desc, wts, a)
    L = desc["n_layers"]
    for l, lw in enumerate(wts["layers"]):
        v = layer(desc, lw, v, l == L - 1)
    out = np.einsum("kc,czyx->kzyx", wts["Q"], v) + wts["q"][:, None, None, None]
    return out[0::2] + 1j * out[1::2]
