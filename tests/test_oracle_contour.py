"""Pins for the oracle's threshold-contour width metric (paper, Results,
"Practical assessment of scattered-field convergence" paragraph, equation
logistic_sigmoid).

* the sigmoid: S(I_th) = 1/2, symmetry S(I_th + a) + S(I_th - a) = 1, slope
  1/(4w) at the threshold;
* crossings of a line whose sigmoid samples are chosen by the inverse
  sigmoid (so that the linear interpolation has a hand-computed answer),
  including a segment that wraps around the periodic line end, a line that
  never crosses and a line that is above threshold everywhere;
* a smooth cosine profile sampled ever finer: the width converges to the
  exact width of its I = I_th contour, at second order;
* translation invariance (a periodic shift by whole samples moves starts,
  keeps widths);
* the deviation: a reference against itself gives 0 everywhere; a known
  widening by 2 nm gives -0.5 nm at wafer scale; a missing counterpart is
  unresolved; statistics count them;
* line placement and the intensity's rounding (re*re + im*im).
"""

import numpy as np
import pytest

from oracle import contour_ref as C


def inv_sigmoid(S):
    S = np.asarray(S, dtype=np.float64)
    return C.I_TH + C.W_SIG * np.log(S / (1.0 - S))


def test_sigmoid_properties():
    assert C.sigmoid(C.I_TH) == 0.5
    a = np.linspace(0.0, 0.3, 7)
    assert np.allclose(C.sigmoid(C.I_TH + a) + C.sigmoid(C.I_TH - a), 1.0, atol=1e-15)
    h = 1e-6
    slope = (C.sigmoid(C.I_TH + h) - C.sigmoid(C.I_TH - h)) / (2 * h)
    assert abs(slope - 1.0 / (4 * C.W_SIG)) < 1e-6


def test_hand_computed_crossings():
    # S samples 0.25 0.75 0.75 0.25 0.25 0.25, h = 2: up-crossing halfway between 0 and 1
    # (x = 1 nm), down-crossing halfway between 2 and 3 (x = 5 nm): one segment of 4 nm
    S = np.array([0.25, 0.75, 0.75, 0.25, 0.25, 0.25])
    segs = C.line_segments(inv_sigmoid(S), 2.0)
    assert len(segs) == 1
    assert abs(segs[0][0] - 1.0) < 1e-12 and abs(segs[0][1] - 4.0) < 1e-12
    # unequal steps: S 0.4 -> 0.9 crosses at t = 0.2; 0.7 -> 0.2 at t = 0.4
    S = np.array([0.4, 0.9, 0.7, 0.2])
    (s, w), = C.line_segments(inv_sigmoid(S), 1.0)
    assert abs(s - 0.2) < 1e-12 and abs(w - (2.4 - 0.2)) < 1e-12


def test_wrapping_segment_and_degenerate_lines():
    # above threshold at the two ends: the segment wraps around
    S = np.array([0.75, 0.25, 0.25, 0.25, 0.75, 0.75])
    segs = C.line_segments(inv_sigmoid(S), 1.0)
    assert len(segs) == 1
    s, w = segs[0]
    assert abs(s - 3.5) < 1e-12 and abs(w - 3.0) < 1e-12   # from 3.5 to 0.5 (+6)
    assert C.line_segments(np.full(8, 0.1), 1.0) == []
    assert C.line_segments(np.full(8, 0.9), 1.0) == []
    # two features
    S = np.array([0.1, 0.9, 0.1, 0.9, 0.9, 0.1, 0.1, 0.1])
    segs = C.line_segments(inv_sigmoid(S), 1.0)
    assert [round(w, 12) for _, w in segs] == [1.0, 2.0]


def test_cosine_profile_converges_to_exact_width():
    # I(x) = I_th + 0.1 cos(2 pi x / L) + 0.05: I = I_th where cos = -1/2,
    # so the above-threshold width is 2L/3 exactly
    L = 60.0
    errs = []
    for n in (15, 30, 60, 120, 240):
        x = (np.arange(n) + 0.37) * (L / n)
        I = C.I_TH + 0.1 * np.cos(2 * np.pi * x / L) + 0.05
        (s, w), = C.line_segments(I, L / n)
        errs.append(abs(w - 2 * L / 3))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3
    assert all(3.5 < a / b < 4.5 for a, b in zip(errs, errs[1:])), errs   # second order


def test_translation_moves_starts_keeps_widths():
    rng = np.random.default_rng(3)
    I = np.convolve(rng.random(64), np.ones(5) / 5, mode="same")
    I = 0.15 + (I - I.mean()) * 2.0
    a = C.line_segments(I, 1.5)
    b = C.line_segments(np.roll(I, 7), 1.5)
    assert len(a) == len(b) > 0
    wa = sorted(w for _, w in a)
    wb = sorted(w for _, w in b)
    assert np.allclose(wa, wb, atol=1e-12)
    sa = sorted((s + 7 * 1.5) % 96.0 for s, _ in a)
    sb = sorted(s for s, _ in b)
    assert np.allclose(sa, sb, atol=1e-12)


def test_deviation_and_stats():
    S0 = np.array([0.1, 0.9, 0.9, 0.1, 0.1, 0.1, 0.9, 0.1])
    ref = [C.line_segments(inv_sigmoid(S0), 2.0)]
    assert C.width_deviation(ref, ref, [16.0]) == [[0.0, 0.0]]
    # the first feature one sample wider (2 nm at h = 2): wafer-scale dd = -2/4
    S1 = np.array([0.1, 0.9, 0.9, 0.9, 0.1, 0.1, 0.9, 0.1])
    k = [C.line_segments(inv_sigmoid(S1), 2.0)]
    dev = C.width_deviation(ref, k, [16.0])
    assert abs(dev[0][0] + 0.5) < 1e-12 and abs(dev[0][1]) < 1e-12
    # the second feature gone: unresolved
    S2 = np.array([0.1, 0.9, 0.9, 0.1, 0.1, 0.1, 0.1, 0.1])
    dev = C.width_deviation(ref, [C.line_segments(inv_sigmoid(S2), 2.0)], [16.0])
    assert dev[0][1] is None and abs(dev[0][0]) < 1e-12
    s1, s2, nres, nun, nbig = C.deviation_stats([[0.5, None, -2.0], [1.5]], thr=1.0)
    assert (nres, nun, nbig) == (3, 1, 2) and s1 == 4.0 and s2 == 0.25 + 4.0 + 2.25


def test_plane_lines_and_intensity():
    assert C.line_positions(1024, 100)[:3] == [5, 15, 25]
    assert C.line_positions(64, 100)[:4] == [0, 0, 1, 2]
    rng = np.random.default_rng(9)
    E = rng.standard_normal((8, 16)) + 1j * rng.standard_normal((8, 16))
    I = C.intensity(E)
    assert np.array_equal(I, E.real * E.real + E.imag * E.imag)
    segs, lengths = C.plane_segments(E, 2.0, 3.0, nlines=4)
    assert len(segs) == 8 and lengths == [32.0] * 4 + [24.0] * 4
    # a horizontal line of the plane is line_segments of that row
    assert segs[1] == C.line_segments(I[C.line_positions(8, 4)[1]], 2.0)
    assert segs[5] == C.line_segments(I[:, C.line_positions(16, 4)[1]], 3.0)
