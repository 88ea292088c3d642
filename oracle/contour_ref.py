"""Plain FP64 CPU reference (the oracle) for the threshold-contour width
metric of the paper's Results section ("Practical assessment of
scattered-field convergence" paragraph, equation logistic_sigmoid, and the
figure that maps the wafer-equivalent width error).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP library.

What it computes:

* the intensity I = |E_y^scat|^2 of a field plane, mapped through the
  logistic sigmoid S(I) = 1 / (1 + exp(-(I - I_th) / w)), I_th = 0.15,
  w = 0.05;
* on each of n horizontal and n vertical scan lines (rows / columns at
  floor((l + 1/2) N / n)), the threshold crossings S = 0.5, i.e. I = I_th;
* the segments where S > 0.5 between an upward and the next downward
  crossing, and their widths d (the threshold-contour widths);
* against a reference (the converged solution), the deviation
  delta d = d_ref - d for every reference segment, divided by the 4x
  demagnification of a 0.33-NA EUV system for wafer-scale numbers; a
  reference segment with no counterpart is "unresolved".

Readings where the paper is silent:
the lines are periodic (the mask cell is periodic); whether a sample is
above threshold is decided on I > I_th (no rounding of the sigmoid can flip
it); the crossing between two samples is placed by linear interpolation of
S; a reference segment is matched to the segment of the other field, on
the same line, that contains its centre.
"""

import numpy as np

I_TH = 0.15
W_SIG = 0.05
DEMAG = 4.0


def intensity(plane):
    """|E|^2 as re*re + im*im, each product rounded (no fused multiply-add)."""
    p = np.asarray(plane, dtype=np.complex128)
    return p.real * p.real + p.imag * p.imag


def sigmoid(I, i_th=I_TH, w=W_SIG):
    """Equation logistic_sigmoid."""
    return 1.0 / (1.0 + np.exp(-(np.asarray(I, dtype=np.float64) - i_th) / w))


def line_positions(n, nlines):
    """Indices of nlines evenly spread scan lines across n rows or columns."""
    return [int((l + 0.5) * n / nlines) for l in range(nlines)]


def line_segments(I_line, h, i_th=I_TH, w=W_SIG):
    """Above-threshold segments of one periodic line of samples spaced h.

    Returns a list of (start, width) in length units, in the order of their
    starts after the first upward crossing from sample 0; [] if the line
    never crosses the threshold."""
    I_line = np.asarray(I_line, dtype=np.float64)
    n = len(I_line)
    S = sigmoid(I_line, i_th, w)
    above = I_line > i_th
    cross = []  # (position, upward?)
    for j in range(n):
        j1 = (j + 1) % n
        if above[j] != above[j1]:
            t = (0.5 - S[j]) / (S[j1] - S[j])
            cross.append(((j + t) * h, bool(above[j1])))
    if not cross:
        return []
    L = n * h
    first = next(i for i, c in enumerate(cross) if c[1])
    m = len(cross)
    segs = []
    for q in range(m // 2):
        u = cross[(first + 2 * q) % m][0]
        d = cross[(first + 2 * q + 1) % m][0]
        width = d - u
        if width < 0:
            width += L
        segs.append((u, width))
    return segs


def plane_segments(plane, dx, dy, nlines=100, i_th=I_TH, w=W_SIG):
    """Segments of the nlines horizontal lines (along x) then the nlines
    vertical lines (along y) of a [ny][nx] field plane; also the line lengths."""
    I = intensity(plane)
    ny, nx = I.shape
    out, lengths = [], []
    for r in line_positions(ny, nlines):
        out.append(line_segments(I[r, :], dx, i_th, w))
        lengths.append(nx * dx)
    for c in line_positions(nx, nlines):
        out.append(line_segments(I[:, c], dy, i_th, w))
        lengths.append(ny * dy)
    return out, lengths


def width_deviation(ref_lines, k_lines, lengths, demag=DEMAG):
    """delta d / demag for every reference segment (None: unresolved).

    The counterpart of a reference segment is the segment of the same line
    of the other field whose interval (periodic) contains the reference
    segment's centre."""
    out = []
    for ref, other, L in zip(ref_lines, k_lines, lengths):
        row = []
        for s, wr in ref:
            c = (s + 0.5 * wr) % L
            match = None
            for sk, wk in other:
                if (c - sk) % L < wk:
                    match = wk
                    break
            row.append(None if match is None else (wr - match) / demag)
        out.append(row)
    return out


def deviation_stats(dev, thr=1.0):
    """(sum |dd|, sum dd^2, resolved, unresolved, count |dd| > thr) over all segments."""
    s1 = s2 = 0.0
    nres = nun = nbig = 0
    for row in dev:
        for v in row:
            if v is None:
                nun += 1
            else:
                nres += 1
                s1 += abs(v)
                s2 += v * v
                nbig += abs(v) > thr
    return s1, s2, nres, nun, nbig
