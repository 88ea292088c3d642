"""Writes the sampled 256 x 256 x 48 reference solutions (c2_linespace_te.txt,
c2_linespace_tm.txt) from the oracle alone.

The problem is the benchmark's first clip: lines and spaces from
psfd_synth.line_space with seed 100, 256 x 256 lateral cells at 2 nm, 32
absorber rows over 60 nm, 6 degrees, the multilayer operator on every
lateral order.  The oracle solves A E = b (paper, section 2.2: the vector
Helmholtz operator with R_ml inside it and the background source, equations
vector_helmholtz_operator and bg_source) with its BiCGSTAB to a relative
residual (equation relative_residual) of 1e-10.  The field is far too large
for a fixture, so the file keeps seeded samples of it: every component at
128 pixels of the observation row (the first row above the absorber) and
single components at 128 voxels anywhere on the grid.

    python tests/golden/make_c2_reference.py 0   # TE, about an hour and a half
    python tests/golden/make_c2_reference.py 1   # TM
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import psfd_ref as R  # noqa: E402
from psfd_synth import config_c2, eps_absorber_default, line_space  # noqa: E402

TOL = 1e-10
SEED_LAYOUT = 100
SEED_SAMPLES = 2026
N_OBS = 128
N_VOX = 128


def problem(pol):
    cfg = dict(config_c2(pol), ml_kz_min=0.0)
    a = line_space(cfg["nx"], cfg["ny"], cfg["dx"], np.random.default_rng(SEED_LAYOUT))
    eps = R.eps_from_fill(cfg, R.smooth_layout(cfg, a), eps_absorber_default())
    return cfg, a, eps


def samples(shape):
    """(observation-row pixels, voxels) drawn from one seeded generator."""
    _, nz, ny, nx = shape
    rng = np.random.default_rng(SEED_SAMPLES)
    obs = [(int(rng.integers(0, ny)), int(rng.integers(0, nx))) for _ in range(N_OBS)]
    vox = [(int(rng.integers(0, 3)), int(rng.integers(0, nz)), int(rng.integers(0, ny)),
            int(rng.integers(0, nx))) for _ in range(N_VOX)]
    return obs, vox


class _Progress(list):
    def append(self, v):
        super().append(v)
        if len(self) % 100 == 0:
            print(f"  iteration {len(self)}: r_rel {v:.3e}", flush=True)


def main(pol):
    cfg, _, eps = problem(pol)
    P = R.Problem(cfg, eps)
    t0 = time.time()
    E, info = R.solve(P, tol=TOL, maxit=8000, history=_Progress())
    dt = time.time() - t0
    if info["status"] != "converged":
        raise SystemExit(f"oracle did not converge: {info}")
    obs, vox = samples(P.g.shape)
    j = P.g.j_obs
    name = os.path.join(HERE, f"c2_linespace_{'te' if pol == 0 else 'tm'}.txt")
    with open(name, "w") as f:
        f.write("# Sampled oracle solution, 256x256x48 line/space clip (seed 100), "
                f"{'TE' if pol == 0 else 'TM'}, 6 deg, multilayer on every order.\n")
        f.write("# Written by tests/golden/make_c2_reference.py from the oracle alone "
                "(paper, section 2.2, equations vector_helmholtz_operator, bg_source,\n"
                "# relative_residual); BiCGSTAB to r_rel "
                f"{TOL:g}: {info['iters']} iterations, true r_rel {info['rrel']:.3e}, {dt:.0f} s.\n")
        f.write("# obs iy ix  Ex.re Ex.im Ey.re Ey.im Ez.re Ez.im   (observation row, scattered field)\n")
        f.write("# vox c z iy ix  re im\n")
        f.write(f"pol {pol}\nobs_row {j}\n")
        for iy, ix in obs:
            v = E[:, j, iy, ix]
            f.write(f"obs {iy} {ix} " + " ".join(repr(float(x)) for c in v for x in (c.real, c.imag))
                    + "\n")
        for c, z, iy, ix in vox:
            v = E[c, z, iy, ix]
            f.write(f"vox {c} {z} {iy} {ix} {float(v.real)!r} {float(v.imag)!r}\n")
    print(f"wrote {name}: {info}", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]))
