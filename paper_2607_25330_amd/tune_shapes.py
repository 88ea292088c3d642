"""Tune the kernel schedules of the solver's workload shapes on this GPU and write
the table that libpsfd.so reads at start-up (tune_table.txt next to it).

    PSFD_TUNE_FILE= python -m paper_2607_25330_amd.tune_shapes OUT.txt

(PSFD_TUNE_FILE empty: ignore the existing table, time every shape afresh.)
Shapes: (nx, ny, nz_abs, absorber thickness in nm), each in complex128 and in
complex64 plans; the axial size is nz_abs + 16.
"""

import sys

SHAPES = [
    (32, 32, 16, 30.0),      # 32 x 32 x 32
    (64, 64, 32, 60.0),      # the batched workload's lateral sizes, Nz = 48
    (128, 128, 32, 60.0),
    (192, 192, 32, 60.0),
    (256, 256, 32, 60.0),    # the benchmark clip, 256 x 256 x 48
    (1024, 1024, 48, 70.0),  # 1024 x 1024 x 64
]


def main(out):
    import torch

    from . import psfd as P
    from psfd_synth import base_config

    dev = torch.device("cuda:0")
    for nx, ny, nabs, t in SHAPES:
        cfg = base_config(nx, ny, nabs, t)
        eps = torch.full((nabs, ny, nx), 0.9 + 0.05j, dtype=torch.complex128, device=dev)
        for prec in (P.PSFD_C128, P.PSFD_C64_REFINE64):
            plan = P.Plan(cfg, eps, prec)
            sched = plan.tune()
            print(f"{nx}x{ny}x{nabs + 16} prec {prec}: {list(sched)}", flush=True)
            plan.close()
        P.trim_cache()
    P.tune_save(out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "tune_table.txt")
