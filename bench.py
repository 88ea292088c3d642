"""PSFD solves/s at relative residual 1e-6 on one MI355X.

Workload (one "step"): one seeded 256 x 256 mask clip (2 nm pitch, 32
absorber cells over 60 nm, Nz = 48), alternating line/space and contact-hole
layouts, solved for TE and TM at 6 deg incidence: layout smoothing -> plan
(TMM per lateral mode) -> source -> right-preconditioned BiCGSTAB to a true
FP64 relative residual of 1e-6 -> field.  Two solves per step.

The headline value is the mixed path (complex64 operator, preconditioner and
Krylov vectors inside FP64 iterative refinement); the plain FP64 path is
timed on the same layouts and reported beside it.  Inputs (binary layouts)
are resident on the device before the timed region starts.

Prints one JSON line.  `--gpus N` with N > 1 is not supported (one GPU).
"""

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PSFD solves/s at rel. residual 1e-6 (mixed/batched vs FP64 plain); HBM GB/s"
HBM_PEAK_GBS = 8000.0
# Grazing cutoff of the multilayer response (|kz| < ML_KZ_MIN k0 gets none); 0 is the
# operator as defined (every order with |kz| >= 1e-9 k0 reflected); --ml-kz-min sets it.
ML_KZ_MIN = 0.0


def workload_name():
    cut = ("no grazing cutoff" if ML_KZ_MIN == 0.0 else f"grazing cutoff |kz|<{ML_KZ_MIN:g}k0")
    return ("256x256 lateral @2nm, 32 absorber cells / 60 nm (Nz=48), seeded line/space + "
            f"contact layouts, TE+TM, 6 deg, {cut}, tol 1e-6, plan+TMM+source+solve")


def layouts(n, nx, ny, dx):
    import numpy as np
    from psfd_synth import contact_holes, line_space
    out = []
    for i in range(n):
        rng = np.random.default_rng(100 + i)
        out.append(line_space(nx, ny, dx, rng) if i % 2 == 0 else contact_holes(nx, ny, dx, rng))
    return out


def run_steps(psfd, cfgs, a_dev, idx, prec, tol, maxit, profile=None, sched=None):
    """Solve every (layout, polarisation); returns list of infos and profile sums."""
    from psfd_synth import eps_absorber_default
    eps_abs = eps_absorber_default()
    infos = []
    prof = [0.0, 0, 0.0]
    for i in idx:
        for cfg in cfgs:
            eps = psfd.psfd_layout_eps(cfg, a_dev[i], eps_abs)
            plan = psfd.Plan(cfg, eps, prec)
            if sched is not None:
                plan.set_schedule(sched)
            if profile:
                plan.profile_enable(profile)
            _, info = plan.solve(tol=tol, maxit=maxit, check=False)
            if str(info["status"]).startswith("ERR"):
                raise RuntimeError(f"solve failed: {info['status']}: {psfd.lib().psfd_last_error().decode()}")
            if profile:
                ms, n, b = plan.profile_read()
                prof[0] += ms
                prof[1] += n
                prof[2] += b
            plan.close()
            infos.append(info)
    return infos, prof


def cpu_leg(iters_proj, sample_iters, layout_index=0):
    """Oracle timing on the host: setup + `sample_iters` BiCGSTAB iterations of one
    layout of the same workload (TE), projected to a full solve with the GPU's FP64
    iteration count.  The oracle as it stands: numpy FP64, pocketfft (one thread);
    the caller pins the BLAS/OpenMP threads to 1."""
    import numpy as np
    from oracle import psfd_ref as R
    from psfd_synth import config_c2, eps_absorber_default
    cfg = dict(config_c2(0), ml_kz_min=ML_KZ_MIN)
    a = layouts(layout_index + 1, cfg["nx"], cfg["ny"], cfg["dx"])[layout_index]
    t0 = time.perf_counter()
    P = R.Problem(cfg, R.eps_from_fill(cfg, R.smooth_layout(cfg, a), eps_absorber_default()))
    b = R.rhs(P)
    t1 = time.perf_counter()
    bnorm = float(np.linalg.norm(b))
    _, iters, _ = R.bicgstab_core(lambda u: R.apply_A(P, u), lambda u: R.apply_M(P, u), b, bnorm,
                                  1e-30, sample_iters)
    t2 = time.perf_counter()
    per_iter = (t2 - t1) / max(iters, 1)
    setup = t1 - t0
    return {"solve_s": setup + per_iter * iters_proj, "s_per_iteration": per_iter,
            "setup_s": setup, "iters": iters, "wall_s": t2 - t0}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(iters_proj, sample_iters, workers):
    """The oracle on the host, two modes: one process (one core), and `workers`
    single-threaded processes on different layouts at once (all cores of the
    share: aggregate solves/s).  Each process projects a full solve from a sample
    of iterations."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
               MKL_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")

    def spawn(k):
        return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--ml-kz-min", str(ML_KZ_MIN),
                                 "--cpu-leg", str(iters_proj), "--cpu-sample-iters", str(sample_iters),
                                 "--cpu-layout", str(k)], stdout=subprocess.PIPE,
                                stderr=subprocess.PIPE, text=True, env=env)

    def gather(procs):
        out = []
        for p in procs:
            so, se = p.communicate(timeout=900)
            if p.returncode != 0:
                raise RuntimeError(se[-500:])
            out.append(json.loads(so.strip().splitlines()[-1]))
        return out
    t = time.perf_counter()
    one = gather([spawn(0)])[0]
    t_one = time.perf_counter() - t
    t = time.perf_counter()
    many = gather([spawn(k % 4) for k in range(workers)])
    t_many = time.perf_counter() - t
    agg = sum(1.0 / r["solve_s"] for r in many)
    return {"value": round(agg, 6), "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": (f"numpy FP64 oracle (one thread per process), {workers} processes at once on "
                       f"the workload's layouts 0-3 (TE): setup + {sample_iters} BiCGSTAB iterations "
                       f"each, projected to {iters_proj:.0f} iterations (GPU FP64 mean); aggregate of "
                       f"the {workers} projected solve rates; wall {t_many:.1f} s"),
            "projected": True,
            "single_core": {"value": round(1.0 / one["solve_s"], 6), "unit": "solves/s", "cores": 1,
                            "s_per_iteration": round(one["s_per_iteration"], 3),
                            "setup_s": round(one["setup_s"], 2), "wall_s": round(t_one, 1)},
            "all_cores_s_per_iteration_mean": round(sum(r["s_per_iteration"] for r in many) / workers, 3),
            "host": {"os_cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
                     "threads_per_process": 1, "fft": "numpy.fft (pocketfft)"}}


# the files each timed kernel class is compiled from (the counter summaries record a hash)
KERNEL_SOURCES = {
    "xinv": ["cplx.h", "fft_core.h", "fft_lateral.hip", "psfd_internal.h", "reduce.h"],
    "xfwd": ["cplx.h", "fft_core.h", "fft_lateral.hip", "psfd_internal.h", "reduce.h"],
    "yfft": ["cplx.h", "fft_core.h", "fft_lateral.hip", "psfd_internal.h"],
    "axial": ["cplx.h", "fft_core.h", "lane_fft.h", "axial.hip", "psfd_internal.h"],
}
KERNEL_NAMES = {"axial": "k_axial_reg / k_axial (axial column kernel)", "xinv": "k_xfft_inv",
                "xfwd": "k_xfft_fwd", "yfft": "k_yfft"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_256x256x48_mixed.md")


def _sources_hash(kernel):
    """SHA-256 over a kernel class's sources (file name + bytes, sorted by name)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(KERNEL_SOURCES[kernel]):
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2607_25330_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _traffic_text():
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        return f.read()


def measured_traffic(kernel, sched):
    """HBM bytes per launch of `kernel` (schedule index `sched`) from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a device copy's readings),
    or None when there is none or the kernel's sources changed since."""
    import re
    text = _traffic_text()
    if text is None:
        return None
    sha = re.search(r"^sources_sha256 %s: ([0-9a-f]{64})$" % re.escape(kernel), text, re.M)
    row = re.search(r"^traffic_bytes_per_launch %s sched %d: ([0-9.eE+]+)$" % (re.escape(kernel), sched),
                    text, re.M)
    if not sha or not row or sha.group(1) != _sources_hash(kernel):
        return None
    return float(row.group(1))


def measured_iteration_traffic():
    """Counter bytes of one complex64 BiCGSTAB iteration (all its kernels) from the
    committed summary, or None when any kernel class changed since."""
    import re
    text = _traffic_text()
    if text is None:
        return None
    for k in KERNEL_SOURCES:
        sha = re.search(r"^sources_sha256 %s: ([0-9a-f]{64})$" % re.escape(k), text, re.M)
        if not sha or sha.group(1) != _sources_hash(k):
            return None
    row = re.search(r"^traffic_bytes_per_iteration: ([0-9.eE+]+)$", text, re.M)
    return float(row.group(1)) if row else None


def copy_peak_gbs(dev, mib=1024, reps=5):
    """Device-to-device copy rate (read + write bytes / time) of a `mib` MiB buffer."""
    import torch
    n = mib * 1024 * 1024 // 16
    src = torch.ones(n, dtype=torch.complex128, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 1e30
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    return 2.0 * mib * 1024 * 1024 / (best * 1e-3) / 1e9


def _sync_time(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def workload_c1(psfd, args):
    """32x32 lateral, 16 absorber cells / 30 nm (Nz = 32), 6 deg TE, plain FP64 to 1e-10."""
    import numpy as np
    import torch
    from psfd_synth import config_c1, eps_absorber_default, rect_layout
    dev = torch.device("cuda:0")
    cfg = config_c1(0)
    lays = [torch.from_numpy(rect_layout(32, 32, np.random.default_rng(s))).to(dev)
            for s in range(args.warmup + args.steps)]

    def one(a):
        eps = psfd.psfd_layout_eps(cfg, a, eps_absorber_default())
        plan = psfd.Plan(cfg, eps, psfd.PSFD_C128)
        _, info = plan.solve(tol=1e-10, maxit=args.maxit, check=False)
        plan.close()
        return info
    for a in lays[args.steps:]:
        one(a)
    infos, dt = _sync_time(lambda: [one(a) for a in lays[:args.steps]])
    return {"metric": METRIC, "value": round(args.steps / dt, 3), "unit": "solves/s",
            "ms_per_solve": round(1e3 * dt / args.steps, 2), "dtype": "f64",
            "config": {"workload": "32x32x(16+16), 2 nm, 30 nm absorber, 6 deg TE, FP64, tol 1e-10, "
                                   "seeded rectangles (seeds 0..)"},
            "iters": [i["iters"] for i in infos],
            "converged": all(i["status"] == "OK" for i in infos)}


def workload_c3(psfd, args):
    """Batched uneven solves: seeded rectangle clips of {64,128,192,256}^2 x 48 x 5 angles x 2
    polarisations, mixed precision and plain FP64, each through psfd_solve_batch; solves/s and
    the cost per voxel-iteration (to compare with the single 256^2 solve)."""
    import numpy as np
    import torch
    from psfd_synth import base_config, config_c3_sizes, eps_absorber_default, rect_layout
    dev = torch.device("cuda:0")
    # the solver reports each Krylov run's end on stderr (progress of a long batch)
    os.environ.setdefault("PSFD_TRACE", "1")
    sizes, angles, pols = config_c3_sizes()
    rng = np.random.default_rng(300)
    cfgs, eps, per_size = [], [], {}
    for c in range(args.c3_clips):
        n = int(rng.choice(sizes))
        per_size[n] = per_size.get(n, 0) + 1
        a = torch.from_numpy(rect_layout(n, n, np.random.default_rng(1000 + c))).to(dev)
        for th in angles:
            for pol in pols:
                cfg = dict(base_config(n, n, 32, 60.0, theta_deg=th, pol=pol), ml_kz_min=ML_KZ_MIN)
                cfgs.append(cfg)
                eps.append(psfd.psfd_layout_eps(cfg, a, eps_absorber_default()))
    vox = [c["nx"] * c["ny"] * (c["nz_abs"] + 16) for c in cfgs]
    legs = {}
    for name, prec in (("mixed", psfd.PSFD_C64_REFINE64), ("fp64", psfd.PSFD_C128)):
        batch = psfd.Batch(cfgs, eps, prec=prec)
        (E, infos), dt = _sync_time(lambda: batch.solve(tol=args.tol, maxit=args.maxit, check=False))
        batch.close()
        del E
        vit = sum(v * i["iters"] for v, i in zip(vox, infos))
        legs[name] = {"solves_per_s": round(len(cfgs) / dt, 3), "seconds": round(dt, 2),
                      "iters_mean": round(sum(i["iters"] for i in infos) / len(infos), 1),
                      "iters_max": max(i["iters"] for i in infos),
                      "converged": sum(i["status"] == "OK" for i in infos),
                      "ns_per_voxel_iteration": round(1e9 * dt / vit, 4)}
        _log(f"c3 {name}: {legs[name]}")
    cut = "no grazing cutoff" if ML_KZ_MIN == 0 else f"grazing cutoff {ML_KZ_MIN:g}"
    return {"metric": METRIC, "value": legs["mixed"]["solves_per_s"], "unit": "solves/s",
            "dtype": "f32+f64", "legs": legs,
            "mixed_vs_fp64": round(legs["fp64"]["seconds"] / legs["mixed"]["seconds"], 3),
            "config": {"workload": f"{args.c3_clips} seeded rectangle clips, lateral sizes from "
                                   "{64,128,192,256}^2, Nz 48, x 5 angles (0-10 deg) x TE/TM, "
                                   f"tol {args.tol:g}, batched (psfd_solve_batch), " + cut,
                       "solves": len(cfgs), "clips_per_size": per_size, "voxels": sum(vox),
                       "workers": int(os.environ.get("PSFD_BATCH_WORKERS", "2"))}}


def _smooth_noise(shape, seed, dev, sigma_cells=8.0):
    """Seeded complex noise on the device, Gaussian-filtered over the lateral axes
    (periodic, std sigma_cells) - the warm-start perturbation at full size."""
    import torch
    g = torch.Generator(device=dev).manual_seed(seed)
    z = torch.complex(torch.randn(shape, generator=g, device=dev, dtype=torch.float64),
                      torch.randn(shape, generator=g, device=dev, dtype=torch.float64))
    fy = torch.fft.fftfreq(shape[-2], device=dev, dtype=torch.float64)
    fx = torch.fft.fftfreq(shape[-1], device=dev, dtype=torch.float64)
    h = torch.exp(-2.0 * (torch.pi * sigma_cells) ** 2 * (fy[:, None] ** 2 + fx[None, :] ** 2))
    for c in range(shape[0]):
        z[c] = torch.fft.ifft2(torch.fft.fft2(z[c]) * h)
    return z


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload_c4(psfd, args):
    """1024x1024 lateral, 48 absorber cells / 70 nm (Nz = 64), curvilinear layout, 6 deg, TE and
    TM: FP64 reference to 1e-9, then mixed solves (complex64 Krylov; and the bf16 preconditioner
    trial, the damped spectrum held in bfloat16) from null and from a warm start (reference +
    smooth complex noise scaled to r_rel ~ 0.1), and the plain FP64 solve."""
    import numpy as np
    import torch
    from psfd_synth import config_c4, curvilinear, eps_absorber_default
    dev = torch.device("cuda:0")
    # the solver reports its residual every 512 iterations on stderr (long solves at this size)
    os.environ.setdefault("PSFD_TRACE", "2")
    a = torch.from_numpy(curvilinear(1024, 1024, np.random.default_rng(400))).to(dev)
    out = {"metric": METRIC, "unit": "solves/s", "dtype": "f32+f64",
           "config": {"workload": "1024x1024x(48+16), 2 nm, 70 nm absorber, curvilinear, 6 deg, "
                                  "no grazing cutoff, tol %g" % args.tol}, "legs": {}}
    for pol in (0, 1):
        cfg = dict(config_c4(pol), ml_kz_min=ML_KZ_MIN)
        eps = psfd.psfd_layout_eps(cfg, a, eps_absorber_default())
        ref = psfd.Plan(cfg, eps, psfd.PSFD_C128)

        (E_ref, i_ref), t_ref = _sync_time(lambda: ref.solve(tol=1e-9, maxit=args.maxit, check=False))
        _log(f"c4 pol {pol} fp64 reference: {i_ref['iters']} it, {t_ref:.2f} s, {i_ref['status']}")
        b = ref.rhs()
        bn = float(torch.linalg.vector_norm(b))
        d = _smooth_noise((3, ref.nz, 1024, 1024), 401 + pol, dev)
        r_d, _ = ref.residual(d, b=torch.zeros_like(b))  # -A d
        s = 0.1 * bn / float(torch.linalg.vector_norm(r_d))
        x0 = (E_ref + s * d).contiguous()
        del d, r_d
        _, rr0 = ref.residual(x0)
        leg = {"fp64_ref_iters": i_ref["iters"], "fp64_ref_s": round(t_ref, 3),
               "x0_rrel": round((rr0 ** 0.5) / bn, 4)}
        for name, prec, warm in [("mixed_null", psfd.PSFD_C64_REFINE64, False),
                                 ("mixed_warm", psfd.PSFD_C64_REFINE64, True),
                                 ("bf16pc_warm", psfd.PSFD_C64_BF16PC_REFINE64, True),
                                 ("fp64_null", psfd.PSFD_C128, False)]:
            plan = psfd.Plan(cfg, eps, prec)
            (E, info), dt = _sync_time(lambda: plan.solve(x0=x0 if warm else None, tol=args.tol,
                                                          maxit=args.maxit, check=False))
            _log(f"c4 pol {pol} {name}: {info['iters']} it, {dt:.2f} s, {info['status']}")
            err = float(torch.linalg.vector_norm(E - E_ref) / torch.linalg.vector_norm(E_ref))
            leg[name] = {"iters": info["iters"], "s": round(dt, 3), "status": info["status"],
                         "rrel": info["rrel"], "field_err_vs_ref": err}
            plan.close()
            del E
        ref.close()
        out["legs"]["TE" if pol == 0 else "TM"] = leg
    te = out["legs"]["TE"]["mixed_warm"]["s"] + out["legs"]["TM"]["mixed_warm"]["s"]
    out["value"] = round(2 / te, 4)
    return out


def workload_c5(psfd, args):
    """Gradients: 16 clips 128x128x(32+16), TE 6 deg; gradient of the summed observation-row
    intensity w.r.t. eps through the autograd wrapper (mixed forward + adjoint solves)."""
    import numpy as np
    import torch
    from paper_2607_25330_amd.autograd import scattered_field
    from psfd_synth import config_c5, eps_absorber_default, rect_layout
    dev = torch.device("cuda:0")
    cfg = dict(config_c5(), ml_kz_min=ML_KZ_MIN)
    jobs = cfg["nz_pml"] + cfg["nz_gap_bot"] + cfg["nz_abs"]
    eps = [psfd.psfd_layout_eps(cfg, torch.from_numpy(rect_layout(128, 128, np.random.default_rng(500 + c))).to(dev),
                                eps_absorber_default()) for c in range(16)]

    def grads():
        out = []
        for e in eps:
            x = e.clone().requires_grad_(True)
            E = scattered_field(x, cfg, prec=psfd.PSFD_C64_REFINE64, tol=args.tol)
            (E[:, jobs].abs() ** 2).sum().backward()
            out.append(x.grad)
        return out
    grads()
    g, dt = _sync_time(grads)
    return {"metric": "gradient evaluations/s (forward + adjoint solve)", "value": round(16 / dt, 3),
            "unit": "gradients/s", "dtype": "f32+f64",
            "config": {"workload": "16 seeded rectangle clips 128x128x(32+16), TE 6 deg, d(sum |E|^2 "
                                   "on the observation row)/d eps, mixed, tol %g" % args.tol}}


def workload_fd(psfd, args):
    """Standard full-domain PSFD (the whole 40-bilayer Mo/Si stack discretised on the grid, no
    multilayer operator) next to the background-decomposed solve.
    (1) bare stack, 16x16 lateral, 1 and 0.5 nm grids (Nz 324 / 648), TE at the four angles a
        150 nm periodic cell represents: reflection against the transfer matrix, iterations, time;
    (2) one seeded absorber layout, 128x128 lateral at 1 nm, 50 nm absorber, TE normal incidence:
        background-decomposed grid (Nz 96) against the full-domain grid with the stack under the
        absorber (Nz 384): iterations, solve time, device memory, specular reflection at the
        absorber's top face, and the tall axial kernel's bandwidth (launch-packet events).  The
        decomposed grid runs on the operator as defined and, for comparison, with a 0.1 k0
        grazing cutoff."""
    import math
    import numpy as np
    import torch
    from psfd_synth import (FULL_DOMAIN_THETAS_DEG, base_config, eps_absorber_default,
                            full_domain_config, full_domain_stack, rect_layout)
    dev = torch.device("cuda:0")
    eps_l, d_l = full_domain_stack()
    out = {"metric": "full-domain vs background-decomposed PSFD", "unit": "solves/s",
           "dtype": "f64", "legs": {"bare_stack": [], "absorber": {}},
           "config": {"workload": "bare 40-bilayer Mo/Si stack, 16x16 lateral, dz 1 and 0.5 nm, TE, "
                                  "4 angles, tol 1e-8; 128x128x(50 nm absorber) at 1 nm, TE normal "
                                  "incidence, decomposed (Nz 96, no grazing cutoff, and cutoff 0.1 "
                                  "for comparison) vs full-domain (Nz 384), tol %g"
                                  % args.tol}}
    t_bare = 0.0
    for dz in (1.0, 0.5):
        for th in FULL_DOMAIN_THETAS_DEG:
            cfg = full_domain_config(dz, th, 0, nx=16)
            eps = psfd.psfd_layered_eps(cfg, eps_l, d_l, dev)
            plan = psfd.Plan(cfg, eps, psfd.PSFD_C128)
            plan.solve(tol=1e-8, maxit=args.maxit)
            (E, info), dt = _sync_time(lambda: plan.solve(tol=1e-8, maxit=args.maxit))
            r = plan.specular(E)
            plan.close()
            r_tmm = _tmm_te(psfd, cfg, eps_l, d_l, dev)
            t_bare += dt
            leg = {"dz": dz, "theta_deg": round(th, 2), "nz": plan.nz, "iters": info["iters"],
                   "ms": round(1e3 * dt, 2), "R": round(abs(r) ** 2, 5),
                   "arg_r": round(math.atan2(r.imag, r.real), 4), "R_tmm": round(abs(r_tmm) ** 2, 5),
                   "arg_r_tmm": round(math.atan2(r_tmm.imag, r_tmm.real), 4),
                   "abs_r_minus_tmm": float(abs(r - r_tmm))}
            _log(f"fd bare dz {dz} theta {th:.2f}: {leg}")
            out["legs"]["bare_stack"].append(leg)
    # (2) absorber layout on the stack
    a = torch.from_numpy(rect_layout(128, 128, np.random.default_rng(700), wmin=8, wmax=48)).to(dev)
    cfg_d = base_config(128, 128, 50, 50.0, dx=1.0, theta_deg=0.0, pol=0, nz_pml=12, nz_gap=11)
    cfg_f = dict(cfg_d, ml_eps=[], ml_thick=[], eps_sub=1.0 + 0j, nz_abs=330, nz_gap_bot=15,
                 nz_gap_top=15)
    eps_abs = psfd.psfd_layout_eps(cfg_d, a, eps_absorber_default())
    cfg_s = dict(cfg_f, nz_abs=280)
    eps_f = torch.cat([psfd.psfd_layered_eps(cfg_s, eps_l, d_l, dev), eps_abs], dim=0).contiguous()
    res = {}
    cfg_dc = dict(cfg_d, ml_kz_min=0.1)
    for name, cfg, eps in (("decomposed", cfg_d, eps_abs), ("decomposed_cutoff_0.1", cfg_dc, eps_abs),
                           ("full_domain", cfg_f, eps_f)):
        for prec_name, prec in (("fp64", psfd.PSFD_C128), ("mixed", psfd.PSFD_C64_REFINE64)):
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            plan = psfd.Plan(cfg, eps, prec)
            (E, info), dt = _sync_time(lambda: plan.solve(tol=args.tol, maxit=args.maxit, check=False))
            used = (free0 - torch.cuda.mem_get_info()[0]) / 2 ** 30
            r = plan.specular(E)
            leg = {"nz": plan.nz, "iters": info["iters"], "status": info["status"],
                   "s": round(dt, 3), "device_GiB": round(used, 2), "R": round(abs(r) ** 2, 5),
                   "arg_r": round(math.atan2(r.imag, r.real), 4)}
            if prec_name == "fp64":
                plan.profile_enable("axial")
                for _ in range(10):
                    plan.apply(E)
                torch.cuda.synchronize()
                ms, nl, by = plan.profile_read()
                plan.profile_enable("off")
                leg["axial_us"] = round(1e3 * ms / max(nl, 1), 2)
                leg["axial_GBs"] = round(by / max(ms, 1e-12) / 1e6, 1)
            _log(f"fd absorber {name} {prec_name}: {leg}")
            res[f"{name}_{prec_name}"] = leg
            plan.close()
            del E
    out["legs"]["absorber"] = res
    out["value"] = round(8 / t_bare, 3)
    fl = res.get("full_domain_fp64", {})
    if "axial_GBs" in fl:
        out["roofline"] = {"bound": "hbm", "achieved": fl["axial_GBs"], "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(fl["axial_GBs"] / HBM_PEAK_GBS, 4),
                           "traffic": None, "kernel": "axial (LDS-staged, Nz 384, FP64 A apply)",
                           "avg_launch_us": fl["axial_us"]}
    return out


def workload_contour(psfd, args):
    """Practical convergence by threshold-contour widths: 8 seeded 256x256x48 clips (line/space
    and contacts alternating), TE 6 deg, grazing cutoff --ml-kz-min.  Reference: FP64 solve to r_rel 1e-7.
    Mixed solves stopped after k iterations (k = 50 ... 1600) and run to 1e-6: |delta d| at wafer
    scale (/4) over 100 horizontal + 100 vertical scan lines of |E_y|^2 on the observation row
    (S(I) with I_th 0.15, w 0.05), and the metric kernels' own time for the 8 planes."""
    import numpy as np
    import torch
    from psfd_synth import config_c2, eps_absorber_default
    dev = torch.device("cuda:0")
    cfg = dict(config_c2(0), ml_kz_min=ML_KZ_MIN)
    nx, ny, dx = cfg["nx"], cfg["ny"], cfg["dx"]
    jobs = cfg["nz_pml"] + cfg["nz_gap_bot"] + cfg["nz_abs"]
    lays = [torch.from_numpy(a).to(dev) for a in layouts(8, nx, ny, dx)]
    eps = [psfd.psfd_layout_eps(cfg, a, eps_absorber_default()) for a in lays]
    refs = []
    for e in eps:
        plan = psfd.Plan(cfg, e, psfd.PSFD_C128)
        E, info = plan.solve(tol=1e-7, maxit=args.maxit)
        refs.append(E[1, jobs].clone())
        plan.close()
    ref_planes = torch.stack(refs)
    seg_ref = psfd.contour_segments(ref_planes, dx, dx)
    checkpoints = [50, 100, 200, 400, 800, 1600, None]
    legs = []
    for k in checkpoints:
        planes, iters, rrel = [], [], []
        for e in eps:
            plan = psfd.Plan(cfg, e, psfd.PSFD_C64_REFINE64)
            E, info = plan.solve(tol=1e-6 if k is None else 1e-12, maxit=args.maxit if k is None else k,
                                 check=False)
            planes.append(E[1, jobs].clone())
            iters.append(info["iters"])
            rrel.append(info["rrel"])
            plan.close()
        seg_k = psfd.contour_segments(torch.stack(planes), dx, dx)
        _, st = psfd.contour_deviation(seg_ref, seg_k, nx, ny, dx, dx, demag=4.0, thr=1.0)
        leg = {"iters": "to 1e-6" if k is None else k, "mean_iters": float(np.mean(iters)),
               "median_rrel": float(np.median(rrel)), "mean_abs_dd_nm": st["mean_abs"],
               "std_abs_dd_nm": st["std_abs"], "resolved": st["resolved"],
               "unresolved": st["unresolved"], "above_1nm": st["above_thr"]}
        _log(f"contour k={k}: {leg}")
        legs.append(leg)
    # metric kernels alone (8 planes, 200 lines each)
    for _ in range(3):
        psfd.contour_deviation(seg_ref, psfd.contour_segments(ref_planes, dx, dx), nx, ny, dx, dx)
    (_, dt) = _sync_time(lambda: [psfd.contour_segments(ref_planes, dx, dx) for _ in range(20)])
    seg_t = dt / 20
    (_, dt2) = _sync_time(lambda: [psfd.contour_deviation(seg_ref, seg_ref, nx, ny, dx, dx)
                                   for _ in range(20)])
    return {"metric": "threshold-contour width deviation vs iterations", "unit": "planes/s",
            "value": round(8 / seg_t, 1), "dtype": "f64", "legs": legs,
            "segments_ms_8_planes": round(1e3 * seg_t, 4),
            "roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "traffic": None,
                         "kernel": "contour segments (8 planes, 200 lines of 256 samples each)",
                         "achieved": round(8 * 200 * 256 * 16 / seg_t / 1e9, 1),
                         "frac": round(8 * 200 * 256 * 16 / seg_t / 1e9 / HBM_PEAK_GBS, 5),
                         "note": "one launch per call: latency-bound, not bandwidth-bound"},
            "deviation_ms_8_planes": round(1e3 * dt2 / 20, 4),
            "segments_per_ref_plane": float(seg_ref[1].sum().item()) / 8,
            "config": {"workload": f"8 seeded 256x256x(32+16) clips, TE 6 deg, cutoff {ML_KZ_MIN:g}; "
                                   "reference FP64 1e-7; mixed stopped at k iterations; 100+100 scan "
                                   "lines, I_th 0.15, w 0.05, /4 demag"}}


def workload_pino(psfd, args):
    """The paper's physics loss with the high-frequency penalty, as PINO training evaluates it:
    16 seeded 128x128x(32+16) clips, TE 6 deg, one field per clip (a solve's output plus smooth
    noise, standing in for a network prediction); loss + gradients with respect to the field and
    the permittivity through the autograd wrapper (w0 1, eta_hf 10 nm, lambda_hf 0.01).  Also
    the loss kernels' own time: residual, weighted spectral pass, gradient combine, adjoint."""
    import numpy as np
    import torch
    from paper_2607_25330_amd.autograd import pino_loss
    from psfd_synth import config_c5, eps_absorber_default, rect_layout
    dev = torch.device("cuda:0")
    cfg = dict(config_c5(), ml_kz_min=ML_KZ_MIN)
    w0, eta, lam = 1.0, 10.0, 0.01
    eps = [psfd.psfd_layout_eps(cfg, torch.from_numpy(rect_layout(128, 128, np.random.default_rng(900 + c))).to(dev),
                                eps_absorber_default()) for c in range(16)]
    fields = []
    for c, e in enumerate(eps):
        plan = psfd.Plan(cfg, e, psfd.PSFD_C64_REFINE64)
        E, _ = plan.solve(tol=1e-6, maxit=args.maxit)
        plan.close()
        fields.append((E + 0.05 * _smooth_noise(E.shape, 950 + c, dev, sigma_cells=4.0)).contiguous())

    def step():
        out = []
        for E, e in zip(fields, eps):
            Et = E.clone().requires_grad_(True)
            et = e.clone().requires_grad_(True)
            J = pino_loss(Et, et, cfg, w0, eta, lam)
            J.backward()
            out.append((float(J), Et.grad, et.grad))
        return out
    step()
    res, dt = _sync_time(step)
    # the library calls alone on one plan (no plan setup, no autograd bookkeeping)
    plan = psfd.Plan(cfg, eps[0], psfd.PSFD_C128)
    E = fields[0]
    for _ in range(3):
        _, g = plan.pino_loss(E, w0, eta, lam)
        plan.adjoint(g)
    (_, dt_loss) = _sync_time(lambda: [plan.pino_loss(E, w0, eta, lam) for _ in range(20)])
    (_, dt_adj) = _sync_time(lambda: [plan.adjoint(g) for _ in range(20)])
    (_, dt_apply) = _sync_time(lambda: [plan.apply(E) for _ in range(20)])
    plan.close()
    vox = 3 * 128 * 128 * 48
    return {"metric": "physics-loss evaluations/s (loss + field and permittivity gradients)",
            "value": round(16 / dt, 2), "unit": "evaluations/s", "dtype": "f64",
            "loss_ms": round(1e3 * dt_loss / 20, 3), "adjoint_ms": round(1e3 * dt_adj / 20, 3),
            "apply_ms": round(1e3 * dt_apply / 20, 3),
            "loss_terms_clip0": {"J": res[0][0]}, "voxels": vox,
            "roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "traffic": None,
                         "kernel": "one psfd_pino_loss call (FP64), counted as its 8 field passes "
                                   "(read E, b; write r; read r, write H r; read r, H r, write g)",
                         "achieved": round(8 * 16 * vox / (dt_loss / 20) / 1e9, 1),
                         "frac": round(8 * 16 * vox / (dt_loss / 20) / 1e9 / HBM_PEAK_GBS, 4)},
            "config": {"workload": "16 seeded rectangle clips 128x128x(32+16), TE 6 deg, field = "
                                   "mixed solve + smooth noise; J = (1/N)||r||^2 + (lambda/N)"
                                   "||w F3 r||^2, w0 1, eta 10 nm, lambda 0.01; autograd"}}


def workload_ffno(psfd, args):
    """Factorised Fourier neural operator forward pass (seeded random weights; no trained
    weights exist): d_v 32, d_h 64, 4 layers, modes kx 12, |ky| 12, kz 8, on the 256x256x48
    solver grid and on the paper's 1200x1200x100 inference grid.  The dominant kernel is the
    fused axial branch + MLP (2 d_v d_h multiply-adds per voxel for the MLP); it is timed with
    torch events around the whole forward pass and reported against the FP32 vector peak."""
    import numpy as np
    import torch
    from psfd_synth import ffno_desc, ffno_weights
    dev = torch.device("cuda:0")
    out = {"metric": "F-FNO forward passes/s", "unit": "forwards/s", "dtype": "f32", "legs": {}}
    grids = {"256x256x48": (256, 256, 48), "1200x1200x100": (1200, 1200, 100)}
    for name in args.ffno_grids.split(","):
        nx, ny, nz = grids[name]
        d = ffno_desc(nx, ny, nz, d_v=32, d_h=64, n_layers=4, kx_max=12, ky_max=12, kz_max=8)
        w = torch.from_numpy(ffno_weights(d, 1234)).to(dev)
        net = psfd.Ffno(d, w)
        g = torch.Generator(device=dev).manual_seed(5)
        a = torch.rand((nz, ny, nx), generator=g, device=dev, dtype=torch.float32)
        E = net(a)
        for _ in range(2):
            net(a, out=E)
        reps = 5 if nx < 1000 else 2
        _, dt = _sync_time(lambda: [net(a, out=E) for _ in range(reps)])
        vox = nx * ny * nz
        mlp_flop = 4 * vox * 2 * 2 * 32 * 64
        leg = {"ms": round(1e3 * dt / reps, 3), "voxels": vox, "mlp_tflop": round(mlp_flop / 1e12, 3),
               "mlp_tflops_if_all_time": round(mlp_flop / (dt / reps) / 1e12, 2),
               "workspace_GiB": round(net.workspace.numel() / 2 ** 30, 2),
               "finite": bool(torch.isfinite(E.real).all().item())}
        _log(f"ffno {name}: {leg}")
        out["legs"][name] = leg
        del net, E, a
        torch.cuda.empty_cache()
    last = out["legs"].get("1200x1200x100") or next(iter(out["legs"].values()))
    out["value"] = round(1e3 / last["ms"], 3)
    mlp = last["mlp_tflop"] / (last["ms"] / 1e3)
    out["roofline"] = {"bound": "alu", "unit": "TFLOP/s", "peak": 157.3, "traffic": None,
                       "kernel": "whole forward pass, counted as its MLP flops only",
                       "achieved": round(mlp, 2), "frac": round(mlp / 157.3, 4),
                       "note": "per-kernel figures in the rocprofv3 summary"}
    out["config"] = {"workload": "F-FNO d_v 32, d_h 64, 4 layers, modes (12, 12, 8), random "
                                 "weights; 256x256x48 and 1200x1200x100 (value: the latter)"}
    return out


def workload_paper_grid(psfd, args):
    """The paper's solver workload at the nearest supported grid: its 1200x1200 nm cell at
    1 nm and 100 axial rows of 2 nm become 1024x1024 lateral (1.17 nm) x 96 rows (2 nm): a 50 nm
    absorber (25 rows), 12-row PMLs, gaps; TE normal incidence, grazing cutoff --ml-kz-min; one seeded
    curvilinear layout.  Mixed and FP64 solves to r_rel 5e-2 (the paper's criterion for its
    iteration counts) and to 1e-4 (iteration budget 4000): iterations, seconds, seconds per
    iteration."""
    import numpy as np
    import torch
    from psfd_synth import base_config, curvilinear, eps_absorber_default
    dev = torch.device("cuda:0")
    cfg = dict(base_config(1024, 1024, 25, 50.0, dx=1200.0 / 1024, theta_deg=0.0, pol=0,
                           nz_pml=12, nz_gap=23), ml_kz_min=ML_KZ_MIN)
    cfg["nz_gap_top"] = 96 - 25 - 24 - 23
    a = torch.from_numpy(curvilinear(1024, 1024, np.random.default_rng(1200))).to(dev)
    eps = psfd.psfd_layout_eps(cfg, a, eps_absorber_default())
    out = {"metric": "seconds per BiCGSTAB iteration at the paper's solver grid (stand-in)",
           "unit": "s/iteration", "higher_is_better": False, "dtype": "f32+f64", "legs": {}}
    runs = [("mixed", psfd.PSFD_C64_REFINE64, 5e-2, 2000), ("fp64", psfd.PSFD_C128, 5e-2, 2000),
            ("mixed", psfd.PSFD_C64_REFINE64, 1e-4, 4000), ("fp64", psfd.PSFD_C128, 1e-4, 4000)]
    for prec_name, prec, tol, maxit in runs:
        plan = psfd.Plan(cfg, eps, prec)
        plan.solve(tol=0.5, maxit=2, check=False)   # first-use allocations and graph capture
        (E, info), dt = _sync_time(lambda: plan.solve(tol=tol, maxit=maxit, check=False))
        plan.close()
        leg = {"iters": info["iters"], "s": round(dt, 3), "status": info["status"],
               "rrel": info["rrel"], "s_per_iter": round(dt / max(info["iters"], 1), 5)}
        _log(f"paper grid {prec_name} tol {tol}: {leg}")
        out["legs"][f"{prec_name}_tol{tol:g}"] = leg
        del E
    out["value"] = out["legs"]["mixed_tol0.05"]["s_per_iter"]
    out["config"] = {"workload": "1024x1024x96 (1.17 x 1.17 x 2 nm), 50 nm absorber, TE normal "
                                 f"incidence, curvilinear layout, cutoff {ML_KZ_MIN:g}; the paper: "
                                 "1200x1200x100 at 1 x 1 x 2 nm"}
    return out


def _tmm_te(psfd, cfg, eps_l, d_l, dev):
    """Transfer-matrix reflection of the bare stack between vacuum half-spaces (TE), from the
    library's own per-mode table of a plan that carries the stack as its multilayer."""
    import torch
    c = dict(cfg, ml_eps=list(eps_l), ml_thick=list(d_l), eps_sub=1.0 + 0j, nz_abs=8,
             nz_gap_bot=2, nz_gap_top=2)
    c["nz_pml"] = (32 - 12) // 2
    plan = psfd.Plan(c, torch.ones((8, c["ny"], c["nx"]), dtype=torch.complex128, device=dev))
    rte, _ = plan.ml_reflection()
    r = complex(rte[0, 0].item())
    plan.close()
    return r


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--ml-kz-min", type=float, default=0.0,
                    help="grazing cutoff of the multilayer response in units of k0 (0: none)")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--maxit", type=int, default=20000)
    ap.add_argument("--roofline-kernel", default="xinv", choices=["axial", "yfft", "xfwd", "xinv"],
                    help="kernel class timed for the roofline object (the dominant one by rocprof)")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the untimed kernel-timing leg (no roofline object)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 leg")
    ap.add_argument("--no-tune", action="store_true",
                    help="default kernel schedules instead of the autotuner's (psfd_tune)")
    ap.add_argument("--schedule", default=None,
                    help="fixed kernel schedule of the mixed leg, 'xf,xi,y,ax' (no tuning)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=4)
    ap.add_argument("--cpu-leg", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-layout", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="oracle processes of the all-core CPU baseline (the box's CPU share)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (for counter calibration)")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "fd", "contour", "pino", "ffno",
                                                 "paper_grid"],
                    help="c2 (default) is the headline line; the others print their own line")
    ap.add_argument("--c3-clips", type=int, default=64)
    ap.add_argument("--ffno-grids", default="256x256x48,1200x1200x100",
                    help="grids of the ffno workload (comma-separated)")
    args = ap.parse_args()
    global ML_KZ_MIN
    ML_KZ_MIN = args.ml_kz_min

    if args.cpu_leg is not None:
        print(json.dumps(cpu_leg(args.cpu_leg, args.cpu_sample_iters, args.cpu_layout)))
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the PSFD solve here is a single-GPU path "
              "(independent solves shard trivially across GPUs). "
              "Run with --gpus 1.", file=sys.stderr)
        return 2

    forced = tuple(int(v) for v in args.schedule.split(",")) if args.schedule else None
    if not args.no_tune and forced is None:
        # plans pick up the autotuner's schedules (tuned once per shape, before timing)
        os.environ["PSFD_TUNE"] = "1"
    import torch
    import paper_2607_25330_amd as psfd
    from psfd_synth import config_c2

    if args.workload != "c2":
        fn = {"c1": workload_c1, "c3": workload_c3, "c4": workload_c4, "c5": workload_c5,
              "fd": workload_fd, "contour": workload_contour, "pino": workload_pino,
              "ffno": workload_ffno, "paper_grid": workload_paper_grid}[args.workload]
        res = fn(psfd, args)
        res.setdefault("higher_is_better", True)
        res.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
                    "vs_baseline": None})
        print(json.dumps(res), flush=True)
        return 0

    dev = torch.device("cuda:0")
    cfgs = [dict(config_c2(pol), ml_kz_min=ML_KZ_MIN) for pol in (0, 1)]
    nx, ny, dx = cfgs[0]["nx"], cfgs[0]["ny"], cfgs[0]["dx"]
    K, W = args.steps, args.warmup
    a_dev = [torch.from_numpy(a).to(dev) for a in layouts(W + K, nx, ny, dx)]
    torch.cuda.synchronize()
    print(f"bench: workload ready ({W} warmup + {K} timed steps, 2 solves each)",
          file=sys.stderr, flush=True)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * 1024 * 1024 // 16
        src = torch.ones(n, dtype=torch.complex128, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    prec_mixed = psfd.PSFD_C64_REFINE64
    schedules = {}
    if forced is not None:
        schedules["mixed"] = list(forced)
    elif not args.no_tune:
        from psfd_synth import eps_absorber_default
        eps0 = psfd.psfd_layout_eps(cfgs[0], a_dev[0], eps_absorber_default())
        for name, prec in (("mixed", prec_mixed), ("fp64", psfd.PSFD_C128)):
            plan = psfd.Plan(cfgs[0], eps0, prec)
            schedules[name] = list(plan.tune())
            plan.close()
        del eps0
        torch.cuda.synchronize()
    if W:
        run_steps(psfd, cfgs, a_dev, range(K, K + W), prec_mixed, args.tol, args.maxit, sched=forced)
        if not args.no_fp64:
            run_steps(psfd, cfgs, a_dev, range(K, K + W), psfd.PSFD_C128, args.tol, args.maxit)
    torch.cuda.synchronize()

    # ---- timed: mixed precision (headline); both timed legs replay graph-captured chunks
    t0 = time.perf_counter()
    infos_m, _ = run_steps(psfd, cfgs, a_dev, range(K), prec_mixed, args.tol, args.maxit,
                           sched=forced)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    print(f"bench: mixed leg {t_mixed:.3f} s", file=sys.stderr, flush=True)

    res = {}
    if not args.no_fp64:
        t0 = time.perf_counter()
        infos_d, _ = run_steps(psfd, cfgs, a_dev, range(K), psfd.PSFD_C128, args.tol, args.maxit)
        torch.cuda.synchronize()
        t_fp64 = time.perf_counter() - t0
        print(f"bench: fp64 leg {t_fp64:.3f} s", file=sys.stderr, flush=True)
        res["fp64"] = (t_fp64, infos_d)

    # ---- untimed: the same mixed solves again with the roofline kernel's launches timed
    # by HIP events that its launch packets record on the solver's stream (the chunks
    # then run without graph replay; the kernels are the same)
    prof_kernel = None if args.no_profile else args.roofline_kernel
    prof = (0.0, 0, 0.0)
    if prof_kernel is not None:
        # (the first four steps: the kernel's average per launch does not need all of them)
        infos_p, prof = run_steps(psfd, cfgs, a_dev, range(min(K, 4)), prec_mixed, args.tol,
                                  args.maxit, profile=prof_kernel, sched=forced)
        torch.cuda.synchronize()
        print(f"bench: profiled leg: {prof[1]} launches of {prof_kernel}", file=sys.stderr, flush=True)

    # ---- untimed: one complex64 operator apply, the device copy rate
    nz = cfgs[0]["nz_abs"] + 16
    vox = nx * ny * nz                      # voxels of one problem
    eps0 = psfd.psfd_layout_eps(cfgs[0], a_dev[0], __import__("psfd_synth").eps_absorber_default())
    plan = psfd.Plan(cfgs[0], eps0, prec_mixed)
    if forced is not None:
        plan.set_schedule(forced)
    elif schedules:
        plan.set_schedule(schedules["mixed"])
    xa = torch.randn(plan.shape, dtype=torch.complex64, device=dev)
    ya = torch.empty_like(xa)
    for _ in range(3):
        plan.apply_c64(xa, out=ya)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(20):
        plan.apply_c64(xa, out=ya)
    ev1.record()
    torch.cuda.synchronize()
    apply_us = 1e3 * ev0.elapsed_time(ev1) / 20
    plan.close()
    del xa, ya, eps0
    copy_gbs = copy_peak_gbs(dev)

    nsolve = 2 * K
    ok_m = all(i["status"] == "OK" and i["rrel"] <= args.tol for i in infos_m)
    value = nsolve / t_mixed
    it_m = max(1, sum(i["iters"] for i in infos_m))
    # algorithmic bytes: one complex64 A.M apply moves 48 B per voxel
    # (read x, write y: 3 components x 8 B each way); one BiCGSTAB iteration 480 B.
    alg_apply = 48.0 * vox
    alg_iter = 480.0 * vox
    roofline = None
    if prof_kernel is not None:
        ms, nl, by = prof
        knob = {"xfwd": 0, "xinv": 1, "yfft": 2, "axial": 3}[prof_kernel]
        kernel_sched = schedules["mixed"][knob] if schedules else (forced[knob] if forced else 0)
        avg_s = 1e-3 * ms / max(nl, 1)
        achieved = alg_apply / avg_s / 1e9 if ms > 0 else 0.0
        traffic = measured_traffic(prof_kernel, kernel_sched)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic,
                    "kernel": KERNEL_NAMES[prof_kernel], "kernel_class": prof_kernel,
                    "sched": kernel_sched, "launches": nl, "avg_launch_us": round(1e6 * avg_s, 2),
                    "alg_bytes_per_launch": alg_apply,
                    "alg_basis": f"48 B/voxel (one complex64 A.M apply) x {vox} voxels per launch",
                    "own_bytes_per_launch": round(by / max(nl, 1)),
                    "own_gbs": round(by / max(nl, 1) / avg_s / 1e9, 1) if ms > 0 else None,
                    "traffic_gbs": round(traffic / avg_s / 1e9, 1) if traffic and ms > 0 else None,
                    "copy_peak_gbs": round(copy_gbs, 1),
                    "frac_of_copy_peak": round(achieved / copy_gbs, 4) if copy_gbs else None}
    it_traffic = measured_iteration_traffic()
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": round(1e3 * t_mixed / K, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": workload_name(), "solves_per_step": 2, "grid": [nx, ny, nz],
                   "ml_kz_min": ML_KZ_MIN,
                   "precision": "complex64 operator/Krylov, FP64 residual + refinement"},
        "converged": ok_m,
        "iters_mixed": [i["iters"] for i in infos_m],
        "rrel_mixed_max": max(i["rrel"] for i in infos_m),
        "roofline": roofline,
        "apply_roofline": {"unit": "one complex64 operator apply A x", "alg_bytes": alg_apply,
                           "us": round(apply_us, 1),
                           "achieved_gbs": round(alg_apply / (apply_us * 1e-6) / 1e9, 1),
                           "frac": round(alg_apply / (apply_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
        "iteration_roofline": {"unit": "one BiCGSTAB iteration (2 A.M applies + updates)",
                               "alg_bytes": alg_iter,
                               "us": round(1e6 * t_mixed / it_m, 1),
                               "achieved_gbs": round(alg_iter / (t_mixed / it_m) / 1e9, 1),
                               "frac": round(alg_iter / (t_mixed / it_m) / 1e9 / HBM_PEAK_GBS, 4),
                               "counter_bytes": it_traffic,
                               "counter_over_alg": round(it_traffic / alg_iter, 3) if it_traffic else None,
                               "note": "time per iteration includes plan, source and the FP64 reliable updates"},
        "schedules": schedules or ("forced" if forced else "default"),
    }
    if "fp64" in res:
        t_fp64, infos_d = res["fp64"]
        out["fp64_plain"] = {"value": round(nsolve / t_fp64, 4), "unit": "solves/s",
                             "ms_per_step": round(1e3 * t_fp64 / K, 2),
                             "iters": [i["iters"] for i in infos_d],
                             "converged": all(i["status"] == "OK" for i in infos_d)}
        out["mixed_vs_fp64"] = round(t_fp64 / t_mixed, 3)
    if not args.no_cpu_baseline:
        iters_proj = (sum(i["iters"] for i in res["fp64"][1]) / nsolve if "fp64" in res
                      else sum(i["iters"] for i in infos_m) / nsolve)
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        try:
            out["cpu_baseline"] = cpu_baseline(iters_proj, args.cpu_sample_iters, args.cpu_workers)
        except Exception as exc:  # noqa: BLE001 - report, do not lose the GPU line
            out["cpu_baseline"] = {"error": str(exc)[-500:]}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
