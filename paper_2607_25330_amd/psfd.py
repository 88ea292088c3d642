"""Thin ctypes binding of libpsfd.so (the C ABI in include/psfd.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  The
library must be built (``__graft_entry__.build()`` or
``python -m paper_2607_25330_amd.build``); importing works without it, but
the first call raises ``PsfdLibraryMissing``.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_DEFAULT_LIB = os.path.join(_HERE, "libpsfd.so")
# PSFD_LIBRARY selects another build of the same library (same ABI).
LIB_PATH = os.environ.get("PSFD_LIBRARY", _DEFAULT_LIB)
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "psfd.h")

PSFD_OK, PSFD_ERR_ARG, PSFD_ERR_ALLOC, PSFD_ERR_HIP, PSFD_NOT_CONVERGED, PSFD_BREAKDOWN = range(6)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_ALLOC", 3: "ERR_HIP", 4: "NOT_CONVERGED",
                5: "BREAKDOWN"}
PSFD_C128, PSFD_C64_REFINE64, PSFD_C64_BF16PC_REFINE64 = 0, 1, 2


class PsfdLibraryMissing(ImportError):
    pass


class PsfdError(RuntimeError):
    def __init__(self, func, status, msg):
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
c_dp = ctypes.POINTER(c_double)


class Desc(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nz_abs", c_int32), ("nz_gap_bot", c_int32),
        ("nz_gap_top", c_int32), ("nz_pml", c_int32),
        ("dx", c_double), ("dy", c_double), ("dz", c_double), ("lambda_", c_double),
        ("theta", c_double), ("phi", c_double), ("pol", c_int32),
        ("eps_bg", c_double),
        ("n_ml", c_int32), ("ml_eps", c_dp), ("ml_thick", c_dp), ("eps_sub", c_double * 2),
        ("pml_sigma0", c_double), ("pml_order", c_int32), ("precond", c_int32),
        ("pc_mmin", c_double), ("pc_kref", c_double), ("pc_gamma", c_double), ("pc_reg", c_double),
        ("prec", c_int32), ("ml_kz_min", c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("status", c_int32), ("restarts", c_int32),
                ("applies", c_int32), ("rrel_true", c_double), ("rrel_hist_last", c_double)]


class FfnoDesc(ctypes.Structure):
    _fields_ = [(n, c_int32) for n in ("nx", "ny", "nz", "d_v", "d_h", "n_layers", "kx_max",
                                         "ky_max", "kz_max")]


_SIGS = {
    "psfd_layout_eps": [ctypes.POINTER(Desc), c_void_p, c_dp, c_double, c_void_p, c_void_p],
    "psfd_layout_eps_noalloc": [ctypes.POINTER(Desc), c_void_p, c_dp, c_double, c_void_p, c_void_p],
    "psfd_plan": [ctypes.POINTER(Desc), c_void_p, c_void_p, ctypes.POINTER(c_void_p)],
    "psfd_set_eps": [c_void_p, c_void_p],
    "psfd_rhs": [c_void_p, c_void_p],
    "psfd_apply": [c_void_p, c_void_p, c_void_p],
    "psfd_adjoint": [c_void_p, c_void_p, c_void_p],
    "psfd_precond": [c_void_p, c_void_p, c_void_p],
    "psfd_apply_c64": [c_void_p, c_void_p, c_void_p],
    "psfd_adjoint_c64": [c_void_p, c_void_p, c_void_p],
    "psfd_precond_c64": [c_void_p, c_void_p, c_void_p],
    "psfd_solve": [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32, c_int32,
                   ctypes.POINTER(Info)],
    "psfd_solve_shadow": [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32, c_int32,
                          c_void_p, ctypes.POINTER(Info)],
    "psfd_ml_reflection": [c_void_p, c_void_p, c_void_p],
    "psfd_residual": [c_void_p, c_void_p, c_void_p, c_void_p, c_dp],
    "psfd_eps_grad": [c_void_p, c_void_p, c_void_p, c_double, c_void_p],
    "psfd_plan_batch": [c_int32, ctypes.POINTER(Desc), ctypes.POINTER(c_void_p), c_void_p,
                        ctypes.POINTER(c_void_p)],
    "psfd_solve_batch": [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_double,
                         c_int32, ctypes.POINTER(Info)],
    "psfd_profile_enable": [c_void_p, c_int32],
    "psfd_profile_read": [c_void_p, c_dp, ctypes.POINTER(c_int64), c_dp],
    "psfd_layered_eps": [ctypes.POINTER(Desc), c_int32, c_dp, c_dp, c_void_p, c_void_p],
    "psfd_specular": [c_void_p, c_void_p, c_dp],
    "psfd_contour_segments": [c_void_p, c_int32, c_int32, c_int32, c_int64, c_double, c_double,
                              c_int32, c_double, c_double, c_int32, c_void_p, c_void_p, c_void_p],
    "psfd_contour_deviation": [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32,
                               c_double, c_double, c_int32, c_int32, c_double, c_double, c_void_p,
                               c_dp, c_void_p],
    "psfd_pino_loss": [c_void_p, c_void_p, c_double, c_double, c_double, c_dp, c_void_p],
    "psfd_ffno_sizes": [ctypes.POINTER(FfnoDesc), ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)],
    "psfd_ffno_forward": [ctypes.POINTER(FfnoDesc), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "psfd_tune": [c_void_p],
    "psfd_tune_save": [ctypes.c_char_p],
    "psfd_schedule": [c_void_p, ctypes.POINTER(c_int32)],
    "psfd_set_schedule": [c_void_p, ctypes.POINTER(c_int32)],
}

# kernel ids for Plan.profile_enable
PROFILE_KERNELS = {"off": 0, "axial": 1, "yfft": 2, "xfwd": 3, "xinv": 4}

_lib = None


def lib():
    """Load libpsfd.so (raises PsfdLibraryMissing if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PsfdLibraryMissing(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int32
        L.psfd_field_size.argtypes = [c_void_p]
        L.psfd_field_size.restype = c_int64
        L.psfd_destroy.argtypes = [c_void_p]
        L.psfd_destroy.restype = None
        L.psfd_trim_cache.argtypes = []
        L.psfd_trim_cache.restype = None
        L.psfd_last_error.argtypes = []
        L.psfd_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != PSFD_OK:
        raise PsfdError(name, st, lib().psfd_last_error().decode())
    return st


def make_desc(cfg, prec=PSFD_C128):
    """psfd_desc from a configuration dict (keys as in psfd_synth.configs); returns (desc, keepalive)."""
    n_ml = len(cfg["ml_eps"])
    eps_arr = (c_double * max(2 * n_ml, 1))(*[v for e in cfg["ml_eps"] for v in (e.real, e.imag)])
    d_arr = (c_double * max(n_ml, 1))(*cfg["ml_thick"])
    es = complex(cfg["eps_sub"])
    d = Desc(
        nx=cfg["nx"], ny=cfg["ny"], nz_abs=cfg["nz_abs"], nz_gap_bot=cfg["nz_gap_bot"],
        nz_gap_top=cfg["nz_gap_top"], nz_pml=cfg["nz_pml"],
        dx=cfg["dx"], dy=cfg["dy"], dz=cfg["dz"], lambda_=cfg["lam"],
        theta=cfg["theta"], phi=cfg["phi"], pol=cfg["pol"], eps_bg=float(cfg["eps_bg"]),
        n_ml=n_ml, ml_eps=ctypes.cast(eps_arr, c_dp), ml_thick=ctypes.cast(d_arr, c_dp),
        eps_sub=(c_double * 2)(es.real, es.imag),
        pml_sigma0=cfg["pml_sigma0"], pml_order=cfg["pml_order"], precond=int(cfg["precond"]),
        pc_mmin=cfg["pc_mmin"], pc_kref=cfg["pc_kref"], pc_gamma=cfg["pc_gamma"],
        pc_reg=cfg["pc_reg"], prec=int(prec), ml_kz_min=float(cfg.get("ml_kz_min", 0.0)))
    return d, (eps_arr, d_arr)


def _stream_handle():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return c_void_p(t.data_ptr())


def nz_of(cfg):
    return cfg["nz_abs"] + cfg["nz_gap_bot"] + cfg["nz_gap_top"] + 2 * cfg["nz_pml"]


def psfd_layout_eps(cfg, a_bin, eps_abs, sigma=None):
    """Smoothed-layout permittivity on absorber rows, (nz_abs, ny, nx) complex128."""
    d, keep = make_desc(cfg)
    a = a_bin.to(torch.float64).contiguous()
    out = torch.empty((cfg["nz_abs"], cfg["ny"], cfg["nx"]), dtype=torch.complex128, device=a.device)
    e = complex(eps_abs)
    ea = (c_double * 2)(e.real, e.imag)
    sig = cfg.get("smooth_sigma", 1.0) if sigma is None else sigma
    _call("psfd_layout_eps", ctypes.byref(d), _ptr(a, torch.float64, (cfg["ny"], cfg["nx"]), "a_bin"),
          ctypes.cast(ea, c_dp), c_double(sig), _ptr(out, torch.complex128), _stream_handle())
    return out


def psfd_layout_eps_noalloc(cfg, a_bin, eps_abs, sigma=None, out=None):
    """psfd_layout_eps through the allocation-free entry point (nx * ny <= 512^2);
    queued on the current stream, no synchronisation."""
    d, keep = make_desc(cfg)
    a = a_bin.to(torch.float64).contiguous()
    if out is None:
        out = torch.empty((cfg["nz_abs"], cfg["ny"], cfg["nx"]), dtype=torch.complex128,
                          device=a.device)
    e = complex(eps_abs)
    ea = (c_double * 2)(e.real, e.imag)
    sig = cfg.get("smooth_sigma", 1.0) if sigma is None else sigma
    _call("psfd_layout_eps_noalloc", ctypes.byref(d),
          _ptr(a, torch.float64, (cfg["ny"], cfg["nx"]), "a_bin"), ctypes.cast(ea, c_dp),
          c_double(sig), _ptr(out, torch.complex128, (cfg["nz_abs"], cfg["ny"], cfg["nx"]), "out"),
          _stream_handle())
    return out


def tune_save(path):
    """Write the process's kernel-schedule table (psfd_tune_save) to `path`."""
    _call("psfd_tune_save", os.fsencode(str(path)))


def trim_cache():
    """Free the device blocks the library keeps from destroyed plans."""
    lib().psfd_trim_cache()


def psfd_layered_eps(cfg, layers_eps, layers_thick, device):
    """Row-mean permittivity of a planar stack hanging from the top face of the
    absorber region (full-domain discretisation), (nz_abs, ny, nx) complex128."""
    d, keep = make_desc(cfg)
    n = len(layers_eps)
    if len(layers_thick) != n:
        raise ValueError("layers_eps and layers_thick differ in length")
    le = (c_double * max(1, 2 * n))(*[v for e in layers_eps for v in (complex(e).real, complex(e).imag)])
    ld = (c_double * max(1, n))(*[float(t) for t in layers_thick])
    out = torch.empty((cfg["nz_abs"], cfg["ny"], cfg["nx"]), dtype=torch.complex128, device=device)
    _call("psfd_layered_eps", ctypes.byref(d), c_int32(n), ctypes.cast(le, c_dp),
          ctypes.cast(ld, c_dp), _ptr(out, torch.complex128), _stream_handle())
    return out


def contour_segments(planes, dx, dy, nlines=100, i_th=0.15, w=0.05, max_seg=None):
    """Threshold-contour segments of [ny][nx] or [B][ny][nx] complex128 planes.

    Returns (seg [B][2 nlines][max_seg][2] (start, width) float64, nseg [B][2 nlines] int32);
    horizontal lines first."""
    p = planes if planes.dim() == 3 else planes.unsqueeze(0)
    if p.dtype != torch.complex128 or not p.is_cuda:
        raise TypeError("planes must be a complex128 CUDA tensor")
    if p.stride(2) != 1 or p.stride(1) != p.shape[2]:
        raise ValueError("each plane must be contiguous")
    B, ny, nx = p.shape
    ms = max(nx, ny) // 2 if max_seg is None else int(max_seg)
    seg = torch.zeros((B, 2 * nlines, ms, 2), dtype=torch.float64, device=p.device)
    nseg = torch.zeros((B, 2 * nlines), dtype=torch.int32, device=p.device)
    _call("psfd_contour_segments", c_void_p(p.data_ptr()), c_int32(nx), c_int32(ny), c_int32(B),
          c_int64(p.stride(0)), c_double(dx), c_double(dy), c_int32(nlines), c_double(i_th),
          c_double(w), c_int32(ms), c_void_p(seg.data_ptr()), c_void_p(nseg.data_ptr()),
          _stream_handle())
    return seg, nseg


def contour_deviation(ref, other, nx, ny, dx, dy, demag=4.0, thr=1.0):
    """(d_ref - d) / demag per reference segment and the statistics, from two
    contour_segments results of the same sizes.  Returns (delta, stats dict)."""
    sr, nr = ref
    sk, nk = other
    if sr.shape != sk.shape or nr.shape != nk.shape:
        raise ValueError("reference and field segments differ in shape")
    B, nl2, ms, _ = sr.shape
    delta = torch.empty((B, nl2, ms), dtype=torch.float64, device=sr.device)
    st = (c_double * 5)()
    _call("psfd_contour_deviation", c_void_p(sr.data_ptr()), c_void_p(nr.data_ptr()),
          c_void_p(sk.data_ptr()), c_void_p(nk.data_ptr()), c_int32(nx), c_int32(ny), c_int32(B),
          c_double(dx), c_double(dy), c_int32(nl2 // 2), c_int32(ms), c_double(demag),
          c_double(thr), c_void_p(delta.data_ptr()), ctypes.cast(st, c_dp), _stream_handle())
    n = st[2]
    mean = st[0] / n if n else float("nan")
    var = st[1] / n - mean * mean if n else float("nan")
    return delta, {"sum_abs": st[0], "sum_sq": st[1], "resolved": int(st[2]),
                   "unresolved": int(st[3]), "above_thr": int(st[4]), "mean_abs": mean,
                   "std_abs": (max(var, 0.0)) ** 0.5 if n else float("nan")}


class Ffno:
    """Factorised Fourier neural operator forward pass (psfd_ffno_forward) with its own
    workspace; `weights` is a flat float32 CUDA tensor in the documented layout."""

    def __init__(self, desc, weights):
        self.desc = FfnoDesc(**{k: int(desc[k]) for k, _ in FfnoDesc._fields_})
        nw, nb = c_int64(), c_int64()
        _call("psfd_ffno_sizes", ctypes.byref(self.desc), ctypes.byref(nw), ctypes.byref(nb))
        if weights.dtype != torch.float32 or not weights.is_cuda or weights.numel() != nw.value:
            raise ValueError(f"weights must be a float32 CUDA tensor of {nw.value} elements")
        self.weights = weights.contiguous()
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=weights.device)
        self.shape = (3, desc["nz"], desc["ny"], desc["nx"])

    def __call__(self, a, out=None):
        a = a.to(torch.float32).contiguous()
        if tuple(a.shape) != self.shape[1:]:
            raise ValueError(f"a must have shape {self.shape[1:]}")
        E = torch.empty(self.shape, dtype=torch.complex128, device=a.device) if out is None else out
        _call("psfd_ffno_forward", ctypes.byref(self.desc), c_void_p(self.weights.data_ptr()),
              c_void_p(a.data_ptr()), _ptr(E, torch.complex128, self.shape, "E"),
              c_void_p(self.workspace.data_ptr()), _stream_handle())
        return E


class Plan:
    """A psfd_plan bound to the current torch stream."""

    def __init__(self, cfg, eps, prec=PSFD_C128):
        self.cfg = dict(cfg)
        self.prec = prec
        self.nz = nz_of(cfg)
        self.shape = (3, self.nz, cfg["ny"], cfg["nx"])
        self.eps_shape = (cfg["nz_abs"], cfg["ny"], cfg["nx"])
        d, keep = make_desc(cfg, prec)
        h = c_void_p()
        _call("psfd_plan", ctypes.byref(d), _ptr(eps, torch.complex128, self.eps_shape, "eps"),
              _stream_handle(), ctypes.byref(h))
        self._h = h
        self.device = eps.device

    def _field(self, dtype=torch.complex128):
        return torch.empty(self.shape, dtype=dtype, device=self.device)

    def _unary(self, name, x, out, dtype):
        y = self._field(dtype) if out is None else out
        _call(name, self._h, _ptr(x, dtype, self.shape, "x"), _ptr(y, dtype, self.shape, "y"))
        return y

    def apply(self, x, out=None):
        return self._unary("psfd_apply", x, out, torch.complex128)

    def adjoint(self, x, out=None):
        return self._unary("psfd_adjoint", x, out, torch.complex128)

    def precond(self, x, out=None):
        return self._unary("psfd_precond", x, out, torch.complex128)

    def apply_c64(self, x, out=None):
        return self._unary("psfd_apply_c64", x, out, torch.complex64)

    def adjoint_c64(self, x, out=None):
        return self._unary("psfd_adjoint_c64", x, out, torch.complex64)

    def precond_c64(self, x, out=None):
        return self._unary("psfd_precond_c64", x, out, torch.complex64)

    def rhs(self, out=None):
        b = self._field() if out is None else out
        _call("psfd_rhs", self._h, _ptr(b, torch.complex128, self.shape, "b"))
        return b

    def set_eps(self, eps):
        _call("psfd_set_eps", self._h, _ptr(eps, torch.complex128, self.eps_shape, "eps"))

    def ml_reflection(self):
        n = (self.cfg["ny"], self.cfg["nx"])
        rte = torch.empty(n, dtype=torch.complex128, device=self.device)
        rpe = torch.empty(n, dtype=torch.complex128, device=self.device)
        _call("psfd_ml_reflection", self._h, _ptr(rte, torch.complex128), _ptr(rpe, torch.complex128))
        return rte, rpe

    def pino_loss(self, E, w0=1.0, eta=0.0, lam=0.0, grad=True):
        """(J, residual term, penalty term) of the physics loss and, with grad=True, the field
        g = (1/N) (b - A E) + lam H (b - A E) its gradients are built from."""
        out = (c_double * 3)()
        g = self._field() if grad else None
        _call("psfd_pino_loss", self._h, _ptr(E, torch.complex128, self.shape, "E"), c_double(w0),
              c_double(eta), c_double(lam), ctypes.cast(out, c_dp),
              c_void_p(None) if g is None else _ptr(g, torch.complex128, self.shape, "g"))
        return (out[0], out[1], out[2]), g

    def specular(self, E):
        """Specular (0, 0)-order reflection coefficient at the absorber region's top face."""
        r = (c_double * 2)()
        _call("psfd_specular", self._h, _ptr(E, torch.complex128, self.shape, "E"),
              ctypes.cast(r, c_dp))
        return complex(r[0], r[1])

    def solve(self, b=None, x0=None, tol=1e-6, maxit=20000, adjoint=False, out=None,
              check=True, shadow=None):
        """Returns (E, info dict).  With check=False a non-converged solve returns its status.
        shadow: the first Krylov run's shadow residual (psfd_solve_shadow)."""
        E = self._field() if out is None else out
        info = Info()
        bp = c_void_p(None) if b is None else _ptr(b, torch.complex128, self.shape, "b")
        xp = c_void_p(None) if x0 is None else _ptr(x0, torch.complex128, self.shape, "x0")
        Ep = _ptr(E, torch.complex128, self.shape, "E")
        if shadow is None:
            name = "psfd_solve"
            st = lib().psfd_solve(self._h, bp, xp, Ep, c_double(tol), c_int32(maxit),
                                  c_int32(1 if adjoint else 0), ctypes.byref(info))
        else:
            name = "psfd_solve_shadow"
            sp = _ptr(shadow, torch.complex128, self.shape, "shadow")
            st = lib().psfd_solve_shadow(self._h, bp, xp, Ep, c_double(tol), c_int32(maxit),
                                         c_int32(1 if adjoint else 0), sp, ctypes.byref(info))
        if check and st != PSFD_OK:
            raise PsfdError(name, st, lib().psfd_last_error().decode())
        return E, {"iters": info.iters, "status": STATUS_NAMES.get(st, st),
                   "restarts": info.restarts, "applies": info.applies,
                   "rrel": info.rrel_true, "rrel_rec": info.rrel_hist_last}

    def residual(self, E, b=None, out=None):
        """(r, ||r||^2) with r = b - A E in FP64 (b = None: the analytic source)."""
        r = self._field() if out is None else out
        n2 = c_double()
        bp = c_void_p(None) if b is None else _ptr(b, torch.complex128, self.shape, "b")
        _call("psfd_residual", self._h, bp, _ptr(E, torch.complex128, self.shape, "E"),
              _ptr(r, torch.complex128, self.shape, "r"), ctypes.byref(n2))
        return r, n2.value

    def eps_grad(self, E, u, scale, out=None):
        """scale * sum_alpha u_alpha conj(Psi_alpha(E)) on absorber voxels (nz_abs, ny, nx)."""
        g = torch.empty(self.eps_shape, dtype=torch.complex128, device=self.device) if out is None else out
        _call("psfd_eps_grad", self._h, _ptr(E, torch.complex128, self.shape, "E"),
              _ptr(u, torch.complex128, self.shape, "u"), c_double(scale),
              _ptr(g, torch.complex128, self.eps_shape, "grad"))
        return g

    @property
    def k0(self):
        return 2.0 * 3.141592653589793 / self.cfg["lam"]

    def tune(self):
        """psfd_tune: pick the fastest kernel schedules for this shape (cached per process)."""
        _call("psfd_tune", self._h)
        return self.schedule()

    def schedule(self):
        """psfd_schedule: (forward x, inverse x, y, axial) schedule indices."""
        out = (c_int32 * 4)()
        _call("psfd_schedule", self._h, out)
        return tuple(out)

    def set_schedule(self, sched):
        """psfd_set_schedule: (forward x, inverse x, y, axial) schedule indices."""
        _call("psfd_set_schedule", self._h, (c_int32 * 4)(*[int(v) for v in sched]))

    def profile_enable(self, kernel):
        """Time every launch of one kernel class with HIP events (see PROFILE_KERNELS)."""
        _call("psfd_profile_enable", self._h, c_int32(PROFILE_KERNELS.get(kernel, kernel)))

    def profile_read(self):
        """(total ms, launches, algorithmic bytes) of the timed launches."""
        ms, n, b = c_double(), c_int64(), c_double()
        _call("psfd_profile_read", self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b))
        return ms.value, n.value, b.value

    def field_size(self):
        return int(lib().psfd_field_size(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psfd_destroy(self._h)
            self._h = c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """psfd_plan_batch / psfd_solve_batch over independent problems of any sizes."""

    def __init__(self, cfgs, eps_list, prec=PSFD_C128):
        n = len(cfgs)
        if n == 0 or len(eps_list) != n:
            raise ValueError("need one permittivity per configuration")
        descs = (Desc * n)()
        self._keep = []
        self.shapes = []
        ptrs = (c_void_p * n)()
        for i, (cfg, eps) in enumerate(zip(cfgs, eps_list)):
            d, keep = make_desc(cfg, prec)
            descs[i] = d
            self._keep.append(keep)
            self.shapes.append((3, nz_of(cfg), cfg["ny"], cfg["nx"]))
            ptrs[i] = _ptr(eps, torch.complex128, (cfg["nz_abs"], cfg["ny"], cfg["nx"]), "eps")
        self._eps = list(eps_list)  # must stay alive until solve returns
        self.device = eps_list[0].device
        self.n = n
        h = c_void_p()
        _call("psfd_plan_batch", c_int32(n), descs, ptrs, _stream_handle(), ctypes.byref(h))
        self._h = h

    def solve(self, x0=None, tol=1e-6, maxit=20000, check=True):
        E = [torch.empty(sh, dtype=torch.complex128, device=self.device) for sh in self.shapes]
        Ep = (c_void_p * self.n)(*[e.data_ptr() for e in E])
        if x0 is None:
            xp = ctypes.cast(None, ctypes.POINTER(c_void_p))
        else:
            xp = (c_void_p * self.n)(*[0 if x is None else _ptr(x, torch.complex128, sh, "x0").value
                                       for x, sh in zip(x0, self.shapes)])
        infos = (Info * self.n)()
        st = lib().psfd_solve_batch(self._h, xp, Ep, c_double(tol), c_int32(maxit), infos)
        if check and st != PSFD_OK:
            raise PsfdError("psfd_solve_batch", st, lib().psfd_last_error().decode())
        out = [{"iters": i.iters, "status": STATUS_NAMES.get(i.status, i.status),
                "restarts": i.restarts, "rrel": i.rrel_true} for i in infos]
        return E, out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().psfd_destroy(self._h)
            self._h = c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Module-level names matching the C ABI.
def psfd_plan(cfg, eps, prec=PSFD_C128):
    return Plan(cfg, eps, prec)


def psfd_apply(plan, x, y=None):
    return plan.apply(x, y)


def psfd_adjoint(plan, x, y=None):
    return plan.adjoint(x, y)


def psfd_precond(plan, x, y=None):
    return plan.precond(x, y)


def psfd_rhs(plan, b=None):
    return plan.rhs(b)


def psfd_solve(plan, b=None, x0=None, tol=1e-6, maxit=20000, adjoint=False):
    return plan.solve(b, x0, tol, maxit, adjoint)


def psfd_destroy(plan):
    plan.close()


def psfd_plan_batch(cfgs, eps_list, prec=PSFD_C128):
    return Batch(cfgs, eps_list, prec)


def psfd_solve_batch(batch, x0=None, tol=1e-6, maxit=20000):
    return batch.solve(x0, tol, maxit)


def psfd_residual(plan, E, b=None):
    return plan.residual(E, b)


def psfd_eps_grad(plan, E, u, scale):
    return plan.eps_grad(E, u, scale)
