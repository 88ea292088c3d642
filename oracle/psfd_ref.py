"""Plain FP64 CPU reference (the oracle) for the background-decomposed,
right-preconditioned PSFD full-vector scattering solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library: it is numpy
complex128 throughout, with numpy.fft as its only transform.

What it computes (paper, Methodology section 2.2 and Results, "PINO
warm-start" paragraph):

* the vector Helmholtz operator  L = curl curl - k0^2 eps  (equation
  vector_helmholtz_operator), every derivative pseudo-spectral, with PML
  coordinate stretching along z;
* background decomposition: the grid covers the absorber region only; the
  multilayer enters through the reflection operator R_ml, which maps the
  tangential field at the multilayer interface to the reflected background
  field (upgoing/downgoing split, TE/TM split, transfer-matrix reflection,
  analytic phase-matched propagation);
* the background source  b = k0^2 d_eps (E_inc + E_ML)  (equation
  bg_source), with R_ml inside the operator so that the multilayer response
  is re-evaluated from the current field at every iteration (self-consistent
  coupling, no finite-order Born approximation);
* the spectral damping preconditioner M (equations spectral_damping_action
  and spectral_damping_mask) used as a right preconditioner with the affine
  warm start  E = E_base + M y,  A M y = b - A E_base  (equations
  right_correction_solution and right_preconditioned_system);
* BiCGSTAB stopped on the relative residual ||b - A E|| / ||b|| (equation
  relative_residual).

Where the paper defers details to its companion PSFD paper (not available),
each reading used here is stated where it is used (grid, PML, basis, TMM convention, ...).

Array layout: fields are complex arrays of shape (3, nz, ny, nx): component,
axial row (bottom to top), y, x.  The permittivity is given on absorber
rows only, shape (nz_abs, ny, nx).
"""

import numpy as np

# --------------------------------------------------------------------------
# Geometry and wavenumbers
# --------------------------------------------------------------------------


def principal_sqrt(w):
    """Square root on the branch Im >= 0 (Re >= 0 on the real axis).

    Outgoing / decaying branch for axial wavenumbers with time factor
    exp(-i omega t).  Signed zeros are normalised so that a negative real
    argument always maps to +i sqrt(|w|)."""
    q = np.sqrt(np.asarray(w, dtype=np.complex128))
    flip = (q.imag < 0) | ((q.imag == 0) & (q.real < 0))
    return np.where(flip, -q, q)


class Grid:
    """Axial rows, lateral Bloch wavenumbers, PML stretch, incidence.

    Axial rows from the bottom: PML | gap | absorber | gap | PML.  Rows are
    cell-centred; z = 0 is the absorber's bottom face, which is where the
    multilayer interface z_ml sits.  The evaluation row for the
    multilayer split is the last bottom-gap row (z = -dz/2); the observation
    row is the first top-gap row.  The z axis is periodic, so the two PML
    slabs are contiguous across the wrap.
    """

    def __init__(self, cfg):
        self.cfg = cfg
        self.nx, self.ny = cfg["nx"], cfg["ny"]
        self.nz_abs = cfg["nz_abs"]
        self.npml = cfg["nz_pml"]
        self.nz = cfg["nz_abs"] + cfg["nz_gap_bot"] + cfg["nz_gap_top"] + 2 * cfg["nz_pml"]
        self.dx, self.dy, self.dz = cfg["dx"], cfg["dy"], cfg["dz"]
        self.j0 = cfg["nz_pml"] + cfg["nz_gap_bot"]          # first absorber row
        self.abs_rows = np.arange(self.j0, self.j0 + self.nz_abs)
        self.j_ev = self.j0 - 1
        self.j_obs = self.j0 + self.nz_abs
        self.z = (np.arange(self.nz) - self.j0 + 0.5) * self.dz

        self.k0 = 2.0 * np.pi / cfg["lam"]
        self.eps_bg = float(cfg["eps_bg"])
        self.kbg = self.k0 * np.sqrt(self.eps_bg)
        th, ph = cfg["theta"], cfg["phi"]
        self.theta, self.phi = th, ph
        self.kx0 = self.kbg * np.sin(th) * np.cos(ph)
        self.ky0 = self.kbg * np.sin(th) * np.sin(ph)
        self.kz0 = self.kbg * np.cos(th)

        # Bloch-shifted lateral wavenumbers (numpy fftfreq order, Nyquist at -N/2).
        self.kx = self.kx0 + 2.0 * np.pi * np.fft.fftfreq(self.nx, d=self.dx)
        self.ky = self.ky0 + 2.0 * np.pi * np.fft.fftfreq(self.ny, d=self.dy)
        self.kz = 2.0 * np.pi * np.fft.fftfreq(self.nz, d=self.dz)

        self.s = pml_stretch(self.nz, self.npml, self.dz, cfg["pml_sigma0"], cfg["pml_order"])

    @property
    def shape(self):
        return (3, self.nz, self.ny, self.nx)


def pml_stretch(nz, npml, dz, sigma0, order):
    """Complex coordinate stretch s(z) = 1 + i sigma0 (d/D)^p in PML rows.

    Paper, section 2.2 (derivatives "with PML coordinate stretching"); the
    profile is not printed, a polynomial grading is used.  d is the distance
    of the row centre into the PML from its inner edge, D its thickness."""
    s = np.ones(nz, dtype=np.complex128)
    if npml == 0:
        return s
    D = npml * dz
    for j in range(npml):
        d = (npml - j - 0.5) * dz
        s[j] = 1.0 + 1j * sigma0 * (d / D) ** order
    for j in range(nz - npml, nz):
        d = (j - (nz - npml) + 0.5) * dz
        s[j] = 1.0 + 1j * sigma0 * (d / D) ** order
    return s


# --------------------------------------------------------------------------
# Geometry -> material (paper, section 2.1 last paragraphs and Results,
# "PINO surrogate": the binary indicator is Gaussian-smoothed on the grid and
# the same smoothing is applied for the PSFD solver)
# --------------------------------------------------------------------------


def smooth_layout(cfg, a_bin):
    """Periodic Gaussian smoothing of the binary indicator, clipped to [0, 1].

    The smoothing width is not printed in the paper; sigma is
    cfg['smooth_sigma'] lateral cells.  Transfer function
    exp(-(sx^2 kx^2 + sy^2 ky^2)/2) on the unshifted DFT wavenumbers."""
    ny, nx = a_bin.shape
    sx = cfg["smooth_sigma"] * cfg["dx"]
    sy = cfg["smooth_sigma"] * cfg["dy"]
    kxt = 2.0 * np.pi * np.fft.fftfreq(nx, d=cfg["dx"])
    kyt = 2.0 * np.pi * np.fft.fftfreq(ny, d=cfg["dy"])
    H = np.exp(-0.5 * (sx * sx * kxt[None, :] ** 2 + sy * sy * kyt[:, None] ** 2))
    a = np.fft.ifft2(np.fft.fft2(np.asarray(a_bin, dtype=np.float64)) * H).real
    return np.clip(a, 0.0, 1.0)


def eps_from_fill(cfg, a, eps_abs):
    """eps = eps_bg + a (eps_abs - eps_bg) on every absorber row (extruded layout)."""
    e2 = cfg["eps_bg"] + a * (eps_abs - cfg["eps_bg"])
    return np.broadcast_to(e2, (cfg["nz_abs"],) + a.shape).astype(np.complex128).copy()


# --------------------------------------------------------------------------
# Multilayer reflection by the transfer-matrix method (paper, section 2.2,
# definition of R_ml, step (iii); stack from the Results section)
# --------------------------------------------------------------------------


def tmm_reflection(k0, kt2, eps_top, layers_eps, layers_d, eps_sub, pol):
    """Reflection coefficient of a planar stack seen from the top medium.

    Abeles characteristic matrices, layers listed top to bottom, time factor
    exp(-i omega t).  For layer j: q_j = kz_j (TE, pol=0) or kz_j/eps_j
    (TM, pol=1, magnetic-field reflection), delta_j = kz_j d_j and
    M_j = [[cos delta, -(i/q) sin delta], [-i q sin delta, cos delta]].
    With M the ordered product, r = (q0 M11 + q0 qs M12 - M21 - qs M22) /
    (q0 M11 + q0 qs M12 + M21 + qs M22).  The product is rescaled after each
    layer (r is invariant to a common factor) so evanescent modes stay finite.
    """
    kt2 = np.asarray(kt2, dtype=np.float64)

    def q_of(eps):
        kz = principal_sqrt(k0 * k0 * eps - kt2)
        return kz, (kz if pol == 0 else kz / eps)

    _, q0 = q_of(eps_top)
    _, qs = q_of(eps_sub)
    m11 = np.ones(kt2.shape, np.complex128)
    m12 = np.zeros(kt2.shape, np.complex128)
    m21 = np.zeros(kt2.shape, np.complex128)
    m22 = np.ones(kt2.shape, np.complex128)
    for eps_j, d_j in zip(layers_eps, layers_d):
        kz, q = q_of(eps_j)
        dl = kz * d_j
        c, s = np.cos(dl), np.sin(dl)
        a11, a12, a21, a22 = c, -1j * s / q, -1j * q * s, c
        m11, m12, m21, m22 = (m11 * a11 + m12 * a21, m11 * a12 + m12 * a22,
                              m21 * a11 + m22 * a21, m21 * a12 + m22 * a22)
        scale = np.maximum.reduce([np.abs(m11), np.abs(m12), np.abs(m21), np.abs(m22)])
        m11, m12, m21, m22 = m11 / scale, m12 / scale, m21 / scale, m22 / scale
    num = q0 * m11 + q0 * qs * m12 - m21 - qs * m22
    den = q0 * m11 + q0 * qs * m12 + m21 + qs * m22
    return num / den


def ml_reflection(g, cfg, kt2=None):
    """Per-lateral-mode multilayer reflection of tangential E: (r_TE, r_pE).

    r_pE = -r_TM^H converts the magnetic-field TM coefficient to the
    tangential-electric-field amplitude convention used by R_ml."""
    if kt2 is None:
        kt2 = g.kx[None, :] ** 2 + g.ky[:, None] ** 2
    args = (g.k0, kt2, g.eps_bg, cfg["ml_eps"], cfg["ml_thick"], cfg["eps_sub"])
    r_te = tmm_reflection(*args, pol=0)
    r_pe = -tmm_reflection(*args, pol=1)
    return r_te, r_pe


# --------------------------------------------------------------------------
# The R_ml chain on lateral Fourier coefficients (paper, section 2.2 steps
# (i)-(iv)).
# --------------------------------------------------------------------------


class Basis:
    """Per-mode TE/TM basis and background axial wavenumber.

    s_hat = (-ky, kx, 0)/kt, t_hat = (kx, ky, 0)/kt; at kt = 0 the basis of
    the incidence plane is used.  kz = sqrt(kbg^2 - kt^2) with Im kz >= 0.
    Grazing modes, |kz| < max(ml_kz_min, 1e-9) k0, get no multilayer
    response (the paper is silent on grazing orders).

    The TM amplitude of the downgoing field is read from the whole field
    vector at the evaluation row: a downgoing TM wave of tangential amplitude
    a has E_t = a t_hat and E_z = (kt/kz) a, and a is the least-squares fit
    of that polarisation to (t_hat . E_t, E_z).  For a field that is one
    downgoing wave this is t_hat . E_t exactly; it differs where the field on
    the evaluation row also holds other content, which for near-grazing orders
    a periodic PML box always does (coordinate stretching does not act on a
    z-constant field).  Read from E_t alone, that content is multiplied by
    kt/kz when the upgoing TM field's E_z is formed."""

    def __init__(self, g):
        KX = np.broadcast_to(g.kx[None, :], (g.ny, g.nx))
        KY = np.broadcast_to(g.ky[:, None], (g.ny, g.nx))
        kt2 = KX * KX + KY * KY
        kt = np.sqrt(kt2)
        zero = kt == 0.0
        ktn = np.where(zero, 1.0, kt)
        self.sx = np.where(zero, -np.sin(g.phi), -KY / ktn)
        self.sy = np.where(zero, np.cos(g.phi), KX / ktn)
        self.tx = np.where(zero, np.cos(g.phi), KX / ktn)
        self.ty = np.where(zero, np.sin(g.phi), KY / ktn)
        self.kt = kt
        self.kt2 = kt2
        self.kzb = principal_sqrt(g.kbg * g.kbg - kt2)
        kz_min = max(float(g.cfg.get("ml_kz_min", 0.0)), 1e-9)
        self.live = np.abs(self.kzb) >= kz_min * g.k0
        kzn = np.where(self.live, self.kzb, 1.0)
        self.ktkz = np.where(self.live, kt / kzn, 0.0)
        # TM amplitude of the downgoing field: least-squares projection of the
        # field vector (t_hat . E_t, E_z) on the polarisation (1, kt/kz) of a
        # downgoing TM wave, a_p = w_t (t_hat . E_t) + w_z E_z.
        den = 1.0 + np.abs(self.ktkz) ** 2
        self.w_t = 1.0 / den
        self.w_z = np.conj(self.ktkz) / den


def downgoing_amplitudes(g, basis, X_ev):
    """TE and TM amplitudes at z_ml of the downgoing field, from the lateral
    Fourier coefficients X_ev (3, ny, nx) of the field on the evaluation row.

    (i) the field there is taken as downgoing, its amplitude at z_ml = 0 is
    the value times exp(-i kz dz/2); (ii) TE: s_hat . E_t; TM: the
    least-squares fit w_t (t_hat . E_t) + w_z E_z (see Basis)."""
    b = basis
    down = np.exp(-1j * b.kzb * (0.5 * g.dz))
    a_s = (b.sx * X_ev[0] + b.sy * X_ev[1]) * down
    a_p = (b.w_t * (b.tx * X_ev[0] + b.ty * X_ev[1]) + b.w_z * X_ev[2]) * down
    return a_s, a_p


def ml_field_hat(g, basis, r_te, r_pe, X_ev, rows):
    """Reflected multilayer field on the given rows, lateral Fourier space.

    X_ev: (3, ny, nx) coefficients of the field at the evaluation row.
    (i)-(ii) downgoing TE/TM amplitudes at z_ml (downgoing_amplitudes);
    (iii) multiply by r_TE, r_pE; (iv) propagate upward:
    E_ML(z) = [a_s s_hat + a_p (t_hat - (kt/kz) z_hat)] exp(i kz z).
    Returns (3, len(rows), ny, nx)."""
    b = basis
    a_s, a_p = downgoing_amplitudes(g, b, X_ev)
    u_s = np.where(b.live, r_te * a_s, 0.0)
    u_p = np.where(b.live, r_pe * a_p, 0.0)
    out = np.zeros((3, len(rows), g.ny, g.nx), np.complex128)
    for i, j in enumerate(rows):
        ph = np.exp(1j * b.kzb * g.z[j])
        out[0, i] = (u_s * b.sx + u_p * b.tx) * ph
        out[1, i] = (u_s * b.sy + u_p * b.ty) * ph
        out[2, i] = (-u_p * b.ktkz) * ph
    return out


def ml_field_hat_adjoint(g, basis, r_te, r_pe, Q, rows):
    """Adjoint of ml_field_hat (same rows): (3, len(rows), ny, nx) -> (3, ny, nx)."""
    b = basis
    c_s = np.zeros((g.ny, g.nx), np.complex128)
    c_p = np.zeros((g.ny, g.nx), np.complex128)
    for i, j in enumerate(rows):
        ph = np.conj(np.exp(1j * b.kzb * g.z[j]))
        c_s += ph * (b.sx * Q[0, i] + b.sy * Q[1, i])
        c_p += ph * (b.tx * Q[0, i] + b.ty * Q[1, i] - np.conj(b.ktkz) * Q[2, i])
    down = np.conj(np.exp(-1j * b.kzb * (0.5 * g.dz)))
    c_s = down * np.where(b.live, np.conj(r_te) * c_s, 0.0)
    c_p = down * np.where(b.live, np.conj(r_pe) * c_p, 0.0)
    wt = np.conj(b.w_t) * c_p
    return np.stack([b.sx * c_s + b.tx * wt, b.sy * c_s + b.ty * wt, np.conj(b.w_z) * c_p])


# --------------------------------------------------------------------------
# Incident field and analytic background source (paper, equation bg_source)
# --------------------------------------------------------------------------


def incident_vectors(g, pol):
    """Polarisation of the incident (downgoing) and reflected (upgoing) plane wave."""
    th, ph = g.theta, g.phi
    if pol == 0:
        e_in = np.array([-np.sin(ph), np.cos(ph), 0.0])
        e_up = e_in.copy()
    else:
        e_in = np.array([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), np.sin(th)])
        e_up = np.array([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
    return e_in, e_up


def background_field(g, cfg, rows=None):
    """E_inc + R_ml E_inc on the given rows, shape (3, len(rows)) (laterally uniform envelope).

    Unit amplitude, phase 0 at x = 0, z = z_ml; E_inc = e exp(-i kz0 z);
    the reflected part is r(theta) e_up exp(+i kz0 z) with r = r_TE or r_pE
    of the incidence mode."""
    if rows is None:
        rows = np.arange(g.nz)
    kt2 = g.kx0 ** 2 + g.ky0 ** 2
    r_te, r_pe = ml_reflection(g, cfg, kt2=np.array(kt2))
    r = r_te if cfg["pol"] == 0 else r_pe
    e_in, e_up = incident_vectors(g, cfg["pol"])
    z = g.z[rows]
    return (e_in[:, None] * np.exp(-1j * g.kz0 * z)[None, :]
            + complex(r) * e_up[:, None] * np.exp(1j * g.kz0 * z)[None, :])


class Problem:
    """Everything a solve needs: grid, permittivity contrast, reflections."""

    def __init__(self, cfg, eps_abs_rows):
        self.cfg = cfg
        self.g = Grid(cfg)
        eps = np.asarray(eps_abs_rows, dtype=np.complex128)
        assert eps.shape == (cfg["nz_abs"], cfg["ny"], cfg["nx"])
        self.deps = eps - cfg["eps_bg"]          # non-zero on absorber rows only
        self.basis = Basis(self.g)
        self.r_te, self.r_pe = ml_reflection(self.g, cfg)


def rhs(P):
    """b = k0^2 d_eps (E_inc + E_ML[E_inc]) (paper, equation bg_source)."""
    g = P.g
    bg = background_field(g, P.cfg, g.abs_rows)                  # (3, nz_abs)
    b = np.zeros(g.shape, np.complex128)
    b[:, g.abs_rows] = g.k0 ** 2 * P.deps[None] * bg[:, :, None, None]
    return b


# --------------------------------------------------------------------------
# Operator A (paper, equation vector_helmholtz_operator with R_ml inside A)
# --------------------------------------------------------------------------


def dz_apply(g, f):
    """D_z = diag(1/s) F_z^-1 diag(i kz) F_z along the axial axis (-3)."""
    F = np.fft.fft(f, axis=-3) * (1j * g.kz)[:, None, None]
    return np.fft.ifft(F, axis=-3) / g.s[:, None, None]


def dz_apply_adjoint_neg(g, f):
    """-(D_z)^H = F_z^-1 diag(i kz) F_z diag(1/conj(s))."""
    F = np.fft.fft(f / np.conj(g.s)[:, None, None], axis=-3) * (1j * g.kz)[:, None, None]
    return np.fft.ifft(F, axis=-3)


def curlcurl_hat(g, Xh, dz):
    """curl curl in (kx, ky, z): each lateral derivative is i*kappa, each axial one dz().

    Row by row the operator matrix of the paper (without the -k0^2 eps
    diagonal): (-dy dy - dz dz, dx dy, dx dz; ...)."""
    KX = g.kx[None, None, :]
    KY = g.ky[None, :, None]
    Ex, Ey, Ez = Xh
    dEx, dEy, dEz = dz(g, Ex), dz(g, Ey), dz(g, Ez)
    ddEx, ddEy = dz(g, dEx), dz(g, dEy)
    cx = KY * KY * Ex - ddEx - KX * KY * Ey + 1j * KX * dEz
    cy = -KX * KY * Ex + KX * KX * Ey - ddEy + 1j * KY * dEz
    cz = 1j * KX * dEx + 1j * KY * dEy + (KX * KX + KY * KY) * Ez
    return np.stack([cx, cy, cz])


def fft2(x):
    return np.fft.fft2(x, axes=(-2, -1))


def ifft2(x):
    return np.fft.ifft2(x, axes=(-2, -1))


def apply_A(P, x):
    """y = A x = F2^-1[CC X] - k0^2 eps x - k0^2 d_eps F2^-1[R_ml X],  X = F2 x."""
    g = P.g
    Xh = fft2(x)
    U = curlcurl_hat(g, Xh, dz_apply) - (g.kbg ** 2) * Xh
    y = ifft2(U)
    V = ml_field_hat(g, P.basis, P.r_te, P.r_pe, Xh[:, g.j_ev], g.abs_rows)
    e_ml = ifft2(V)
    ra = g.abs_rows
    y[:, ra] -= g.k0 ** 2 * P.deps[None] * (x[:, ra] + e_ml)
    return y


def apply_AH(P, x):
    """y = A^H x (adjoint for the inner product sum(conj(u) v) over the grid)."""
    g = P.g
    Xh = fft2(x)
    U = curlcurl_hat(g, Xh, dz_apply_adjoint_neg) - (g.kbg ** 2) * Xh
    ra = g.abs_rows
    dconj = g.k0 ** 2 * np.conj(P.deps)[None]
    Q = fft2(dconj * x[:, ra])
    U[:, g.j_ev] -= ml_field_hat_adjoint(g, P.basis, P.r_te, P.r_pe, Q, ra)
    y = ifft2(U)
    y[:, ra] -= dconj * x[:, ra]
    return y


# --------------------------------------------------------------------------
# Preconditioner (paper, equations spectral_damping_action / _mask)
# --------------------------------------------------------------------------


def damping_multiplier(k2, k_ref, m_min=0.0, gamma=1.0, reg=0.0):
    """m(k) = m_min + (1 - m_min) * {1 if |k| <= k_ref; (k_ref^2/(|k|^2 + reg))^gamma}."""
    k2 = np.asarray(k2, dtype=np.float64)
    with np.errstate(divide="ignore"):
        tail = (k_ref * k_ref / (k2 + reg)) ** gamma
    core = np.where(k2 <= k_ref * k_ref, 1.0, tail)
    return m_min + (1.0 - m_min) * core


def precond_multiplier(P):
    g = P.g
    cfg = P.cfg
    k_ref = cfg["pc_kref"] if cfg["pc_kref"] > 0 else g.kbg
    K2 = (g.kz[:, None, None] ** 2 + g.ky[None, :, None] ** 2 + g.kx[None, None, :] ** 2)
    return damping_multiplier(K2, k_ref, cfg["pc_mmin"], cfg["pc_gamma"], cfg["pc_reg"])


def apply_M(P, x):
    """(M x)_alpha = F3^-1[m(k) F3 x_alpha] for each Cartesian component."""
    m = precond_multiplier(P)
    return np.fft.ifftn(m[None] * np.fft.fftn(x, axes=(1, 2, 3)), axes=(1, 2, 3))


# --------------------------------------------------------------------------
# BiCGSTAB with right preconditioning and affine warm start
# --------------------------------------------------------------------------


def _dot(u, v):
    return np.vdot(u.ravel(), v.ravel())


def _nrm(u):
    return float(np.linalg.norm(u.ravel()))


OMEGA_LIMIT = 0.7


def bicgstab_core(op, prec, r0, bnorm, tol, maxit, history=None):
    """Right-preconditioned BiCGSTAB on  op(prec(y)) = r0,  y0 = 0.

    Van der Vorst recurrences, shadow residual = r0, with the stabilising
    step omega = <t,s>/<t,t> limited as proposed by Sleijpen and van der
    Vorst (1995): if |<t,s>| < kappa ||t|| ||s|| (kappa = 0.7) omega is
    scaled by kappa ||t|| ||s|| / |<t,s>|.  The paper names BiCGSTAB without
    a variant; the limited step has the same fixed point.  Returns
    (y_hat, iterations, status) where y_hat = prec(y) accumulated directly,
    status 'converged', 'maxit' or 'breakdown'."""
    r = r0.copy()
    rh = r0.copy()
    rho_prev = alpha = omega = 1.0 + 0j
    v = np.zeros_like(r0)
    p = np.zeros_like(r0)
    yh = np.zeros_like(r0)
    rho = _dot(rh, r)
    rh_n = _nrm(rh)
    for it in range(1, maxit + 1):
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = prec(p)
        v = op(ph)
        rv = _dot(rh, v)
        if abs(rv) <= 1e-30 * rh_n * _nrm(v):
            return yh, it - 1, "breakdown"
        alpha = rho / rv
        s = r - alpha * v
        sn = _nrm(s)
        if sn / bnorm <= tol:
            yh = yh + alpha * ph
            if history is not None:
                history.append(sn / bnorm)
            return yh, it, "converged"
        sh = prec(s)
        t = op(sh)
        tt = _dot(t, t).real
        if tt == 0:
            yh = yh + alpha * ph
            return yh, it, "breakdown"
        ts = _dot(t, s)
        omega = ts / tt
        # omega limiting: keep |<t,s>| / (||t|| ||s||) from falling below kappa
        c = abs(ts) / (np.sqrt(tt) * sn)
        if 0.0 < c < OMEGA_LIMIT:
            omega *= OMEGA_LIMIT / c
        yh = yh + alpha * ph + omega * sh
        r = s - omega * t
        rn = _nrm(r)
        if history is not None:
            history.append(rn / bnorm)
        if rn / bnorm <= tol:
            return yh, it, "converged"
        rho_prev = rho
        rho = _dot(rh, r)
        if omega == 0 or abs(rho) <= 1e-30 * rh_n * rn:
            return yh, it, "breakdown"
    return yh, maxit, "maxit"


def solve(P, b=None, x0=None, tol=1e-10, maxit=20000, precond=None, adjoint=False,
          history=None, max_restarts=10):
    """Solve A E = b (or A^H E = b) to  ||b - A E|| / ||b|| <= tol.

    Affine right-corrected warm start E = E_base + M y with A M y = b - A E_base;
    E_base = x0 (zero when None).  After each BiCGSTAB run the true residual
    is recomputed; if it exceeds tol the solve restarts from the current E
    (residual replacement, at most max_restarts times).  ||b|| = 0 returns
    E = 0.  Returns (E, info) with info = dict(iters, rrel, status)."""
    op = (lambda u: apply_AH(P, u)) if adjoint else (lambda u: apply_A(P, u))
    use_pc = P.cfg["precond"] if precond is None else precond
    prec = (lambda u: apply_M(P, u)) if use_pc else (lambda u: u)
    if b is None:
        b = rhs(P)
    bnorm = _nrm(b)
    if bnorm == 0.0:
        return np.zeros(P.g.shape, np.complex128), {"iters": 0, "rrel": 0.0, "status": "converged"}
    E = np.zeros(P.g.shape, np.complex128) if x0 is None else np.array(x0, np.complex128)
    iters = 0
    status = "maxit"
    rrel = None
    for _ in range(max_restarts + 1):
        r = b.copy() if (x0 is None and iters == 0) else b - op(E)
        rrel = _nrm(r) / bnorm
        if history is not None and iters == 0:
            history.append(rrel)
        if rrel <= tol:
            status = "converged"
            break
        if iters >= maxit:
            break
        yh, it, st = bicgstab_core(op, prec, r, bnorm, tol, maxit - iters, history)
        E = E + yh
        iters += it
        rrel = _nrm(b - op(E)) / bnorm
        if rrel <= tol:
            status = "converged"
            break
        status = "maxit" if st == "maxit" else status
    return E, {"iters": iters, "rrel": rrel, "status": status}


# --------------------------------------------------------------------------
# Sensitivity to the permittivity (adjoint method)
# --------------------------------------------------------------------------


def local_field(P, E):
    """Psi = E + E_ML[E] + (E_inc + R_ml E_inc) on absorber rows: the field that
    d_eps multiplies in A E - b (equations bg_source and vector_helmholtz_operator
    with R_ml inside A), shape (3, nz_abs, ny, nx)."""
    g = P.g
    Xh = fft2(E)
    V = ml_field_hat(g, P.basis, P.r_te, P.r_pe, Xh[:, g.j_ev], g.abs_rows)
    bg = background_field(g, P.cfg, g.abs_rows)
    return E[:, g.abs_rows] + ifft2(V) + bg[:, :, None, None]


def eps_gradient(P, E, u, scale):
    """scale * sum_alpha u_alpha conj(Psi_alpha) on absorber voxels.

    A E - b depends on eps only through -k0^2 d_eps * Psi(E), so for a loss L
    of the solution E = A^-1 b with gradient g (dL/dRe E + i dL/dIm E), the
    gradient with respect to eps is k0^2 sum_alpha mu_alpha conj(Psi_alpha)
    with mu = A^-H g."""
    return scale * np.sum(u[:, P.g.abs_rows] * np.conj(local_field(P, E)), axis=0)


def residual_loss(P, E):
    """Mean squared residual (1/N) ||A E - b||^2, N = nx ny nz (paper, equation
    loss, first term)."""
    r = apply_A(P, E) - rhs(P)
    return float(np.vdot(r, r).real) / (P.g.nx * P.g.ny * P.g.nz)


def hf_weight(P, w0, eta):
    """w(nu) = w0 + eta |nu| on the bins of the 3-D DFT of a field, shape (nz, ny, nx).

    |nu| = |k| / (2 pi) with k the physical wavenumber of each bin: the
    Bloch-shifted lateral wavenumbers of the grid and the axial ones (the
    paper names the spatial frequency without saying how the Bloch phase
    enters; the damping preconditioner uses the same wavenumbers)."""
    g = P.g
    K2 = g.kz[:, None, None] ** 2 + g.ky[None, :, None] ** 2 + g.kx[None, None, :] ** 2
    return w0 + eta * np.sqrt(K2) / (2.0 * np.pi)


def hf_penalty(P, r, w0, eta, lam):
    """(lam / N) sum_alpha ||w(nu) F3[r_alpha]||^2, F3 the unnormalised 3-D DFT
    (paper, equation loss, second term)."""
    g = P.g
    n = g.nx * g.ny * g.nz
    R3 = np.fft.fftn(r, axes=(1, 2, 3))
    w = hf_weight(P, w0, eta)
    return lam * float(np.sum(np.abs(w[None] * R3) ** 2)) / n


def pino_loss(P, E, w0, eta, lam):
    """The whole physics loss (paper, equation loss) at E: (J, residual term,
    penalty term) with r = A E - b."""
    g = P.g
    n = g.nx * g.ny * g.nz
    r = apply_A(P, E) - rhs(P)
    t1 = float(np.vdot(r, r).real) / n
    t2 = hf_penalty(P, r, w0, eta, lam)
    return t1 + t2, t1, t2


def pino_loss_field(P, E, w0, eta, lam):
    """u = dJ/d conj(r) = (1/N) r + (lam/N) F3^H w^2 F3 r, r = A E - b (F3^H = N F3^-1)."""
    g = P.g
    n = g.nx * g.ny * g.nz
    r = apply_A(P, E) - rhs(P)
    w2 = hf_weight(P, w0, eta) ** 2
    FH = n * np.fft.ifftn(w2[None] * np.fft.fftn(r, axes=(1, 2, 3)), axes=(1, 2, 3))
    return r / n + (lam / n) * FH


def pino_loss_grad(P, E, w0, eta, lam):
    """Gradients of the physics loss in PyTorch's convention (dJ/dRe + i dJ/dIm):
    with respect to E, 2 A^H u; with respect to eps on absorber voxels,
    -2 k0^2 sum_alpha u_alpha conj(Psi_alpha) (A E - b depends on eps through
    -k0^2 d_eps Psi(E)); u = pino_loss_field."""
    u = pino_loss_field(P, E, w0, eta, lam)
    return 2.0 * apply_AH(P, u), eps_gradient(P, E, u, -2.0 * P.g.k0 ** 2)


# --------------------------------------------------------------------------
# Outputs and diagnostics
# --------------------------------------------------------------------------


def intensity_obs(P, E):
    """|E_y^scat|^2 on the observation row (first row above the absorber)."""
    return np.abs(E[1, P.g.j_obs]) ** 2


def reflected_obs(P, E):
    """(E_scat + E_ML) on the observation row, lateral Fourier coefficients / (nx ny).

    E_ML is R_ml applied to the total downgoing field (scattered plus
    incident) at the multilayer interface."""
    g = P.g
    Xh = fft2(E)
    up = ml_field_hat(g, P.basis, P.r_te, P.r_pe, Xh[:, g.j_ev], [g.j_obs])[:, 0]
    tot = (Xh[:, g.j_obs] + up) / (g.nx * g.ny)
    bgr = background_field(g, P.cfg, [g.j_obs])[:, 0]
    e_in, _ = incident_vectors(g, P.cfg["pol"])
    refl_bg = bgr - e_in * np.exp(-1j * g.kz0 * g.z[g.j_obs])
    tot[:, 0, 0] += refl_bg
    return tot


def flux_balance(P, E):
    """(reflected flux + flux into the multilayer) / incident flux, propagating modes.

    Flux weights per unit tangential-E amplitude: kz for TE, kbg^2/kz for TM.
    Reflected amplitudes are read at the observation row, downgoing
    amplitudes (scattered plus incident) at z_ml from the evaluation row."""
    g, b = P.g, P.basis
    prop = (np.abs(b.kzb.imag) < 1e-12 * g.k0) & (b.kzb.real > 0)
    kz = np.where(prop, b.kzb.real, 1.0)
    up = reflected_obs(P, E)
    ph_obs = np.exp(-1j * b.kzb * g.z[g.j_obs])
    us = (b.sx * up[0] + b.sy * up[1]) * ph_obs
    upp = (b.tx * up[0] + b.ty * up[1]) * ph_obs
    w_s, w_p = kz, g.kbg ** 2 / kz
    f_up = np.sum(np.where(prop, w_s * np.abs(us) ** 2 + w_p * np.abs(upp) ** 2, 0.0))
    Xh = fft2(E) / (g.nx * g.ny)
    ds, dp = downgoing_amplitudes(g, b, Xh[:, g.j_ev])
    e_in, _ = incident_vectors(g, P.cfg["pol"])
    ds[0, 0] += b.sx[0, 0] * e_in[0] + b.sy[0, 0] * e_in[1]
    dp[0, 0] += b.w_t[0, 0] * (b.tx[0, 0] * e_in[0] + b.ty[0, 0] * e_in[1]) + b.w_z[0, 0] * e_in[2]
    f_ml = np.sum(np.where(prop, (1 - np.abs(P.r_te) ** 2) * w_s * np.abs(ds) ** 2
                           + (1 - np.abs(P.r_pe) ** 2) * w_p * np.abs(dp) ** 2, 0.0))
    return float((f_up + f_ml) / g.kz0)


# --------------------------------------------------------------------------
# Standard full-domain PSFD, the comparison case of the paper's Results
# section ("Background-decomposition" paragraph and its first figure): the
# multilayer is discretised in eps on the grid and there is no R_ml.  In this
# module that is a Problem whose configuration has no multilayer (r_TE =
# r_TM = 0) and whose "absorber" rows hold the stack.
# --------------------------------------------------------------------------


def layered_eps_rows(nz_abs, dz, layers_eps, layers_d, eps_bg):
    """Permittivity of a planar stack averaged over each absorber row, shape (nz_abs,).

    The stack (layers listed top to bottom) hangs from the top face of the
    region, z = nz_abs dz; whatever it does not cover is background.  Row j
    spans [j dz, (j + 1) dz) and takes the thickness-weighted mean of eps
    over that interval.  The paper does not say how its standard solver
    samples the stack; the mean is the effective permittivity for fields
    tangential to the layers (TE)."""
    top = nz_abs * dz
    out = np.empty(nz_abs, np.complex128)
    for j in range(nz_abs):
        lo, hi = j * dz, (j + 1) * dz
        acc, covered = 0j, 0.0
        z_hi = top
        for e, d in zip(layers_eps, layers_d):
            z_lo = z_hi - d
            ov = max(0.0, min(hi, z_hi) - max(lo, z_lo))
            acc += complex(e) * ov
            covered += ov
            z_hi = z_lo
        out[j] = (acc + eps_bg * (dz - covered)) / dz
    return out


def specular_reflection(P, E):
    """Specular (0, 0)-order reflection coefficient of the whole structure,
    referred to the top face of the absorber region, z_t = nz_abs dz.

    The total upgoing (0, 0) amplitude at the observation row per unit
    incident amplitude (reflected_obs: scattered field, the multilayer
    response to it and the multilayer reflection of the incident wave) is
    projected on s_hat (TE) or on t_hat and divided by -cos(theta) (TM, the
    magnetic-field sign convention of tmm_reflection), then carried from
    the observation row back to the face, where the incident wave has
    phase exp(-i kz0 z_t):  r = value * exp(-i kz0 z_obs) * exp(2 i kz0 z_t)."""
    g, b = P.g, P.basis
    up = reflected_obs(P, E)[:, 0, 0]
    if P.cfg["pol"] == 0:
        val = b.sx[0, 0] * up[0] + b.sy[0, 0] * up[1]
    else:
        val = -(b.tx[0, 0] * up[0] + b.ty[0, 0] * up[1]) / np.cos(g.theta)
    z_t = g.nz_abs * g.dz
    return complex(val * np.exp(-1j * g.kz0 * g.z[g.j_obs]) * np.exp(2j * g.kz0 * z_t))


# --------------------------------------------------------------------------
# Dense forms for tiny grids
# --------------------------------------------------------------------------


def dense_by_columns(P, op=None):
    """Assemble the matrix of op (default A) column by column from unit vectors."""
    op = op or (lambda u: apply_A(P, u))
    shape = P.g.shape
    n = int(np.prod(shape))
    A = np.empty((n, n), np.complex128)
    e = np.zeros(n, np.complex128)
    for k in range(n):
        e[k] = 1.0
        A[:, k] = op(e.reshape(shape)).ravel()
        e[k] = 0.0
    return A


def dft_matrix(n):
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def dense_kronecker(P):
    """A assembled from explicit DFT matrices (no FFT routine involved).

    A = T^-1 C T - k0^2 diag(eps) - k0^2 diag(d_eps) T^-1 R T, where T is
    the lateral DFT on every (component, row) plane, C holds the per-mode
    curl-curl blocks with D_z = diag(1/s) Fz^-1 diag(i kz) Fz, and R maps
    the evaluation-row coefficients to absorber rows."""
    g, b = P.g, P.basis
    nx, ny, nz = g.nx, g.ny, g.nz
    L = nx * ny
    F2 = np.kron(dft_matrix(ny), dft_matrix(nx))
    F2i = np.conj(F2).T / L
    Fz = dft_matrix(nz)
    Dz = np.diag(1.0 / g.s) @ (np.conj(Fz).T / nz) @ np.diag(1j * g.kz) @ Fz
    I = np.eye(nz)
    n = 3 * nz * L
    C = np.zeros((n, n), np.complex128)
    R = np.zeros((n, n), np.complex128)

    def idx(c, q):
        return (c * nz + np.arange(nz)) * L + q

    KX = np.broadcast_to(g.kx[None, :], (ny, nx)).ravel()
    KY = np.broadcast_to(g.ky[:, None], (ny, nx)).ravel()
    r_te, r_pe = P.r_te.ravel(), P.r_pe.ravel()
    sx, sy, tx, ty = b.sx.ravel(), b.sy.ravel(), b.tx.ravel(), b.ty.ravel()
    kzb, ktkz, live = b.kzb.ravel(), b.ktkz.ravel(), b.live.ravel()
    w_t, w_z = b.w_t.ravel(), b.w_z.ravel()
    DD = Dz @ Dz
    for q in range(L):
        kx, ky = KX[q], KY[q]
        blocks = [[ky * ky * I - DD, -kx * ky * I, 1j * kx * Dz],
                  [-kx * ky * I, kx * kx * I - DD, 1j * ky * Dz],
                  [1j * kx * Dz, 1j * ky * Dz, (kx * kx + ky * ky) * I]]
        for c in range(3):
            for c2 in range(3):
                blk = blocks[c][c2] - (g.kbg ** 2 * I if c == c2 else 0.0)
                C[np.ix_(idx(c, q), idx(c2, q))] = blk
        if not live[q]:
            continue
        down = np.exp(-1j * kzb[q] * 0.5 * g.dz)
        ws = [sx[q], sy[q], 0.0]
        wp = [tx[q], ty[q], -ktkz[q]]
        src_s = [sx[q], sy[q], 0.0]
        src_p = [w_t[q] * tx[q], w_t[q] * ty[q], w_z[q]]
        for j in g.abs_rows:
            ph = np.exp(1j * kzb[q] * g.z[j]) * down
            for c in range(3):
                row = (c * nz + j) * L + q
                for c2 in range(3):
                    col = (c2 * nz + g.j_ev) * L + q
                    R[row, col] = ph * (r_te[q] * ws[c] * src_s[c2] + r_pe[q] * wp[c] * src_p[c2])
    T = np.kron(np.eye(3 * nz), F2)
    Ti = np.kron(np.eye(3 * nz), F2i)
    de = np.zeros((3, nz, ny, nx), np.complex128)
    de[:, g.abs_rows] = P.deps[None]
    de = de.ravel()
    A = Ti @ C @ T - g.k0 ** 2 * np.diag(de) - g.k0 ** 2 * (de[:, None] * (Ti @ R @ T))
    return A


def slab_1d_matrix(P):
    """Dense 3nz x 3nz matrix of the (0, 0) lateral mode for a laterally uniform d_eps.

    Explicit D_z matrix and low-rank multilayer coupling; used to pin the
    3-D solve of a uniform slab against a 1-D solve."""
    g, b = P.g, P.basis
    nz = g.nz
    Fz = dft_matrix(nz)
    Dz = np.diag(1.0 / g.s) @ (np.conj(Fz).T / nz) @ np.diag(1j * g.kz) @ Fz
    I = np.eye(nz)
    kx, ky = g.kx[0], g.ky[0]
    DD = Dz @ Dz
    blocks = [[ky * ky * I - DD, -kx * ky * I, 1j * kx * Dz],
              [-kx * ky * I, kx * kx * I - DD, 1j * ky * Dz],
              [1j * kx * Dz, 1j * ky * Dz, (kx * kx + ky * ky) * I]]
    A = np.block(blocks) - g.kbg ** 2 * np.eye(3 * nz)
    de = np.zeros(nz, np.complex128)
    de[g.abs_rows] = P.deps[:, 0, 0]
    A -= g.k0 ** 2 * np.diag(np.tile(de, 3))
    if b.live[0, 0]:
        down = np.exp(-1j * b.kzb[0, 0] * 0.5 * g.dz)
        ws = [b.sx[0, 0], b.sy[0, 0], 0.0]
        wp = [b.tx[0, 0], b.ty[0, 0], -b.ktkz[0, 0]]
        for j in g.abs_rows:
            ph = np.exp(1j * b.kzb[0, 0] * g.z[j]) * down
            src_s = [b.sx[0, 0], b.sy[0, 0], 0.0]
            src_p = [b.w_t[0, 0] * b.tx[0, 0], b.w_t[0, 0] * b.ty[0, 0], b.w_z[0, 0]]
            for c in range(3):
                for c2 in range(3):
                    A[c * nz + j, c2 * nz + g.j_ev] -= g.k0 ** 2 * de[j] * ph * (
                        P.r_te[0, 0] * ws[c] * src_s[c2] + P.r_pe[0, 0] * wp[c] * src_p[c2])
    return A
