/*
 * psfd.h -- C ABI of the MI355X PSFD solver library (libpsfd.so).
 *
 * The library solves the background-decomposed, right-preconditioned
 * pseudo-spectral frequency-domain (PSFD) full-vector scattering equations
 * of an EUV mask absorber above a multilayer mirror:
 *
 *     A E = b,   A = curl curl - k0^2 eps - k0^2 d_eps R_ml,
 *     b = k0^2 d_eps (E_inc + R_ml E_inc)
 *
 * (paper: section 2.2, equations vector_helmholtz_operator and bg_source,
 * and the definition of the multilayer reflection operator R_ml), with
 * BiCGSTAB, the spectral damping right preconditioner M and the affine warm
 * start E = E_base + M y (Results, "PINO warm-start" paragraph, equations
 * spectral_damping_action, spectral_damping_mask, right_preconditioned,
 * right_correction_solution, right_preconditioned_system,
 * relative_residual).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.  Axial rows from the bottom: nz_pml PML | nz_gap_bot gap |
 *   nz_abs absorber | nz_gap_top gap | nz_pml PML;
 *   Nz = nz_abs + nz_gap_bot + nz_gap_top + 2 nz_pml.  Rows are
 *   cell-centred, z = 0 is the absorber's bottom face (the multilayer
 *   interface), the z axis is periodic.  Lateral grid nx x ny, periodic,
 *   with Bloch-shifted wavenumbers for oblique incidence.
 * Field layout.  Structure of arrays [3][Nz][ny][nx] (component x, y, z;
 *   then row; then y; x fastest), each element an interleaved complex pair
 *   (re, im).  Element type complex128 (two doubles) unless an entry point
 *   says complex64.
 * Memory.  Every field pointer is a caller-owned DEVICE pointer on the
 *   device current when the plan was made, 16-byte aligned (8-byte for
 *   complex64).  Inputs and outputs must not overlap unless stated.  The
 *   plan owns its workspace.  Host pointers appear only inside psfd_desc
 *   (the multilayer tables) and for psfd_info.
 * Streams.  Work is enqueued on the HIP stream given to psfd_plan (NULL =
 *   the default stream).  Calls are asynchronous unless stated otherwise;
 *   psfd_solve synchronises the stream to test convergence.
 * Errors.  No exception crosses the ABI.  A non-zero psfd_status is
 *   returned and psfd_last_error() gives a message (thread-local).  Invalid
 *   arguments return PSFD_ERR_ARG before any buffer is touched.
 * Threads.  A plan may be used by one host thread at a time.
 */
#ifndef PSFD_H
#define PSFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psfd_plan* psfd_plan_t;

typedef enum {
  PSFD_OK = 0,
  PSFD_ERR_ARG = 1,        /* invalid argument or unsupported size          */
  PSFD_ERR_ALLOC = 2,      /* device allocation failed                      */
  PSFD_ERR_HIP = 3,        /* a HIP runtime call or kernel launch failed    */
  PSFD_NOT_CONVERGED = 4,  /* maxit reached before the tolerance            */
  PSFD_BREAKDOWN = 5       /* BiCGSTAB broke down and restarts were used up */
} psfd_status;

typedef enum {
  PSFD_C128 = 0,              /* complex128 everywhere                                  */
  PSFD_C64_REFINE64 = 1,      /* complex64 operator/preconditioner/Krylov vectors,
                                 FP64 true residual and refinement updates              */
  PSFD_C64_BF16PC_REFINE64 = 2 /* as 1, with the preconditioner's output spectrum     */
                                /* m(k) F3 x held in bfloat16 (see below)                */
} psfd_precision;

/* PSFD_C64_BF16PC_REFINE64, the bfloat16 preconditioner trial: inside every
 * complex64 M and A.M apply the damped spectrum m(k) F3 x -- the
 * preconditioner's data -- is rounded to bfloat16 right after the damping
 * and used in that form from there on (its x and y components are parked in
 * LDS as packed bfloat16 pairs).  M is then a rounded, not exactly linear,
 * operator; the FP64 reliable updates keep the recursive and the true
 * residual together.  A itself and the FP64 applies are unchanged. */

/* Plan descriptor.  Lengths in nm, angles in radians.
 * Supported sizes: nx, ny in {16, 32, 64, 128, 192, 256, 512, 1024};
 * Nz in {24, 32, 48, 64, 96, 128} (the register-resident and LDS axial
 * kernels) or {192, 256, 324, 384, 576, 648, 768} (tall columns of the
 * full-domain comparison, LDS axial kernel only); nz_abs >= 1; nz_gap_bot >= 1 (the
 * evaluation row of the multilayer split is the last bottom-gap row). */
typedef struct {
  int32_t nx, ny, nz_abs, nz_gap_bot, nz_gap_top, nz_pml;
  double dx, dy, dz, lambda;
  double theta, phi;             /* incidence polar / azimuth angle               */
  int32_t pol;                   /* 0 = TE (s), 1 = TM (p)                        */
  double eps_bg;                 /* real background permittivity of the domain   */
  int32_t n_ml;                  /* number of multilayer layers (may be 0)       */
  const double* ml_eps;          /* host, [n_ml][2] complex permittivity, top->bottom */
  const double* ml_thick;        /* host, [n_ml] thickness                        */
  double eps_sub[2];             /* substrate permittivity (complex)             */
  double pml_sigma0;             /* PML stretch s = 1 + i sigma0 (d/D)^order      */
  int32_t pml_order;
  int32_t precond;               /* 0 = none, 1 = spectral damping M              */
  double pc_mmin, pc_kref, pc_gamma, pc_reg; /* m(k) parameters; pc_kref <= 0 -> k0 sqrt(eps_bg) */
  int32_t prec;                  /* psfd_precision                                */
  double ml_kz_min;              /* lateral modes with |kz| < max(ml_kz_min, 1e-9) k0 get no
                                    multilayer response (grazing orders); 0 = default   */
} psfd_desc;

typedef struct {
  int32_t iters;        /* BiCGSTAB iterations (one = two operator applies)          */
  int32_t status;       /* psfd_status of the solve                                  */
  int32_t restarts;     /* residual replacements / refinement steps taken           */
  int32_t applies;      /* operator applies in the working precision                 */
  double rrel_true;     /* ||b - A E|| / ||b|| recomputed in FP64 at exit            */
  double rrel_hist_last;/* last recursive residual seen by the Krylov loop           */
} psfd_info;

/* Gaussian smoothing of a binary layout and material map (paper, section
 * 2.1 closing paragraphs and Results, "PINO surrogate": the binary indicator
 * is Gaussian-smoothed on the grid, and the same smoothing is applied to the
 * structure of the rigorous PSFD solve).
 *   a_bin_dev  device, [ny][nx] double, values in {0, 1}
 *   eps_abs    absorber permittivity (re, im)
 *   sigma      smoothing width in lateral cells
 *   eps_out    device, [nz_abs][ny][nx] complex128: eps = eps_bg + a (eps_abs - eps_bg),
 *              a = clip(periodic Gaussian smoothing of a_bin, 0, 1), same on every row.
 * Uses d->nx, ny, nz_abs, dx, dy, eps_bg only.  Allocates and frees a
 * temporary workspace and synchronises the stream. */
psfd_status psfd_layout_eps(const psfd_desc* d, const double* a_bin_dev, const double eps_abs[2],
                            double sigma, void* eps_out, void* hip_stream);

/* psfd_layout_eps for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments and result (equal up to the last bits of the twiddles, which
 * are generated on the device here).  It calls no hipMalloc / hipFree and
 * does not synchronise: the work is queued on hip_stream, and eps_out is
 * ready when the stream reaches that point.  Its workspace is a fixed
 * library-owned device array of 8 MiB per GPU (two lateral planes and two
 * twiddle tables), held until the process ends; the caller's current device
 * must be the stream's device.
 * Limits: nx * ny <= 512 * 512 (larger layouts return PSFD_ERR_ARG; use
 * psfd_layout_eps).  Calls on one GPU share the workspace: calls that may
 * overlap in time on one GPU (different streams without ordering between
 * them) race and must be serialised by the caller. */
psfd_status psfd_layout_eps_noalloc(const psfd_desc* d, const double* a_bin_dev,
                                    const double eps_abs[2], double sigma, void* eps_out,
                                    void* hip_stream);

/* Build a plan (paper, section 2.2: lateral Bloch wavenumbers, PML stretch,
 * per-mode multilayer reflections r_TE and r_pE by the transfer-matrix
 * method, permittivity contrast).  eps_abs_dev: device, [nz_abs][ny][nx]
 * complex128 permittivity on absorber rows (copied; the caller may free it).
 * The multilayer tables in d are copied.  The TMM runs on the device. */
psfd_status psfd_plan(const psfd_desc* d, const void* eps_abs_dev, void* hip_stream,
                      psfd_plan_t* out);

/* Replace the permittivity of an existing plan (same sizes).  eps_abs_dev as
 * in psfd_plan.  Used for gradient checks and design loops. */
psfd_status psfd_set_eps(psfd_plan_t p, const void* eps_abs_dev);

/* b = k0^2 d_eps (E_inc + R_ml E_inc) (equation bg_source): incident plane
 * wave of unit amplitude, phase 0 at x = 0, z = 0, and its analytic
 * multilayer reflection.  b: device [3][Nz][ny][nx] complex128 (zero outside
 * absorber rows). */
psfd_status psfd_rhs(psfd_plan_t p, void* b);

/* y = A x (equation vector_helmholtz_operator with R_ml inside the operator:
 * lateral FFTs, axial pseudo-spectral derivatives with PML stretching,
 * curl curl, -k0^2 eps, and -k0^2 d_eps times the reflected multilayer field
 * of x).  x, y: device [3][Nz][ny][nx] complex128, must not overlap. */
psfd_status psfd_apply(psfd_plan_t p, const void* x, void* y);

/* y = A^H x (adjoint for the inner product sum conj(u) v over the grid). */
psfd_status psfd_adjoint(psfd_plan_t p, const void* x, void* y);

/* y = M x: per component F3^-1[m(k) F3 x] (equations spectral_damping_action
 * and spectral_damping_mask, |k| from the Bloch-shifted wavenumbers).  M is
 * Hermitian.  Applied regardless of d->precond. */
psfd_status psfd_precond(psfd_plan_t p, const void* x, void* y);

/* complex64 variants of apply / adjoint / precond (single-precision
 * kernels).  x, y: device [3][Nz][ny][nx] complex64. */
psfd_status psfd_apply_c64(psfd_plan_t p, const void* x, void* y);
psfd_status psfd_adjoint_c64(psfd_plan_t p, const void* x, void* y);
psfd_status psfd_precond_c64(psfd_plan_t p, const void* x, void* y);

/* Solve A E = b (adjoint = 0) or A^H E = b (adjoint = 1) by right-
 * preconditioned BiCGSTAB with the affine warm start E = x0 + M y,
 * A M y = b - A x0 (equations right_correction_solution and
 * right_preconditioned_system), stopping when the FP64 true relative
 * residual ||b - A E|| / ||b|| (equation relative_residual) is <= tol.
 *   b      device complex128 field, or NULL for the analytic source psfd_rhs
 *   x0     device complex128 field, or NULL for E_base = 0
 *   E      device complex128 field (output; may alias x0)
 *   maxit  iteration cap (one iteration = two operator applies)
 *   info   host, optional (may be NULL)
 * ||b|| = 0 gives E = 0, iters = 0, PSFD_OK.  For PSFD_C64_* plans the
 * Krylov iteration runs in complex64 inside an FP64 iterative-refinement
 * loop; it needs more iterations than PSFD_C128 (about 1.2x at 256^2 x 48,
 * up to 2.3x on 1024^2 grids below r_rel 1e-4, where the complex64
 * recursion slows), each at about 0.55x the FP64 cost.  Returns
 * PSFD_NOT_CONVERGED / PSFD_BREAKDOWN when the tolerance was not reached (E
 * then holds the best iterate).  Synchronises the stream. */
psfd_status psfd_solve(psfd_plan_t p, const void* b, const void* x0, void* E, double tol,
                       int32_t maxit, int32_t adjoint, psfd_info* info);

/* psfd_solve with a caller-given shadow residual: BiCGSTAB leaves the choice
 * of the shadow vector r^ open (any r^ with <r^, r0> != 0); psfd_solve takes
 * r^ = r0.  shadow: device complex128 field (single-problem plan), the r^ of
 * the first Krylov run; later runs (restarts from the current field) take
 * their own starting residual.  A shadow with |<r^, r0>| <= 1e-30 ||r^|| ||r0||
 * is a breakdown before the first step: that run ends with no iteration, E is
 * unchanged, and the solve restarts from E with r^ = r (info.restarts counts
 * the extra run).  Other arguments, results and errors as psfd_solve; an x0
 * with a non-finite residual returns PSFD_ERR_ARG before E is written (both
 * entry points). */
psfd_status psfd_solve_shadow(psfd_plan_t p, const void* b, const void* x0, void* E, double tol,
                              int32_t maxit, int32_t adjoint, const void* shadow,
                              psfd_info* info);

/* r = b - A E in FP64 (b = NULL: the analytic source psfd_rhs) and, if
 * norm2 != NULL, ||r||^2 (host, synchronises).  E, r: device complex128
 * fields; r must not overlap E or b.  The residual of equation
 * relative_residual, and the residual term of the physics loss of the paper
 * (section 2.2, equation loss, first term). */
psfd_status psfd_residual(psfd_plan_t p, const void* b, const void* E, void* r, double* norm2);

/* Sensitivity of the PSFD system to the permittivity (adjoint method):
 *   grad[v] = scale * sum_alpha u_alpha(v) conj(Psi_alpha(v)),
 *   Psi = E + R_ml[E] + (E_inc + R_ml E_inc)   on absorber voxels v,
 * i.e. the field that d_eps multiplies in A E - b (equations bg_source and
 * vector_helmholtz_operator with R_ml inside A).  With u = A^{-H} g and
 * scale = k0^2 this is dL/d eps for a loss L(E) whose gradient with respect
 * to the solution E = A^{-1} b is g (PyTorch convention: grad = dL/dRe +
 * i dL/dIm).  E, u: device complex128 fields; grad: device [nz_abs][ny][nx]
 * complex128 (overwritten). */
psfd_status psfd_eps_grad(psfd_plan_t p, const void* E, const void* u, double scale, void* grad);

/* The physics loss of the paper's PINO (section 2.2, equation loss, with its
 * frequency weight w(nu) = w0 + eta_hf |nu|) at a field E:
 *   J = (1/N) sum_alpha ||r_alpha||^2
 *     + (lambda_hf/N) sum_alpha ||w(nu) F3[r_alpha]||^2,   r = A E - b,
 * N = nx ny Nz, F3 the unnormalised 3-D DFT, |nu| = |k| / (2 pi) with k the
 * plan's (Bloch-shifted lateral, axial) wavenumber of each DFT bin, in 1/nm.
 * The paper does not give w0, eta_hf, lambda_hf: they are arguments.
 *   E     device [3][Nz][ny][nx] complex128
 *   loss  host out, [3]: J, the residual term, the penalty term
 *   g     device out or NULL: the field g = (1/N) r' + lambda_hf H r' with
 *         r' = b - A E and H = F3^-1 w^2 F3; the gradients then follow as
 *         dJ/dE = -2 A^H g (psfd_adjoint) and dJ/d eps = psfd_eps_grad(E, g,
 *         2 k0^2) (PyTorch convention grad = dJ/dRe + i dJ/dIm).
 * The penalty is evaluated as lambda_hf <r', H r'> (Parseval), one spectral
 * pass with w^2 as its multiplier whose inner product rides on the last
 * lateral pass.  Single-problem plans; g must not overlap E; synchronises. */
psfd_status psfd_pino_loss(psfd_plan_t p, const void* E, double w0, double eta_hf,
                           double lambda_hf, double loss[3], void* g);

/* Batched solves of independent problems (mask clips x incidence angles x
 * polarisations, uneven sizes allowed).  psfd_plan_batch validates and
 * records n problems: the descriptors and multilayer tables are copied; the
 * permittivity pointers eps_abs_dev[i] (as in psfd_plan) are kept and must
 * stay valid until psfd_solve_batch returns.  The returned handle is only
 * usable with psfd_solve_batch and psfd_destroy.  psfd_solve_batch solves
 * every problem (source b = psfd_rhs of that problem, E_i = x0[i] + M y,
 * as psfd_solve) after the work queued on the batch's stream.  Problems that
 * share everything but angle, polarisation and permittivity are solved as
 * one group (largest first, at most 2^26 voxels and 256 problems per group,
 * PSFD_GROUP_VOXELS / PSFD_GROUP_MAX in the environment): every kernel launch
 * covers the whole group, each problem keeps its own Krylov scalars and
 * refinement and stops on its own, and a 16-iteration chunk of the group is
 * captured once as a HIP graph and replayed.  Mixed-precision groups of more
 * than one problem refine by restarts (inner runs to a loose tolerance, then
 * an FP64 fold and a fresh start) instead of the reliable updates of a
 * single-problem solve, whose host round trips would stop every member;
 * PSFD_RELIABLE=0 / 1 selects one form for all plans.  Each group's kernel schedules
 * come from the autotuner (psfd_tune; PSFD_TUNE=0 disables).  Groups run on a
 * pool of PSFD_BATCH_WORKERS host threads (default 2), each with its own
 * non-blocking stream.  x0 may be NULL (all zero) or hold NULL entries;
 * E[i] are device complex128 fields of problem i's shape; infos is a host
 * array of n entries (required).  Returns PSFD_OK when every problem
 * converged, else the status of the first failing problem (all problems
 * are attempted). */
psfd_status psfd_plan_batch(int32_t n, const psfd_desc* descs, const void* const* eps_abs_dev,
                            void* hip_stream, psfd_plan_t* out);
psfd_status psfd_solve_batch(psfd_plan_t batch, const void* const* x0, void* const* E, double tol,
                             int32_t maxit, psfd_info* infos);

/* Standard full-domain discretisation of a planar stack (paper, Results,
 * "Background-decomposition" paragraph and its first figure: the comparison
 * solver meshes the whole multilayer; with n_ml = 0 and eps_sub = eps_bg the
 * plan has no multilayer operator and the stack lives in the absorber rows).
 *   layers_eps    host, [n_layers][2] permittivities (re, im), top to bottom
 *   layers_thick  host, [n_layers] thicknesses in nm, >= 0
 *   eps_abs_dev   device, [nz_abs][ny][nx] complex128 output: row j, which
 *                 spans [j dz, (j+1) dz) above the region's bottom face, holds
 *                 the thickness-weighted mean permittivity over that interval
 *                 of a stack whose top face is the region's top face
 *                 (z = nz_abs dz); the part no layer covers is eps_bg.  Every
 *                 lateral point of a row gets the same value.
 * Uses d->nx, ny, nz_abs, dz, eps_bg only.  Returns PSFD_ERR_ARG for a
 * negative or non-finite thickness; allocates a temporary and synchronises. */
psfd_status psfd_layered_eps(const psfd_desc* d, int32_t n_layers, const double* layers_eps,
                             const double* layers_thick, void* eps_abs_dev, void* hip_stream);

/* Specular (0, 0)-order reflection coefficient of the structure (absorber
 * region plus the multilayer operator) referred to the top face of the
 * absorber region, z = nz_abs dz (paper, Results, first figure panels c and
 * d compare it with the transfer-matrix value of the bare stack).
 *   E   device [3][Nz][ny][nx] complex128 scattered field of this plan's solve
 *   r   host, out: (re, im).  TE plans: the s-polarised amplitude; TM plans:
 *       the magnetic-field coefficient (sign convention of the transfer matrix).
 * The upgoing (0, 0) amplitude at the observation row is the mean of E over
 * that row plus the multilayer response to E (read at the evaluation row)
 * plus the multilayer reflection of the incident wave; it is carried back to
 * the face.  Single-problem plans only; synchronises the plan's stream. */
psfd_status psfd_specular(psfd_plan_t p, const void* E, double r[2]);

/* Threshold-contour widths (paper, Results, "Practical assessment of
 * scattered-field convergence" paragraph, equation logistic_sigmoid): the
 * intensity I = |v|^2 of each field plane is mapped through
 * S(I) = 1 / (1 + exp(-(I - i_th) / w)) (the paper: i_th = 0.15, w = 0.05),
 * and on nlines horizontal lines (rows floor((l + 1/2) ny / nlines), along
 * x) and then nlines vertical lines (columns floor((l + 1/2) nx / nlines),
 * along y) the segments with S > 1/2 between an upward and the next
 * downward crossing of S = 1/2 are measured.  Lines are periodic; a sample
 * is above threshold when re*re + im*im > i_th (products rounded
 * separately); a crossing is placed by linear interpolation of S.
 *   planes        device, nplanes planes of [ny][nx] complex128 (e.g. E_y on
 *                 the observation row), plane_stride elements apart
 *   seg           device out, [nplanes][2 nlines][max_seg][2] doubles: start
 *                 (from the line's first sample) and width, in nm, in line
 *                 order from the first upward crossing
 *   nseg          device out, [nplanes][2 nlines] int32: segments on each line
 *                 (0: the line never crosses; a count above max_seg means
 *                 only max_seg were stored; max(nx, ny)/2 always suffices)
 * 2 <= nx, ny <= 1024.  Asynchronous on hip_stream. */
psfd_status psfd_contour_segments(const void* planes, int32_t nx, int32_t ny, int32_t nplanes,
                                  int64_t plane_stride, double dx, double dy, int32_t nlines,
                                  double i_th, double w, int32_t max_seg, double* seg,
                                  int32_t* nseg, void* hip_stream);

/* Width deviation against a reference (same paragraph: delta d = d_ref - d,
 * divided by the 4x demagnification for wafer-scale numbers).  For every
 * reference segment the segment of the other field on the same line whose
 * periodic interval holds the reference segment's centre is its
 * counterpart.  Inputs are two outputs of psfd_contour_segments with the
 * same sizes (device).
 *   delta   device out, [nplanes][2 nlines][max_seg]: (d_ref - d) / demag per
 *           reference segment, NaN where there is no counterpart (unresolved),
 *           0 in slots beyond the line's segment count
 *   stats   host out, [5]: sum |delta|, sum delta^2, resolved count,
 *           unresolved count, count of |delta| > thr
 * Allocates a temporary and synchronises hip_stream. */
psfd_status psfd_contour_deviation(const double* seg_ref, const int32_t* nseg_ref,
                                   const double* seg, const int32_t* nseg, int32_t nx, int32_t ny,
                                   int32_t nplanes, double dx, double dy, int32_t nlines,
                                   int32_t max_seg, double demag, double thr, double* delta,
                                   double* stats, void* hip_stream);

/* Factorised Fourier neural operator of the paper's PINO (section 2.1: the
 * lateral and axial Fourier layers, the pointwise MLP with its residual
 * connection, the lifting and decoding layers), forward pass only (a field
 * prediction for the solver's warm start x0).  The paper does not give d_v,
 * d_h, the layer count or the retained modes; they are fields here. */
typedef struct {
  int32_t nx, ny, nz;        /* grid of the prediction, each in 4 .. 8192 (nz <= 4096)      */
  int32_t d_v, d_h;          /* feature / MLP hidden channels: (32, 64), (16, 32) or (8, 16) */
  int32_t n_layers;          /* 1 .. 16                                                    */
  int32_t kx_max, ky_max, kz_max; /* retained modes: kx 0..kx_max of the real-input half
                                     spectrum, |ky| <= ky_max, kz 0..kz_max; 2 k_max < n,
                                     kx_max <= 31, kz_max <= 15                           */
} psfd_ffno_desc;

/* Number of FP32 weights and workspace bytes of a network (host outputs,
 * either may be NULL).  Weight layout, row-major blocks in this order:
 *   P [d_v][4], p [d_v]                       lifting of (a, x/nx, y/ny, z/nz)
 *   per layer: K_xy [d_v][d_v][2 ky_max + 1][kx_max + 1] complex (re, im pairs;
 *              ky index m = ky + ky_max), K_z [d_v][d_v][kz_max + 1] complex,
 *              W1 [d_h][d_v], b1 [d_h], W2 [d_v][d_h], b2 [d_v]
 *   Q [6][d_v], q [6]                          decoding to Ex.re, Ex.im, Ey.re, ... */
psfd_status psfd_ffno_sizes(const psfd_ffno_desc* d, int64_t* n_weights, int64_t* workspace_bytes);

/* Forward pass.  Per layer l:
 *   u_xy = F2^-1[K_xy . F2 v]  on every z slice (truncated real-input DFT;
 *          the half-spectrum inverse drops the imaginary part of kx = 0),
 *   u_z  = F1^-1[K_z . F1 u_xy] along z,
 *   v   <- v + act(W2 gelu(W1 (u_xy + u_z) + b1) + b2), act = gelu (erf form)
 *          except in the last layer,
 * with v0 = P (a, x/nx, y/ny, z/nz) + p and E = Q v + q.
 *   weights    device FP32, layout above, 8-byte aligned
 *   a_in       device FP32 [nz][ny][nx]: the smoothed material indicator
 *   E          device out, [3][nz][ny][nx] complex128 (the solver's field layout)
 *   workspace  device, psfd_ffno_sizes bytes, 256-byte aligned; contents
 *              are overwritten (no allocation happens in this call)
 * Asynchronous on hip_stream. */
psfd_status psfd_ffno_forward(const psfd_ffno_desc* d, const float* weights, const float* a_in,
                              void* E, void* workspace, void* hip_stream);

/* Copy the plan's per-mode multilayer reflections (transfer-matrix method,
 * paper section 2.2 step (iii)): r_te, r_pe device [ny][nx] complex128.
 * r_pe is the tangential-electric-field TM coefficient. */
psfd_status psfd_ml_reflection(psfd_plan_t p, void* r_te, void* r_pe);

/* Kernel timing (measurement aid; not needed for solving).  kernel selects
 * which launches of this plan are bracketed by HIP events on the plan's
 * stream: 0 = off, 1 = axial column kernel, 2 = y-pass FFT, 3 = forward
 * x-pass FFT, 4 = inverse x-pass FFT with the combine epilogue.  Only
 * launches in the plan's working precision are timed (complex64 for the
 * PSFD_C64_* plans, whose FP64 residual applies are not counted).  While
 * timing is on, the solver launches its iteration chunks directly instead of
 * replaying captured graphs (the kernels are the same); launches of
 * iterations queued after the problem stopped (the kernels return at once)
 * are not counted.  Enabling resets the counters.  psfd_profile_read returns
 * (all host pointers):
 * total event time in ms, number of timed launches, and the algorithmic
 * bytes those launches move (each launch counts the complex elements it
 * must read and write once, at its element size). */
psfd_status psfd_profile_enable(psfd_plan_t p, int32_t kernel);
psfd_status psfd_profile_read(psfd_plan_t p, double* total_ms, int64_t* launches, double* bytes);

/* Autotuner (not part of the method: it selects among equivalent kernel
 * schedules).  psfd_tune times the plan's working-precision operator with
 * each candidate schedule of one knob at a time -- radix schedule (radix 8 or
 * radix 4 first) and rows per block of the forward and of the inverse x pass,
 * radix schedule and tile width of the y pass, axial kernel variant
 * (register-resident with L, 2L or L/2 lanes per column, or LDS-staged) -- and
 * keeps the fastest; results are cached per (precision, nx, ny, Nz, nz_abs,
 * group size) for the life of the process.  Synchronises the plan's stream.
 * Schedules change the rounding of the FFTs, never the operator.  A table of
 * earlier choices is read once per process from tune_table.txt next to the
 * library (or the file PSFD_TUNE_FILE names; an empty name disables it):
 * shapes it lists take their schedules without timing, in every plan.  Other
 * shapes use the default schedules unless psfd_tune is called or PSFD_TUNE=1
 * is set (batch groups are tuned unless PSFD_TUNE=0).  With PSFD_TUNE=0 plans
 * created afterwards keep the default schedules, table or not.  psfd_tune_save writes
 * the process's table (the file's entries plus everything tuned since) to
 * `path` (host string), in the file's format: one line per shape,
 * "elem nx ny nz nabs group : xf xi y ax" (elem 4: complex64 plans, 8:
 * complex128; group: problems per plan rounded up to a power of two).
 * psfd_schedule writes the plan's
 * current schedules to
 * sched[4] (host): forward x pass, inverse x pass, y pass (bit 0: radix-4
 * schedule, bit 1: half the rows / tile width), axial variant (0: L lanes,
 * 1: 2L lanes, 2: LDS-staged, 3: L/2 lanes).  psfd_set_schedule sets them
 * (both precisions) from sched[4] (host; values 0..3, else PSFD_ERR_ARG)
 * after draining the plan's stream. */
psfd_status psfd_tune(psfd_plan_t p);
psfd_status psfd_tune_save(const char* path);
psfd_status psfd_schedule(psfd_plan_t p, int32_t* sched);
psfd_status psfd_set_schedule(psfd_plan_t p, const int32_t* sched);

/* Total number of complex elements of one field, 3 * Nz * ny * nx. */
int64_t psfd_field_size(psfd_plan_t p);

/* Destroy a plan: waits for its stream, then gives its device blocks to the
 * library's memory cache (blocks are reused by later plans asking for the
 * same sizes, at most 32 GiB are kept; a failed allocation empties the cache
 * first).  PSFD_CACHE=0 in the environment frees the blocks instead. */
void psfd_destroy(psfd_plan_t p);

/* Free every device block held by the library's memory cache (the caller
 * wants the memory back; no plan needs to be destroyed for this). */
void psfd_trim_cache(void);

/* Message of the last error on this thread ("" if none). */
const char* psfd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSFD_H */
