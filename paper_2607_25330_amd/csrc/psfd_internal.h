// Internal declarations shared by the host driver and the kernel files.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "cplx.h"

namespace psfd {

// Sizes the kernels are instantiated for.
bool lateral_size_ok(int n);
bool axial_size_ok(int n);

// Grid geometry and per-axis tables shared by the operator kernels.
template <typename T>
struct OpTables {
  // A plan holds nprob problems of one shape ("group"); fields are stacked
  // [nprob][3][nz][ny][nx] and spectral workspaces [nprob][3 nz + 3 nabs][ny][nx].
  // Launches cover the whole group; no block straddles two problems.
  int nx, ny, nz, nabs, j0, jev;
  int nprob;
  int64_t pfield;           // elements of one problem's field
  int64_t pspec;            // elements of one problem's spectral workspace
  const T* kx;              // [nprob][nx] Bloch-shifted lateral wavenumbers
  const T* ky;              // [nprob][ny]
  const T* kz;              // [nz] axial wavenumbers (fftfreq order)
  const cplx<T>* inv_s;     // [nz] 1 / s(z), PML stretch
  const T* zabs;            // [nabs] z of the absorber row centres (z_ml = 0)
  const cplx<T>* r_te;      // [nprob][ny][nx] multilayer reflection, TE
  const cplx<T>* r_pe;      // [nprob][ny][nx] multilayer reflection, TM (tangential E)
  const cplx<T>* kd;        // [nprob][nabs][ny][nx] k0^2 (eps - eps_bg)
  const cplx<T>* tw_x;      // twiddles exp(-2 pi i m / nx)
  const cplx<T>* tw_y;
  const cplx<T>* tw_z;
  const T* cphi;            // [nprob] incidence-plane basis at kt = 0
  const T* sphi;
  T kbg2;                   // (k0 sqrt(eps_bg))^2
  T k0;
  T kz_live;                // |kz| below this (absolute) gets no multilayer response
  T dz;
  // spectral damping multiplier m(k)
  T pc_mmin, pc_kref2, pc_gamma, pc_reg;
  int pc_bf16;              // bf16 trial: the preconditioned spectrum m X^ held in bfloat16
  int hf_mode;              // 1: the M-mode multiplier is the loss weight w(nu)^2 instead of m(k)
  T hf_w0, hf_eta;          // w(nu) = hf_w0 + hf_eta |nu|,  |nu| = |k| / (2 pi)
  int ax_lds;               // 1: always use the LDS-staged axial kernel
  // kernel schedules chosen by the autotuner (0 = default): forward x pass,
  // inverse x pass, y pass (bit 0 radix schedule, bit 1 half rows / tile);
  // axial kernel (0 register kernel, 1 register kernel with twice the lanes,
  // 2 LDS-staged kernel, 3 register kernel with half the lanes)
  int sched_xf, sched_xi, sched_y, sched_ax;
  // per-problem skip flags: when non-null and skip[b * skip_stride] != 0 the
  // operator kernels return at once for problem b
  const int* skip;
  int skip_stride;
  // host side: when set, the operator kernel launched with these tables
  // records the events from its own dispatch packet (kernel start / end)
  hipEvent_t prof_start, prof_stop;
};

// Launch `kern` (parenthesised template-id) with the tables `t`; the
// measurement events, when present, are recorded by the launch itself.
#define PSFD_LAUNCH(t, kern, grid, block, st, ...)                                          \
  do {                                                                                      \
    if ((t).prof_start)                                                                     \
      hipExtLaunchKernelGGL(kern, grid, block, 0, st, (t).prof_start, (t).prof_stop, 0,     \
                            __VA_ARGS__);                                                   \
    else                                                                                    \
      hipLaunchKernelGGL(kern, grid, block, 0, st, __VA_ARGS__);                            \
  } while (0)

template <typename T>
__host__ __device__ __forceinline__ bool skipped(const OpTables<T>& t, int b) {
  return t.skip && t.skip[(int64_t)b * t.skip_stride] != 0;
}

enum AxialMode { AX_A = 0, AX_AM = 1, AX_AH = 2, AX_M = 3 };
enum CombineMode { CB_PLAIN = 0, CB_FWD = 1, CB_ADJ = 2 };

struct KState;

// Vector update fused into the forward x pass of an operator apply:
//   PRE_P: p = r + beta (p - omega v)  (p overwritten, then transformed)
//   PRE_S: s = r - alpha v             (s written, then transformed; partials ||s||^2)
enum { PRE_NONE = 0, PRE_P = 1, PRE_S = 2 };
template <typename T>
struct PreOp {
  int mode = PRE_NONE;
  const cplx<T>* r = nullptr;
  cplx<T>* pv = nullptr;  // p (in/out) or s (out)
  const cplx<T>* v = nullptr;
  const KState* ks = nullptr;
  double* part = nullptr;
};
// Inner products fused into the inverse x pass: partials of
//   sum conj(d) y  and  sum |y|^2  over the operator output y.
enum { POST_NONE = 0, POST_DOT = 1 };
template <typename T>
struct PostOp {
  int mode = POST_NONE;
  const cplx<T>* d = nullptr;
  double* part = nullptr;
};

// ---- lateral FFT launchers (fft_lateral.hip)
// Forward x-FFT of rows.  nrows_main rows come straight from `in`; for the
// adjoint, extra = 3 * nabs planes follow whose rows are conj(kd) * in on the
// absorber rows.
// *nblk receives the grid size (number of partials for PRE_S).
template <typename T>
hipError_t launch_xfft_fwd(const OpTables<T>& t, const cplx<T>* in, cplx<T>* out, bool adj_extra,
                           const PreOp<T>& pre, int* nblk, hipStream_t st);
// In-place y-FFT of nplanes planes of ny x nx.
template <typename T>
hipError_t launch_yfft(const OpTables<T>& t, cplx<T>* buf, int nplanes, bool inverse,
                       hipStream_t st);
// Inverse x-FFT of the 3 Nz U planes (+ W planes) with the combine epilogue.
template <typename T>
hipError_t launch_xfft_inv(const OpTables<T>& t, const cplx<T>* UW, cplx<T>* y, int cmode,
                           const cplx<T>* x, const PostOp<T>& post, int* nblk, hipStream_t st);
// Inverse x pass (no combine, scale 1/(nx ny)) over nrows arbitrary rows.
template <typename T>
hipError_t launch_xfft_inv_rows(const OpTables<T>& t, const cplx<T>* in, cplx<T>* out,
                                int64_t nrows, hipStream_t st);
// 2-D FFT of a single plane (layout smoothing).  Forward: in -> out.
// Inverse (unnormalised): y pass in place on `in`, x pass into `out`.
template <typename T>
hipError_t launch_plane_fft(const OpTables<T>& t, cplx<T>* in, cplx<T>* out, bool inverse,
                            hipStream_t st);

// ---- axial launcher (axial.hip)
template <typename T>
hipError_t launch_axial(const OpTables<T>& t, const cplx<T>* S, cplx<T>* UW, int mode,
                        hipStream_t st);

// ---- setup kernels (setup.hip)
struct TmmArgs {
  int nx, ny;
  const double* kx;
  const double* ky;
  double k0, eps_bg;
  int nl;
  const cplx<double>* eps_l;  // device [nl]
  const double* d_l;          // device [nl]
  cplx<double> eps_sub;
};
hipError_t launch_tmm(const TmmArgs& a, cplx<double>* r_te, cplx<double>* r_pe, hipStream_t st);

struct RhsArgs {
  int nx, ny, nz, nabs, j0, pol;
  double k0, kz0, theta, phi;
  const double* zabs;
  const cplx<double>* r_te;  // mode (0, 0) is the incidence mode
  const cplx<double>* r_pe;
  const cplx<double>* kd;
};
template <typename T>
hipError_t launch_rhs(const RhsArgs& a, cplx<T>* b, hipStream_t st);

// grad[v] = scale * sum_a u_a(v) conj(W_a(v) + bg_a(z_v)) on absorber voxels;
// W: [3][nabs][ny][nx] real-space E + E_ML on absorber rows; u: full field.
hipError_t launch_eps_grad(const RhsArgs& a, const cplx<double>* W, const cplx<double>* u,
                           double scale, cplx<double>* grad, hipStream_t st);
hipError_t launch_eps_contrast(const cplx<double>* eps, int n, double k0, double eps_bg,
                               cplx<double>* kd64, cplx<float>* kd32, hipStream_t st);
hipError_t launch_smooth_mult(cplx<double>* plane, int nx, int ny, double dx, double dy,
                              double sigma, hipStream_t st);
hipError_t launch_fill_eps(const cplx<double>* plane, int nx, int ny, int nabs, double scale,
                           double eps_bg, cplx<double> eps_abs, cplx<double>* eps_out,
                           hipStream_t st);
hipError_t launch_real_to_cplx(const double* a, int n, cplx<double>* out, hipStream_t st);
// w[m] = exp(-2 pi i m / n), m < n (w: device)
hipError_t launch_twiddles(cplx<double>* w, int n, hipStream_t st);
// out[j][i] = rows[j] for j < nrows, i < plane (rows: device)
hipError_t launch_fill_rows(const cplx<double>* rows, int64_t plane, int nrows,
                            cplx<double>* out, hipStream_t st);
// ---- threshold-contour width metric (contour.hip)
constexpr int kContourLineMax = 1024;  // longest scan line
struct ContourArgs {
  const cplx<double>* f;   // planes [nplanes] of [ny][nx], plane stride pstride elements
  int64_t pstride;
  int nx, ny, nlines, max_seg;
  double dx, dy, i_th, w;
  double* seg;             // [nplanes][2 nlines][max_seg][2]: start, width
  int32_t* nseg;           // [nplanes][2 nlines]
};
struct DeviationArgs {
  const double* sref;
  const int32_t* nref;
  const double* sk;
  const int32_t* nk;
  int nplanes, nlines, max_seg;
  double len_h, len_v, demag, thr;
  double* delta;           // [nplanes][2 nlines][max_seg]
  double* part;            // [blocks][5]
};
hipError_t launch_contour_segments(const ContourArgs& a, int nplanes, hipStream_t st);
hipError_t launch_contour_deviation(const DeviationArgs& a, int nblocks, hipStream_t st);

// ---- factorised Fourier neural operator inference (ffno.hip)
constexpr int kFfnoMaxLayers = 16;
struct FfnoArgs {
  int nx, ny, nz, dv, dh, nl;
  int mx, my, mz, ky_max;  // retained modes: kx 0..mx-1, ky -ky_max..ky_max (my), kz 0..mz-1
};
struct FfnoPtrs {
  const float *P, *p, *Q, *q;
  const float2* Kxy[kFfnoMaxLayers];
  const float2* Kz[kFfnoMaxLayers];
  const float *W1[kFfnoMaxLayers], *b1[kFfnoMaxLayers], *W2[kFfnoMaxLayers], *b2[kFfnoMaxLayers];
  float *v, *u;            // hidden state and lateral-branch output, [dv][nz][ny][nx]
  float* W2T;              // [nl][dh][dv] transposed MLP output weights
  float2* KzT;             // [nl][mz][dv][dv] axial mixing weights, kz-major
  float2* pz;              // [nz + 3][16] powers w^(kz z) of the axial transforms
  float2* qx;              // [ceil(nx / 16) + 7][16 or 32] powers w^(16 kx j) of the x DFT
  float2* q4;              // [4 ceil(nx / 64) + 4][16 or 32] powers w^(kx (64 j + c)) (nx % 4 == 0)
  float2 *T, *G, *U;       // [dv][nz][ny][mx], [dv][nz][my][mx] x 2
  float2 *W, *Z;           // axial spectra before / after mixing, [dv][mz][ny][nx] each
  float2 *twx, *twy, *twz; // e^{+2 pi i k / n}
};
hipError_t ffno_forward(const FfnoArgs& a, const FfnoPtrs& w, const float* in, cplx<double>* E,
                        hipStream_t st);

// part[q][b], q < 4, b < nblk: partial sums of the plane starting at f + off[q]
struct PlaneSet {
  int64_t off[5];
};
hipError_t launch_plane_sums(const cplx<double>* f, const PlaneSet& ps, int64_t plane, int nblk,
                             cplx<double>* part, hipStream_t st);

// ---- Krylov kernels (krylov.hip)
struct KState {
  double rho[2], rho_prev[2], alpha[2], omega[2];
  double rv[2], ts[2], tt;
  double snorm2, rnorm2, bnorm2, tol2, rh_norm2;
  double red[4];        // generic reduction outputs
  double rmax2, delta2;  // reliable updates: max ||r||^2 since the last one, trigger factor
  double rfold2;         // ||r||^2 at the run's start or its last residual replacement
  int iter, done, status, half;
  int itmax, pad;
};

constexpr int KRED_THREADS = 256;
int red_blocks(int64_t n, int nprob);  // blocks per problem of the streaming vector kernels

// Per-problem scalars set by the host between Krylov runs.
struct ProbParams {
  double bnorm2;  // ||b||^2 of the system the run solves
  double tol2;    // squared relative stopping tolerance; < 0: problem idle (skipped)
  double scale;   // y += scale * x (refinement update)
  double iscale;  // y = iscale * x (normalised residual)
  double itmax;   // iteration budget of the run
  double delta2;  // reliable update when ||r||^2 <= delta2 * (max ||r||^2 since the last one); 0: never
  double mask;    // 0: the host-driven vector kernels leave this problem untouched
  double pad;
};

enum FinStage { FIN_INIT = 0, FIN_ALPHA, FIN_OMEGA, FIN_RHO, FIN_RED0, FIN_REPLACE, FIN_RED3,
                FIN_SHADOW };
// Krylov state of a problem (KState::done)
enum { KS_RUN = 0, KS_CONV = 1, KS_HALF = 2, KS_BREAK = 3, KS_IDLE = 4, KS_MAXIT = 5, KS_UPDATE = 6 };
// One block per problem: sum problem b's `nblocks` partials (they start at
// part + b * nblocks * KPART) and update ks[b] for one stage of the recurrence.
// FIN_OMEGA also sums the ||s||^2 partials of the forward x pass (part2,
// nblocks2 per problem) and takes the half-step decision there.
hipError_t launch_finalize(int stage, KState* ks, const double* part, int nblocks, int nprob,
                           const ProbParams* pp, hipStream_t st, const double* part2 = nullptr,
                           int nblocks2 = 0);

// Streaming vector kernels over a group: n = elements of one problem; problem
// b's vectors start at b * n; grid = nprob * red_blocks(n) blocks.
template <typename T>
hipError_t launch_k_xr_update(cplx<T>* y, cplx<T>* r, const cplx<T>* p, const cplx<T>* s,
                              const cplx<T>* t, const cplx<T>* rh, int64_t n, int nprob,
                              const KState* ks, double* part, hipStream_t st);
template <typename T>
hipError_t launch_k_p_update(cplx<T>* p, const cplx<T>* r, const cplx<T>* v, int64_t n,
                             int nprob, const KState* ks, hipStream_t st);
// Start a BiCGSTAB run: rh = r, p = v = y = 0, partials ||r||^2 (then FIN_INIT).
template <typename T>
hipError_t launch_k_init(cplx<T>* rh, const cplx<T>* r, cplx<T>* p, cplx<T>* v, cplx<T>* y,
                         int64_t n, int nprob, double* part, hipStream_t st);
// out = a - b, partials ||out||^2 (then FIN_RED0); problems with skip[b] != 0
// (skip may be NULL) are left untouched and write no partials
template <typename T>
hipError_t launch_k_residual(cplx<T>* out, const cplx<T>* a, const cplx<T>* b, int64_t n,
                             int nprob, const int* skip, double* part, hipStream_t st);
// partials ||r||^2, sum conj(rh) r of a replaced residual (then FIN_REPLACE)
template <typename T>
hipError_t launch_k_dot_rr(const cplx<T>* rh, const cplx<T>* r, int64_t n, int nprob,
                           double* part, hipStream_t st);
// partials ||a||^2 (then FIN_RED0)
template <typename T>
hipError_t launch_k_norm2(const cplx<T>* a, int64_t n, int nprob, double* part, hipStream_t st);
// y += scale_b * x for problem b (scale from pp[b].scale)
template <typename TY, typename TX>
hipError_t launch_k_axpy(cplx<TY>* y, const cplx<TX>* x, const ProbParams* pp, int64_t n,
                         int nprob, hipStream_t st);
// y = scale_b * x (precision conversion with scaling; pp == nullptr: scale 1)
template <typename TY, typename TX>
hipError_t launch_k_scale_copy(cplx<TY>* y, const cplx<TX>* x, const ProbParams* pp, int64_t n,
                               int nprob, hipStream_t st);

}  // namespace psfd
