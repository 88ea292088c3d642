// Plan-time and source kernels.
//
// * Per-lateral-mode multilayer reflection (transfer-matrix method, paper
//   section 2.2, step (iii) of R_ml) by the bottom-up recursion of interface
//   reflections, which stays finite for strongly evanescent modes (every
//   phase factor exp(2 i kz d) has modulus <= 1).  TE uses q = kz, TM the
//   magnetic-field form q = kz / eps; r_pE = -r_TM^H converts to tangential E.
// * The analytic background source b = k0^2 d_eps (E_inc + R_ml E_inc)
//   (equation bg_source).
// * Permittivity contrast k0^2 (eps - eps_bg) and the Gaussian smoothing of
//   a binary layout (paper, section 2.1 closing paragraphs).
#include "psfd_internal.h"

namespace psfd {

__global__ void k_tmm(const TmmArgs a, cplx<double>* __restrict__ r_te,
                      cplx<double>* __restrict__ r_pe) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.nx * a.ny) return;
  const int ix = idx % a.nx, iy = idx / a.nx;
  const double kt2 = a.kx[ix] * a.kx[ix] + a.ky[iy] * a.ky[iy];
  const double k02 = a.k0 * a.k0;
  for (int pol = 0; pol < 2; ++pol) {
    // start below the stack, in the substrate (no reflection from beneath)
    cplx<double> eps_cur = a.eps_sub;
    cplx<double> kz_cur = sqrt_up(cplx<double>{k02 * eps_cur.re - kt2, k02 * eps_cur.im});
    cplx<double> q_cur = pol == 0 ? kz_cur : cdiv(kz_cur, eps_cur);
    double d_cur = 0.0;
    cplx<double> R = {0.0, 0.0};
    for (int j = a.nl; j >= 0; --j) {
      const cplx<double> eps_j = (j == 0) ? cplx<double>{a.eps_bg, 0.0} : a.eps_l[j - 1];
      const cplx<double> kz_j = sqrt_up(cplx<double>{k02 * eps_j.re - kt2, k02 * eps_j.im});
      const cplx<double> q_j = pol == 0 ? kz_j : cdiv(kz_j, eps_j);
      const cplx<double> r = cdiv(q_j - q_cur, q_j + q_cur);
      const cplx<double> ph = cexpi(2.0 * d_cur * kz_cur);
      const cplx<double> Rp = R * ph;
      R = cdiv(r + Rp, cplx<double>{1.0, 0.0} + r * Rp);
      kz_cur = kz_j;
      q_cur = q_j;
      d_cur = (j == 0) ? 0.0 : a.d_l[j - 1];
    }
    if (pol == 0) r_te[idx] = R;
    else r_pe[idx] = -R;
  }
}

hipError_t launch_tmm(const TmmArgs& a, cplx<double>* r_te, cplx<double>* r_pe, hipStream_t st) {
  const int n = a.nx * a.ny;
  hipLaunchKernelGGL(k_tmm, dim3((n + 127) / 128), dim3(128), 0, st, a, r_te, r_pe);
  return hipGetLastError();
}

template <typename T>
__global__ void k_rhs(const RhsArgs a, cplx<T>* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t plane = (int64_t)a.nx * a.ny;
  const int64_t pidx = i / plane;
  const int64_t inplane = i % plane;
  const int c = (int)(pidx / a.nz), z = (int)(pidx % a.nz);
  cplx<T> out = {T(0), T(0)};
  if (z >= a.j0 && z < a.j0 + a.nabs) {
    const int ja = z - a.j0;
    double sth, cth, sph, cph;
    sincos(a.theta, &sth, &cth);
    sincos(a.phi, &sph, &cph);
    double ein, eup;
    if (a.pol == 0) {
      ein = (c == 0) ? -sph : (c == 1 ? cph : 0.0);
      eup = ein;
    } else {
      ein = (c == 0) ? cth * cph : (c == 1 ? cth * sph : sth);
      eup = (c == 2) ? -sth : ein;
    }
    const double zz = a.zabs[ja];
    const cplx<double> r = (a.pol == 0) ? a.r_te[0] : a.r_pe[0];
    double s, co;
    sincos(a.kz0 * zz, &s, &co);
    const cplx<double> down = {co, -s}, up = {co, s};
    const cplx<double> bg = ein * down + eup * (r * up);
    const cplx<double> v = a.kd[(int64_t)ja * plane + inplane] * bg;
    out = {(T)v.re, (T)v.im};
  }
  b[i] = out;
}

template <typename T>
hipError_t launch_rhs(const RhsArgs& a, cplx<T>* b, hipStream_t st) {
  const int64_t n = (int64_t)3 * a.nz * a.nx * a.ny;
  hipLaunchKernelGGL((k_rhs<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}
template hipError_t launch_rhs<double>(const RhsArgs&, cplx<double>*, hipStream_t);
template hipError_t launch_rhs<float>(const RhsArgs&, cplx<float>*, hipStream_t);

// Background field E_inc + R_ml E_inc, component c, absorber row ja.
__device__ cplx<double> background(const RhsArgs& a, int c, int ja) {
  double sth, cth, sph, cph;
  sincos(a.theta, &sth, &cth);
  sincos(a.phi, &sph, &cph);
  double ein, eup;
  if (a.pol == 0) {
    ein = (c == 0) ? -sph : (c == 1 ? cph : 0.0);
    eup = ein;
  } else {
    ein = (c == 0) ? cth * cph : (c == 1 ? cth * sph : sth);
    eup = (c == 2) ? -sth : ein;
  }
  const double zz = a.zabs[ja];
  const cplx<double> r = (a.pol == 0) ? a.r_te[0] : a.r_pe[0];
  double s, co;
  sincos(a.kz0 * zz, &s, &co);
  const cplx<double> down = {co, -s}, up = {co, s};
  return ein * down + eup * (r * up);
}

__global__ void k_eps_grad(const RhsArgs a, const cplx<double>* __restrict__ W,
                           const cplx<double>* __restrict__ u, double scale,
                           cplx<double>* __restrict__ grad) {
  const int64_t plane = (int64_t)a.nx * a.ny;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.nabs * plane) return;
  const int ja = (int)(i / plane);
  const int64_t inplane = i % plane;
  cplx<double> acc = {0.0, 0.0};
  for (int c = 0; c < 3; ++c) {
    const cplx<double> psi = W[((int64_t)c * a.nabs + ja) * plane + inplane] + background(a, c, ja);
    const cplx<double> uv = u[((int64_t)c * a.nz + a.j0 + ja) * plane + inplane];
    acc = acc + uv * conj(psi);
  }
  grad[i] = scale * acc;
}

hipError_t launch_eps_grad(const RhsArgs& a, const cplx<double>* W, const cplx<double>* u,
                           double scale, cplx<double>* grad, hipStream_t st) {
  const int64_t n = (int64_t)a.nabs * a.nx * a.ny;
  hipLaunchKernelGGL(k_eps_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, W, u,
                     scale, grad);
  return hipGetLastError();
}

__global__ void k_eps_contrast(const cplx<double>* __restrict__ eps, int n, double k02,
                               double eps_bg, cplx<double>* __restrict__ kd64,
                               cplx<float>* __restrict__ kd32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cplx<double> d = {k02 * (eps[i].re - eps_bg), k02 * eps[i].im};
  kd64[i] = d;
  if (kd32) kd32[i] = {(float)d.re, (float)d.im};
}

hipError_t launch_eps_contrast(const cplx<double>* eps, int n, double k0, double eps_bg,
                               cplx<double>* kd64, cplx<float>* kd32, hipStream_t st) {
  hipLaunchKernelGGL(k_eps_contrast, dim3((n + 255) / 256), dim3(256), 0, st, eps, n, k0 * k0,
                     eps_bg, kd64, kd32);
  return hipGetLastError();
}

__global__ void k_smooth_mult(cplx<double>* __restrict__ p, int nx, int ny, double ax,
                              double ay) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx * ny) return;
  const int ix = i % nx, iy = i / nx;
  const double fx = (ix < (nx + 1) / 2) ? ix : ix - nx;
  const double fy = (iy < (ny + 1) / 2) ? iy : iy - ny;
  const double h = exp(-0.5 * (ax * fx * fx + ay * fy * fy));
  p[i] = h * p[i];
}

hipError_t launch_smooth_mult(cplx<double>* plane, int nx, int ny, double dx, double dy,
                              double sigma, hipStream_t st) {
  // exp(-(sx^2 kx^2 + sy^2 ky^2)/2), kx = 2 pi f / (nx dx), sx = sigma dx
  const double two_pi = 6.283185307179586476925;
  const double cx = sigma * dx * two_pi / (nx * dx);
  const double cy = sigma * dy * two_pi / (ny * dy);
  hipLaunchKernelGGL(k_smooth_mult, dim3((nx * ny + 255) / 256), dim3(256), 0, st, plane, nx, ny,
                     cx * cx, cy * cy);
  return hipGetLastError();
}

__global__ void k_fill_eps(const cplx<double>* __restrict__ plane, int n, int nabs, double scale,
                           double eps_bg, cplx<double> eps_abs, cplx<double>* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = plane[i].re * scale;
  a = fmin(fmax(a, 0.0), 1.0);
  const cplx<double> e = {eps_bg + a * (eps_abs.re - eps_bg), a * eps_abs.im};
  for (int j = 0; j < nabs; ++j) out[(int64_t)j * n + i] = e;
}

hipError_t launch_fill_eps(const cplx<double>* plane, int nx, int ny, int nabs, double scale,
                           double eps_bg, cplx<double> eps_abs, cplx<double>* eps_out,
                           hipStream_t st) {
  const int n = nx * ny;
  hipLaunchKernelGGL(k_fill_eps, dim3((n + 255) / 256), dim3(256), 0, st, plane, n, nabs, scale,
                     eps_bg, eps_abs, eps_out);
  return hipGetLastError();
}

__global__ void k_real_to_cplx(const double* __restrict__ a, int n, cplx<double>* __restrict__ o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = {a[i], 0.0};
}

hipError_t launch_real_to_cplx(const double* a, int n, cplx<double>* out, hipStream_t st) {
  hipLaunchKernelGGL(k_real_to_cplx, dim3((n + 255) / 256), dim3(256), 0, st, a, n, out);
  return hipGetLastError();
}

// DFT twiddles w[m] = exp(-2 pi i m / n), m < n, in FP64 on the device.
__global__ void k_twiddles(cplx<double>* __restrict__ w, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)n, &s, &c);
  w[m] = {c, s};
}

hipError_t launch_twiddles(cplx<double>* w, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, st, w, n);
  return hipGetLastError();
}

// Row values broadcast over every lateral point: out[j][i] = rows[j].
__global__ void k_fill_rows(const cplx<double>* __restrict__ rows, int64_t plane,
                            cplx<double>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < plane) out[(int64_t)j * plane + i] = rows[j];
}

hipError_t launch_fill_rows(const cplx<double>* rows, int64_t plane, int nrows,
                            cplx<double>* out, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_rows, dim3((unsigned)((plane + 255) / 256), nrows), dim3(256), 0, st,
                     rows, plane, out);
  return hipGetLastError();
}

// Partial sums of up to four planes of a field: block (b, q) adds the
// elements b * 256 + tid + k * 256 * gridDim.x of plane q and writes one
// complex partial to part[q * gridDim.x + b].
__global__ void __launch_bounds__(256)
k_plane_sums(const cplx<double>* __restrict__ f, PlaneSet ps, int64_t plane,
             cplx<double>* __restrict__ part) {
  const int q = blockIdx.y, tid = threadIdx.x;
  const cplx<double>* p = f + ps.off[q];
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < plane; i += (int64_t)gridDim.x * 256) {
    re += p[i].re;
    im += p[i].im;
  }
  __shared__ double sr[256], si[256];
  sr[tid] = re;
  si[tid] = im;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      sr[tid] += sr[tid + h];
      si[tid] += si[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) part[q * gridDim.x + blockIdx.x] = {sr[0], si[0]};
}

hipError_t launch_plane_sums(const cplx<double>* f, const PlaneSet& ps, int64_t plane, int nblk,
                             cplx<double>* part, hipStream_t st) {
  hipLaunchKernelGGL(k_plane_sums, dim3(nblk, 5), dim3(256), 0, st, f, ps, plane, part);
  return hipGetLastError();
}

}  // namespace psfd
