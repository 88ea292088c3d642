// BiCGSTAB vector updates and inner products (paper: BiCGSTAB with right
// preconditioning, Results section, "PINO warm-start" paragraph; the stop
// test is the relative residual of equation relative_residual).
//
// Every scalar of the recurrence (rho, alpha, omega, the norms) lives in a
// device-side KState in FP64, so an iteration is a fixed sequence of
// launches with no host round trip.  Each reduction kernel writes one FP64
// partial per block; the last block to finish (ticket counter) adds the
// partials in a fixed order, so results are deterministic, and then
// updates the scalars and the convergence / breakdown flags:
//   done = 0 running, 1 converged, 2 pending half step (y += alpha p only),
//   3 breakdown (the host restarts with a fresh shadow residual).
// Kernels return immediately when done is set, so extra launches queued
// after convergence are no-ops.
#include "psfd_internal.h"

namespace psfd {

enum { KS_RUN = 0, KS_CONV = 1, KS_HALF = 2, KS_BREAK = 3 };

static inline int red_blocks(int64_t n) {
  int64_t b = (n + KRED_THREADS - 1) / KRED_THREADS;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

// Block-level sum of NV doubles; thread 0 returns the totals in acc.
template <int NV>
__device__ __forceinline__ void block_sum(double (&acc)[NV]) {
  __shared__ double sm[NV][KRED_THREADS / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    acc[k] = v;
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sm[k][wv] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < KRED_THREADS / 64; ++w) s += sm[k][w];
      acc[k] = s;
    }
  }
}

// Store this block's partials; in the last block thread 0 gets the grand
// totals in acc and the function returns true (for thread 0 only).
template <int NV>
__device__ __forceinline__ bool reduce_grid(double (&acc)[NV], double* part, KState* ks) {
  __shared__ int last;
  block_sum<NV>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[blockIdx.x * NV + k] = acc[k];
    __threadfence();
    const unsigned t = atomicAdd(&ks->ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double tot[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] += part[b * NV + k];
  }
  block_sum<NV>(tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = tot[k];
    ks->ticket = 0u;
    return true;
  }
  return false;
}

__device__ __forceinline__ cplx<double> ld2(const double* a) { return {a[0], a[1]}; }
__device__ __forceinline__ void st2(double* a, cplx<double> v) { a[0] = v.re; a[1] = v.im; }

// ------------------------------------------------------------------ kernels

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_p_update(cplx<T>* __restrict__ p, const cplx<T>* __restrict__ r, const cplx<T>* __restrict__ v,
           int64_t n, const KState* __restrict__ ks) {
  if (ks->done != KS_RUN) return;
  const cplx<double> rho = ld2(ks->rho), rho_p = ld2(ks->rho_prev);
  const cplx<double> al = ld2(ks->alpha), om = ld2(ks->omega);
  const cplx<double> beta = cdiv(rho, rho_p) * cdiv(al, om);
  const cplx<T> b = cast<T>(beta), w = cast<T>(om);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = r[i] + b * (p[i] - w * v[i]);
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_dot_rv(const cplx<T>* __restrict__ rh, const cplx<T>* __restrict__ v, int64_t n, KState* ks,
         double* part) {
  if (ks->done != KS_RUN) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<double> a = cast<double>(rh[i]), b = cast<double>(v[i]);
    acc[0] += a.re * b.re + a.im * b.im;
    acc[1] += a.re * b.im - a.im * b.re;
    acc[2] += b.re * b.re + b.im * b.im;
  }
  if (reduce_grid<3>(acc, part, ks)) {
    const cplx<double> rv = {acc[0], acc[1]};
    st2(ks->rv, rv);
    if (sqrt(norm2(rv)) <= 1e-30 * sqrt(ks->rh_norm2 * acc[2])) {
      ks->status = 1;
      ks->done = KS_BREAK;
    } else {
      st2(ks->alpha, cdiv(ld2(ks->rho), rv));
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_s_update(cplx<T>* __restrict__ s, const cplx<T>* __restrict__ r, const cplx<T>* __restrict__ v,
           int64_t n, KState* ks, double* part) {
  if (ks->done != KS_RUN) return;
  const cplx<T> al = cast<T>(ld2(ks->alpha));
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<T> si = r[i] - al * v[i];
    s[i] = si;
    acc[0] += norm2(cast<double>(si));
  }
  if (reduce_grid<1>(acc, part, ks)) {
    ks->snorm2 = acc[0];
    if (acc[0] <= ks->tol2 * ks->bnorm2) {
      ks->half = 1;
      ks->done = KS_HALF;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_dot_ts(const cplx<T>* __restrict__ t, const cplx<T>* __restrict__ s, int64_t n, KState* ks,
         double* part) {
  if (ks->done != KS_RUN) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<double> a = cast<double>(t[i]), b = cast<double>(s[i]);
    acc[0] += a.re * b.re + a.im * b.im;
    acc[1] += a.re * b.im - a.im * b.re;
    acc[2] += a.re * a.re + a.im * a.im;
  }
  if (reduce_grid<3>(acc, part, ks)) {
    st2(ks->ts, cplx<double>{acc[0], acc[1]});
    ks->tt = acc[2];
    if (acc[2] == 0.0) {
      ks->half = 1;
      ks->status = 1;
      ks->done = KS_HALF;
    } else {
      st2(ks->omega, cplx<double>{acc[0] / acc[2], acc[1] / acc[2]});
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_xr_update(cplx<T>* __restrict__ y, cplx<T>* __restrict__ r, const cplx<T>* __restrict__ p,
            const cplx<T>* __restrict__ s, const cplx<T>* __restrict__ t,
            const cplx<T>* __restrict__ rh, int64_t n, KState* ks, double* part) {
  const int d = ks->done;
  if (d != KS_RUN && d != KS_HALF) return;
  const cplx<T> al = cast<T>(ld2(ks->alpha));
  double acc[3] = {0.0, 0.0, 0.0};
  if (d == KS_HALF) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
      y[i] = y[i] + al * p[i];
  } else {
    const cplx<T> om = cast<T>(ld2(ks->omega));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
      const cplx<T> si = s[i];
      y[i] = y[i] + al * p[i] + om * si;
      const cplx<T> ri = si - om * t[i];
      r[i] = ri;
      const cplx<double> a = cast<double>(rh[i]), b = cast<double>(ri);
      acc[0] += norm2(b);
      acc[1] += a.re * b.re + a.im * b.im;
      acc[2] += a.re * b.im - a.im * b.re;
    }
  }
  if (reduce_grid<3>(acc, part, ks)) {
    ks->iter += 1;
    if (d == KS_HALF) {
      ks->rnorm2 = ks->snorm2;
      ks->done = ks->status ? KS_BREAK : KS_CONV;
      return;
    }
    ks->rnorm2 = acc[0];
    const cplx<double> rho_new = {acc[1], acc[2]};
    ks->rho_prev[0] = ks->rho[0];
    ks->rho_prev[1] = ks->rho[1];
    st2(ks->rho, rho_new);
    if (acc[0] <= ks->tol2 * ks->bnorm2) {
      ks->done = KS_CONV;
    } else {
      const cplx<double> om = ld2(ks->omega);
      if ((om.re == 0.0 && om.im == 0.0) ||
          sqrt(norm2(rho_new)) <= 1e-30 * sqrt(ks->rh_norm2 * acc[0])) {
        ks->status = 1;
        ks->done = KS_BREAK;
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_init(cplx<T>* __restrict__ rh, const cplx<T>* __restrict__ r, cplx<T>* __restrict__ p,
       cplx<T>* __restrict__ v, cplx<T>* __restrict__ y, int64_t n, KState* ks, double* part,
       double bnorm2, double tol2) {
  double acc[1] = {0.0};
  const cplx<T> zero = {T(0), T(0)};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<T> ri = r[i];
    rh[i] = ri;
    p[i] = zero;
    v[i] = zero;
    y[i] = zero;
    acc[0] += norm2(cast<double>(ri));
  }
  if (reduce_grid<1>(acc, part, ks)) {
    ks->rho[0] = acc[0];
    ks->rho[1] = 0.0;
    ks->rho_prev[0] = ks->alpha[0] = ks->omega[0] = 1.0;
    ks->rho_prev[1] = ks->alpha[1] = ks->omega[1] = 0.0;
    ks->rh_norm2 = acc[0];
    ks->rnorm2 = acc[0];
    ks->bnorm2 = bnorm2;
    ks->tol2 = tol2;
    ks->done = KS_RUN;
    ks->half = 0;
    ks->status = 0;
    ks->iter = 0;
  }
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_residual(cplx<T>* __restrict__ out, const cplx<T>* __restrict__ a, const cplx<T>* __restrict__ b,
           int64_t n, KState* ks, double* part) {
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<T> d = a[i] - b[i];
    out[i] = d;
    acc[0] += norm2(cast<double>(d));
  }
  if (reduce_grid<1>(acc, part, ks)) ks->red[0] = acc[0];
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_norm2(const cplx<T>* __restrict__ a, int64_t n, KState* ks, double* part) {
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc[0] += norm2(cast<double>(a[i]));
  if (reduce_grid<1>(acc, part, ks)) ks->red[0] = acc[0];
}

template <typename TY, typename TX>
__global__ void __launch_bounds__(KRED_THREADS)
k_axpy(cplx<TY>* __restrict__ y, const cplx<TX>* __restrict__ x, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<TY> xv = cast<TY>(x[i]);
    y[i] = y[i] + TY(a) * xv;
  }
}

template <typename TY, typename TX>
__global__ void __launch_bounds__(KRED_THREADS)
k_scale_copy(cplx<TY>* __restrict__ y, const cplx<TX>* __restrict__ x, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<double> xv = cast<double>(x[i]);
    y[i] = cast<TY>(a * xv);
  }
}

// ---------------------------------------------------------------- launchers
#define KGRID dim3(red_blocks(n)), dim3(KRED_THREADS), 0, st

template <typename T>
hipError_t launch_k_p_update(cplx<T>* p, const cplx<T>* r, const cplx<T>* v, int64_t n,
                             KState* ks, hipStream_t st) {
  hipLaunchKernelGGL((k_p_update<T>), KGRID, p, r, v, n, ks);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_dot_rv(const cplx<T>* rh, const cplx<T>* v, int64_t n, KState* ks,
                           double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_dot_rv<T>), KGRID, rh, v, n, ks, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_s_update(cplx<T>* s, const cplx<T>* r, const cplx<T>* v, int64_t n,
                             KState* ks, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_s_update<T>), KGRID, s, r, v, n, ks, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_dot_ts(const cplx<T>* t, const cplx<T>* s, int64_t n, KState* ks,
                           double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_dot_ts<T>), KGRID, t, s, n, ks, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_xr_update(cplx<T>* y, cplx<T>* r, const cplx<T>* p, const cplx<T>* s,
                              const cplx<T>* t, const cplx<T>* rh, int64_t n, KState* ks,
                              double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_xr_update<T>), KGRID, y, r, p, s, t, rh, n, ks, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_init(cplx<T>* rh, const cplx<T>* r, cplx<T>* p, cplx<T>* v, cplx<T>* y,
                         int64_t n, KState* ks, double* part, double bnorm2, double tol2,
                         hipStream_t st) {
  hipLaunchKernelGGL((k_init<T>), KGRID, rh, r, p, v, y, n, ks, part, bnorm2, tol2);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_residual(cplx<T>* out, const cplx<T>* a, const cplx<T>* b, int64_t n,
                             KState* ks, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_residual<T>), KGRID, out, a, b, n, ks, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_norm2(const cplx<T>* a, int64_t n, KState* ks, double* part,
                          hipStream_t st) {
  hipLaunchKernelGGL((k_norm2<T>), KGRID, a, n, ks, part);
  return hipGetLastError();
}
template <typename TY, typename TX>
hipError_t launch_k_axpy(cplx<TY>* y, const cplx<TX>* x, double a, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_axpy<TY, TX>), KGRID, y, x, a, n);
  return hipGetLastError();
}
template <typename TY, typename TX>
hipError_t launch_k_scale_copy(cplx<TY>* y, const cplx<TX>* x, double a, int64_t n,
                               hipStream_t st) {
  hipLaunchKernelGGL((k_scale_copy<TY, TX>), KGRID, y, x, a, n);
  return hipGetLastError();
}

#define PSFD_INST_K(T)                                                                        \
  template hipError_t launch_k_p_update<T>(cplx<T>*, const cplx<T>*, const cplx<T>*, int64_t, \
                                           KState*, hipStream_t);                             \
  template hipError_t launch_k_dot_rv<T>(const cplx<T>*, const cplx<T>*, int64_t, KState*,    \
                                         double*, hipStream_t);                               \
  template hipError_t launch_k_s_update<T>(cplx<T>*, const cplx<T>*, const cplx<T>*, int64_t, \
                                           KState*, double*, hipStream_t);                    \
  template hipError_t launch_k_dot_ts<T>(const cplx<T>*, const cplx<T>*, int64_t, KState*,    \
                                         double*, hipStream_t);                               \
  template hipError_t launch_k_xr_update<T>(cplx<T>*, cplx<T>*, const cplx<T>*,               \
                                            const cplx<T>*, const cplx<T>*, const cplx<T>*,   \
                                            int64_t, KState*, double*, hipStream_t);          \
  template hipError_t launch_k_init<T>(cplx<T>*, const cplx<T>*, cplx<T>*, cplx<T>*,          \
                                       cplx<T>*, int64_t, KState*, double*, double, double,   \
                                       hipStream_t);                                          \
  template hipError_t launch_k_residual<T>(cplx<T>*, const cplx<T>*, const cplx<T>*, int64_t, \
                                           KState*, double*, hipStream_t);                    \
  template hipError_t launch_k_norm2<T>(const cplx<T>*, int64_t, KState*, double*, hipStream_t);

PSFD_INST_K(double)
PSFD_INST_K(float)

template hipError_t launch_k_axpy<double, double>(cplx<double>*, const cplx<double>*, double,
                                                  int64_t, hipStream_t);
template hipError_t launch_k_axpy<double, float>(cplx<double>*, const cplx<float>*, double,
                                                 int64_t, hipStream_t);
template hipError_t launch_k_scale_copy<float, double>(cplx<float>*, const cplx<double>*, double,
                                                       int64_t, hipStream_t);
template hipError_t launch_k_scale_copy<double, float>(cplx<double>*, const cplx<float>*, double,
                                                       int64_t, hipStream_t);
template hipError_t launch_k_scale_copy<double, double>(cplx<double>*, const cplx<double>*,
                                                        double, int64_t, hipStream_t);

}  // namespace psfd
