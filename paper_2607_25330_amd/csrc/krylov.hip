// BiCGSTAB vector kernels and scalar finalisation (paper: BiCGSTAB with right
// preconditioning, Results section, "PINO warm-start" paragraph; stop test on
// the relative residual of equation relative_residual).
//
// Every scalar of the recurrence (rho, alpha, omega, norms) lives in a
// device-side KState in FP64, so an iteration is a fixed sequence of
// launches with no host round trip.  Kernels that contribute to an inner
// product write one FP64 partial per block; a one-block finalize kernel adds
// them in a fixed order and updates the scalars and the flags:
//   done = 0 running, 1 converged, 2 pending half step (y += alpha p only),
//   3 breakdown or divergence (the host restarts from the current field),
//   4 idle (the problem is not part of this run),
//   5 iteration budget of the run used up,
//   6 reliable update due: the recursive residual fell by the factor delta
//     since the last true residual; the host folds the iterate into the
//     high-precision solution, recomputes the true residual, replaces r with
//     it (FIN_REPLACE: rho = <rh, r>) and the recurrence continues with its
//     search direction p and shadow residual rh kept.
// A plan may hold a group of problems: every kernel here covers all of them,
// each block working for one problem (its index from the block index), and
// the finalize kernel runs one block per problem.
// Operator kernels skip when done != 0, so launches queued after
// convergence cost almost nothing.
//
// The stabilising step omega = <t,s>/<t,t> is limited as proposed by
// Sleijpen and van der Vorst (1995): when |<t,s>| < kappa ||t|| ||s||,
// omega is scaled by kappa ||t|| ||s|| / |<t,s>| (kappa = 0.7).  This keeps
// the BiCGSTAB recurrences and fixed point and avoids the stagnation of the
// plain form on strongly indefinite systems.
#include "psfd_internal.h"
#include "reduce.h"

namespace psfd {

constexpr double kOmegaLimit = 0.7;
// Reliable updates are due when the recursive residual has fallen by the
// factor delta below its value at the run's start or last replacement, or,
// after a spike of more than sqrt(kSpike2) over that value, by delta below
// the spike (the rounding gap between the recursive and the true residual
// grows with the largest residual seen, so a large spike calls for an
// earlier replacement).  Measured on the benchmark clips and the batched
// uneven workload: the spike rule alone (van der Vorst and Ye's running
// maximum) fires updates that the fold check rejects, the progress rule
// alone lets the gap grow on the small grids; together they keep both.
constexpr double kSpike2 = 10.0;

int red_blocks(int64_t n, int nprob) {
  // at most 8192 blocks per problem (enough waves in flight to keep the
  // streaming kernels at the copy rate) and 128k blocks per launch, so that
  // groups of up to 16 problems use the per-problem grid of a single solve
  int64_t b = (n + KRED_THREADS - 1) / KRED_THREADS;
  int64_t cap = 131072 / (nprob > 0 ? nprob : 1);
  if (cap > 8192) cap = 8192;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

__device__ __forceinline__ cplx<double> ld2(const double* a) { return {a[0], a[1]}; }
__device__ __forceinline__ void st2(double* a, cplx<double> v) { a[0] = v.re; a[1] = v.im; }

// ---------------------------------------------------------------- finalize
// Sum of nblocks partials (NV values each) over the block; thread 0 gets the totals.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int nblocks,
                                             double (&acc)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  // the loads of four partials are issued before their sums (latency, not
  // bandwidth, bounds this loop); the order of the additions is unchanged
  int b = threadIdx.x;
  for (; b + 3 * 1024 < nblocks; b += 4 * 1024) {
    double v[4][NV];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) v[u][k] = part[(size_t)(b + u * 1024) * KPART + k];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k] += v[u][k];
  }
  for (; b < nblocks; b += 1024) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += part[(size_t)b * KPART + k];
  }
  __shared__ double sm[NV][16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sm[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = 0.0;
      for (int w = 0; w < 16; ++w) t += sm[k][w];
      acc[k] = t;
    }
  }
}

template <int STAGE>
__global__ void __launch_bounds__(1024)
k_finalize(KState* ks_all, const double* __restrict__ part_all, int nblocks,
           const ProbParams* __restrict__ pp, const double* __restrict__ part2_all,
           int nblocks2) {
  KState* ks = ks_all + blockIdx.x;
  const double* part = part_all + (size_t)blockIdx.x * nblocks * KPART;
  const int d = ks->done;
  bool run;
  if (STAGE == FIN_INIT || STAGE == FIN_RED0 || STAGE == FIN_RED3) run = true;
  else if (STAGE == FIN_RHO) run = (d == KS_RUN || d == KS_HALF);
  else if (STAGE == FIN_REPLACE) run = (d == KS_UPDATE);
  else if (STAGE == FIN_SHADOW) run = (d == KS_RUN);
  else run = (d == KS_RUN);
  if (!run) return;
  constexpr int NV = (STAGE == FIN_INIT || STAGE == FIN_RED0) ? 1 : 3;
  double s2[1] = {0.0};
  if constexpr (STAGE == FIN_OMEGA) {
    if (part2_all) sum_partials<1>(part2_all + (size_t)blockIdx.x * nblocks2 * KPART, nblocks2, s2);
    __syncthreads();
  }
  double acc[NV];
  sum_partials<NV>(part, nblocks, acc);
  if (threadIdx.x != 0) return;
  if constexpr (STAGE == FIN_INIT) {
    const ProbParams q = pp[blockIdx.x];
    ks->rho[0] = acc[0];
    ks->rho[1] = 0.0;
    ks->rho_prev[0] = ks->alpha[0] = ks->omega[0] = 1.0;
    ks->rho_prev[1] = ks->alpha[1] = ks->omega[1] = 0.0;
    ks->rh_norm2 = acc[0];
    ks->rnorm2 = acc[0];
    ks->bnorm2 = q.bnorm2;
    ks->tol2 = q.tol2;
    ks->itmax = (int)q.itmax;
    ks->delta2 = q.delta2;
    ks->rmax2 = acc[0];
    ks->rfold2 = acc[0];
    ks->done = (q.tol2 < 0.0) ? KS_IDLE : (ks->itmax <= 0 ? KS_MAXIT : KS_RUN);
    ks->half = 0;
    ks->status = 0;
    ks->iter = 0;
  } else if constexpr (STAGE == FIN_RED0) {
    ks->red[0] = acc[0];
  } else if constexpr (STAGE == FIN_RED3) {
    ks->red[0] = acc[0];
    ks->red[1] = acc[1];
    ks->red[2] = acc[2];
  } else if constexpr (STAGE == FIN_ALPHA) {
    const cplx<double> rv = {acc[0], acc[1]};
    st2(ks->rv, rv);
    if (!(sqrt(norm2(rv)) > 1e-30 * sqrt(ks->rh_norm2 * acc[2]))) {
      ks->status = 1;
      ks->done = KS_BREAK;
    } else {
      st2(ks->alpha, cdiv(ld2(ks->rho), rv));
    }
  } else if constexpr (STAGE == FIN_OMEGA) {
    if (part2_all) {  // half-step test on ||s|| (partials of the forward x pass)
      ks->snorm2 = s2[0];
      if (s2[0] <= ks->tol2 * ks->bnorm2) {
        ks->half = 1;
        ks->done = KS_HALF;
        return;
      }
      if (!(s2[0] < 1e24 * ks->bnorm2)) {
        ks->status = 2;  // diverged (or not finite)
        ks->done = KS_BREAK;
        return;
      }
    }
    // partials hold sum conj(s) t; <t, s> is its conjugate
    const cplx<double> ts = {acc[0], -acc[1]};
    const double tt = acc[2];
    st2(ks->ts, ts);
    ks->tt = tt;
    if (!(tt > 0.0)) {
      ks->half = 1;
      ks->status = 1;
      ks->done = KS_HALF;
    } else {
      cplx<double> om = {ts.re / tt, ts.im / tt};
      const double c = sqrt(norm2(ts)) / sqrt(tt * ks->snorm2);
      if (c < kOmegaLimit && c > 0.0) om = (kOmegaLimit / c) * om;
      st2(ks->omega, om);
    }
  } else if constexpr (STAGE == FIN_RHO) {
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
    } else if (ks->iter >= ks->itmax) {
      ks->done = KS_MAXIT;
    } else if (!(acc[0] < 1e8 * ks->rfold2)) {
      // diverging: the residual has grown 1e4-fold since the run's start or
      // its last replacement (or is not finite)
      ks->status = 2;
      ks->done = KS_BREAK;
    } else {
      const cplx<double> om = ld2(ks->omega);
      if ((om.re == 0.0 && om.im == 0.0) ||
          !(sqrt(norm2(rho_new)) > 1e-30 * sqrt(ks->rh_norm2 * acc[0]))) {
        ks->status = 1;
        ks->done = KS_BREAK;
      } else if (ks->delta2 > 0.0 &&
                 (acc[0] <= ks->delta2 * ks->rfold2 ||
                  (ks->rmax2 >= kSpike2 * ks->rfold2 && acc[0] <= ks->delta2 * ks->rmax2))) {
        ks->done = KS_UPDATE;
      }
    }
    if (acc[0] > ks->rmax2) ks->rmax2 = acc[0];
  } else if constexpr (STAGE == FIN_SHADOW) {
    // a caller-given shadow residual replaced rh after FIN_INIT: partials
    // ||r||^2, sum conj(rh) r; ||rh||^2 is in red[0] (FIN_RED0 before this).
    // rho = <rh, r> = 0 is a breakdown of the recurrence before its first step.
    ks->rh_norm2 = ks->red[0];
    const cplx<double> rho = {acc[1], acc[2]};
    st2(ks->rho, rho);
    if (!(sqrt(norm2(rho)) > 1e-30 * sqrt(ks->rh_norm2 * acc[0]))) {
      ks->status = 1;
      ks->done = KS_BREAK;
    }
  } else if constexpr (STAGE == FIN_REPLACE) {
    // r was replaced by the true residual (host): partials ||r||^2, <rh, r>
    ks->rnorm2 = acc[0];
    ks->rmax2 = acc[0];
    ks->rfold2 = acc[0];
    st2(ks->rho, cplx<double>{acc[1], acc[2]});
    ks->done = (acc[0] <= ks->tol2 * ks->bnorm2) ? KS_CONV : KS_RUN;
  }
}

hipError_t launch_finalize(int stage, KState* ks, const double* part, int nblocks, int nprob,
                           const ProbParams* pp, hipStream_t st, const double* part2,
                           int nblocks2) {
  dim3 g(nprob), b(1024);
#define PSFD_FIN(S) hipLaunchKernelGGL(k_finalize<S>, g, b, 0, st, ks, part, nblocks, pp, part2, nblocks2)
  switch (stage) {
    case FIN_INIT: PSFD_FIN(FIN_INIT); break;
    case FIN_ALPHA: PSFD_FIN(FIN_ALPHA); break;
    case FIN_OMEGA: PSFD_FIN(FIN_OMEGA); break;
    case FIN_RHO: PSFD_FIN(FIN_RHO); break;
    case FIN_SHADOW: PSFD_FIN(FIN_SHADOW); break;
    case FIN_REPLACE: PSFD_FIN(FIN_REPLACE); break;
    case FIN_RED3: PSFD_FIN(FIN_RED3); break;
    default: PSFD_FIN(FIN_RED0); break;
  }
#undef PSFD_FIN
  return hipGetLastError();
}

// ------------------------------------------------------------- vector kernels
// Block -> (problem pb, block within the problem lb); problem pb's elements
// start at pb * n; element loop i = lb * NT + tid, step bpp * NT.
#define PSFD_GROUP_LOOP(i)                                                           \
  const int bpp = gridDim.x / nprob;                                                 \
  const int pb = blockIdx.x / bpp, lb = blockIdx.x % bpp;                            \
  const int64_t off = (int64_t)pb * n;                                               \
  for (int64_t i = off + (int64_t)lb * blockDim.x + threadIdx.x; i < off + n;        \
       i += (int64_t)bpp * blockDim.x)

// y += alpha p + omega s;  r = s - omega t;  partials ||r||^2, sum conj(rh) r.
// In the pending-half-step state only y += alpha p.
template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_xr_update(cplx<T>* __restrict__ y, cplx<T>* __restrict__ r, const cplx<T>* __restrict__ p,
            const cplx<T>* __restrict__ s, const cplx<T>* __restrict__ t,
            const cplx<T>* __restrict__ rh, int64_t n, int nprob, const KState* __restrict__ ks_all,
            double* __restrict__ part) {
  const KState* ks = ks_all + blockIdx.x / (gridDim.x / nprob);
  const int d = ks->done;
  if (d != KS_RUN && d != KS_HALF) return;
  const cplx<T> al = cast<T>(ld2(ks->alpha));
  double acc[3] = {0.0, 0.0, 0.0};
  if (d == KS_HALF) {
    PSFD_GROUP_LOOP(i) y[i] = y[i] + al * p[i];
  } else {
    const cplx<T> om = cast<T>(ld2(ks->omega));
    // two elements per trip: all ten loads are issued before the first use
    const int bpp = gridDim.x / nprob;
    const int64_t off = (int64_t)(blockIdx.x / bpp) * n;
    const int64_t step = (int64_t)bpp * blockDim.x;
    for (int64_t i = (int64_t)(blockIdx.x % bpp) * blockDim.x + threadIdx.x; i < n; i += 2 * step) {
      const bool two = i + step < n;
      const int64_t i0 = off + i, i1 = off + (two ? i + step : i);
      const cplx<T> s0 = s[i0], s1 = s[i1], t0 = t[i0], t1 = t[i1];
      const cplx<T> y0 = y[i0], y1 = y[i1], p0 = p[i0], p1 = p[i1];
      const cplx<T> h0 = rh[i0], h1 = rh[i1];
      const cplx<T> r0 = s0 - om * t0;
      y[i0] = y0 + al * p0 + om * s0;
      r[i0] = r0;
      const cplx<double> a0 = cast<double>(h0), b0 = cast<double>(r0);
      acc[0] += norm2(b0);
      acc[1] += a0.re * b0.re + a0.im * b0.im;
      acc[2] += a0.re * b0.im - a0.im * b0.re;
      if (two) {
        const cplx<T> r1 = s1 - om * t1;
        y[i1] = y1 + al * p1 + om * s1;
        r[i1] = r1;
        const cplx<double> a1 = cast<double>(h1), b1 = cast<double>(r1);
        acc[0] += norm2(b1);
        acc[1] += a1.re * b1.re + a1.im * b1.im;
        acc[2] += a1.re * b1.im - a1.im * b1.re;
      }
    }
  }
  block_partials<3, KRED_THREADS>(acc, part);
}

// p = r + beta (p - omega v) as a separate pass (used where the update cannot be
// fused into the forward x pass).
template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_p_update(cplx<T>* __restrict__ p, const cplx<T>* __restrict__ r, const cplx<T>* __restrict__ v,
           int64_t n, int nprob, const KState* __restrict__ ks_all) {
  const KState* ks = ks_all + blockIdx.x / (gridDim.x / nprob);
  if (ks->done != KS_RUN) return;
  const cplx<double> beta = cdiv(ld2(ks->rho), ld2(ks->rho_prev)) * cdiv(ld2(ks->alpha), ld2(ks->omega));
  const cplx<T> b = cast<T>(beta), w = cast<T>(ld2(ks->omega));
  PSFD_GROUP_LOOP(i) p[i] = r[i] + b * (p[i] - w * v[i]);
}

// rh = r; p = v = y = 0; partials ||r||^2.
template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_init(cplx<T>* __restrict__ rh, const cplx<T>* __restrict__ r, cplx<T>* __restrict__ p,
       cplx<T>* __restrict__ v, cplx<T>* __restrict__ y, int64_t n, int nprob,
       double* __restrict__ part) {
  double acc[1] = {0.0};
  const cplx<T> zero = {T(0), T(0)};
  PSFD_GROUP_LOOP(i) {
    const cplx<T> ri = r[i];
    rh[i] = ri;
    p[i] = zero;
    v[i] = zero;
    y[i] = zero;
    acc[0] += norm2(cast<double>(ri));
  }
  block_partials<1, KRED_THREADS>(acc, part);
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_residual(cplx<T>* __restrict__ out, const cplx<T>* __restrict__ a, const cplx<T>* __restrict__ b,
           int64_t n, int nprob, const int* __restrict__ skip, double* __restrict__ part) {
  // problems flagged in skip (whose operator apply was skipped) are left alone
  if (skip && skip[blockIdx.x / (gridDim.x / nprob)]) return;
  double acc[1] = {0.0};
  PSFD_GROUP_LOOP(i) {
    const cplx<T> d = a[i] - b[i];
    out[i] = d;
    acc[0] += norm2(cast<double>(d));
  }
  block_partials<1, KRED_THREADS>(acc, part);
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_dot_rr(const cplx<T>* __restrict__ rh, const cplx<T>* __restrict__ r, int64_t n, int nprob,
         double* __restrict__ part) {
  double acc[3] = {0.0, 0.0, 0.0};
  PSFD_GROUP_LOOP(i) {
    const cplx<double> a = cast<double>(rh[i]), b = cast<double>(r[i]);
    acc[0] += norm2(b);
    acc[1] += a.re * b.re + a.im * b.im;
    acc[2] += a.re * b.im - a.im * b.re;
  }
  block_partials<3, KRED_THREADS>(acc, part);
}

template <typename T>
__global__ void __launch_bounds__(KRED_THREADS)
k_norm2(const cplx<T>* __restrict__ a, int64_t n, int nprob, double* __restrict__ part) {
  double acc[1] = {0.0};
  PSFD_GROUP_LOOP(i) acc[0] += norm2(cast<double>(a[i]));
  block_partials<1, KRED_THREADS>(acc, part);
}

template <typename TY, typename TX>
__global__ void __launch_bounds__(KRED_THREADS)
k_axpy(cplx<TY>* __restrict__ y, const cplx<TX>* __restrict__ x,
       const ProbParams* __restrict__ pp, int64_t n, int nprob) {
  const double a = pp[blockIdx.x / (gridDim.x / nprob)].scale;
  if (a == 0.0) return;
  PSFD_GROUP_LOOP(i) {
    const cplx<TY> xv = cast<TY>(x[i]);
    y[i] = y[i] + TY(a) * xv;
  }
}

template <typename TY, typename TX>
__global__ void __launch_bounds__(KRED_THREADS)
k_scale_copy(cplx<TY>* __restrict__ y, const cplx<TX>* __restrict__ x,
             const ProbParams* __restrict__ pp, int64_t n, int nprob) {
  double a = 1.0;
  if (pp) {
    const ProbParams& q = pp[blockIdx.x / (gridDim.x / nprob)];
    if (q.mask == 0.0) return;
    a = q.iscale;
  }
  PSFD_GROUP_LOOP(i) {
    const cplx<double> xv = cast<double>(x[i]);
    y[i] = cast<TY>(a * xv);
  }
}

// ---------------------------------------------------------------- launchers
#define KGRID dim3(nprob * red_blocks(n, nprob)), dim3(KRED_THREADS), 0, st

template <typename T>
hipError_t launch_k_xr_update(cplx<T>* y, cplx<T>* r, const cplx<T>* p, const cplx<T>* s,
                              const cplx<T>* t, const cplx<T>* rh, int64_t n, int nprob,
                              const KState* ks, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_xr_update<T>), KGRID, y, r, p, s, t, rh, n, nprob, ks, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_p_update(cplx<T>* p, const cplx<T>* r, const cplx<T>* v, int64_t n,
                             int nprob, const KState* ks, hipStream_t st) {
  hipLaunchKernelGGL((k_p_update<T>), KGRID, p, r, v, n, nprob, ks);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_init(cplx<T>* rh, const cplx<T>* r, cplx<T>* p, cplx<T>* v, cplx<T>* y,
                         int64_t n, int nprob, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_init<T>), KGRID, rh, r, p, v, y, n, nprob, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_residual(cplx<T>* out, const cplx<T>* a, const cplx<T>* b, int64_t n,
                             int nprob, const int* skip, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_residual<T>), KGRID, out, a, b, n, nprob, skip, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_dot_rr(const cplx<T>* rh, const cplx<T>* r, int64_t n, int nprob,
                           double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_dot_rr<T>), KGRID, rh, r, n, nprob, part);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_k_norm2(const cplx<T>* a, int64_t n, int nprob, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_norm2<T>), KGRID, a, n, nprob, part);
  return hipGetLastError();
}
template <typename TY, typename TX>
hipError_t launch_k_axpy(cplx<TY>* y, const cplx<TX>* x, const ProbParams* pp, int64_t n,
                         int nprob, hipStream_t st) {
  hipLaunchKernelGGL((k_axpy<TY, TX>), KGRID, y, x, pp, n, nprob);
  return hipGetLastError();
}
template <typename TY, typename TX>
hipError_t launch_k_scale_copy(cplx<TY>* y, const cplx<TX>* x, const ProbParams* pp, int64_t n,
                               int nprob, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_copy<TY, TX>), KGRID, y, x, pp, n, nprob);
  return hipGetLastError();
}

#define PSFD_INST_K(T)                                                                        \
  template hipError_t launch_k_xr_update<T>(cplx<T>*, cplx<T>*, const cplx<T>*,               \
                                            const cplx<T>*, const cplx<T>*, const cplx<T>*,   \
                                            int64_t, int, const KState*, double*, hipStream_t); \
  template hipError_t launch_k_p_update<T>(cplx<T>*, const cplx<T>*, const cplx<T>*, int64_t, \
                                           int, const KState*, hipStream_t);                  \
  template hipError_t launch_k_init<T>(cplx<T>*, const cplx<T>*, cplx<T>*, cplx<T>*,          \
                                       cplx<T>*, int64_t, int, double*, hipStream_t);         \
  template hipError_t launch_k_residual<T>(cplx<T>*, const cplx<T>*, const cplx<T>*, int64_t, \
                                           int, const int*, double*, hipStream_t);            \
  template hipError_t launch_k_norm2<T>(const cplx<T>*, int64_t, int, double*, hipStream_t);   \
  template hipError_t launch_k_dot_rr<T>(const cplx<T>*, const cplx<T>*, int64_t, int, double*, \
                                         hipStream_t);

PSFD_INST_K(double)
PSFD_INST_K(float)

#define PSFD_INST_AX(TY, TX)                                                                  \
  template hipError_t launch_k_axpy<TY, TX>(cplx<TY>*, const cplx<TX>*, const ProbParams*,    \
                                            int64_t, int, hipStream_t);                       \
  template hipError_t launch_k_scale_copy<TY, TX>(cplx<TY>*, const cplx<TX>*,                 \
                                                  const ProbParams*, int64_t, int, hipStream_t);
PSFD_INST_AX(double, double)
PSFD_INST_AX(double, float)
PSFD_INST_AX(float, double)
PSFD_INST_AX(float, float)

}  // namespace psfd
