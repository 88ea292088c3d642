// Threshold-contour width metric on field planes (paper, Results,
// "Practical assessment of scattered-field convergence" paragraph and its
// equation logistic_sigmoid).
//
// Segments: one wavefront per scan line.  The 64 lanes walk the line in
// chunks; each lane tests whether the threshold lies between its sample and
// the next one (the line is periodic), a ballot and a population count give
// every crossing its index in line order, and the crossings (position,
// direction) are stored in LDS.  The segments (an upward crossing to the
// next downward one) are then written in parallel.  A sample is above
// threshold when I = re*re + im*im > I_th, each product rounded on its own
// (no fused multiply-add), so the segment structure does not depend on how
// the sigmoid rounds; the crossing is placed by linear interpolation of
// S(I) = 1 / (1 + exp(-(I - I_th) / w)) between the two samples.
//
// Deviation: one thread per reference segment slot finds the segment of the
// other plane, on the same line, whose periodic interval holds the
// reference segment's centre, writes (d_ref - d) / demag (NaN when there is
// none) and adds to per-block FP64 partials of the statistics.
#include <hip/hip_runtime.h>

#include <cmath>

#include "psfd_internal.h"

namespace psfd {

namespace {

__device__ __forceinline__ double intensity_rn(cplx<double> v) {
  return __dadd_rn(__dmul_rn(v.re, v.re), __dmul_rn(v.im, v.im));
}

__device__ __forceinline__ double logistic(double I, double i_th, double w) {
  return 1.0 / (1.0 + exp(-(I - i_th) / w));
}

__global__ void __launch_bounds__(64) k_contour_segments(const ContourArgs a) {
  const int line = blockIdx.x;  // 0 .. 2 nlines - 1: horizontal lines first
  const int pl = blockIdx.y;
  const int lane = threadIdx.x;
  const bool horiz = line < a.nlines;
  const int l = horiz ? line : line - a.nlines;
  const int n = horiz ? a.nx : a.ny;
  const int across = horiz ? a.ny : a.nx;
  const int at = (int)((l + 0.5) * across / a.nlines);
  const int64_t step = horiz ? 1 : a.nx;
  const cplx<double>* v = a.f + (int64_t)pl * a.pstride + (horiz ? (int64_t)at * a.nx : (int64_t)at);
  const double h = horiz ? a.dx : a.dy;

  __shared__ double xpos[kContourLineMax];
  __shared__ int xup[kContourLineMax];
  int count = 0;  // crossings found so far (the same in every lane)
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int j = c0 + lane;
    bool cross = false;
    double p = 0.0;
    int up = 0;
    if (j < n) {
      const int j1 = (j + 1 == n) ? 0 : j + 1;
      const double I0 = intensity_rn(v[j * step]);
      const double I1 = intensity_rn(v[j1 * step]);
      const bool a0 = I0 > a.i_th, a1 = I1 > a.i_th;
      if (a0 != a1) {
        const double s0 = logistic(I0, a.i_th, a.w), s1 = logistic(I1, a.i_th, a.w);
        p = (j + (0.5 - s0) / (s1 - s0)) * h;
        up = a1 ? 1 : 0;
        cross = true;
      }
    }
    const unsigned long long m = __ballot(cross);
    const int idx = count + __popcll(m & ((1ull << lane) - 1ull));
    if (cross) {
      xpos[idx] = p;
      xup[idx] = up;
    }
    count += __popcll(m);
  }
  __syncthreads();
  const int nseg = count / 2;
  const int64_t lg = (int64_t)pl * 2 * a.nlines + line;
  if (lane == 0) a.nseg[lg] = nseg;
  if (count == 0) return;
  int first = count;
  for (int i = lane; i < count; i += 64)
    if (xup[i] && i < first) first = i;
  for (int o = 32; o > 0; o >>= 1) first = min(first, __shfl_xor(first, o));
  const double L = n * h;
  double* out = a.seg + lg * a.max_seg * 2;
  for (int q = lane; q < nseg && q < a.max_seg; q += 64) {
    const double u = xpos[(first + 2 * q) % count];
    const double d = xpos[(first + 2 * q + 1) % count];
    double wd = d - u;
    if (wd < 0) wd += L;
    out[2 * q] = u;
    out[2 * q + 1] = wd;
  }
}

__global__ void __launch_bounds__(256) k_contour_deviation(const DeviationArgs a) {
  const int tid = threadIdx.x;
  const int64_t items = (int64_t)a.nplanes * 2 * a.nlines * a.max_seg;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // sum |dd|, sum dd^2, resolved, unresolved, |dd| > thr
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < items; i += (int64_t)gridDim.x * 256) {
    const int q = (int)(i % a.max_seg);
    const int64_t lg = i / a.max_seg;
    const int line = (int)(lg % (2 * a.nlines));
    const int nr = min(a.nref[lg], a.max_seg);
    if (q >= nr) {
      a.delta[i] = 0.0;
      continue;
    }
    const double L = line < a.nlines ? a.len_h : a.len_v;
    const double s = a.sref[2 * i], wr = a.sref[2 * i + 1];
    const double c = fmod(s + 0.5 * wr, L);
    const int nk = min(a.nk[lg], a.max_seg);
    const double* sk = a.sk + lg * a.max_seg * 2;
    double wk = -1.0;
    for (int t = 0; t < nk; ++t) {
      double dlt = fmod(c - sk[2 * t], L);
      if (dlt < 0) dlt += L;
      if (dlt < sk[2 * t + 1]) {
        wk = sk[2 * t + 1];
        break;
      }
    }
    if (wk < 0) {
      a.delta[i] = __builtin_nan("");
      acc[3] += 1.0;
    } else {
      const double dd = (wr - wk) / a.demag;
      a.delta[i] = dd;
      acc[0] += fabs(dd);
      acc[1] += dd * dd;
      acc[2] += 1.0;
      if (fabs(dd) > a.thr) acc[4] += 1.0;
    }
  }
  __shared__ double red[5][256];
  for (int k = 0; k < 5; ++k) red[k][tid] = acc[k];
  __syncthreads();
  for (int hh = 128; hh > 0; hh >>= 1) {
    if (tid < hh)
      for (int k = 0; k < 5; ++k) red[k][tid] += red[k][tid + hh];
    __syncthreads();
  }
  if (tid < 5) a.part[(int64_t)blockIdx.x * 5 + tid] = red[tid][0];
}

}  // namespace

hipError_t launch_contour_segments(const ContourArgs& a, int nplanes, hipStream_t st) {
  hipLaunchKernelGGL(k_contour_segments, dim3(2 * a.nlines, nplanes), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_contour_deviation(const DeviationArgs& a, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_contour_deviation, dim3(nblocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace psfd
