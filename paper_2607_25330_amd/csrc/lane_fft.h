// Register-resident FFT of short columns split over L lanes of a wavefront.
//
// A column of length N = L * E is held by L consecutive lanes (a lane group
// inside one quad or octet); lane t keeps elements n = t + L m, m = 0..E-1, in
// registers.  With n = t + L m and k = k2 + E k1 the DFT factorises as
//   X[k2 + E k1] = sum_t w_L^(t k1) w_N^(t k2) sum_m x[t + L m] w_E^(m k2):
//   1. an E-point DFT over each lane's own registers (compile-time Stockham,
//      twiddles are immediates),
//   2. a multiply by the lane twiddle w_N^(t k2),
//   3. an L-point DFT across the lane group, done as log2(L) radix-2
//      decimation-in-frequency butterflies between lanes t and t ^ h
//      (DPP quad permutes for h = 1, 2; ds_swizzle for h >= 4).
// Lane t then holds X[k2 + E brev(t)] for k2 = 0..E-1 ("k layout").  The
// inverse runs the mirror image (decimation in time across lanes, conjugate
// twiddles, inverse E-point DFT) and returns to the "z layout".  Both are
// unnormalised.  Every lane of the wavefront must be active.
#pragma once
#include "fft_core.h"

namespace psfd {

// ---------------------------------------------------------- constexpr roots
// cos and sin of 2 pi a / b, evaluated at compile time: octant reduction on
// the exact fraction, then Taylor series on |angle| <= pi/4.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double y) {
  double term = y, sum = y;
  for (int n = 1; n < 14; ++n) {
    term *= -y * y / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double y) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -y * y / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// cos (which = 0) or sin (which = 1) of 2 pi a / b.  With A = a mod b the
// octant is o = floor(8 A / b) and the remainder x = pi (8 A - o b) / (4 b)
// lies in [0, pi/4); odd octants use y = pi/4 - x and the next quarter turn.
constexpr double root_2pi(long a, long b, int which) {
  long A = a % b;
  if (A < 0) A += b;
  const long o = (8 * A) / b;
  const long num = 8 * A - o * b;  // in [0, b)
  double c = 0.0, s = 0.0;
  long j = 0;
  if (o % 2 == 0) {
    const double x = kPi * (double)num / (4.0 * (double)b);
    c = taylor_cos(x);
    s = taylor_sin(x);
    j = o / 2;
  } else {
    const double y = kPi * (double)(b - num) / (4.0 * (double)b);
    c = taylor_cos(y);
    s = -taylor_sin(y);
    j = o / 2 + 1;
  }
  double rc = c, rs = s;
  switch (j % 4) {
    case 1: rc = -s; rs = c; break;
    case 2: rc = -c; rs = -s; break;
    case 3: rc = s; rs = -c; break;
    default: break;
  }
  return which == 0 ? rc : rs;
}

template <int B>
struct UnitRoots {  // exp(-2 pi i a / B), a = 0..B-1
  struct Tab {
    double c[B], s[B];
  };
  static constexpr Tab make() {
    Tab t{};
    for (int a = 0; a < B; ++a) {
      t.c[a] = root_2pi(a, B, 0);
      t.s[a] = -root_2pi(a, B, 1);
    }
    return t;
  }
  static constexpr Tab tab = make();
};

// ------------------------------------------------ E-point DFT in registers
template <typename T, int E, int I, bool INV>
__device__ __forceinline__ void reg_passes(cplx<T> (&v)[E]) {
  if constexpr (I < Radices<E>::P.np) {
    constexpr int R = Radices<E>::P.r[I];
    constexpr int NS = Radices<E>::P.ns[I];
    cplx<T> o[E];
#pragma unroll
    for (int j = 0; j < E / R; ++j) {
      const int k = j % NS;
      cplx<T> x[R];
#pragma unroll
      for (int q = 0; q < R; ++q) x[q] = v[j + q * (E / R)];
      if constexpr (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          const int a = (q * k) % (NS * R);
          const T c = (T)UnitRoots<NS * R>::tab.c[a];
          const T s = (T)UnitRoots<NS * R>::tab.s[a];
          x[q] = x[q] * cplx<T>{c, INV ? -s : s};
        }
      }
      Dft<T, R, INV>::run(x);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) o[base + q * NS] = x[q];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = o[e];
    reg_passes<T, E, I + 1, INV>(v);
  }
}

// ------------------------------------------------------ lane exchange
template <int H>
__device__ __forceinline__ int lane_xor_i(int i) {
  if constexpr (H == 1) return __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, true);  // quad_perm 1,0,3,2
  else if constexpr (H == 2) return __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, true);  // 2,3,0,1
  else return __builtin_amdgcn_ds_swizzle(i, (H << 10) | 0x1F);  // bit mode, xor_mask = H
}
template <int H>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(lane_xor_i<H>(__float_as_int(v)));
}
template <int H>
__device__ __forceinline__ double lane_xor(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_xor_i<H>((int)(b & 0xffffffffLL));
  const int hi = lane_xor_i<H>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int H, typename T>
__device__ __forceinline__ cplx<T> lane_xor(cplx<T> v) {
  return {lane_xor<H>(v.re), lane_xor<H>(v.im)};
}

// Sum of v over the L lanes of a group (every lane gets the sum).
template <int L, typename T>
__device__ __forceinline__ cplx<T> lane_group_sum(cplx<T> v) {
  if constexpr (L >= 2) v = v + lane_xor<1>(v);
  if constexpr (L >= 4) v = v + lane_xor<2>(v);
  if constexpr (L >= 8) v = v + lane_xor<4>(v);
  if constexpr (L >= 16) v = v + lane_xor<8>(v);
  return v;
}

template <int L>
__device__ __forceinline__ int lane_brev(int t) {
  int r = 0;
#pragma unroll
  for (int b = 1; b < L; b <<= 1) r = (r << 1) | ((t & b) ? 1 : 0);
  return r;
}

template <typename T, int N, int L>
struct LaneFft {
  static constexpr int E = N / L;
  static constexpr int P = (L == 1) ? 0 : (L == 2) ? 1 : (L == 4) ? 2 : (L == 8) ? 3 : 4;
  static_assert((1 << P) == L && N % L == 0, "lane count must be a power of two dividing N");
  cplx<T> tw[E];   // w_N^(t k2)
  cplx<T> cw[P];   // stage s (h = 2^s): w_2h^(t mod h) on the lanes with bit s set, else 1
  T sg[P];         // +1 on the lanes with bit s clear, -1 otherwise
  bool rot;        // span-2 stage twiddle is not 1 (t mod 4 == 3)

  // tw_n: table exp(-2 pi i m / N), m = 0..N-1
  __device__ __forceinline__ void init(const cplx<T>* __restrict__ tw_n, int t) {
    rot = (t & 3) == 3;
#pragma unroll
    for (int k2 = 0; k2 < E; ++k2) tw[k2] = tw_n[t * k2];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int h = 1 << s;
      sg[s] = (t & h) ? T(-1) : T(1);
      cw[s] = (t & h) ? tw_n[(t & (h - 1)) * (N / (2 * h))] : cplx<T>{T(1), T(0)};
    }
  }

  // z layout -> k layout
  __device__ __forceinline__ void fwd(cplx<T> (&v)[E]) const {
    reg_passes<T, E, 0, false>(v);
#pragma unroll
    for (int k2 = 1; k2 < E; ++k2) v[k2] = v[k2] * tw[k2];
    stages_fwd<P - 1>(v);
  }
  // k layout -> z layout
  __device__ __forceinline__ void inv(cplx<T> (&v)[E]) const {
    stages_inv<0>(v);
#pragma unroll
    for (int k2 = 1; k2 < E; ++k2) v[k2] = cmulc(tw[k2], v[k2]);
    reg_passes<T, E, 0, true>(v);
  }

 private:
  // The span-2 stage's twiddle is 1 or -i (forward) / +i (inverse): a swap
  // with a sign instead of a complex product.
  __device__ __forceinline__ cplx<T> rot_fwd(cplx<T> a) const {
    return rot ? cplx<T>{a.im, -a.re} : a;
  }
  __device__ __forceinline__ cplx<T> rot_inv(cplx<T> a) const {
    return rot ? cplx<T>{-a.im, a.re} : a;
  }
  template <int S>
  __device__ __forceinline__ void stages_fwd(cplx<T> (&v)[E]) const {
    if constexpr (S >= 0) {
      constexpr int H = 1 << S;
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) {
        const cplx<T> p = lane_xor<H>(v[k2]);
        cplx<T> r = p + sg[S] * v[k2];
        if constexpr (H == 2) r = rot_fwd(r);
        else if constexpr (H > 2) r = r * cw[S];
        v[k2] = r;
      }
      stages_fwd<S - 1>(v);
    }
  }
  template <int S>
  __device__ __forceinline__ void stages_inv(cplx<T> (&v)[E]) const {
    if constexpr (S < P) {
      constexpr int H = 1 << S;
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) {
        cplx<T> a = v[k2];
        if constexpr (H == 2) a = rot_inv(a);
        else if constexpr (H > 2) a = cmulc(cw[S], a);
        const cplx<T> p = lane_xor<H>(a);
        v[k2] = p + sg[S] * a;
      }
      stages_inv<S + 1>(v);
    }
  }
};

}  // namespace psfd
