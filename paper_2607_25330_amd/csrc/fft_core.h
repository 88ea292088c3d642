// Batched in-place Stockham FFT on data held in LDS.
//
// A transform of length N = 2^a 3^b is factored into radix-8/4/2/3 passes.
// Pass p with radix R and span NS (product of the earlier radices) reads the
// R inputs j + q N/R of butterfly j, multiplies input q by w^(q k) with
// k = j mod NS and w = exp(-+ 2 pi i / (NS R)), does a radix-R DFT and
// writes output q to (j / NS) NS R + k + q NS; after the last pass the data
// is in natural order (Stockham autosort, no bit reversal).
//
// Radix schedule S: 0 prefers radix 8 (fewest passes), 1 prefers radix 4
// (fewer registers and shorter butterflies, one more LDS pass); factors of 3
// always take radix-3 passes last.  The autotuner picks S per shape.
//
// Work split: every transform is handled by TPR = N / EPT threads, EPT being
// the lcm of the pass radices, so each thread owns EPT elements in every
// pass.  A pass loads all of a thread's inputs into registers, synchronises,
// then writes its outputs: a single LDS buffer suffices.  The caller's
// address functor maps (transform b, element i) to an LDS offset, which lets
// the same routine serve contiguous rows, strided columns and per-column
// axial vectors.
#pragma once
#include "cplx.h"

namespace psfd {

struct RadixPlan {
  int n, np, ept;
  int r[8];
  int ns[8];
};

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
constexpr int lcm_c(int a, int b) { return a / gcd_c(a, b) * b; }

constexpr RadixPlan make_radix_plan(int n, int sched = 0) {
  RadixPlan p{};
  p.n = n;
  int m = n, a = 0, b = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  int n8 = a / 3, rem = a % 3, k = 0;
  if (sched == 1) {
    for (int i = 0; i < a / 2; ++i) p.r[k++] = 4;
    if (a % 2) p.r[k++] = 2;
  } else if (rem == 1 && n8 > 0) {
    for (int i = 0; i < n8 - 1; ++i) p.r[k++] = 8;
    p.r[k++] = 4;
    p.r[k++] = 4;
  } else if (rem == 1) {
    p.r[k++] = 2;
  } else {
    for (int i = 0; i < n8; ++i) p.r[k++] = 8;
    if (rem == 2) p.r[k++] = 4;
  }
  for (int i = 0; i < b; ++i) p.r[k++] = 3;
  p.np = k;
  int ns = 1, e = 1;
  for (int i = 0; i < k; ++i) {
    p.ns[i] = ns;
    ns *= p.r[i];
    e = lcm_c(e, p.r[i]);
  }
  p.ept = e;
  return p;
}

template <int N, int S = 0>
struct Radices {
  static constexpr RadixPlan P = make_radix_plan(N, S);
  static constexpr int EPT = P.ept;
  static constexpr int TPR = N / P.ept;
};

// ---------------------------------------------------------------- small DFTs
template <typename T, int R, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<T, 2, INV> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T, bool INV>
struct Dft<T, 3, INV> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const T h = T(0.86602540378443864676);  // sin(pi/3)
    const T s = INV ? h : -h;
    cplx<T> t = v[1] + v[2], d = v[1] - v[2];
    cplx<T> m = v[0] - T(0.5) * t;
    cplx<T> e = mul_i(s * d);
    v[0] = v[0] + t;
    v[1] = m + e;
    v[2] = m - e;
  }
};

template <typename T, bool INV>
struct Dft<T, 4, INV> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
    cplx<T> t2 = v[1] + v[3], t3 = v[1] - v[3];
    cplx<T> r = INV ? mul_i(t3) : -mul_i(t3);
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + r;
    v[3] = t1 - r;
  }
};

template <typename T, bool INV>
struct Dft<T, 8, INV> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4, INV>::run(e);
    Dft<T, 4, INV>::run(o);
    const T c = T(0.70710678118654752440);
    // o[k] *= w^k, w = exp(-+ i pi / 4)
    cplx<T> o1 = INV ? cplx<T>{c * (o[1].re - o[1].im), c * (o[1].re + o[1].im)}
                     : cplx<T>{c * (o[1].re + o[1].im), c * (o[1].im - o[1].re)};
    cplx<T> o2 = INV ? mul_i(o[2]) : -mul_i(o[2]);
    cplx<T> o3 = INV ? cplx<T>{-c * (o[3].re + o[3].im), c * (o[3].re - o[3].im)}
                     : cplx<T>{c * (o[3].im - o[3].re), -c * (o[3].re + o[3].im)};
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
  }
};

// ---------------------------------------------------------- address functors
template <int PITCH>
struct AddrRow {  // transform b is a contiguous row
  __device__ __forceinline__ int operator()(int b, int i) const { return b * PITCH + i; }
};
// Contiguous rows with one element of padding per 256 bytes, so that the
// stride-R writes of the first Stockham passes spread over all LDS banks.
template <int N, int PADP>
struct AddrRowPad {
  static constexpr int PITCH = N + N / PADP;
  __device__ __forceinline__ int operator()(int b, int i) const { return b * PITCH + i + i / PADP; }
};
template <typename T>
constexpr int lds_pad_period() { return 256 / (int)sizeof(cplx<T>); }

template <int PITCH>
struct AddrCol {  // transform b is a column of a [N][PITCH] tile
  __device__ __forceinline__ int operator()(int b, int i) const { return i * PITCH + b; }
};
template <int TX, int PITCH, int VS>
struct AddrVec {  // transform b = (vector, column): [vector][i][column]
  __device__ __forceinline__ int operator()(int b, int i) const {
    return (b / TX) * VS + i * PITCH + (b % TX);
  }
};

// ---------------------------------------------------------------- one pass
template <typename T, int N, int R, int NS, int NB, int NT, bool INV, bool BFAST, int S, class Addr>
__device__ __forceinline__ void stockham_pass(cplx<T>* s, const cplx<T>* __restrict__ tw,
                                              Addr addr, int tid) {
  constexpr int EPT = Radices<N, S>::EPT;
  constexpr int TPR = Radices<N, S>::TPR;
  constexpr int NW = NB * TPR;
  constexpr int WPT = (NW + NT - 1) / NT;
  constexpr int BPI = EPT / R;
  cplx<T> v[WPT][EPT];
#pragma unroll
  for (int w = 0; w < WPT; ++w) {
    const int item = tid + w * NT;
    if ((NW % NT == 0) || item < NW) {
      const int b = BFAST ? item % NB : item / TPR;
      const int t = BFAST ? item / NB : item % TPR;
#pragma unroll
      for (int u = 0; u < BPI; ++u) {
        const int j = t + u * TPR;
#pragma unroll
        for (int q = 0; q < R; ++q) v[w][u * R + q] = s[addr(b, j + q * (N / R))];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < WPT; ++w) {
    const int item = tid + w * NT;
    if ((NW % NT == 0) || item < NW) {
      const int b = BFAST ? item % NB : item / TPR;
      const int t = BFAST ? item / NB : item % TPR;
#pragma unroll
      for (int u = 0; u < BPI; ++u) {
        const int j = t + u * TPR;
        const int k = j % NS;
        cplx<T> x[R];
#pragma unroll
        for (int q = 0; q < R; ++q) x[q] = v[w][u * R + q];
        if constexpr (NS > 1) {
#pragma unroll
          for (int q = 1; q < R; ++q) {
            cplx<T> wq = tw[q * k * (N / (NS * R))];
            if (INV) wq = conj(wq);
            x[q] = x[q] * wq;
          }
        }
        Dft<T, R, INV>::run(x);
        const int base = (j / NS) * NS * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) s[addr(b, base + q * NS)] = x[q];
      }
    }
  }
  __syncthreads();
}

// Passes I .. np - 2 (all but the last).
template <typename T, int N, int I, int NB, int NT, bool INV, bool BFAST, int S, class Addr>
__device__ __forceinline__ void stockham_mid(cplx<T>* s, const cplx<T>* __restrict__ tw, Addr addr,
                                             int tid) {
  if constexpr (I < Radices<N, S>::P.np - 1) {
    constexpr int R = Radices<N, S>::P.r[I];
    constexpr int NS = Radices<N, S>::P.ns[I];
    stockham_pass<T, N, R, NS, NB, NT, INV, BFAST, S>(s, tw, addr, tid);
    stockham_mid<T, N, I + 1, NB, NT, INV, BFAST, S>(s, tw, addr, tid);
  }
}

template <typename T, int N, int I, int NB, int NT, bool INV, bool BFAST, int S, class Addr>
__device__ __forceinline__ void stockham_passes(cplx<T>* s, const cplx<T>* __restrict__ tw,
                                                Addr addr, int tid) {
  if constexpr (I < Radices<N, S>::P.np) {
    constexpr int R = Radices<N, S>::P.r[I];
    constexpr int NS = Radices<N, S>::P.ns[I];
    stockham_pass<T, N, R, NS, NB, NT, INV, BFAST, S>(s, tw, addr, tid);
    stockham_passes<T, N, I + 1, NB, NT, INV, BFAST, S>(s, tw, addr, tid);
  }
}

// Items per thread of an NB-transform batch split over NT threads.
template <int N, int NB, int NT, int S>
constexpr int lds_fft_items() {
  return (NB * Radices<N, S>::TPR + NT - 1) / NT;
}

// lds_fft with the first pass fed from registers and the last pass left in
// registers: two LDS round trips (and two barriers) fewer.  Item w of the
// thread is item = tid + w * NT, i.e. transform b and thread-in-transform t
// as in stockham_pass.  On entry v[w][u * R0 + q] holds element
// j + q N / R0 of transform b (j = t + u TPR, R0 the first radix); on exit
// v[w][u * RL + q] holds output element j + q N / RL (RL the last radix).
// Needs at least two passes; synchronises like lds_fft.
template <typename T, int N, int NB, int NT, bool INV, bool BFAST, int S, class Addr, int WPT,
          int EPT>
__device__ __forceinline__ void lds_fft_regs(cplx<T> (&v)[WPT][EPT], cplx<T>* s,
                                             const cplx<T>* __restrict__ tw, Addr addr, int tid) {
  constexpr RadixPlan PL = Radices<N, S>::P;
  static_assert(PL.np >= 2, "at least two passes");
  static_assert(EPT == Radices<N, S>::EPT && WPT == lds_fft_items<N, NB, NT, S>(),
                "register array of the batch split");
  constexpr int TPR = Radices<N, S>::TPR;
  constexpr int NW = NB * TPR;
  constexpr int R0 = PL.r[0];
  constexpr int RL = PL.r[PL.np - 1];
  // first pass (span 1: no twiddles), from registers into LDS
#pragma unroll
  for (int w = 0; w < WPT; ++w) {
    const int item = tid + w * NT;
    if ((NW % NT == 0) || item < NW) {
      const int b = BFAST ? item % NB : item / TPR;
      const int t = BFAST ? item / NB : item % TPR;
#pragma unroll
      for (int u = 0; u < EPT / R0; ++u) {
        const int j = t + u * TPR;
        cplx<T> x[R0];
#pragma unroll
        for (int q = 0; q < R0; ++q) x[q] = v[w][u * R0 + q];
        Dft<T, R0, INV>::run(x);
#pragma unroll
        for (int q = 0; q < R0; ++q) s[addr(b, j * R0 + q)] = x[q];
      }
    }
  }
  __syncthreads();
  // middle passes in LDS
  if constexpr (PL.np > 2) stockham_mid<T, N, 1, NB, NT, INV, BFAST, S>(s, tw, addr, tid);
  // last pass (span N / RL), from LDS into registers
#pragma unroll
  for (int w = 0; w < WPT; ++w) {
    const int item = tid + w * NT;
    if ((NW % NT == 0) || item < NW) {
      const int b = BFAST ? item % NB : item / TPR;
      const int t = BFAST ? item / NB : item % TPR;
#pragma unroll
      for (int u = 0; u < EPT / RL; ++u) {
        const int j = t + u * TPR;  // < N / RL: the butterfly index and its twiddle power
        cplx<T> x[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q) x[q] = s[addr(b, j + q * (N / RL))];
#pragma unroll
        for (int q = 1; q < RL; ++q) {
          cplx<T> wq = tw[q * j];
          if (INV) wq = conj(wq);
          x[q] = x[q] * wq;
        }
        Dft<T, RL, INV>::run(x);
#pragma unroll
        for (int q = 0; q < RL; ++q) v[w][u * RL + q] = x[q];
      }
    }
  }
}

// NB transforms of length N in LDS; unnormalised in both directions.
// tw: table exp(-2 pi i m / N), m = 0..N-1.  Must be called by all NT
// threads of the block (it synchronises).  BFAST: consecutive threads take
// consecutive transforms (strided layouts) rather than consecutive
// elements of one transform (contiguous rows).
template <typename T, int N, int NB, int NT, bool INV, bool BFAST, int S = 0, class Addr>
__device__ __forceinline__ void lds_fft(cplx<T>* s, const cplx<T>* __restrict__ tw, Addr addr,
                                        int tid) {
  stockham_passes<T, N, 0, NB, NT, INV, BFAST, S>(s, tw, addr, tid);
}

}  // namespace psfd
