// Lateral (x, y) FFT passes of the operator apply.
//
// Every field is [3][Nz][ny][nx] with x fastest.  The 2-D lateral transform
// of every (component, row) plane is done in two HBM passes: an x pass over
// contiguous rows (a block owns B whole rows, fully coalesced) and a y pass
// over a tile of TX adjacent columns of one plane (each tile row is a
// contiguous TX-element segment).  The inverse x pass carries the pointwise
// epilogue of the operator:  y = F2^-1[U] - k0^2 d_eps F2^-1[W]  on absorber
// rows (forward operator) or  y = F2^-1[U] - conj(k0^2 d_eps) x  (adjoint).
#include "fft_core.h"
#include "psfd_internal.h"
#include "reduce.h"

namespace psfd {

bool lateral_size_ok(int n) {
  switch (n) {
    case 16: case 32: case 64: case 128: case 192: case 256: case 512: case 1024: return true;
    default: return false;
  }
}

template <typename T>
constexpr int x_elems() { return sizeof(T) == 8 ? 2048 : 4096; }

// Schedules (chosen per shape by the autotuner, default 0):
//   x passes: bit 0 = radix schedule S, bit 1 = half the rows per block;
//   y pass:   bit 0 = radix schedule S, bit 1 = half the tile width.
template <typename T, int N, int HALF = 0, int S = 0>
constexpr int x_rows() {
  int b = 1;
  while (2 * b * N <= x_elems<T>()) b *= 2;
  return (HALF && b > 1 && (b / 2) * Radices<N, S>::TPR >= 64) ? b / 2 : b;
}

// rows per block of the inverse x pass: the combine needs a second buffer (W rows)
template <typename T, int N, int CM, int S = 0, int HALF = 0>
constexpr int xinv_rows() {
  constexpr int b = x_rows<T, N, HALF, S>();
  return (CM == CB_FWD && b > 1 && (b / 2) * Radices<N, S>::TPR >= 64) ? b / 2 : b;
}

template <typename T, int N, int S = 0, int HALF = 0>
constexpr int y_tile() {
  int tx = 65536 / (N * (int)sizeof(cplx<T>));
  if (tx > 16) tx = 16;
  while (tx > 1 && tx * Radices<N, S>::TPR > 1024) tx /= 2;
  if (HALF && tx > 1 && (tx / 2) * Radices<N, S>::TPR >= 64) tx /= 2;
  return tx;
}

// ------------------------------------------------------------------ kernels

// A launch covers nprob problems: each problem owns bpp consecutive blocks
// (bpp = ceil(rows per problem / rows per block)), so no block straddles two
// problems and block partials stay per problem.
struct RowGroup {
  int nprob = 1;
  int bpp = 1;
  int64_t nmain = 0;       // rows per problem taken straight from the input stack
  int64_t ntot = 0;        // rows per problem in total (adjoint: + 3 nabs ny extra rows)
  int64_t in_stride = 0;   // elements per problem of the input stack
  int64_t out_stride = 0;  // elements per problem of the output stack
  int64_t kd_stride = 0;   // elements per problem of kd
  const int* skip = nullptr;
  int skip_stride = 0;
};

template <typename T>
__device__ __forceinline__ cplx<double> ldks(const double* a) { return {a[0], a[1]}; }

template <typename T, int N, int B, int PRE, int S>
__global__ void __launch_bounds__((B * Radices<N, S>::TPR))
k_xfft_fwd(const cplx<T>* __restrict__ in_all, cplx<T>* __restrict__ out_all,
           const cplx<T>* __restrict__ tw, const RowGroup g, int ny, int nz, int j0, int nabs,
           const cplx<T>* __restrict__ kd_all, const PreOp<T> pre) {
  const int pb = blockIdx.x / g.bpp;
  if (g.skip && g.skip[(int64_t)pb * g.skip_stride]) return;
  constexpr int NT = B * Radices<N, S>::TPR;
  using Addr = AddrRowPad<N, lds_pad_period<T>()>;
  __shared__ cplx<T> s[B * Addr::PITCH];
  __shared__ cplx<T> tws[N];
  __shared__ int64_t rsrc[B];  // element offset of the source row (-1: past the end)
  __shared__ int64_t rkd[B];   // element offset of the conj(kd) row (-1: none)
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)(blockIdx.x % g.bpp) * B;
  const cplx<T>* in = in_all + pb * g.in_stride;
  cplx<T>* out = out_all + pb * g.out_stride;
  const cplx<T>* kd = kd_all + pb * g.kd_stride;
  for (int i = tid; i < N; i += NT) tws[i] = tw[i];
  if (tid < B) {
    const int64_t row = row0 + tid;
    int64_t src = -1, kro = -1;
    if (row < g.nmain) {
      src = row * N;
    } else if (row < g.ntot) {
      const int64_t r = row - g.nmain;
      const int plane = (int)(r / ny), yy = (int)(r % ny);
      const int c = plane / nabs, ja = plane % nabs;
      src = ((int64_t)(c * nz + j0 + ja) * ny + yy) * N;
      kro = ((int64_t)ja * ny + yy) * N;
    }
    rsrc[tid] = src;
    rkd[tid] = kro;
  }
  // scalars of the fused vector update (the input stack is the vector stack)
  cplx<T> c1 = {T(0), T(0)}, c2 = {T(0), T(0)};
  const int64_t vo = pb * g.in_stride;
  if constexpr (PRE == PRE_P) {
    const KState* ks = pre.ks + pb;
    const cplx<double> rho = ldks<T>(ks->rho), rho_p = ldks<T>(ks->rho_prev);
    const cplx<double> al = ldks<T>(ks->alpha), om = ldks<T>(ks->omega);
    c1 = cast<T>(cdiv(rho, rho_p) * cdiv(al, om));  // beta
    c2 = cast<T>(om);
  } else if constexpr (PRE == PRE_S) {
    c1 = cast<T>(ldks<T>((pre.ks + pb)->alpha));
  }
  auto value = [&](int64_t idx) -> cplx<T> {
    if constexpr (PRE == PRE_P) return pre.r[vo + idx] + c1 * (pre.pv[vo + idx] - c2 * pre.v[vo + idx]);
    else if constexpr (PRE == PRE_S) return pre.r[vo + idx] - c1 * pre.v[vo + idx];
    else return in[idx];
  };
  __syncthreads();
  // Thread t of row b loads the inputs of its first Stockham butterflies
  // (elements t + u TPR + q N / R0: consecutive threads, consecutive
  // elements), applies the fused update to them, and after the last pass
  // stores its outputs (t + u TPR + q N / RL) straight from registers.
  constexpr RadixPlan PL = Radices<N, S>::P;
  constexpr int TPR = Radices<N, S>::TPR;
  constexpr int EPT = Radices<N, S>::EPT;
  constexpr int R0 = PL.r[0], RL = PL.r[PL.np - 1];
  static_assert(lds_fft_items<N, B, NT, S>() == 1, "one item per thread");
  const int b = tid / TPR, t = tid % TPR;
  const int64_t src = rsrc[b], kro = rkd[b];
  cplx<T> v[1][EPT];
#pragma unroll
  for (int u = 0; u < EPT / R0; ++u)
#pragma unroll
    for (int q = 0; q < R0; ++q) {
      const int xi = t + u * TPR + q * (N / R0);
      cplx<T> val = {T(0), T(0)};
      if (src >= 0) val = kro < 0 ? value(src + xi) : cmulc(kd[kro + xi], value(src + xi));
      v[0][u * R0 + q] = val;
    }
  double acc[1] = {0.0};
  if constexpr (PRE != PRE_NONE) {
    if (src >= 0 && kro < 0) {
#pragma unroll
      for (int u = 0; u < EPT / R0; ++u)
#pragma unroll
        for (int q = 0; q < R0; ++q) {
          const int xi = t + u * TPR + q * (N / R0);
          pre.pv[vo + src + xi] = v[0][u * R0 + q];
          if constexpr (PRE == PRE_S) acc[0] += norm2(cast<double>(v[0][u * R0 + q]));
        }
    }
  }
  if constexpr (PRE == PRE_S) block_partials<1, NT>(acc, pre.part);
  lds_fft_regs<T, N, B, NT, false, false, S>(v, s, tws, Addr{}, tid);
  const int64_t row = row0 + b;
  if (row < g.ntot) {
#pragma unroll
    for (int u = 0; u < EPT / RL; ++u)
#pragma unroll
      for (int q = 0; q < RL; ++q) out[row * N + t + u * TPR + q * (N / RL)] = v[0][u * RL + q];
  }
}

template <typename T, int N, int B, int CM, int POST, int S>
__global__ void __launch_bounds__((B * Radices<N, S>::TPR))
k_xfft_inv(const cplx<T>* __restrict__ UW_all, cplx<T>* __restrict__ y_all,
           const cplx<T>* __restrict__ tw, const RowGroup g, int ny, int nz, int j0, int nabs,
           T scale, const cplx<T>* __restrict__ kd_all, const cplx<T>* __restrict__ x_all,
           const PostOp<T> post) {
  const int pb = blockIdx.x / g.bpp;
  if (g.skip && g.skip[(int64_t)pb * g.skip_stride]) return;
  constexpr int NT = B * Radices<N, S>::TPR;
  constexpr int NBUF = (CM == CB_FWD) ? 2 : 1;
  using Addr = AddrRowPad<N, lds_pad_period<T>()>;
  __shared__ cplx<T> s[NBUF * B * Addr::PITCH];
  __shared__ cplx<T> tws[N];
  __shared__ int64_t rw[B];   // element offset of the W row (-1: not an absorber row)
  __shared__ int64_t rkd[B];  // element offset of the kd row (-1: none)
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)(blockIdx.x % g.bpp) * B;
  const int64_t nrows = g.ntot;
  const cplx<T>* UW = UW_all + pb * g.in_stride;
  const int64_t fo = pb * g.out_stride;  // y, x and the dot partner share the field stack
  cplx<T>* y = y_all + fo;
  const cplx<T>* kd = kd_all + pb * g.kd_stride;
  for (int i = tid; i < N; i += NT) tws[i] = tw[i];
  if (tid < B) {
    const int64_t row = row0 + tid;
    int64_t wo = -1, ko = -1;
    if (row < nrows && CM != CB_PLAIN) {
      const int plane = (int)(row / ny), yy = (int)(row % ny);
      const int c = plane / nz, z = plane % nz;
      if (z >= j0 && z < j0 + nabs) {
        wo = ((int64_t)3 * nz * ny + (int64_t)(c * nabs + z - j0) * ny + yy) * N;
        ko = ((int64_t)(z - j0) * ny + yy) * N;
      }
    }
    rw[tid] = wo;
    rkd[tid] = ko;
  }
  __syncthreads();
  // Thread t of row b loads the inputs of its first Stockham butterflies of
  // the U row (and of the W row, the block's second batch of B rows: the
  // same thread runs both), requests the epilogue operands (kd, x for the
  // adjoint, the dot partner d) of the elements its last butterflies will
  // produce, and combines and stores those outputs from registers.
  constexpr RadixPlan PL = Radices<N, S>::P;
  constexpr int TPR = Radices<N, S>::TPR;
  constexpr int EPT = Radices<N, S>::EPT;
  constexpr int R0 = PL.r[0], RL = PL.r[PL.np - 1];
  static_assert(lds_fft_items<N, NBUF * B, NT, S>() == NBUF, "one item per row batch");
  const int b = tid / TPR, t = tid % TPR;
  const int64_t row = row0 + b;
  const bool live = row < nrows;
  const int64_t wo = rw[b], ko = rkd[b];
  const cplx<T> z0 = {T(0), T(0)};
  cplx<T> v[NBUF][EPT];
#pragma unroll
  for (int u = 0; u < EPT / R0; ++u)
#pragma unroll
    for (int q = 0; q < R0; ++q) {
      const int xi = t + u * TPR + q * (N / R0);
      v[0][u * R0 + q] = live ? UW[row * N + xi] : z0;
      if constexpr (CM == CB_FWD) v[NBUF - 1][u * R0 + q] = (live && wo >= 0) ? UW[wo + xi] : z0;
    }
  cplx<T> rkv[EPT], rxv[EPT], rdv[EPT];
#pragma unroll
  for (int u = 0; u < EPT / RL; ++u)
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      const int k = u * RL + q;
      const int xo = t + u * TPR + q * (N / RL);
      const int64_t idx = row * N + xo;
      rkv[k] = z0;
      rxv[k] = z0;
      rdv[k] = z0;
      if (live) {
        if (CM != CB_PLAIN && ko >= 0) {
          rkv[k] = kd[ko + xo];
          if (CM == CB_ADJ) rxv[k] = x_all[fo + idx];
        }
        if constexpr (POST == POST_DOT) rdv[k] = post.d[fo + idx];
      }
    }
  lds_fft_regs<T, N, NBUF * B, NT, true, false, S>(v, s, tws, Addr{}, tid);
  double acc[3] = {0.0, 0.0, 0.0};
  if (live) {
#pragma unroll
    for (int u = 0; u < EPT / RL; ++u)
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        const int k = u * RL + q;
        const int64_t idx = row * N + t + u * TPR + q * (N / RL);
        cplx<T> o = scale * v[0][k];
        if (CM != CB_PLAIN && ko >= 0) {
          if (CM == CB_FWD) o = o - scale * (rkv[k] * v[NBUF - 1][k]);
          else o = o - cmulc(rkv[k], rxv[k]);
        }
        y[idx] = o;
        if constexpr (POST == POST_DOT) {
          const cplx<double> a = cast<double>(rdv[k]), bb = cast<double>(o);
          acc[0] += a.re * bb.re + a.im * bb.im;
          acc[1] += a.re * bb.im - a.im * bb.re;
          acc[2] += bb.re * bb.re + bb.im * bb.im;
        }
      }
  }
  if constexpr (POST == POST_DOT) block_partials<3, NT>(acc, post.part);
}

// y pass: problem pb's planes start at pb * stride; grid.y = nprob * nplanes.
// The tile's columns go straight from the global loads into the first
// Stockham pass and from the last pass into the global stores (the loads of
// a thread are the inputs of its first butterflies, its stores the outputs
// of its last ones; consecutive threads take consecutive columns, so every
// access covers TX adjacent columns of one row).
template <typename T, int N, int TX, bool INV, int S>
__global__ void __launch_bounds__((TX * Radices<N, S>::TPR))
k_yfft(cplx<T>* __restrict__ buf, const cplx<T>* __restrict__ tw, int nx, int nplanes,
       int64_t stride, const int* __restrict__ skip, int skip_stride) {
  const int pb = blockIdx.y / nplanes;
  if (skip && skip[(int64_t)pb * skip_stride]) return;
  constexpr RadixPlan PL = Radices<N, S>::P;
  constexpr int TPR = Radices<N, S>::TPR;
  constexpr int EPT = Radices<N, S>::EPT;
  constexpr int NT = TX * TPR;
  constexpr int R0 = PL.r[0], RL = PL.r[PL.np - 1];
  static_assert(lds_fft_items<N, TX, NT, S>() == 1, "one item per thread");
  __shared__ cplx<T> s[N * TX];
  __shared__ cplx<T> tws[N];
  const int tid = threadIdx.x;
  const int64_t base = pb * stride + (int64_t)(blockIdx.y % nplanes) * N * nx +
                       (int64_t)blockIdx.x * TX;
  for (int i = tid; i < N; i += NT) tws[i] = tw[i];
  const int b = tid % TX, t = tid / TX;  // column of the tile, thread within the column
  cplx<T> v[1][EPT];
#pragma unroll
  for (int u = 0; u < EPT / R0; ++u)
#pragma unroll
    for (int q = 0; q < R0; ++q)
      v[0][u * R0 + q] = buf[base + (int64_t)(t + u * TPR + q * (N / R0)) * nx + b];
  lds_fft_regs<T, N, TX, NT, INV, true, S>(v, s, tws, AddrCol<TX>{}, tid);
#pragma unroll
  for (int u = 0; u < EPT / RL; ++u)
#pragma unroll
    for (int q = 0; q < RL; ++q)
      buf[base + (int64_t)(t + u * TPR + q * (N / RL)) * nx + b] = v[0][u * RL + q];
}

// ---------------------------------------------------------------- launchers

template <typename T>
static RowGroup group_of(const OpTables<T>& t, int64_t nmain, int64_t ntot, int64_t in_stride,
                         int64_t out_stride, int rows_per_block) {
  RowGroup g;
  g.nprob = t.nprob;
  g.bpp = (int)((ntot + rows_per_block - 1) / rows_per_block);
  g.nmain = nmain;
  g.ntot = ntot;
  g.in_stride = in_stride;
  g.out_stride = out_stride;
  g.kd_stride = (int64_t)t.nabs * t.nx * t.ny;
  g.skip = t.skip;
  g.skip_stride = t.skip_stride;
  return g;
}

template <typename T, int N, int S, int HALF>
static hipError_t xfwd_v(const OpTables<T>& t, const cplx<T>* in, cplx<T>* out, int64_t nmain,
                         int64_t ntot, int64_t in_stride, int64_t out_stride, const PreOp<T>& pre,
                         int* nblk_out, hipStream_t st) {
  constexpr int B = x_rows<T, N, HALF, S>();
  constexpr int NT = B * Radices<N, S>::TPR;
  static_assert(NT <= 1024, "block too large");
  const RowGroup g = group_of(t, nmain, ntot, in_stride, out_stride, B);
  if (nblk_out) *nblk_out = g.bpp;
  dim3 grid((unsigned)((int64_t)g.bpp * g.nprob)), b(NT);
  switch (pre.mode) {
    case PRE_P:
      PSFD_LAUNCH(t, (k_xfft_fwd<T, N, B, PRE_P, S>), grid, b, st, in, out, t.tw_x, g, t.ny,
                         t.nz, t.j0, t.nabs, t.kd, pre);
      break;
    case PRE_S:
      PSFD_LAUNCH(t, (k_xfft_fwd<T, N, B, PRE_S, S>), grid, b, st, in, out, t.tw_x, g, t.ny,
                         t.nz, t.j0, t.nabs, t.kd, pre);
      break;
    default:
      PSFD_LAUNCH(t, (k_xfft_fwd<T, N, B, PRE_NONE, S>), grid, b, st, in, out, t.tw_x, g,
                         t.ny, t.nz, t.j0, t.nabs, t.kd, pre);
      break;
  }
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t xfwd_n(const OpTables<T>& t, const cplx<T>* in, cplx<T>* out, int64_t nmain,
                         int64_t ntot, int64_t in_stride, int64_t out_stride, const PreOp<T>& pre,
                         int* nblk_out, hipStream_t st) {
  switch (t.sched_xf & 3) {
    case 1: return xfwd_v<T, N, 1, 0>(t, in, out, nmain, ntot, in_stride, out_stride, pre, nblk_out, st);
    case 2: return xfwd_v<T, N, 0, 1>(t, in, out, nmain, ntot, in_stride, out_stride, pre, nblk_out, st);
    case 3: return xfwd_v<T, N, 1, 1>(t, in, out, nmain, ntot, in_stride, out_stride, pre, nblk_out, st);
    default: return xfwd_v<T, N, 0, 0>(t, in, out, nmain, ntot, in_stride, out_stride, pre, nblk_out, st);
  }
}

template <typename T, int N, int CM, int S, int HALF>
static void xinv_launch(const OpTables<T>& t, const cplx<T>* UW, cplx<T>* y, int64_t nrows,
                        int64_t in_stride, int64_t out_stride, const cplx<T>* x, T scale,
                        const PostOp<T>& post, int* nblk_out, hipStream_t st) {
  constexpr int B = xinv_rows<T, N, CM, S, HALF>();
  constexpr int NT = B * Radices<N, S>::TPR;
  static_assert(NT <= 1024, "block too large");
  const RowGroup g = group_of(t, nrows, nrows, in_stride, out_stride, B);
  if (nblk_out) *nblk_out = g.bpp;
  dim3 grid((unsigned)((int64_t)g.bpp * g.nprob)), b(NT);
  if (post.mode == POST_DOT)
    PSFD_LAUNCH(t, (k_xfft_inv<T, N, B, CM, POST_DOT, S>), grid, b, st, UW, y, t.tw_x, g,
                       t.ny, t.nz, t.j0, t.nabs, scale, t.kd, x, post);
  else
    PSFD_LAUNCH(t, (k_xfft_inv<T, N, B, CM, POST_NONE, S>), grid, b, st, UW, y, t.tw_x, g,
                       t.ny, t.nz, t.j0, t.nabs, scale, t.kd, x, post);
}

template <typename T, int N, int S, int HALF>
static void xinv_v(const OpTables<T>& t, const cplx<T>* UW, cplx<T>* y, int64_t nrows,
                   int64_t in_stride, int64_t out_stride, int cmode, const cplx<T>* x, T scale,
                   const PostOp<T>& post, int* nblk_out, hipStream_t st) {
  switch (cmode) {
    case CB_PLAIN: xinv_launch<T, N, CB_PLAIN, S, HALF>(t, UW, y, nrows, in_stride, out_stride, x, scale, post, nblk_out, st); break;
    case CB_FWD: xinv_launch<T, N, CB_FWD, S, HALF>(t, UW, y, nrows, in_stride, out_stride, x, scale, post, nblk_out, st); break;
    default: xinv_launch<T, N, CB_ADJ, S, HALF>(t, UW, y, nrows, in_stride, out_stride, x, scale, post, nblk_out, st); break;
  }
}

template <typename T, int N>
static hipError_t xinv_n(const OpTables<T>& t, const cplx<T>* UW, cplx<T>* y, int64_t nrows,
                         int64_t in_stride, int64_t out_stride, int cmode, const cplx<T>* x,
                         T scale, const PostOp<T>& post, int* nblk_out, hipStream_t st) {
  switch (t.sched_xi & 3) {
    case 1: xinv_v<T, N, 1, 0>(t, UW, y, nrows, in_stride, out_stride, cmode, x, scale, post, nblk_out, st); break;
    case 2: xinv_v<T, N, 0, 1>(t, UW, y, nrows, in_stride, out_stride, cmode, x, scale, post, nblk_out, st); break;
    case 3: xinv_v<T, N, 1, 1>(t, UW, y, nrows, in_stride, out_stride, cmode, x, scale, post, nblk_out, st); break;
    default: xinv_v<T, N, 0, 0>(t, UW, y, nrows, in_stride, out_stride, cmode, x, scale, post, nblk_out, st); break;
  }
  return hipGetLastError();
}

template <typename T, int N, int S, int HALF>
static hipError_t y_v(const OpTables<T>& t, cplx<T>* buf, int nplanes, int64_t stride, bool inv,
                      hipStream_t st) {
  constexpr int TX = y_tile<T, N, S, HALF>();
  constexpr int NT = TX * Radices<N, S>::TPR;
  static_assert(NT <= 1024, "block too large");
  if (t.nx % TX) return hipErrorInvalidValue;
  dim3 g(t.nx / TX, (unsigned)(nplanes * t.nprob));
  if (inv)
    PSFD_LAUNCH(t, (k_yfft<T, N, TX, true, S>), g, dim3(NT), st, buf, t.tw_y, t.nx, nplanes,
                       stride, t.skip, t.skip_stride);
  else
    PSFD_LAUNCH(t, (k_yfft<T, N, TX, false, S>), g, dim3(NT), st, buf, t.tw_y, t.nx, nplanes,
                       stride, t.skip, t.skip_stride);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t y_n(const OpTables<T>& t, cplx<T>* buf, int nplanes, int64_t stride, bool inv,
                      hipStream_t st) {
  switch (t.sched_y & 3) {
    case 1: return y_v<T, N, 1, 0>(t, buf, nplanes, stride, inv, st);
    case 2: return y_v<T, N, 0, 1>(t, buf, nplanes, stride, inv, st);
    case 3: return y_v<T, N, 1, 1>(t, buf, nplanes, stride, inv, st);
    default: return y_v<T, N, 0, 0>(t, buf, nplanes, stride, inv, st);
  }
}

#define PSFD_LATERAL_SWITCH(N, CALL)              \
  switch (N) {                                    \
    case 16: return CALL(16);                     \
    case 32: return CALL(32);                     \
    case 64: return CALL(64);                     \
    case 128: return CALL(128);                   \
    case 192: return CALL(192);                   \
    case 256: return CALL(256);                   \
    case 512: return CALL(512);                   \
    case 1024: return CALL(1024);                 \
    default: return hipErrorInvalidValue;         \
  }

template <typename T>
hipError_t launch_xfft_fwd(const OpTables<T>& t, const cplx<T>* in, cplx<T>* out, bool adj_extra,
                           const PreOp<T>& pre, int* nblk, hipStream_t st) {
  const int64_t nmain = (int64_t)3 * t.nz * t.ny;
  const int64_t ntot = nmain + (adj_extra ? (int64_t)3 * t.nabs * t.ny : 0);
#define CALL_X(NN) xfwd_n<T, NN>(t, in, out, nmain, ntot, t.pfield, t.pspec, pre, nblk, st)
  PSFD_LATERAL_SWITCH(t.nx, CALL_X)
#undef CALL_X
}

template <typename T>
hipError_t launch_yfft(const OpTables<T>& t, cplx<T>* buf, int nplanes, bool inverse,
                       hipStream_t st) {
#define CALL_Y(NN) y_n<T, NN>(t, buf, nplanes, t.pspec, inverse, st)
  PSFD_LATERAL_SWITCH(t.ny, CALL_Y)
#undef CALL_Y
}

template <typename T>
hipError_t launch_xfft_inv(const OpTables<T>& t, const cplx<T>* UW, cplx<T>* y, int cmode,
                           const cplx<T>* x, const PostOp<T>& post, int* nblk, hipStream_t st) {
  const int64_t nrows = (int64_t)3 * t.nz * t.ny;
  const T scale = T(1) / (T(t.nx) * T(t.ny));
#define CALL_XI(NN) xinv_n<T, NN>(t, UW, y, nrows, t.pspec, t.pfield, cmode, x, scale, post, nblk, st)
  PSFD_LATERAL_SWITCH(t.nx, CALL_XI)
#undef CALL_XI
}

template <typename T>
hipError_t launch_xfft_inv_rows(const OpTables<T>& t, const cplx<T>* in, cplx<T>* out,
                                int64_t nrows, hipStream_t st) {
  const T scale = T(1) / (T(t.nx) * T(t.ny));
  OpTables<T> one = t;  // a single problem, no skip
  one.nprob = 1;
  one.skip = nullptr;
#define CALL_XR(NN) xinv_n<T, NN>(one, in, out, nrows, 0, 0, CB_PLAIN, nullptr, scale, PostOp<T>{}, nullptr, st)
  PSFD_LATERAL_SWITCH(t.nx, CALL_XR)
#undef CALL_XR
}

template <typename T>
hipError_t launch_plane_fft(const OpTables<T>& t, cplx<T>* in, cplx<T>* out, bool inverse,
                            hipStream_t st) {
  hipError_t e;
  OpTables<T> one = t;  // a single plane of a single problem
  one.nprob = 1;
  one.skip = nullptr;
  if (!inverse) {
#define CALL_PX(NN) xfwd_n<T, NN>(one, in, out, t.ny, t.ny, 0, 0, PreOp<T>{}, nullptr, st)
    e = [&]() -> hipError_t { PSFD_LATERAL_SWITCH(t.nx, CALL_PX) }();
#undef CALL_PX
    if (e != hipSuccess) return e;
    return [&]() -> hipError_t {
#define CALL_PY(NN) y_n<T, NN>(one, out, 1, 0, false, st)
      PSFD_LATERAL_SWITCH(t.ny, CALL_PY)
#undef CALL_PY
    }();
  }
  // inverse: y pass in place on `in`, then x pass into `out` (unnormalised)
  e = [&]() -> hipError_t {
#define CALL_PYI(NN) y_n<T, NN>(one, in, 1, 0, true, st)
    PSFD_LATERAL_SWITCH(t.ny, CALL_PYI)
#undef CALL_PYI
  }();
  if (e != hipSuccess) return e;
#define CALL_PXI(NN) xinv_n<T, NN>(one, in, out, t.ny, 0, 0, CB_PLAIN, nullptr, T(1), PostOp<T>{}, nullptr, st)
  PSFD_LATERAL_SWITCH(t.nx, CALL_PXI)
#undef CALL_PXI
}

template hipError_t launch_xfft_fwd<double>(const OpTables<double>&, const cplx<double>*,
                                            cplx<double>*, bool, const PreOp<double>&, int*,
                                            hipStream_t);
template hipError_t launch_xfft_fwd<float>(const OpTables<float>&, const cplx<float>*,
                                           cplx<float>*, bool, const PreOp<float>&, int*,
                                           hipStream_t);
template hipError_t launch_yfft<double>(const OpTables<double>&, cplx<double>*, int, bool,
                                        hipStream_t);
template hipError_t launch_yfft<float>(const OpTables<float>&, cplx<float>*, int, bool,
                                       hipStream_t);
template hipError_t launch_xfft_inv<double>(const OpTables<double>&, const cplx<double>*,
                                            cplx<double>*, int, const cplx<double>*,
                                            const PostOp<double>&, int*, hipStream_t);
template hipError_t launch_xfft_inv<float>(const OpTables<float>&, const cplx<float>*,
                                           cplx<float>*, int, const cplx<float>*,
                                           const PostOp<float>&, int*, hipStream_t);
template hipError_t launch_xfft_inv_rows<double>(const OpTables<double>&, const cplx<double>*,
                                                 cplx<double>*, int64_t, hipStream_t);
template hipError_t launch_plane_fft<double>(const OpTables<double>&, cplx<double>*,
                                             cplx<double>*, bool, hipStream_t);

}  // namespace psfd
