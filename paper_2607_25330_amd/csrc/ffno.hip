// Inference of the factorised Fourier neural operator of the paper's PINO
// (section 2.1): lifting, L layers of [lateral truncated spectral conv on
// every z slice -> axial truncated spectral conv -> pointwise MLP with a
// residual connection], decoding to the three complex field components.
//
// Hidden state: d_v real channels, FP32, channel planes [d_v][nz][ny][nx].
// The retained spectra are small (kx = 0..kx_max of the real-input half
// spectrum, |ky| <= ky_max, kz = 0..kz_max), so the transforms are direct
// truncated DFT sums (one FP32 table value e^{2 pi i j / n} per sample, built
// on the device in FP64, its powers by repeated multiplication):
// any grid size works and no full-size spectrum is ever stored.
//   x DFT:  T[c][z][y][kx]  = sum_x v e^{-2 pi i kx x / nx}   (one row per thread)
//   y DFT:  G[c][z][m][kx]  = sum_y T e^{-2 pi i ky y / ny},   ky = m - ky_max
//   mix:    U[o][z][m][kx]  = sum_i K_xy[o][i][m][kx] G[i][z][m][kx]
//   y iDFT: T2[o][z][y][kx] = sum_m U e^{+2 pi i ky y / ny}
//   x iDFT: u[o][z][y][x]   = (Re T2[..][0] + 2 sum_{kx>0} Re(T2 e^{+2 pi i kx x/nx})) / (nx ny)
// The axial branch runs as three coalesced passes over the columns (forward
// z DFT, channel mixing per kz, inverse z DFT added in place to u_xy); the
// MLP and the residual update then run one voxel per thread with the
// weights as scalar operands (W2 is transposed once per call into the
// workspace so that both products read contiguous rows).
#include <hip/hip_runtime.h>

#include "psfd_internal.h"

namespace psfd {

namespace {

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

__global__ void k_ffno_twiddles(float2* tw, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincospi(2.0 * (double)i / (double)n, &s, &c);
  tw[i] = make_float2((float)c, (float)s);  // e^{+2 pi i i / n}
}

__global__ void k_ffno_lift(const FfnoArgs a, const float* __restrict__ P, const float* __restrict__ p,
                            const float* __restrict__ in, float* __restrict__ v) {
  const int64_t vox = (int64_t)a.nz * a.ny * a.nx;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < vox;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(q % a.nx);
    const int y = (int)((q / a.nx) % a.ny);
    const int z = (int)(q / ((int64_t)a.nx * a.ny));
    const float f0 = in[q], f1 = (float)x / a.nx, f2 = (float)y / a.ny, f3 = (float)z / a.nz;
    for (int c = 0; c < a.dv; ++c)
      v[(int64_t)c * vox + q] = P[4 * c] * f0 + P[4 * c + 1] * f1 + P[4 * c + 2] * f2 +
                                P[4 * c + 3] * f3 + p[c];
  }
}

__device__ __forceinline__ float2 cmul2(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// T[row][kx] = sum_x v[row][x] w^(-kx x), w = e^{2 pi i / nx}, rows of v
// (row = (c, z, y)).  kXL lanes share a row (a wave takes 64 / kXL rows and
// reads each of them front to back) and lane l sums the samples
// x = l + kXL j.  The power splits as w^(kx x) = w^(kx l) w^(kx kXL j): the
// second factor is the same for the whole wave and comes from a table
// (qx[j][kx], exact twiddles) read as scalar loads (whole table rows), so a
// sample costs two multiply-adds per kx,
//   S_l[kx] = sum_j v(l + kXL j) conj(qx[j][kx]);
// each lane then applies its own conj(w^(kx l)) once per row and the kXL
// lanes are summed by butterflies.  The loads of kXB samples per lane are
// issued together.  The inner loop carries no bounds tests: the table is
// padded to whole batches, samples past the row end are loaded in bounds and
// multiplied by zero, and all MXM modes are summed (the ones at or above mx
// are not stored).
constexpr int kXL = 16;
constexpr int kXB = 4;

__host__ __device__ constexpr int xdft_table_rows(int nx) {
  return ((nx + kXL - 1) / kXL + kXB - 1) / kXB * kXB;
}

__global__ void k_ffno_xpowers(const float2* __restrict__ twx, int nx, int mxm,
                               float2* __restrict__ qx) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= xdft_table_rows(nx) * mxm) return;
  const int j = e / mxm, kx = e % mxm;
  qx[e] = twx[(int)(((int64_t)kx * kXL * j) % nx)];
}

template <int MXM>
__global__ void __launch_bounds__(256) k_ffno_xdft(const FfnoArgs a, const float* __restrict__ v,
                                                   const float2* __restrict__ twx,
                                                   const float2* __restrict__ qx,
                                                   float2* __restrict__ T, int64_t nrows) {
  constexpr int RPB = 256 / kXL;  // rows per block and step
  const int nx = a.nx, mx = a.mx;
  const int l = threadIdx.x % kXL;
  const int nj = (nx + kXL - 1) / kXL;
  float2 pl[MXM];  // w^(kx l), the same for every row this thread takes
#pragma unroll
  for (int k = 0; k < MXM; ++k) pl[k] = k < mx ? twx[(k * l) % nx] : make_float2(1.f, 0.f);
  for (int64_t base = (int64_t)blockIdx.x * RPB; base < nrows; base += (int64_t)gridDim.x * RPB) {
    const int64_t row = base + threadIdx.x / kXL;
    const bool live = row < nrows;
    const float* src = v + (live ? row : 0) * nx;
    float sr[MXM], si[MXM];
#pragma unroll
    for (int k = 0; k < MXM; ++k) sr[k] = si[k] = 0.f;
    for (int j0 = 0; j0 < nj; j0 += kXB) {
      float val[kXB];
#pragma unroll
      for (int u = 0; u < kXB; ++u) {  // in-bounds load times a 0/1 mask: no branch
        const int x = l + kXL * (j0 + u);
        val[u] = src[min(x, nx - 1)] * ((live && x < nx) ? 1.f : 0.f);
      }
      // the table row is the same for the whole wave: scalar loads
      const int jq = __builtin_amdgcn_readfirstlane(j0);
#pragma unroll
      for (int u = 0; u < kXB; ++u) {
        const float2* q = qx + (jq + u) * MXM;
#pragma unroll
        for (int k = 0; k < MXM; ++k) {
          const float2 w = q[k];
          sr[k] += val[u] * w.x;  // the forward sum takes the conjugate power
          si[k] -= val[u] * w.y;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < MXM; ++k) {
      if (k < mx) {
        // conj(w^(kx l)) S_l, then the sum over the kXL lanes of the row
        float re = pl[k].x * sr[k] + pl[k].y * si[k];
        float im = pl[k].x * si[k] - pl[k].y * sr[k];
#pragma unroll
        for (int off = 1; off < kXL; off <<= 1) {
          re += __shfl_xor(re, off, kXL);
          im += __shfl_xor(im, off, kXL);
        }
        if (live && (k % kXL) == l) T[row * mx + k] = make_float2(re, im);
      }
    }
  }
}

// The same sum with vector loads, for rows whose length is a multiple of 4
// (16-byte aligned rows): lane l of a row reads the 4 samples
// x = 64 j + 4 l + c, c = 0..3, in one load, and the power splits as
// w^(kx x) = w^(4 kx l) w^(kx (64 j + c)); the second factor comes from the
// table q4[4 j + c][kx] (scalar loads), the first is applied once per row.
constexpr int kXB4 = 2;  // vector loads per lane issued together

__host__ __device__ constexpr int xdft4_table_rows(int nx) {
  return 4 * (((nx + 4 * kXL - 1) / (4 * kXL) + kXB4 - 1) / kXB4 * kXB4);
}

__global__ void k_ffno_xpowers4(const float2* __restrict__ twx, int nx, int mxm,
                                float2* __restrict__ q4) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= xdft4_table_rows(nx) * mxm) return;
  const int m = e / mxm, kx = e % mxm;
  const int64_t x = 4 * (int64_t)kXL * (m / 4) + m % 4;
  q4[e] = twx[(int)(((int64_t)kx * x) % nx)];
}

template <int MXM>
__global__ void __launch_bounds__(256) k_ffno_xdft4(const FfnoArgs a, const float* __restrict__ v,
                                                    const float2* __restrict__ twx,
                                                    const float2* __restrict__ q4,
                                                    float2* __restrict__ T, int64_t nrows) {
  constexpr int RPB = 256 / kXL;
  const int nx = a.nx, mx = a.mx;
  const int l = threadIdx.x % kXL;
  const int nj = (nx + 4 * kXL - 1) / (4 * kXL);
  float2 pl[MXM];  // w^(4 kx l)
#pragma unroll
  for (int k = 0; k < MXM; ++k) pl[k] = k < mx ? twx[(4 * k * l) % nx] : make_float2(1.f, 0.f);
  for (int64_t base = (int64_t)blockIdx.x * RPB; base < nrows; base += (int64_t)gridDim.x * RPB) {
    const int64_t row = base + threadIdx.x / kXL;
    const bool live = row < nrows;
    const float* src = v + (live ? row : 0) * nx;
    float sr[MXM], si[MXM];
#pragma unroll
    for (int k = 0; k < MXM; ++k) sr[k] = si[k] = 0.f;
    for (int j0 = 0; j0 < nj; j0 += kXB4) {
      float4 val[kXB4];
#pragma unroll
      for (int u = 0; u < kXB4; ++u) {  // in-bounds load times a 0/1 mask: no branch
        const int x0 = 4 * l + 4 * kXL * (j0 + u);
        const float4 t = *reinterpret_cast<const float4*>(src + min(x0, nx - 4));
        const float m = (live && x0 < nx) ? 1.f : 0.f;
        val[u] = make_float4(t.x * m, t.y * m, t.z * m, t.w * m);
      }
      const int jq = __builtin_amdgcn_readfirstlane(j0);  // wave-uniform: scalar table loads
#pragma unroll
      for (int u = 0; u < kXB4; ++u) {
        const float vc[4] = {val[u].x, val[u].y, val[u].z, val[u].w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float2* q = q4 + (4 * (jq + u) + c) * MXM;
#pragma unroll
          for (int k = 0; k < MXM; ++k) {
            const float2 w = q[k];
            sr[k] += vc[c] * w.x;  // the forward sum takes the conjugate power
            si[k] -= vc[c] * w.y;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < MXM; ++k) {
      if (k < mx) {
        float re = pl[k].x * sr[k] + pl[k].y * si[k];
        float im = pl[k].x * si[k] - pl[k].y * sr[k];
#pragma unroll
        for (int off = 1; off < kXL; off <<= 1) {
          re += __shfl_xor(re, off, kXL);
          im += __shfl_xor(im, off, kXL);
        }
        if (live && (k % kXL) == l) T[row * mx + k] = make_float2(re, im);
      }
    }
  }
}

template <int MXM>
void xdft_launch(const FfnoArgs& a, const FfnoPtrs& w, int64_t nrows, hipStream_t st) {
  const dim3 g((unsigned)std::min<int64_t>((nrows + 15) / 16, 16384));
  if (a.nx % 4 == 0)
    hipLaunchKernelGGL((k_ffno_xdft4<MXM>), g, dim3(256), 0, st, a, w.v, w.twx, w.q4, w.T, nrows);
  else
    hipLaunchKernelGGL((k_ffno_xdft<MXM>), g, dim3(256), 0, st, a, w.v, w.twx, w.qx, w.T, nrows);
}

// G[c][z][m][kx] = sum_y T[c][z][y][kx] e^{-2 pi i ky y / ny}
__global__ void k_ffno_ydft(const FfnoArgs a, const float2* __restrict__ T,
                            const float2* __restrict__ twy, float2* __restrict__ G) {
  const int mx = a.mx, my = a.my, ny = a.ny;
  const int64_t items = (int64_t)a.dv * a.nz * my * mx;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < items;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int kx = (int)(q % mx);
    const int m = (int)((q / mx) % my);
    const int64_t cz = q / ((int64_t)mx * my);
    const int ky = m - a.ky_max;
    const int step = ((ky % ny) + ny) % ny;
    const float2* t = T + cz * ny * mx + kx;
    float re = 0.f, im = 0.f;
    int ph = 0;
    for (int y = 0; y < ny; ++y) {
      const float2 w = twy[ph];  // e^{+i theta}; the forward sum takes its conjugate
      const float2 s = t[(int64_t)y * mx];
      re += s.x * w.x + s.y * w.y;
      im += s.y * w.x - s.x * w.y;
      ph += step;
      if (ph >= ny) ph -= ny;
    }
    G[q] = make_float2(re, im);
  }
}

// U[o][z][m][kx] = sum_i K[o][i][m][kx] G[i][z][m][kx]
__global__ void k_ffno_mix_xy(const FfnoArgs a, const float2* __restrict__ K,
                              const float2* __restrict__ G, float2* __restrict__ U) {
  const int modes = a.my * a.mx;
  const int64_t per_c = (int64_t)a.nz * modes;
  const int64_t items = (int64_t)a.dv * per_c;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < items;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int md = (int)(q % modes);
    const int64_t zq = (q / modes) % a.nz;
    const int o = (int)(q / per_c);
    float re = 0.f, im = 0.f;
    for (int i = 0; i < a.dv; ++i) {
      const float2 k = K[((int64_t)o * a.dv + i) * modes + md];
      const float2 g = G[(int64_t)i * per_c + zq * modes + md];
      re += k.x * g.x - k.y * g.y;
      im += k.x * g.y + k.y * g.x;
    }
    U[q] = make_float2(re, im);
  }
}

// T2[o][z][y][kx] = sum_m U[o][z][m][kx] e^{+2 pi i ky y / ny}
__global__ void k_ffno_yidft(const FfnoArgs a, const float2* __restrict__ U,
                             const float2* __restrict__ twy, float2* __restrict__ T2) {
  const int mx = a.mx, my = a.my, ny = a.ny;
  const int64_t items = (int64_t)a.dv * a.nz * ny * mx;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < items;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int kx = (int)(q % mx);
    const int y = (int)((q / mx) % ny);
    const int64_t cz = q / ((int64_t)mx * ny);
    const float2* u = U + cz * my * mx + kx;
    float re = 0.f, im = 0.f;
    // table index of ky y mod ny for ky = -ky_max, then stepped by y per mode
    int ph = (int)((((int64_t)(-a.ky_max) * y) % ny + ny) % ny);
    for (int m = 0; m < my; ++m) {
      const float2 w = twy[ph];
      ph += y;
      if (ph >= ny) ph -= ny;
      const float2 s = u[(int64_t)m * mx];
      re += s.x * w.x - s.y * w.y;
      im += s.x * w.y + s.y * w.x;
    }
    T2[q] = make_float2(re, im);
  }
}

// u[o][z][y][x] = (Re T2[..][0] + 2 sum_{kx>0} Re(T2[..][kx] e^{+2 pi i kx x / nx})) / (nx ny)
// With the split of the x DFT (kXL lanes per row, lane l writes x = l + kXL j,
// w^(kx x) = w^(kx l) w^(kx kXL j)), each lane forms R_l[kx] = T2[kx] w^(kx l)
// (doubled for kx > 0) once per row; an output sample then costs two
// multiply-adds per kx with the wave-uniform table value qx[j][kx] (scalar
// loads, the table of the forward pass):
//   u(l + kXL j) = (Re R_l[0] + sum_{kx>0} Re(R_l[kx] qx[j][kx])) / (nx ny).
// Modes at and above mx have R = 0; the stores are masked at the row end.
template <int MXM>
__global__ void __launch_bounds__(256) k_ffno_xidft(const FfnoArgs a, const float2* __restrict__ T2,
                                                    const float2* __restrict__ twx,
                                                    const float2* __restrict__ qx,
                                                    float* __restrict__ u, int64_t nrows) {
  constexpr int RPB = 256 / kXL;  // rows per block and step
  const int nx = a.nx, mx = a.mx;
  const int l = threadIdx.x % kXL;
  const int nj = (nx + kXL - 1) / kXL;
  const float norm = 1.0f / ((float)nx * (float)a.ny);
  float2 pl[MXM];  // w^(kx l)
#pragma unroll
  for (int k = 0; k < MXM; ++k) pl[k] = k < mx ? twx[(k * l) % nx] : make_float2(0.f, 0.f);
  for (int64_t base = (int64_t)blockIdx.x * RPB; base < nrows; base += (int64_t)gridDim.x * RPB) {
    const int64_t row = base + threadIdx.x / kXL;
    const bool live = row < nrows;
    const float2* t = T2 + (live ? row : 0) * mx;
    float rr[MXM], ri[MXM];
#pragma unroll
    for (int k = 0; k < MXM; ++k) {
      const float2 tv = k < mx ? t[k] : make_float2(0.f, 0.f);
      const float f = k == 0 ? 1.f : 2.f;
      rr[k] = f * (tv.x * pl[k].x - tv.y * pl[k].y);
      ri[k] = f * (tv.x * pl[k].y + tv.y * pl[k].x);
    }
    float* dst = u + (live ? row : 0) * nx;
    for (int j0 = 0; j0 < nj; j0 += kXB) {
      const int jq = __builtin_amdgcn_readfirstlane(j0);  // wave-uniform: scalar table loads
#pragma unroll
      for (int uu = 0; uu < kXB; ++uu) {
        const float2* q = qx + (jq + uu) * MXM;
        float acc = rr[0];  // qx[j][0] = 1
#pragma unroll
        for (int k = 1; k < MXM; ++k) {
          const float2 w = q[k];
          acc += rr[k] * w.x - ri[k] * w.y;
        }
        const int x = l + kXL * (j0 + uu);
        if (live && x < nx) dst[x] = acc * norm;
      }
    }
  }
}

// The inverse x DFT with 16-byte stores for rows whose length is a multiple
// of 4: lane l writes x = 64 j + 4 l + c, c = 0..3, from R_l[kx] =
// T2[kx] w^(4 kx l) (doubled for kx > 0) and the table q4[4 j + c][kx] of
// the forward pass.
template <int MXM>
__global__ void __launch_bounds__(256) k_ffno_xidft4(const FfnoArgs a, const float2* __restrict__ T2,
                                                     const float2* __restrict__ twx,
                                                     const float2* __restrict__ q4,
                                                     float* __restrict__ u, int64_t nrows) {
  constexpr int RPB = 256 / kXL;
  const int nx = a.nx, mx = a.mx;
  const int l = threadIdx.x % kXL;
  const int nj = (nx + 4 * kXL - 1) / (4 * kXL);
  const float norm = 1.0f / ((float)nx * (float)a.ny);
  float2 pl[MXM];  // w^(4 kx l)
#pragma unroll
  for (int k = 0; k < MXM; ++k) pl[k] = k < mx ? twx[(4 * k * l) % nx] : make_float2(0.f, 0.f);
  for (int64_t base = (int64_t)blockIdx.x * RPB; base < nrows; base += (int64_t)gridDim.x * RPB) {
    const int64_t row = base + threadIdx.x / kXL;
    const bool live = row < nrows;
    const float2* t = T2 + (live ? row : 0) * mx;
    float rr[MXM], ri[MXM];
#pragma unroll
    for (int k = 0; k < MXM; ++k) {
      const float2 tv = k < mx ? t[k] : make_float2(0.f, 0.f);
      const float f = k == 0 ? 1.f : 2.f;
      rr[k] = f * (tv.x * pl[k].x - tv.y * pl[k].y);
      ri[k] = f * (tv.x * pl[k].y + tv.y * pl[k].x);
    }
    float* dst = u + (live ? row : 0) * nx;
    for (int j = 0; j < nj; ++j) {
      const int jq = __builtin_amdgcn_readfirstlane(j);  // wave-uniform: scalar table loads
      float out[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float2* q = q4 + (4 * jq + c) * MXM;
        float acc = rr[0] * q[0].x - ri[0] * q[0].y;
#pragma unroll
        for (int k = 1; k < MXM; ++k) {
          const float2 w = q[k];
          acc += rr[k] * w.x - ri[k] * w.y;
        }
        out[c] = acc * norm;
      }
      const int x0 = 4 * l + 4 * kXL * j;
      if (live && x0 < nx)
        *reinterpret_cast<float4*>(dst + x0) = make_float4(out[0], out[1], out[2], out[3]);
    }
  }
}

// Axial branch in three coalesced passes over the columns (col = y nx + x,
// consecutive threads on consecutive columns):
//   forward:  W[c][kz][col] = sum_z u[c][z][col] w^(-kz z)
//   mixing:   Z[o][kz][col] = sum_i K_z[o][i][kz] W[i][kz][col]   (one thread per column,
//             kz = blockIdx.y, the d_v inputs in registers)
//   inverse:  u[o][z][col] += (Re Z[o][0] + 2 sum_{kz>0} Re(Z[o][kz] w^(kz z))) / nz
// so that u holds s = u_xy + u_z afterwards.  The powers w^(kz z) depend on
// z only: they are tabulated once per forward pass (PZ[z][kz], repeated
// multiplication of the table value w^z) and, z being the same for every
// thread of a pass step, read as scalar loads, as are the mixing weights
// (a kz-major copy KzT[kz][o][i] of K_z).  The column loads of four z rows
// are issued together.
constexpr int kZPow = 16;  // row stride of the power table (kz_max <= 15)

constexpr int kZB = 4;  // z rows per batch of column loads
__host__ __device__ constexpr int zdft_table_rows(int nz) { return (nz + kZB - 1) / kZB * kZB; }

// pz[z][kz] = w^(kz z) for kz < mz (the last power repeated above), rows up to
// a whole batch (rows past nz hold finite values that meet zero samples)
__global__ void k_ffno_zpowers(const float2* __restrict__ twz, int nz, int mz,
                               float2* __restrict__ pz) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= zdft_table_rows(nz)) return;
  const float2 w1 = z < nz ? twz[z] : make_float2(1.f, 0.f);
  float2 p = make_float2(1.f, 0.f);
  for (int kz = 0; kz < kZPow; ++kz) {
    pz[z * kZPow + kz] = p;
    if (kz + 1 < mz) p = cmul2(p, w1);
  }
}

// KzT[kz][o][i] = Kz[o][i][kz] (one layer)
__global__ void k_ffno_kz_major(const float2* __restrict__ Kz, int dv, int mz,
                                float2* __restrict__ KzT) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dv * dv * mz) return;
  KzT[(int64_t)(e % mz) * dv * dv + e / mz] = Kz[e];
}

__global__ void __launch_bounds__(256)
k_ffno_zdft(const FfnoArgs a, const float* __restrict__ u, const float2* __restrict__ pz,
            float2* __restrict__ W) {
  const int64_t plane = (int64_t)a.ny * a.nx;
  const int64_t items = (int64_t)a.dv * plane;
  const int nz = a.nz, mz = a.mz;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < items;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = q / plane, col = q % plane;
    const float* src = u + c * plane * nz + col;
    float2 acc[kZPow];
#pragma unroll
    for (int kz = 0; kz < kZPow; ++kz) acc[kz] = make_float2(0.f, 0.f);
    for (int z0 = 0; z0 < nz; z0 += kZB) {
      float val[kZB];
#pragma unroll
      for (int j = 0; j < kZB; ++j) val[j] = (z0 + j < nz) ? src[(int64_t)(z0 + j) * plane] : 0.f;
#pragma unroll
      for (int j = 0; j < kZB; ++j) {
        const float2* pw = pz + (z0 + j) * kZPow;
#pragma unroll
        for (int kz = 0; kz < kZPow; ++kz) {  // every row entry: no bounds tests in the loop
          const float2 p = pw[kz];
          acc[kz].x += val[j] * p.x;
          acc[kz].y -= val[j] * p.y;
        }
      }
    }
    float2* dst = W + c * mz * plane + col;
#pragma unroll
    for (int kz = 0; kz < kZPow; ++kz)
      if (kz < mz) dst[(int64_t)kz * plane] = acc[kz];
  }
}

template <int DV>
__global__ void __launch_bounds__(256)
k_ffno_zmix(const FfnoArgs a, const float2* __restrict__ KzT, const float2* __restrict__ W,
            float2* __restrict__ Z) {
  const int64_t plane = (int64_t)a.ny * a.nx;
  const int mz = a.mz;
  const int kz = blockIdx.y;
  const float2* K = KzT + (int64_t)kz * DV * DV;
  for (int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; col < plane;
       col += (int64_t)gridDim.x * blockDim.x) {
    float2 w[DV];
#pragma unroll
    for (int i = 0; i < DV; ++i) w[i] = W[((int64_t)i * mz + kz) * plane + col];
#pragma unroll 1
    for (int o = 0; o < DV; ++o) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int i = 0; i < DV; ++i) {
        const float2 k = K[o * DV + i];
        re += k.x * w[i].x - k.y * w[i].y;
        im += k.x * w[i].y + k.y * w[i].x;
      }
      Z[((int64_t)o * mz + kz) * plane + col] = make_float2(re, im);
    }
  }
}

__global__ void __launch_bounds__(256)
k_ffno_zidft(const FfnoArgs a, const float2* __restrict__ Z, const float2* __restrict__ pz,
             float* __restrict__ u) {
  const int64_t plane = (int64_t)a.ny * a.nx;
  const int64_t items = (int64_t)a.dv * plane;
  const int nz = a.nz, mz = a.mz;
  const float inz = 1.0f / nz;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < items;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = q / plane, col = q % plane;
    const float2* zs = Z + o * mz * plane + col;
    float2 zk[kZPow];
#pragma unroll
    for (int kz = 0; kz < kZPow; ++kz) zk[kz] = kz < mz ? zs[(int64_t)kz * plane] : make_float2(0.f, 0.f);
    float* dst = u + o * plane * nz + col;
    for (int z0 = 0; z0 < nz; z0 += kZB) {
      float old[kZB];
#pragma unroll
      for (int j = 0; j < kZB; ++j) old[j] = (z0 + j < nz) ? dst[(int64_t)(z0 + j) * plane] : 0.f;
#pragma unroll
      for (int j = 0; j < kZB; ++j) {
        const float2* pw = pz + (z0 + j) * kZPow;
        float acc = zk[0].x;
#pragma unroll
        for (int kz = 1; kz < kZPow; ++kz) {  // zk is zero at and above mz
          const float2 p = pw[kz];
          acc += 2.0f * (zk[kz].x * p.x - zk[kz].y * p.y);
        }
        if (z0 + j < nz) dst[(int64_t)(z0 + j) * plane] = old[j] + acc * inz;
      }
    }
  }
}

// Pointwise MLP with residual: v <- v + act(W2 gelu(W1 s + b1) + b2), one
// voxel per thread (channel planes, coalesced); the weights are the same for
// every thread, so they come as scalar loads and enter the multiply-adds as
// scalar operands (no LDS traffic; staging them in LDS and reading them as
// broadcasts took 26.4 against 21.5 ms per layer at 1200x1200x100).  W2 is
// used transposed ([d_h][d_v]) so that both products walk contiguous rows
// while only s, o and one hidden unit are live.
template <int DV, int DH>
__global__ void __launch_bounds__(256)
k_ffno_mlp(const FfnoArgs a, const float* __restrict__ s_in, float* __restrict__ v,
           const float* __restrict__ W1, const float* __restrict__ b1,
           const float* __restrict__ W2T, const float* __restrict__ b2, int last) {
  // every index into the weights is the same for the whole wave: scalar loads
  const float* w1s = W1;
  const float* w2s = W2T;
  const float* b1s = b1;
  const float* b2s = b2;
  const int64_t vox = (int64_t)a.nz * a.ny * a.nx;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < vox;
       q += (int64_t)gridDim.x * blockDim.x) {
    float s[DV], o[DV];
#pragma unroll
    for (int i = 0; i < DV; ++i) {
      s[i] = s_in[(int64_t)i * vox + q];
      o[i] = b2s[i];
    }
#pragma unroll 1
    for (int j = 0; j < DH; ++j) {
      float acc = b1s[j];
#pragma unroll
      for (int i = 0; i < DV; ++i) acc += w1s[j * DV + i] * s[i];
      const float h = gelu(acc);
#pragma unroll
      for (int i = 0; i < DV; ++i) o[i] += w2s[j * DV + i] * h;
    }
#pragma unroll
    for (int i = 0; i < DV; ++i) v[(int64_t)i * vox + q] += last ? o[i] : gelu(o[i]);
  }
}

// out[j][i] = in[i][j] for an [rows][cols] matrix
__global__ void k_ffno_transpose(const float* __restrict__ in, int rows, int cols,
                                 float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int i = e / cols, j = e % cols;
  out[j * rows + i] = in[e];
}

__global__ void k_ffno_decode(const FfnoArgs a, const float* __restrict__ Q,
                              const float* __restrict__ qb, const float* __restrict__ v,
                              cplx<double>* __restrict__ E) {
  const int64_t vox = (int64_t)a.nz * a.ny * a.nx;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < vox;
       q += (int64_t)gridDim.x * blockDim.x) {
    float acc[6];
    for (int k = 0; k < 6; ++k) acc[k] = qb[k];
    for (int c = 0; c < a.dv; ++c) {
      const float val = v[(int64_t)c * vox + q];
      for (int k = 0; k < 6; ++k) acc[k] += Q[k * a.dv + c] * val;
    }
    for (int k = 0; k < 3; ++k) E[(int64_t)k * vox + q] = {(double)acc[2 * k], (double)acc[2 * k + 1]};
  }
}

unsigned grid_for(int64_t items) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, 8192));
}

template <int DV, int DH>
hipError_t axial_mlp_launch(const FfnoArgs& a, const FfnoPtrs& w, int layer, int last, hipStream_t st) {
  const int64_t plane = (int64_t)a.ny * a.nx;
  const int64_t vox = plane * a.nz;
  hipLaunchKernelGGL(k_ffno_zdft, dim3(grid_for((int64_t)DV * plane)), dim3(256), 0, st, a, w.u,
                     w.pz, w.W);
  hipLaunchKernelGGL((k_ffno_zmix<DV>), dim3(grid_for(plane), (unsigned)a.mz), dim3(256), 0, st, a,
                     w.KzT + (size_t)layer * a.mz * DV * DV, w.W, w.Z);
  hipLaunchKernelGGL(k_ffno_zidft, dim3(grid_for((int64_t)DV * plane)), dim3(256), 0, st, a, w.Z,
                     w.pz, w.u);
  hipLaunchKernelGGL((k_ffno_mlp<DV, DH>), dim3(grid_for(vox)), dim3(256), 0, st, a, w.u, w.v,
                     w.W1[layer], w.b1[layer], w.W2T + (size_t)layer * DV * DH, w.b2[layer], last);
  return hipGetLastError();
}

}  // namespace

hipError_t ffno_forward(const FfnoArgs& a, const FfnoPtrs& w, const float* in, cplx<double>* E,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_ffno_twiddles, dim3((a.nx + 255) / 256), dim3(256), 0, st, w.twx, a.nx);
  hipLaunchKernelGGL(k_ffno_twiddles, dim3((a.ny + 255) / 256), dim3(256), 0, st, w.twy, a.ny);
  hipLaunchKernelGGL(k_ffno_twiddles, dim3((a.nz + 255) / 256), dim3(256), 0, st, w.twz, a.nz);
  {
    const int mxm = a.mx <= 16 ? 16 : 32, nj = xdft_table_rows(a.nx);
    hipLaunchKernelGGL(k_ffno_xpowers, dim3((nj * mxm + 255) / 256), dim3(256), 0, st, w.twx, a.nx,
                       mxm, w.qx);
    if (a.nx % 4 == 0) {
      const int n4 = xdft4_table_rows(a.nx);
      hipLaunchKernelGGL(k_ffno_xpowers4, dim3((n4 * mxm + 255) / 256), dim3(256), 0, st, w.twx,
                         a.nx, mxm, w.q4);
    }
  }
  hipLaunchKernelGGL(k_ffno_zpowers, dim3((zdft_table_rows(a.nz) + 255) / 256), dim3(256), 0, st,
                     w.twz, a.nz, a.mz, w.pz);
  for (int l = 0; l < a.nl; ++l) {
    hipLaunchKernelGGL(k_ffno_transpose, dim3((a.dv * a.dh + 255) / 256), dim3(256), 0, st,
                       w.W2[l], a.dv, a.dh, w.W2T + (size_t)l * a.dv * a.dh);
    hipLaunchKernelGGL(k_ffno_kz_major, dim3((a.dv * a.dv * a.mz + 255) / 256), dim3(256), 0, st,
                       w.Kz[l], a.dv, a.mz, w.KzT + (size_t)l * a.mz * a.dv * a.dv);
  }
  const int64_t vox = (int64_t)a.nz * a.ny * a.nx;
  hipLaunchKernelGGL(k_ffno_lift, dim3(grid_for(vox)), dim3(256), 0, st, a, w.P, w.p, in, w.v);
  const int64_t nrows = (int64_t)a.dv * a.nz * a.ny;
  for (int l = 0; l < a.nl; ++l) {
    if (a.mx <= 16) xdft_launch<16>(a, w, nrows, st);
    else xdft_launch<32>(a, w, nrows, st);
    hipLaunchKernelGGL(k_ffno_ydft, dim3(grid_for((int64_t)a.dv * a.nz * a.my * a.mx)), dim3(256),
                       0, st, a, w.T, w.twy, w.G);
    hipLaunchKernelGGL(k_ffno_mix_xy, dim3(grid_for((int64_t)a.dv * a.nz * a.my * a.mx)),
                       dim3(256), 0, st, a, w.Kxy[l], w.G, w.U);
    hipLaunchKernelGGL(k_ffno_yidft, dim3(grid_for((int64_t)a.dv * a.nz * a.ny * a.mx)), dim3(256),
                       0, st, a, w.U, w.twy, w.T);
    const dim3 gi((unsigned)std::min<int64_t>((nrows + 15) / 16, 16384));
    if (a.nx % 4 == 0) {
      if (a.mx <= 16)
        hipLaunchKernelGGL(k_ffno_xidft4<16>, gi, dim3(256), 0, st, a, w.T, w.twx, w.q4, w.u, nrows);
      else
        hipLaunchKernelGGL(k_ffno_xidft4<32>, gi, dim3(256), 0, st, a, w.T, w.twx, w.q4, w.u, nrows);
    } else if (a.mx <= 16) {
      hipLaunchKernelGGL(k_ffno_xidft<16>, gi, dim3(256), 0, st, a, w.T, w.twx, w.qx, w.u, nrows);
    } else {
      hipLaunchKernelGGL(k_ffno_xidft<32>, gi, dim3(256), 0, st, a, w.T, w.twx, w.qx, w.u, nrows);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int last = l == a.nl - 1;
    if (a.dv == 32 && a.dh == 64) e = axial_mlp_launch<32, 64>(a, w, l, last, st);
    else if (a.dv == 16 && a.dh == 32) e = axial_mlp_launch<16, 32>(a, w, l, last, st);
    else if (a.dv == 8 && a.dh == 16) e = axial_mlp_launch<8, 16>(a, w, l, last, st);
    else e = hipErrorInvalidValue;
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ffno_decode, dim3(grid_for(vox)), dim3(256), 0, st, a, w.Q, w.q, w.v, E);
  return hipGetLastError();
}

}  // namespace psfd
