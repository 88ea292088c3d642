// Axial column kernel: everything the operator does along z for one lateral
// Fourier mode (kx, ky), fused in one pass over the lateral spectrum.
//
// Input S holds the lateral Fourier coefficients X(kx, ky, z) of the three
// components.  With D = diag(1/s) G, G = F_z^-1 diag(i kz) F_z (PML-stretched
// pseudo-spectral d/dz), curl curl per mode is
//   Ux = ky^2 Px - kx ky Py + D(-D Px + i kx Pz)
//   Uy = -kx ky Px + kx^2 Py + D(-D Py + i ky Pz)
//   Uz = i kx D Px + i ky D Py + kt^2 Pz
// (the operator matrix of the paper's vector Helmholtz equation written as
// curl of curl, four G applications per column), minus kbg^2 P.  P = X for
// the plain operator and P = M X for the fused operator-times-preconditioner
// (F_z, multiply by the damping m(k), and the D of P shares that forward
// transform).  The multilayer branch takes P at the evaluation row (taken as
// downgoing there) and splits it into TE and TM amplitudes: TE = s . P_t, TM
// = the least-squares fit of the downgoing TM polarisation (1, kt/kz) to
// (t . P_t, P_z), i.e. w_t (t . P_t) + w_z P_z with w_t = 1 / (1 + |kt/kz|^2),
// w_z = conj(kt/kz) w_t; it multiplies them by r_TE / r_pE and propagates
// them up to the absorber rows:
//   W = P + E_ML on absorber rows,  so that  y = F2^-1[U] - k0^2 d_eps F2^-1[W].
// The adjoint replaces D by -D^H = G diag(1/conj(s)) and the multilayer
// branch by its adjoint applied to F2[conj(k0^2 d_eps) x] (extra input planes),
// which lands on the evaluation row.
#include <type_traits>

#include "fft_core.h"
#include "lane_fft.h"
#include "psfd_internal.h"

namespace psfd {

bool axial_size_ok(int n) {
  switch (n) {
    case 24: case 32: case 48: case 64: case 96: case 128:
    case 192: case 256: case 324: case 384: case 576: case 648: case 768: return true;
    default: return false;
  }
}

template <typename T>
struct ColInfo {
  T kx, ky, kt2, sx, sy, tx, ty;
  T kzr, kzi;          // background axial wavenumber kzr + i kzi (one of them is 0)
  cplx<T> ktkz, down;  // kt / kz,  exp(-i kz dz / 2)
  T wt;                // TM amplitude weights: a_p = wt (t . P_t) + wz P_z
  cplx<T> wz;
  cplx<T> rte, rpe;
  cplx<T> a0, a1, a2;  // forward: upgoing (TE, TM) amplitudes; adjoint: evaluation-row terms (x, y, z)
  int live;
};

__device__ __forceinline__ float round_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}
__device__ __forceinline__ double round_bf16(double x) { return (double)round_bf16((float)x); }
template <typename T>
__device__ __forceinline__ cplx<T> round_bf16(cplx<T> v) { return {round_bf16(v.re), round_bf16(v.im)}; }
// A complex value whose parts are bfloat16 numbers, packed into 32 bits and back.
__device__ __forceinline__ uint32_t pack_bf16(cplx<float> v) {
  return (__float_as_uint(v.re) >> 16) | (__float_as_uint(v.im) & 0xFFFF0000u);
}
__device__ __forceinline__ cplx<float> unpack_bf16(uint32_t u) {
  return {__uint_as_float(u << 16), __uint_as_float(u & 0xFFFF0000u)};
}

template <typename T>
__device__ __forceinline__ T damping(T k2, const OpTables<T>& t) {
  T core = T(1);
  if (k2 > t.pc_kref2) {
    const T q = t.pc_kref2 / (k2 + t.pc_reg);
    core = (t.pc_gamma == T(1)) ? q : pow(q, t.pc_gamma);
  }
  return t.pc_mmin + (T(1) - t.pc_mmin) * core;
}

// Multiplier of the M mode: the damping m(k), or for the physics loss's
// high-frequency penalty the squared weight w(nu)^2 = (w0 + eta |k| / 2 pi)^2.
template <typename T>
__device__ __forceinline__ T spec_mult(T k2, const OpTables<T>& t) {
  if (t.hf_mode) {
    const T wgt = t.hf_w0 + t.hf_eta * sqrt(k2) * T(0.15915494309189533577);
    return wgt * wgt;
  }
  return damping(k2, t);
}

// exp(i kz z) for kz = kzr + i kzi
template <typename T>
__device__ __forceinline__ cplx<T> up_phase(const ColInfo<T>& c, T z) {
  T s, co;
  sc(c.kzr * z, &s, &co);
  const T m = exp(-c.kzi * z);
  return {m * co, m * s};
}

template <typename T>
__device__ void column_info(ColInfo<T>& c, const OpTables<T>& t, int pb, int ix, int iy) {
  c.kx = t.kx[(int64_t)pb * t.nx + ix];
  c.ky = t.ky[(int64_t)pb * t.ny + iy];
  c.kt2 = c.kx * c.kx + c.ky * c.ky;
  const T kt = sqrt(c.kt2);
  if (kt == T(0)) {
    const T cp = t.cphi[pb], sp = t.sphi[pb];
    c.sx = -sp; c.sy = cp; c.tx = cp; c.ty = sp;
  } else {
    c.sx = -c.ky / kt; c.sy = c.kx / kt; c.tx = c.kx / kt; c.ty = c.ky / kt;
  }
  const T q2 = t.kbg2 - c.kt2;
  if (q2 >= T(0)) { c.kzr = sqrt(q2); c.kzi = T(0); }
  else { c.kzr = T(0); c.kzi = sqrt(-q2); }
  const T kzabs = c.kzr + c.kzi;
  c.live = kzabs >= t.kz_live;
  if (!c.live) c.ktkz = {T(0), T(0)};
  else if (c.kzi == T(0)) c.ktkz = {kt / c.kzr, T(0)};
  else c.ktkz = {T(0), -kt / c.kzi};
  c.wt = T(1) / (T(1) + c.ktkz.re * c.ktkz.re + c.ktkz.im * c.ktkz.im);
  c.wz = {c.wt * c.ktkz.re, -c.wt * c.ktkz.im};
  const T h = T(0.5) * t.dz;
  T s, co;
  sc(c.kzr * h, &s, &co);
  const T m = exp(c.kzi * h);
  c.down = {m * co, -m * s};
  const int64_t mode = ((int64_t)pb * t.ny + iy) * t.nx + ix;
  c.rte = t.r_te[mode];
  c.rpe = t.r_pe[mode];
}

// Columns up to 128 rows keep the z tables (twiddles, 1/s, kz) in LDS next
// to the column tile; taller columns (the full-domain grids that discretise
// a whole multilayer) read them through the caches so that one or two
// columns of five vectors still fit the 64 KiB a block may declare.
template <int NZ>
constexpr bool ax_tables_in_lds() { return NZ <= 128; }

template <typename T, int NZ>
constexpr int ax_tile() {
  int tx = sizeof(T) == 8 ? 8 : 16;
  while (tx > 1 && 5 * NZ * tx * (int)sizeof(cplx<T>) > 65536) tx /= 2;
  return tx;
}

template <typename T, int NZ, int TX, int MODE>
__global__ void __launch_bounds__(256)
k_axial(const cplx<T>* __restrict__ S_all, cplx<T>* __restrict__ UW_all, const OpTables<T> t) {
  const int pb = blockIdx.y / t.ny;
  if (skipped(t, pb)) return;
  const cplx<T>* S = S_all + pb * t.pspec;
  cplx<T>* UW = UW_all + pb * t.pspec;
  constexpr int NT = 256;
  constexpr int PITCH = TX;
  constexpr int VS = NZ * PITCH;
  constexpr int NV = (MODE == AX_M) ? 3 : 5;
  using Addr = AddrVec<TX, PITCH, VS>;
  constexpr bool TL = ax_tables_in_lds<NZ>();
  constexpr int NTAB = TL ? NZ : 1;
  __shared__ cplx<T> buf[NV * VS];
  __shared__ ColInfo<T> ci[TX];
  __shared__ cplx<T> twz_s[NTAB];
  __shared__ cplx<T> invs_s[NTAB];
  __shared__ T kzs_s[NTAB];
  const cplx<T>* twz = TL ? twz_s : t.tw_z;
  const cplx<T>* invs = TL ? invs_s : t.inv_s;
  const T* kzs = TL ? kzs_s : t.kz;

  const int tid = threadIdx.x;
  const int iy = blockIdx.y % t.ny;
  // Workgroups go to the 8 XCDs round-robin by linear id; with gridDim.x a
  // multiple of 8 the tiles of one XCD are made neighbours along x, so that
  // the narrow column tiles of neighbouring blocks share that XCD's L2 lines.
  const int bx = (gridDim.x % 8 == 0) ? (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8
                                      : blockIdx.x;
  const int kx0 = bx * TX;
  const int64_t plane = (int64_t)t.nx * t.ny;
  const int64_t colbase = (int64_t)iy * t.nx + kx0;
  const T inz = T(1) / T(NZ);
  // pointwise stages: each thread keeps one column and walks z
  constexpr int ZS = NT / TX;
  const int cc = tid % TX, z0 = tid / TX;

  for (int e = tid; e < 3 * NZ * TX; e += NT) {
    const int c = e / (NZ * TX), rem = e % (NZ * TX);
    const int z = rem / TX, cc = rem % TX;
    buf[c * VS + z * PITCH + cc] = S[(int64_t)(c * NZ + z) * plane + colbase + cc];
  }
  if (tid < TX) column_info(ci[tid], t, pb, kx0 + tid, iy);
  if constexpr (TL) {
    for (int i = tid; i < NZ; i += NT) {
      twz_s[i] = t.tw_z[i];
      invs_s[i] = t.inv_s[i];
      kzs_s[i] = t.kz[i];
    }
  }
  __syncthreads();

  if constexpr (MODE == AX_AM || MODE == AX_M) {
    lds_fft<T, NZ, 3 * TX, NT, false, true>(buf, twz, Addr{}, tid);
    const T kt2 = ci[cc].kt2;
    for (int l = z0; l < NZ; l += ZS) {
      const T kzl = kzs[l];
      const T m = (MODE == AX_M ? spec_mult(kt2 + kzl * kzl, t) : damping(kt2 + kzl * kzl, t)) * inz;
      cplx<T>* b0 = &buf[l * PITCH + cc];
      cplx<T> p0 = m * b0[0], p1 = m * b0[VS], p2 = m * b0[2 * VS];
      if (sizeof(T) == 4 && t.pc_bf16 && !t.hf_mode) {  // bf16 trial: M's spectrum in bfloat16
        p0 = round_bf16(p0);
        p1 = round_bf16(p1);
        p2 = round_bf16(p2);
      }
      b0[0] = p0;
      b0[VS] = p1;
      b0[2 * VS] = p2;
      if constexpr (MODE == AX_AM) {
        b0[3 * VS] = kzl * mul_i(p0);
        b0[4 * VS] = kzl * mul_i(p1);
      }
    }
    __syncthreads();
    lds_fft<T, NZ, (MODE == AX_AM ? 5 : 3) * TX, NT, true, true>(buf, twz, Addr{}, tid);
    if constexpr (MODE == AX_M) {
      for (int e = tid; e < 3 * NZ * TX; e += NT) {
        const int c = e / (NZ * TX), rem = e % (NZ * TX);
        const int z = rem / TX, cc = rem % TX;
        UW[(int64_t)(c * NZ + z) * plane + colbase + cc] = buf[c * VS + z * PITCH + cc];
      }
      return;
    }
  } else {
    for (int z = z0; z < NZ; z += ZS) {
      cplx<T> a = buf[z * PITCH + cc], b = buf[VS + z * PITCH + cc];
      if constexpr (MODE == AX_AH) {
        const cplx<T> is = invs[z];
        a = cmulc(is, a);
        b = cmulc(is, b);
      }
      buf[3 * VS + z * PITCH + cc] = a;
      buf[4 * VS + z * PITCH + cc] = b;
    }
    __syncthreads();
    lds_fft<T, NZ, 2 * TX, NT, false, true>(buf + 3 * VS, twz, Addr{}, tid);
    for (int l = z0; l < NZ; l += ZS) {
      const T f = kzs[l] * inz;
      buf[3 * VS + l * PITCH + cc] = f * mul_i(buf[3 * VS + l * PITCH + cc]);
      buf[4 * VS + l * PITCH + cc] = f * mul_i(buf[4 * VS + l * PITCH + cc]);
    }
    __syncthreads();
    lds_fft<T, NZ, 2 * TX, NT, true, true>(buf + 3 * VS, twz, Addr{}, tid);
  }

  // Multilayer branch amplitudes (one thread per column).
  if (tid < TX) {
    ColInfo<T>& c = ci[tid];
    if constexpr (MODE != AX_AH) {
      const cplx<T> px = buf[t.jev * PITCH + tid], py = buf[VS + t.jev * PITCH + tid];
      const cplx<T> pz = buf[2 * VS + t.jev * PITCH + tid];
      const cplx<T> as = (c.sx * px + c.sy * py) * c.down;
      const cplx<T> ap = (c.wt * (c.tx * px + c.ty * py) + c.wz * pz) * c.down;
      c.a0 = c.live ? c.rte * as : cplx<T>{T(0), T(0)};
      c.a1 = c.live ? c.rpe * ap : cplx<T>{T(0), T(0)};
    } else {
      cplx<T> cs = {T(0), T(0)}, cp = {T(0), T(0)};
      for (int ja = 0; ja < t.nabs; ++ja) {
        const cplx<T> qx = S[(int64_t)(3 * NZ + ja) * plane + colbase + tid];
        const cplx<T> qy = S[(int64_t)(3 * NZ + t.nabs + ja) * plane + colbase + tid];
        const cplx<T> qz = S[(int64_t)(3 * NZ + 2 * t.nabs + ja) * plane + colbase + tid];
        const cplx<T> ph = conj(up_phase(c, t.zabs[ja]));
        cs = cs + ph * (c.sx * qx + c.sy * qy);
        cp = cp + ph * (c.tx * qx + c.ty * qy - cmulc(c.ktkz, qz));
      }
      cs = c.live ? cmulc(c.rte, cs) : cplx<T>{T(0), T(0)};
      cp = c.live ? cmulc(c.rpe, cp) : cplx<T>{T(0), T(0)};
      c.a0 = cmulc(c.down, c.sx * cs + (c.tx * c.wt) * cp);
      c.a1 = cmulc(c.down, c.sy * cs + (c.ty * c.wt) * cp);
      c.a2 = cmulc(c.down, cmulc(c.wz, cp));
    }
  }

  // Uz and the inner curl vectors w = -D P_t + i k_t P_z.
  const T ckx = ci[cc].kx, cky = ci[cc].ky, ckt2 = ci[cc].kt2;
  cplx<T> uz_ev = {T(0), T(0)};  // adjoint: U_z of the evaluation row, completed below
  for (int z = z0; z < NZ; z += ZS) {
    const int o = z * PITCH + cc;
    cplx<T> dpx = buf[3 * VS + o], dpy = buf[4 * VS + o];
    if constexpr (MODE != AX_AH) {
      const cplx<T> is = invs[z];
      dpx = dpx * is;
      dpy = dpy * is;
    }
    const cplx<T> pz = buf[2 * VS + o];
    const cplx<T> uz = ckx * mul_i(dpx) + cky * mul_i(dpy) + (ckt2 - t.kbg2) * pz;
    UW[(int64_t)(2 * NZ + z) * plane + colbase + cc] = uz;
    if (z == t.jev) uz_ev = uz;
    cplx<T> wx = ckx * mul_i(pz) - dpx;
    cplx<T> wy = cky * mul_i(pz) - dpy;
    if constexpr (MODE == AX_AH) {
      const cplx<T> is = invs[z];
      wx = cmulc(is, wx);
      wy = cmulc(is, wy);
    }
    buf[3 * VS + o] = wx;
    buf[4 * VS + o] = wy;
  }
  __syncthreads();
  lds_fft<T, NZ, 2 * TX, NT, false, true>(buf + 3 * VS, twz, Addr{}, tid);
  for (int l = z0; l < NZ; l += ZS) {
    const T f = kzs[l] * inz;
    buf[3 * VS + l * PITCH + cc] = f * mul_i(buf[3 * VS + l * PITCH + cc]);
    buf[4 * VS + l * PITCH + cc] = f * mul_i(buf[4 * VS + l * PITCH + cc]);
  }
  __syncthreads();
  lds_fft<T, NZ, 2 * TX, NT, true, true>(buf + 3 * VS, twz, Addr{}, tid);

  const cplx<T> ca0 = ci[cc].a0, ca1 = ci[cc].a1, ca2 = ci[cc].a2;
  for (int z = z0; z < NZ; z += ZS) {
    const int o = z * PITCH + cc;
    cplx<T> dwx = buf[3 * VS + o], dwy = buf[4 * VS + o];
    if constexpr (MODE != AX_AH) {
      const cplx<T> is = invs[z];
      dwx = dwx * is;
      dwy = dwy * is;
    }
    const cplx<T> px = buf[o], py = buf[VS + o];
    cplx<T> ux = (cky * cky - t.kbg2) * px - (ckx * cky) * py + dwx;
    cplx<T> uy = (ckx * ckx - t.kbg2) * py - (ckx * cky) * px + dwy;
    if constexpr (MODE == AX_AH) {
      if (z == t.jev) {
        ux = ux - ca0;
        uy = uy - ca1;
        // the same thread wrote U_z of this row in the first pass
        UW[(int64_t)(2 * NZ + z) * plane + colbase + cc] = uz_ev - ca2;
      }
    }
    UW[(int64_t)z * plane + colbase + cc] = ux;
    UW[(int64_t)(NZ + z) * plane + colbase + cc] = uy;
  }

  if constexpr (MODE != AX_AH) {
    const ColInfo<T> c = ci[cc];
    for (int ja = z0; ja < t.nabs; ja += ZS) {
      const int z = t.j0 + ja;
      const cplx<T> ph = up_phase(c, t.zabs[ja]);
      const cplx<T> vs = c.a0 * ph, vp = c.a1 * ph;
      const cplx<T> vx = c.sx * vs + c.tx * vp;
      const cplx<T> vy = c.sy * vs + c.ty * vp;
      const cplx<T> vz = -(c.ktkz * vp);
      const int o = z * PITCH + cc;
      const int64_t wb = (int64_t)3 * NZ;
      UW[(wb + ja) * plane + colbase + cc] = buf[o] + vx;
      UW[(wb + t.nabs + ja) * plane + colbase + cc] = buf[VS + o] + vy;
      UW[(wb + 2 * t.nabs + ja) * plane + colbase + cc] = buf[2 * VS + o] + vz;
    }
  }
}


// ------------------------------------------------------------------------
// Register-resident variant for the forward modes (A, AM, M): L lanes own a
// column (lane t keeps z = t + L m), every z transform is a LaneFft, so the
// column never goes through LDS; the only barrier follows the staging of the
// z tables in LDS.  Same
// arithmetic as k_axial above, in the order that keeps at most five column
// vectors live: P^ (k layout) -> D P -> P_z -> U_z and w -> D w -> P_x, P_y
// -> U_x, U_y and the absorber-row W planes.
// Element (row r, column g) of a plane stack lives at r * plane + g; with
// r = r0 + lt (lt the lane within the column's group) the offset splits into
// a wave-uniform part r0 * plane and a per-lane byte offset
// (lt * plane + g) * sizeof, below 4 GiB for every supported size: each
// access is a scalar base plus one 32-bit lane offset.
// BF (complex64, A.M and M modes): the bf16 preconditioner trial; the damped
// spectrum P^ = m X^ is rounded to bfloat16 right after the damping and its
// x, y components are parked in LDS as packed bfloat16 pairs.
template <typename T, int NZ, int L, int MODE, bool BF = false>
__global__ void __launch_bounds__(256)
k_axial_reg(const cplx<T>* __restrict__ S_all, cplx<T>* __restrict__ UW_all, const OpTables<T> t) {
  constexpr int E = NZ / L;
  const int64_t plane = (int64_t)t.nx * t.ny;
  const int lt = threadIdx.x & (L - 1);
  const int64_t gg = (int64_t)blockIdx.x * (256 / L) + (threadIdx.x / L);
  // a block's 256 / L columns lie in one problem (plane is a multiple of 256)
  const int pb = (int)(gg / plane);
  if (skipped(t, pb)) return;
  const int64_t g = gg - pb * plane;
  const cplx<T>* S = S_all + pb * t.pspec;
  cplx<T>* UW = UW_all + pb * t.pspec;
  const int64_t pbytes = plane * (int64_t)sizeof(cplx<T>);
  const uint32_t lane_bo = (uint32_t)((lt * plane + g) * (int64_t)sizeof(cplx<T>));
  auto ld = [&](int64_t row) -> cplx<T> {  // row of lane 0 of the group
    return *reinterpret_cast<const cplx<T>*>(reinterpret_cast<const char*>(S) + row * pbytes + lane_bo);
  };
  auto stv = [&](int64_t row, cplx<T> v) {
    *reinterpret_cast<cplx<T>*>(reinterpret_cast<char*>(UW) + row * pbytes + lane_bo) = v;
  };
  const T inz = T(1) / T(NZ);
  // the z tables (twiddles, kz, 1/s) in LDS: every lane reads them at its own
  // index many times, and LDS reads keep those lookups off the vector memory
  // path that carries the column data
  __shared__ cplx<T> twz_s[NZ], invs_s[NZ];
  __shared__ T kz_s[NZ];
  for (int i = threadIdx.x; i < NZ; i += 256) {
    twz_s[i] = t.tw_z[i];
    invs_s[i] = t.inv_s[i];
    kz_s[i] = t.kz[i];
  }
  __syncthreads();
  LaneFft<T, NZ, L> F;
  F.init(twz_s, lt);
  const int kofs = E * lane_brev<L>(lt);  // k of register k2 is k2 + kofs

  cplx<T> px[E], py[E], pz[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    px[m] = ld(L * m);
    py[m] = ld(NZ + L * m);
    pz[m] = ld(2 * NZ + L * m);
  }
  const int ix = (int)(g % t.nx), iy = (int)(g / t.nx);
  const T kx = t.kx[(int64_t)pb * t.nx + ix], ky = t.ky[(int64_t)pb * t.ny + iy];
  const T kt2 = kx * kx + ky * ky;

  if constexpr (MODE == AX_M) {
    F.fwd(px);
    F.fwd(py);
    F.fwd(pz);
#pragma unroll
    for (int k2 = 0; k2 < E; ++k2) {
      const T kzl = kz_s[k2 + kofs];
      const T m = spec_mult(kt2 + kzl * kzl, t) * inz;
      px[k2] = m * px[k2];
      py[k2] = m * py[k2];
      pz[k2] = m * pz[k2];
      if constexpr (BF) {
        px[k2] = round_bf16(px[k2]);
        py[k2] = round_bf16(py[k2]);
        pz[k2] = round_bf16(pz[k2]);
      }
    }
    F.inv(px);
    F.inv(py);
    F.inv(pz);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      stv(L * m, px[m]);
      stv(NZ + L * m, py[m]);
      stv(2 * NZ + L * m, pz[m]);
    }
    return;
  } else {
    // Column data parked in LDS: each lane stores and reloads only its own
    // slots ([slot][register][lane], conflict-free), so no barrier is needed.
    using Park = typename std::conditional<BF, uint32_t, cplx<T>>::type;
    __shared__ Park park[2 * E * 256];
    auto park_st = [&](int slot, const cplx<T>(&v)[E]) {
#pragma unroll
      for (int k = 0; k < E; ++k) {
        if constexpr (BF) park[(slot * E + k) * 256 + threadIdx.x] = pack_bf16(v[k]);
        else park[(slot * E + k) * 256 + threadIdx.x] = v[k];
      }
    };
    auto park_ld = [&](int slot, cplx<T>(&v)[E]) {
#pragma unroll
      for (int k = 0; k < E; ++k) {
        if constexpr (BF) v[k] = unpack_bf16(park[(slot * E + k) * 256 + threadIdx.x]);
        else v[k] = park[(slot * E + k) * 256 + threadIdx.x];
      }
    };
    // P at the evaluation row (the multilayer branch reads it there)
    cplx<T> ex = {T(0), T(0)}, ey = {T(0), T(0)}, ez = {T(0), T(0)};
    cplx<T> dx[E], dy[E];
    if constexpr (MODE == AX_AM) {
      F.fwd(px);
      F.fwd(py);
      F.fwd(pz);
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) {
        const T kzl = kz_s[k2 + kofs];
        const T m = damping(kt2 + kzl * kzl, t) * inz;
        px[k2] = m * px[k2];
        py[k2] = m * py[k2];
        pz[k2] = m * pz[k2];
        if constexpr (BF) {
          px[k2] = round_bf16(px[k2]);
          py[k2] = round_bf16(py[k2]);
          pz[k2] = round_bf16(pz[k2]);
        }
      }
      // P(jev) = sum_k P^[k] exp(+2 pi i k jev / NZ): this lane's terms, then the group sum
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) {
        const cplx<T> w = conj(twz_s[((k2 + kofs) * t.jev) % NZ]);
        ex = ex + px[k2] * w;
        ey = ey + py[k2] * w;
        ez = ez + pz[k2] * w;
      }
      ex = lane_group_sum<L>(ex);
      ey = lane_group_sum<L>(ey);
      ez = lane_group_sum<L>(ez);
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) dx[k2] = kz_s[k2 + kofs] * mul_i(px[k2]);
      park_st(0, px);
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) dy[k2] = kz_s[k2 + kofs] * mul_i(py[k2]);
      park_st(1, py);
      F.inv(pz);
    } else {
      const int mj = t.jev / L, tj = t.jev % L;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        if (m == mj) {
          ex = px[m];
          ey = py[m];
          ez = pz[m];
        }
      }
      ex = {__shfl(ex.re, tj, L), __shfl(ex.im, tj, L)};
      ey = {__shfl(ey.re, tj, L), __shfl(ey.im, tj, L)};
      ez = {__shfl(ez.re, tj, L), __shfl(ez.im, tj, L)};
#pragma unroll
      for (int m = 0; m < E; ++m) {
        dx[m] = px[m];
        dy[m] = py[m];
      }
      park_st(0, px);
      park_st(1, py);
      F.fwd(dx);
      F.fwd(dy);
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) {
        const T f = kz_s[k2 + kofs] * inz;
        dx[k2] = f * mul_i(dx[k2]);
        dy[k2] = f * mul_i(dy[k2]);
      }
    }
    F.inv(dx);
    F.inv(dy);

    // multilayer amplitudes from P at the evaluation row
    ColInfo<T> c;
    column_info(c, t, pb, ix, iy);
    const cplx<T> as = (c.sx * ex + c.sy * ey) * c.down;
    const cplx<T> ap = (c.wt * (c.tx * ex + c.ty * ey) + c.wz * ez) * c.down;
    const cplx<T> a0 = c.live ? c.rte * as : cplx<T>{T(0), T(0)};
    const cplx<T> a1 = c.live ? c.rpe * ap : cplx<T>{T(0), T(0)};
    // exp(i kz z_abs) on this lane's absorber rows (z = lt + L m, every L-th
    // row): evaluated at the first one, then stepped by exp(i kz L dz)
    const int zf = t.j0 + ((lt - t.j0) % L + L) % L;
    const cplx<T> ph0 = up_phase(c, (T(zf - t.j0) + T(0.5)) * t.dz);
    const cplx<T> step = up_phase(c, T(L) * t.dz);
    const int64_t wb = (int64_t)3 * NZ - t.j0;  // W row of z is wb + (z - j0) + comp * nabs

    // U_z, the inner curl vectors w = -D P_t + i k_t P_z, and the W_z rows
    {
      cplx<T> ph = ph0;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int z = lt + L * m;
        const cplx<T> is = invs_s[z];
        const cplx<T> dpx = dx[m] * is, dpy = dy[m] * is;
        stv(2 * NZ + L * m, kx * mul_i(dpx) + ky * mul_i(dpy) + (kt2 - t.kbg2) * pz[m]);
        dx[m] = kx * mul_i(pz[m]) - dpx;
        dy[m] = ky * mul_i(pz[m]) - dpy;
        const int ja = z - t.j0;
        if (ja >= 0 && ja < t.nabs) {
          stv(wb + 2 * t.nabs + L * m, pz[m] - c.ktkz * (a1 * ph));
          ph = ph * step;
        }
      }
    }
    F.fwd(dx);
    F.fwd(dy);
#pragma unroll
    for (int k2 = 0; k2 < E; ++k2) {
      const T f = kz_s[k2 + kofs] * inz;
      dx[k2] = f * mul_i(dx[k2]);
      dy[k2] = f * mul_i(dy[k2]);
    }
    F.inv(dx);
    F.inv(dy);

    // U_x = (ky^2 - kbg^2) P_x - kx ky P_y + D w_x,  U_y = -kx ky P_x + (kx^2 - kbg^2) P_y + D w_y:
    // P_x first (then its W rows), P_y second
    const T cxx = ky * ky - t.kbg2, cxy = -(kx * ky), cyy = kx * kx - t.kbg2;
    {
      cplx<T>(&q)[E] = pz;  // P_z is no longer needed: reuse its registers
      park_ld(0, q);
      if constexpr (MODE == AX_AM) F.inv(q);
      cplx<T> ph = ph0;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int z = lt + L * m;
        const cplx<T> is = invs_s[z];
        dx[m] = dx[m] * is + cxx * q[m];
        dy[m] = dy[m] * is + cxy * q[m];
        const int ja = z - t.j0;
        if (ja >= 0 && ja < t.nabs) {
          const cplx<T> vs = a0 * ph, vp = a1 * ph;
          stv(wb + L * m, q[m] + (c.sx * vs + c.tx * vp));
          ph = ph * step;
        }
      }
      park_ld(1, q);
      if constexpr (MODE == AX_AM) F.inv(q);
      ph = ph0;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int z = lt + L * m;
        stv(L * m, dx[m] + cxy * q[m]);
        stv(NZ + L * m, dy[m] + cyy * q[m]);
        const int ja = z - t.j0;
        if (ja >= 0 && ja < t.nabs) {
          const cplx<T> vs = a0 * ph, vp = a1 * ph;
          stv(wb + t.nabs + L * m, q[m] + (c.sy * vs + c.ty * vp));
          ph = ph * step;
        }
      }
    }
  }
}

template <typename T, int NZ>
constexpr int ax_lanes() {
  // lanes per column for the register kernel (0: LDS kernel only): at most
  // 6 (FP32) or 3 (FP64) elements per lane keep the kernel near 128 VGPRs
  constexpr int emax = sizeof(T) == 4 ? 6 : 3;
  if (NZ > 64) return 0;
  int l = 1;
  while ((NZ / l > emax || NZ % l) && l < 16) l *= 2;
  return l;
}

template <typename T, int NZ, int L>
static hipError_t axial_reg_launch(const OpTables<T>& t, const cplx<T>* S, cplx<T>* UW, int mode,
                                   hipStream_t st) {
  const int64_t cols = (int64_t)t.nx * t.ny;
  if ((cols * L) % 256) return hipErrorInvalidValue;
  dim3 g((unsigned)(cols * L / 256 * t.nprob)), b(256);
  constexpr bool F32 = sizeof(T) == 4;
  const bool bf = F32 && t.pc_bf16 && !t.hf_mode;
  switch (mode) {
    case AX_A: PSFD_LAUNCH(t, (k_axial_reg<T, NZ, L, AX_A>), g, b, st, S, UW, t); break;
    case AX_AM:
      if (bf) PSFD_LAUNCH(t, (k_axial_reg<T, NZ, L, AX_AM, F32>), g, b, st, S, UW, t);
      else PSFD_LAUNCH(t, (k_axial_reg<T, NZ, L, AX_AM>), g, b, st, S, UW, t);
      break;
    default:
      if (bf) PSFD_LAUNCH(t, (k_axial_reg<T, NZ, L, AX_M, F32>), g, b, st, S, UW, t);
      else PSFD_LAUNCH(t, (k_axial_reg<T, NZ, L, AX_M>), g, b, st, S, UW, t);
      break;
  }
  return hipGetLastError();
}

// sched_ax: 0 register kernel (L lanes per column), 1 register kernel with
// 2L lanes, 2 LDS-staged kernel, 3 register kernel with L/2 lanes.  The adjoint and Nz > 64 always use the LDS
// kernel; PSFD_AXIAL_LDS forces it everywhere.
template <typename T, int NZ>
static hipError_t axial_n(const OpTables<T>& t, const cplx<T>* S, cplx<T>* UW, int mode,
                          hipStream_t st) {
  constexpr int L = ax_lanes<T, NZ>();
  if constexpr (L > 0) {
    if (!t.ax_lds && mode != AX_AH && t.sched_ax != 2) {
      constexpr int L2 = (2 * L <= 16 && NZ % (2 * L) == 0) ? 2 * L : L;
      constexpr int Lh = (L >= 4 && NZ % (L / 2) == 0 && NZ / (L / 2) <= 16) ? L / 2 : L;
      if (t.sched_ax == 1) return axial_reg_launch<T, NZ, L2>(t, S, UW, mode, st);
      if (t.sched_ax == 3) return axial_reg_launch<T, NZ, Lh>(t, S, UW, mode, st);
      return axial_reg_launch<T, NZ, L>(t, S, UW, mode, st);
    }
  }
  constexpr int TX = ax_tile<T, NZ>();
  if (t.nx % TX) return hipErrorInvalidValue;
  dim3 g(t.nx / TX, t.ny * t.nprob), b(256);
  switch (mode) {
    case AX_A: PSFD_LAUNCH(t, (k_axial<T, NZ, TX, AX_A>), g, b, st, S, UW, t); break;
    case AX_AM: PSFD_LAUNCH(t, (k_axial<T, NZ, TX, AX_AM>), g, b, st, S, UW, t); break;
    case AX_AH: PSFD_LAUNCH(t, (k_axial<T, NZ, TX, AX_AH>), g, b, st, S, UW, t); break;
    default: PSFD_LAUNCH(t, (k_axial<T, NZ, TX, AX_M>), g, b, st, S, UW, t); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axial(const OpTables<T>& t, const cplx<T>* S, cplx<T>* UW, int mode,
                        hipStream_t st) {
  switch (t.nz) {
    case 24: return axial_n<T, 24>(t, S, UW, mode, st);
    case 32: return axial_n<T, 32>(t, S, UW, mode, st);
    case 48: return axial_n<T, 48>(t, S, UW, mode, st);
    case 64: return axial_n<T, 64>(t, S, UW, mode, st);
    case 96: return axial_n<T, 96>(t, S, UW, mode, st);
    case 128: return axial_n<T, 128>(t, S, UW, mode, st);
    case 192: return axial_n<T, 192>(t, S, UW, mode, st);
    case 256: return axial_n<T, 256>(t, S, UW, mode, st);
    case 324: return axial_n<T, 324>(t, S, UW, mode, st);
    case 384: return axial_n<T, 384>(t, S, UW, mode, st);
    case 576: return axial_n<T, 576>(t, S, UW, mode, st);
    case 648: return axial_n<T, 648>(t, S, UW, mode, st);
    case 768: return axial_n<T, 768>(t, S, UW, mode, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_axial<double>(const OpTables<double>&, const cplx<double>*,
                                         cplx<double>*, int, hipStream_t);
template hipError_t launch_axial<float>(const OpTables<float>&, const cplx<float>*,
                                        cplx<float>*, int, hipStream_t);

}  // namespace psfd
