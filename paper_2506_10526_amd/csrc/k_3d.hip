// 3D bispectrum kernels for gfx950.
//
// Data flow (one pass per kernel, every intermediate in HBM):
//   delay transform along nu of the weighted cube, kept for |eta| <= H only
//   -> per shell j and delay plane eta in [0, H_j]: inverse C2C along v, then along u
//      (the shell's uv window is |qu|, |qv| <= vmax; negative qv come from Hermitian symmetry)
//   -> per shell, inverse C2R along eta (the Hermitian half kept is eta >= 0)
//   -> pair x shell contraction over voxels on MFMA.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "bs_kernels.h"

namespace {

__device__ __forceinline__ int sidx(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }
__device__ __forceinline__ int wrap(int q, int n) { return q < 0 ? q + n : q; }
// Workgroups are dispatched to the eight XCDs in turn (id mod 8).  This maps the dispatch id to a
// logical block so that every XCD runs one contiguous range of logical blocks: neighbours that
// share cache lines then meet in the same L2.
__device__ __forceinline__ int xcd_block(int id, int nb) {
  const int q = nb >> 3, r = nb & 7, x = id & 7, j = id >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
}
// two floats as packed bf16 (round to nearest even): x in the low half, y in the high half
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned v4u_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint32_t dft_pk(float x, float y) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{x, y}, bf16x2_t));
}
// A constant in a VGPR.  The asm is not volatile, so the compiler may share and hoist it.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t c) {
  uint32_t r;
  asm("" : "=v"(r) : "0"(c));
  return r;
}
// Split of two floats into packed bf16 hi = rne(x) and lo = rne(x - hi) (x in the low halves);
// x - hi is exact (hi lies within a factor two of x and shares its grid), and v_dot2_f32_bf16 of
// the packed hi with (-1, 0) or (0, -1), plus x or y, forms it in one instruction (a bf16 product
// by -1 and one addition whose exact result is representable).  The (-1, 0) operand must sit in a
// register: as the inline constant -1.0 this instruction does not read it as bf16 -1 in the low
// half and 0 in the high half.
__device__ __forceinline__ void dft_split2(float x, float y, uint32_t& hp, uint32_t& lp) {
  hp = dft_pk(x, y);
  const bf16x2_t h = __builtin_bit_cast(bf16x2_t, hp);
  const bf16x2_t mlo = __builtin_bit_cast(bf16x2_t, in_vgpr(0x0000BF80u));
  const bf16x2_t mhi = __builtin_bit_cast(bf16x2_t, in_vgpr(0xBF800000u));
  lp = dft_pk(__builtin_amdgcn_fdot2_f32_bf16(h, mlo, x, false), __builtin_amdgcn_fdot2_f32_bf16(h, mhi, y, false));
}

// --------------------------------------------------------------- delay transform
// Vt(eta, U) = sum_nu w(nu) m(U) V(U, nu) e^{-2 pi i eta nu / nc}, with the v = 0 column
// symmetrised per channel.  Block: NL consecutive qv of one qu row, all channels.
template <typename T, int IP>   // IP: in-place FFT butterflies per thread (2 or 4), 0 = two buffers
__global__ __launch_bounds__(256) void k3_delay(Delay3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Shell3Geom& g = a.g;
  const int nc = g.nc, n = g.n, nh = g.nh;
  // logical block (ub, v-block), v-blocks of one uv row consecutive on one XCD: the NL-column
  // reads of neighbouring blocks fill the same cache lines
  const int nvblk = (g.nvb + a.NL - 1) / a.NL;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int ub = lb / nvblk;
  const int qu = ub - g.vmax;
  const int iu = wrap(qu, n), iun = wrap(-qu, n);
  const int v0 = (lb - ub * nvblk) * a.NL;
  const int nl = min(a.NL, g.nvb - v0);
  const int ld = nc + 1;
  Cx<T>* A = (Cx<T>*)smem_raw;
  Cx<T>* Bf = A + (size_t)a.NL * ld;
  // the FFT's twiddle table (nc entries) in LDS after the line buffers, loaded with the lines
  Cx<T>* twl = A + (size_t)a.NL * ld * (IP > 0 ? 1 : 2);
  for (int e = threadIdx.x; e < nc; e += blockDim.x) twl[e] = ((const Cx<T>*)a.tw)[e];
  const Cx<T>* vis = (const Cx<T>*)a.vis;
  // eight elements per thread in flight before their LDS stores
  const float rnl = 1.0f / (float)nl;
  for (int e0 = threadIdx.x; e0 < nl * nc; e0 += 8 * blockDim.x) {
    Cx<T> x[8], y[8];
    int nuu[8], lu[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * blockDim.x;
      int nu = 0, l = 0;
      if (e < nl * nc) fdivmod(e, nl, rnl, nu, l);
      nuu[u] = e < nl * nc ? nu : -1;
      lu[u] = l;
      const int v = v0 + l;
      x[u] = y[u] = cmk(T(0), T(0));
      if (e < nl * nc) {
        x[u] = vis[((size_t)nu * n + iu) * nh + v];
        if (v == 0) y[u] = vis[((size_t)nu * n + iun) * nh];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int nu = nuu[u], l = lu[u], v = v0 + l;
      if (nu < 0) continue;
      const T cw = a.chw ? T(a.chw[nu]) : T(1);
      const T m = g.uvm ? T(g.uvm[(size_t)iu * nh + v]) : T(1);
      Cx<T> xv = cscale(x[u], cw * m);
      if (v == 0) {
        const T mn = g.uvm ? T(g.uvm[(size_t)iun * nh]) : T(1);
        xv = cscale(cadd(xv, cconj(cscale(y[u], cw * mn))), T(0.5));
      }
      A[(size_t)l * ld + nu] = xv;
    }
  }
  __syncthreads();
  Cx<T>* r = A;
  if constexpr (IP > 0) lds_fft_ip<-1, T, IP>(A, a.plan, nl, twl, 1, ld);
  else r = lds_fft<-1, T>(A, Bf, a.plan, nl, twl, 1, ld);
  Cx<T>* out = (Cx<T>*)a.out;
  const int ne = 2 * g.H + 1;
  for (int e = threadIdx.x; e < ne * nl; e += blockDim.x) {
    int ec, l;
    fdivmod(e, nl, rnl, ec, l);
    int eta = ec - g.H;
    int idx = eta < 0 ? eta + nc : eta;
    out[((size_t)ec * g.nub + ub) * g.nvb + v0 + l] = r[(size_t)l * ld + idx];
  }
}

// --------------------------------------------------------------- v pass
// Input value of shell j at (eta >= 0, qu, qv): data Vt or the unit indicator.
// Membership of (eta >= 0, qu, qv) in shell j (shell table and uv support), then its input value:
// data Vt or the unit indicator.
// With a.shell_iv the shell's cells at this |eta| are the range [s_lo, s_hi] of s (no table read).
__device__ __forceinline__ bool shell_member(const Pass3Args& a, int shell, int eta, int qu, int qv, int s_lo, int s_hi) {
  const Shell3Geom& g = a.g;
  if (qv > g.vmax || qv < -g.vmax) return false;
  const int s = qu * qu + qv * qv;
  if (s < 1 || s > g.smax) return false;
  bool in = a.shell_iv ? s >= s_lo && s <= s_hi : g.lut[(size_t)eta * g.S1 + s] == shell;
  if (g.uvm) {
    const int hu = qv >= 0 ? qu : -qu, hv = qv >= 0 ? qv : -qv;  // stored half-plane cell
    in = in && g.uvm[(size_t)wrap(hu, g.n) * g.nh + hv];
  }
  return in;
}
template <typename T>
__device__ __forceinline__ Cx<T> shell_data(const Pass3Args& a, int eta, int qu, int qv) {
  const Shell3Geom& g = a.g;
  if (a.indicator) return cmk(T(1), T(0));
  const Cx<T>* D = (const Cx<T>*)a.in;
  if (qv >= 0) return D[((size_t)(eta + g.H) * g.nub + (qu + g.vmax)) * g.nvb + qv];
  return cconj(D[((size_t)(g.H - eta) * g.nub + (-qu + g.vmax)) * g.nvb + (-qv)]);
}

template <typename T, int IP>
__global__ __launch_bounds__(256) void k3_vpass(Pass3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Shell3Geom& g = a.g;
  // consecutive work items (neighbouring qu blocks, whose output rows share cache lines) on one XCD
  const Work3 w = a.work[xcd_block(blockIdx.x, gridDim.x)];
  const int shell = a.shell_of_block[w.j];
  const int n = g.n, ld = n + 1;
  const int nl = min(a.NL, g.nub - w.start);
  Cx<T>* A = (Cx<T>*)smem_raw;
  Cx<T>* Bf = A + (size_t)a.NL * ld;
  // the FFT's twiddle table (n entries) in LDS after the line buffers, loaded with the lines
  Cx<T>* twl = A + (size_t)a.NL * ld * (IP > 0 ? 1 : 2);
  for (int e = threadIdx.x; e < n; e += blockDim.x) twl[e] = ((const Cx<T>*)a.tw)[e];
  const int s_lo = w.pad & 0xffff, s_hi = (int)((unsigned)w.pad >> 16);
  // column i (qv) of the block's qu rows, eight rows at a time: the shell-table and mask reads of
  // all eight first, then the data reads of the members, then the LDS stores
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int qv = sidx(i, n);
    for (int l0 = 0; l0 < nl; l0 += 8) {
      bool mem[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        mem[u] = l0 + u < nl && shell_member(a, shell, w.eta, w.start + l0 + u - g.vmax, qv, s_lo, s_hi);
      Cx<T> v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = mem[u] ? shell_data<T>(a, w.eta, w.start + l0 + u - g.vmax, qv) : cmk(T(0), T(0));
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (l0 + u < nl) A[(size_t)(l0 + u) * ld + i] = v[u];
    }
  }
  __syncthreads();
  Cx<T>* r = A;
  if constexpr (IP > 0) lds_fft_ip<+1, T, IP>(A, a.plan, nl, twl, 1, ld);
  else r = lds_fft<+1, T>(A, Bf, a.plan, nl, twl, 1, ld);
  // T_j[x_v][eta][qu]: consecutive threads write consecutive qu rows of one x_v
  const int hp1 = a.hj[w.j] + 1;
  Cx<T>* out = (Cx<T>*)a.out + a.off_out[w.j];
  const float rnl = 1.0f / (float)nl;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int i, l;
    fdivmod(e, nl, rnl, i, l);
    out[((size_t)i * hp1 + w.eta) * g.nub + w.start + l] = r[(size_t)l * ld + i];
  }
}

// --------------------------------------------------------------- u pass
// Work item (j, x_v = w.start, eta0 = w.eta): the delay planes eta0.. of one x_v column.
// Output G_j[line = x_u n + x_v][eta] keeps each line's delay spectrum contiguous.
template <typename T, int IP>
__global__ __launch_bounds__(256) void k3_upass(Pass3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Shell3Geom& g = a.g;
  const Work3 w = a.work[blockIdx.x];
  const int n = g.n, ld = n + 1;
  const int hp1 = a.hj[w.j] + 1;
  const int xv = w.start, e0 = w.eta;
  const int nl = min(a.NL, hp1 - e0);
  Cx<T>* A = (Cx<T>*)smem_raw;
  Cx<T>* Bf = A + (size_t)a.NL * ld;
  // the FFT's twiddle table (n entries) in LDS after the line buffers, loaded with the lines
  Cx<T>* twl = A + (size_t)a.NL * ld * (IP > 0 ? 1 : 2);
  for (int e = threadIdx.x; e < n; e += blockDim.x) twl[e] = ((const Cx<T>*)a.tw)[e];
  const Cx<T>* in = (const Cx<T>*)a.in + a.off_in[w.j] + ((size_t)xv * hp1 + e0) * g.nub;
  // column i of every plane: eight loads in flight per thread before their LDS stores
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int qu = sidx(i, n);
    const bool inw = qu >= -g.vmax && qu <= g.vmax;
    const Cx<T>* src = in + (inw ? qu + g.vmax : 0);
    for (int l0 = 0; l0 < nl; l0 += 8) {
      Cx<T> v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = inw && l0 + u < nl ? src[(size_t)(l0 + u) * g.nub] : cmk(T(0), T(0));
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (l0 + u < nl) A[(size_t)(l0 + u) * ld + i] = v[u];
    }
  }
  __syncthreads();
  Cx<T>* r = A;
  if constexpr (IP > 0) lds_fft_ip<+1, T, IP>(A, a.plan, nl, twl, 1, ld);
  else r = lds_fft<+1, T>(A, Bf, a.plan, nl, twl, 1, ld);
  if constexpr (std::is_same<T, float>::value) {
    if (a.gs) {
      // bf16 hi/lo A-fragments of K-step s = e0 / 16 for the n / 16 line groups of this x_v column:
      // lane group g (lanes 16 g .. 16 g + 15) holds modes 16 s + 4 g .. +3.  This item writes its
      // planes' groups that hold at least one mode (<= H_j); groups wholly past H_j are never
      // written (the synthesis kernel keeps them zero in LDS and does not copy them).
      const int S = (hp1 + 15) >> 4, s = e0 >> 4, nxub = n >> 4;
      const int g0 = (e0 & 15) >> 2, gpl = min(a.NL >> 2, (hp1 - e0 + 3) >> 2);
      uint4* out = (uint4*)a.gs + a.off_gs[w.j];
      const float sc = (float)a.scale;
      const float rgr = 1.0f / (float)(16 * gpl);
      for (int e = threadIdx.x; e < nxub * 16 * gpl; e += blockDim.x) {
        int xub, lr;
        fdivmod(e, 16 * gpl, rgr, xub, lr);
        const int lane = g0 * 16 + lr;
        const int xu = xub * 16 + (lane & 15), q0 = 4 * (lane >> 4) - (e0 & 15);
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int q = q0 + c;   // mode e0 + q
          float re = 0.f, im = 0.f;
          if (q < nl) {
            const Cx<float> z = r[(size_t)q * ld + xu];
            const bool dc = e0 + q == 0;
            re = z.x * (dc ? sc : 2.f * sc);
            im = dc ? 0.f : z.y * (2.f * sc);
          }
          dft_split2(re, im, hw[c], lw[c]);
        }
        uint4* o = out + ((size_t)(xv * nxub + xub) * S + s) * 128;
        o[lane] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        o[64 + lane] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
      }
      return;
    }
  }
  Cx<T>* out = (Cx<T>*)a.out + a.off_out[w.j];
  const float rnl = 1.0f / (float)nl;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int i, l;
    fdivmod(e, nl, rnl, i, l);
    out[((size_t)i * n + xv) * hp1 + e0 + l] = r[(size_t)l * ld + i];
  }
}

// --------------------------------------------------------------- eta pass (C2R)
// Writes the real fields F_j[x_eta][line] (used for the field output and the FP64 counts).
template <typename T>
__global__ __launch_bounds__(256) void k3_etapass(Pass3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Shell3Geom& g = a.g;
  const Work3 w = a.work[blockIdx.x];
  const int n = g.n;
  const long long n2 = (long long)n * n;
  const int nl = (int)min((long long)a.NL, n2 - w.start);
  const int Mh = a.M / 2;
  const int ld = Mh + 1;
  const int Hj = a.hj[w.j];
  Cx<T>* A = (Cx<T>*)smem_raw;
  Cx<T>* Bf = A + (size_t)a.NL * ld;
  const Cx<T>* in = (const Cx<T>*)a.in + a.off_in[w.j] + (size_t)w.start * (Hj + 1);
  const Cx<T>* tw = (const Cx<T>*)a.tw;  // table of length M
  for (int e = threadIdx.x; e < nl * Mh; e += blockDim.x) {
    int l = e / Mh, k = e - l * Mh;
    const Cx<T>* gl = in + (size_t)l * (Hj + 1);
    auto get = [&](int eta) -> Cx<T> { return eta <= Hj ? gl[eta] : cmk(T(0), T(0)); };
    A[(size_t)l * ld + k] = c2r_pack<T>(k, Mh, get, tw, 1);
  }
  __syncthreads();
  Cx<T>* r = lds_fft<+1, T>(A, Bf, a.plan, nl, tw, 2, ld);
  T* out = (T*)a.out + (size_t)w.j * a.fstride + w.start;
  const T sc = T(a.scale);
  for (int e = threadIdx.x; e < nl * Mh; e += blockDim.x) {
    int k = e / nl, l = e - k * nl;
    Cx<T> z = r[(size_t)l * ld + k];
    out[(size_t)(2 * k) * n2 + l] = z.x * sc;
    out[(size_t)(2 * k + 1) * n2 + l] = z.y * sc;
  }
}

// --------------------------------------------------------------- contraction
// C[p][c] = sum_x F_a(x) F_b(x) F_c(x) for every pair p = (a, b) and field c, as a GEMM
// with M = pairs, N = fields, K = voxels: 16 x 16 MFMA tiles, up to 7 x 2 tiles per wave.
// A block streams its voxel range through LDS in slabs of 128 voxels (32 per wave).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int C3_RT = 7, C3_CT = 2, C3_SLAB = 128, C3_LDS = C3_SLAB + 4;


// hi = rne_bf16(v), lo = rne_bf16(v - hi) for eight floats, two conversions per instruction
__device__ __forceinline__ void split8(const float* v, bf16x8& h, bf16x8& l) {
  uint32_t hw[4], lw[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    dft_split2(v[2 * q], v[2 * q + 1], hw[q], lw[q]);
  }
  h = __builtin_bit_cast(bf16x8, v4u_t{hw[0], hw[1], hw[2], hw[3]});
  l = __builtin_bit_cast(bf16x8, v4u_t{lw[0], lw[1], lw[2], lw[3]});
}

template <int MODE>
using acc_t = typename std::conditional<MODE == 0, f64x4, f32x4>::type;

// One 32-voxel step of one wave: voxels v0 .. v0+31 of the LDS field rows sF + j*ld
// (j < nbu; rows beyond nbu read as zero).  A rows are the pair products F_a F_b, B columns
// the fields F_c; sp holds the pair table (-1 = padding row).
template <int MODE, typename T>
__device__ __forceinline__ void con3_step(const T* __restrict__ sF, int ld, int nbu, int v0, const int* sp, int RT,
                                          int CT, acc_t<MODE> (&acc)[C3_RT][C3_CT]) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  if constexpr (MODE == 2) {
    const int vb = v0 + kq * 8;
    bf16x8 bh[C3_CT], bl[C3_CT];
#pragma unroll
    for (int ct = 0; ct < C3_CT; ++ct) {
      float v[8];
      const int c = ct * 16 + r16;
      if (c < nbu) {
        const T* src = &sF[(size_t)c * ld + vb];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (float)src[q];
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = 0.f;
      }
      split8(v, bh[ct], bl[ct]);
    }
#pragma unroll
    for (int rt = 0; rt < C3_RT; ++rt) {
      if (rt < RT) {
        int p = rt * 16 + r16;
        int pa = sp[2 * p], pb = sp[2 * p + 1];
        float v[8];
        if (pa >= 0) {
          const T* sa = &sF[(size_t)pa * ld + vb];
          const T* sb = &sF[(size_t)pb * ld + vb];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = (float)sa[q] * (float)sb[q];
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = 0.f;
        }
        bf16x8 ah, al;
        split8(v, ah, al);
#pragma unroll
        for (int ct = 0; ct < C3_CT; ++ct) {
          if (ct < CT) {
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ct], acc[rt][ct], 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ct], acc[rt][ct], 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ct], acc[rt][ct], 0, 0, 0);
          }
        }
      }
    }
  } else {
#pragma unroll 2
    for (int ks = 0; ks < 8; ++ks) {
      const int vx = v0 + ks * 4 + kq;
      T bv[C3_CT];
#pragma unroll
      for (int ct = 0; ct < C3_CT; ++ct) {
        const int c = ct * 16 + r16;
        bv[ct] = c < nbu ? sF[(size_t)c * ld + vx] : T(0);
      }
#pragma unroll
      for (int rt = 0; rt < C3_RT; ++rt) {
        if (rt < RT) {
          int p = rt * 16 + r16;
          int pa = sp[2 * p], pb = sp[2 * p + 1];
          T av = pa >= 0 ? sF[(size_t)pa * ld + vx] * sF[(size_t)pb * ld + vx] : T(0);
#pragma unroll
          for (int ct = 0; ct < C3_CT; ++ct) {
            if (ct < CT) {
              if constexpr (MODE == 0)
                acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[ct], acc[rt][ct], 0, 0, 0);
              else
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[ct], acc[rt][ct], 0, 0, 0);
            }
          }
        }
      }
    }
  }
}

template <int MODE>
__device__ __forceinline__ void con3_flush(acc_t<MODE> (&acc)[C3_RT][C3_CT], double (&acc64)[C3_RT][C3_CT][4]) {
#pragma unroll
  for (int i = 0; i < C3_RT; ++i)
#pragma unroll
    for (int j = 0; j < C3_CT; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) { acc64[i][j][q] += (double)acc[i][j][q]; acc[i][j][q] = 0; }
}

// Reduce the four waves' sums in a fixed order into red[112][32] and store them as this
// block's partial sums.  red must be zeroed and visible to all threads before the call.
template <int MODE>
__device__ __forceinline__ void con3_store(acc_t<MODE> (&acc)[C3_RT][C3_CT], double (&acc64)[C3_RT][C3_CT][4],
                                           double* red, double* out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r16 = lane & 15, kq = lane >> 4;
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int i = 0; i < C3_RT; ++i)
#pragma unroll
        for (int j = 0; j < C3_CT; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            // 16x16 MFMA output rows: 4*(lane/16)+q for the f32/bf16 forms, lane/16+4*q for f64
            int p = i * 16 + (MODE == 0 ? kq + 4 * q : kq * 4 + q), c = j * 16 + r16;
            red[p * 32 + c] += acc64[i][j][q] + (double)acc[i][j][q];
          }
    }
    __syncthreads();
  }
  for (int e = tid; e < 112 * 32; e += 256) out[e] = red[e];
}

// Contraction over precomputed fields F[j][vox] streamed through LDS in 128-voxel slabs.
template <int MODE, typename T>  // MODE 0: FP64 MFMA, 1: FP32 MFMA, 2: split-BF16 MFMA
__global__ __launch_bounds__(256) void k3_contract(Con3Args a) {
  __shared__ T sF[32 * C3_LDS];
  __shared__ int sp[2 * 112];
  __shared__ double red[112 * 32];
  const int tid = threadIdx.x, wave = tid >> 6;
  for (int e = tid; e < 2 * 112; e += 256) sp[e] = e < 2 * a.npairs ? a.pairs[e] : -1;
  for (int e = tid; e < 112 * 32; e += 256) red[e] = 0.0;
  const int RT = (a.npairs + 15) / 16, CT = (a.nbu + 15) / 16;
  acc_t<MODE> acc[C3_RT][C3_CT];
  double acc64[C3_RT][C3_CT][4];
#pragma unroll
  for (int i = 0; i < C3_RT; ++i)
#pragma unroll
    for (int j = 0; j < C3_CT; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) { acc[i][j][q] = 0; acc64[i][j][q] = 0.0; }
  const long long x_beg = (long long)blockIdx.x * a.chunk;
  const long long x_end = x_beg + a.chunk < a.vox ? x_beg + a.chunk : a.vox;
  const T* F = (const T*)a.F;
  int since = 0;
  __syncthreads();
  for (long long x0 = x_beg; x0 < x_end; x0 += C3_SLAB) {
    for (int e = tid; e < a.nbu * C3_SLAB; e += 256) {
      int j = e / C3_SLAB, v = e - j * C3_SLAB;
      long long x = x0 + v;
      sF[j * C3_LDS + v] = x < x_end ? F[(size_t)j * a.vox + x] : T(0);
    }
    __syncthreads();
    con3_step<MODE, T>(sF, C3_LDS, a.nbu, wave * 32, sp, RT, CT, acc);
    __syncthreads();
    since += C3_SLAB;
    // FP32 forms: FP64 flush every 512 voxels.  FP64 form (the triangle counts): every slab, so
    // that no accumulation chain is longer than one slab plus the slab count of the block.
    if (since >= (MODE == 0 ? C3_SLAB : 512)) { since = 0; con3_flush<MODE>(acc, acc64); }
  }
  con3_store<MODE>(acc, acc64, red, a.partial + (size_t)blockIdx.x * 112 * 32);
}

// Fused C2R along eta + contraction.  A block owns a range of (x_u, x_v) lines; for each line
// it unpacks every shell's delay spectrum G_j[line][0..H_j] (Hermitian half eta >= 0), runs the
// M/2-point inverse FFT of the C2R packing for all shells at once in LDS (the complex result
// read as floats is the real field x_eta = 0..M-1), and contracts the M voxels of the line.
// The next line's spectra are fetched into registers while the current line is processed, and
// twiddles and per-shell metadata live in LDS, so no dependent global load sits in the loop.
constexpr int FUSED_STAGE = 512;   // max sum_j (H_j + 1) held per line

template <int MODE>
__global__ __launch_bounds__(256) void k3_fused(Fused3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int nbu = a.nbu, M = a.M, Mh = M / 2, ld = Mh + Mh / 16 + 2;   // room for the padded FFT layout
  Cx<float>* A = (Cx<float>*)smem_raw;
  Cx<float>* Bf = A + (size_t)nbu * ld;
  Cx<float>* tw = Bf + (size_t)nbu * ld;                    // [M]
  Cx<float>* stage = tw + M;                                  // [2][FUSED_STAGE]
  int* sp = (int*)(stage + 2 * FUSED_STAGE);                  // [224]
  int* pre = sp + 224;                                        // [33] prefix of H_j + 1
  int* sj = pre + 33;                                         // [FUSED_STAGE] shell of a stage slot
  for (int e = tid; e < 2 * 112; e += 256) sp[e] = e < 2 * a.npairs ? a.pairs[e] : -1;
  for (int e = tid; e < M; e += 256) tw[e] = ((const Cx<float>*)a.tw)[e];
  if (tid == 0) {
    int acc = 0;
    for (int j = 0; j < nbu; ++j) { pre[j] = acc; acc += a.hj[j] + 1; }
    pre[nbu] = acc;
  }
  __syncthreads();
  const int L = pre[nbu];
  for (int e = tid; e < L; e += 256) {
    int j = 0;
    while (pre[j + 1] <= e) ++j;
    sj[e] = j;
  }
  const int RT = (a.npairs + 15) / 16, CT = (nbu + 15) / 16;
  acc_t<MODE> acc[C3_RT][C3_CT];
  double acc64[C3_RT][C3_CT][4];
#pragma unroll
  for (int i = 0; i < C3_RT; ++i)
#pragma unroll
    for (int j = 0; j < C3_CT; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) { acc[i][j][q] = 0; acc64[i][j][q] = 0.0; }
  const Cx<float>* G = (const Cx<float>*)a.G;
  const float sc = (float)a.scale;
  const float rMh = 1.0f / (float)Mh, rM = 1.0f / (float)M;
  const int nlow = a.nlow, nfft = nbu - nlow;
  // the FFT result buffer: A after an even number of Stockham passes, Bf after an odd one
  float* Rf = (float*)((a.plan.nr & 1) ? Bf : A);
  const long long l_beg = (long long)blockIdx.x * a.lines_per_block;
  const long long l_end = l_beg + a.lines_per_block < a.nlines ? l_beg + a.lines_per_block : a.nlines;
  __syncthreads();
  // global address of stage slot e for `line`
  auto slot_src = [&](int e, long long line) -> const Cx<float>* {
    int j = sj[e];
    return G + a.offG[j] + (size_t)line * (pre[j + 1] - pre[j]) + (e - pre[j]);
  };
  // prime stage 0 with the first line
  if (l_beg < l_end)
    for (int e = tid; e < L; e += 256) stage[e] = *slot_src(e, l_beg);
  int cur = 0;
  int since = 0;
  __syncthreads();
  for (long long line = l_beg; line < l_end; ++line) {
    // prefetch the next line (at most two slots per thread)
    Cx<float> pf0 = cmk(0.f, 0.f), pf1 = cmk(0.f, 0.f);
    const bool more = line + 1 < l_end;
    if (more) {
      if (tid < L) pf0 = *slot_src(tid, line + 1);
      if (tid + 256 < L) pf1 = *slot_src(tid + 256, line + 1);
    }
    const Cx<float>* st = stage + cur * FUSED_STAGE;
    // shells with a wide delay support: C2R packing, then the M/2-point FFT of all of them at once
    for (int e = tid; e < nfft * Mh; e += 256) {
      int jj, k;
      fdivmod(e, Mh, rMh, jj, k);
      const int j = nlow + jj;
      const int p0 = pre[j], hp1 = pre[j + 1] - p0;
      auto get = [&](int eta) -> Cx<float> { return eta < hp1 ? st[p0 + eta] : cmk(0.f, 0.f); };
      Cx<float> z = c2r_pack<float>(k, Mh, get, tw, 1);
      A[(size_t)j * ld + k] = cmk(z.x * sc, z.y * sc);
    }
    // shells with |eta| <= FUSED_DIRECT_H: x(t) = sc (Re G_0 + 2 sum_q Re(G_q e^{+2 pi i q t / M})),
    // written straight into the rows of the buffer the FFT result lands in
    for (int e = tid; e < nlow * M; e += 256) {
      int j, t;
      fdivmod(e, M, rM, j, t);
      const int p0 = pre[j], h = pre[j + 1] - p0 - 1;
      float x = st[p0].x;
      int m = 0;
      for (int q = 1; q <= h; ++q) {
        m += t;
        if (m >= M) m -= M;
        const Cx<float> g = st[p0 + q], w = tw[m];   // w = e^{-2 pi i m / M}
        x += 2.0f * (g.x * w.x + g.y * w.y);          // Re(g conj(w))
      }
      Rf[2 * (size_t)j * ld + t] = x * sc;
    }
    __syncthreads();
    if (nfft > 0) lds_fft<+1, float, true>(A + (size_t)nlow * ld, Bf + (size_t)nlow * ld, a.plan, nfft, tw, 2, ld);
    const float* Fl = Rf;   // row j: floats [2 j ld, 2 j ld + M)
    for (int v0 = wave * 32; v0 < M; v0 += 128) con3_step<MODE, float>(Fl, 2 * ld, nbu, v0, sp, RT, CT, acc);
    if (more) {
      Cx<float>* nx = stage + (cur ^ 1) * FUSED_STAGE;
      if (tid < L) nx[tid] = pf0;
      if (tid + 256 < L) nx[tid + 256] = pf1;
    }
    cur ^= 1;
    __syncthreads();
    since += M / 4;   // voxels per wave per line
    if (since >= 512) { since = 0; con3_flush<MODE>(acc, acc64); }
  }
  double* red = (double*)smem_raw;   // reuse the FFT buffers
  for (int e = tid; e < 112 * 32; e += 256) red[e] = 0.0;
  __syncthreads();
  con3_store<MODE>(acc, acc64, red, a.partial + (size_t)blockIdx.x * 112 * 32);
}

// Split-BF16 fused kernel: the C2R along eta as MFMA GEMMs against a twiddle-fragment table, then
// the pair x field contraction.  A block of DFT_WAVES waves owns a range of line groups
// (16 consecutive x_u of one x_v).  For each group it copies the group's spectrum fragments (all
// fields, all K-steps) into LDS with 16-byte buffer loads; each wave then takes t-tiles of 16
// delay samples and computes, for every field j, F_j[16 lines][16 t] = sum over K-steps of three
// MFMAs (lo.hi, hi.lo, hi.hi), four fields at a time so that consecutive MFMAs are independent
// (missing K-steps read a zero fragment).  Lane l then holds F_j at lines 4 (l / 16) + i,
// t = l % 16 (i = 0..3); quarter i passes through the wave's own LDS rows (voxel l) into the
// contraction, whose pair rows and padding (a zero row) are resolved once per lane.  The copy of
// the next group's fragments is issued once every wave has finished its last synthesis of the
// current group and lands while that tile is contracted.  Each wave adds its FP32 sums into its
// own FP64 slot of `partial` every a.flush_vox voxels.
typedef __attribute__((address_space(3))) void lds_void_t;

// Contraction of one 16 x 16 synthesis tile (256 voxels, dk[j] for field j) into acc, in four
// quarters of 64 voxels staged in rows sF[j * DFT_LDQ + v] (v < 64): RTN pair row tiles (row
// offsets oa / ob per lane, zero row for padding) and two field column tiles (offsets oc).  Steps
// (32 voxels, pair row tile) are issued as: LDS reads of the next step, products and splits of
// this step, its six MFMAs; sched_barrier keeps that order (the compiler would otherwise wait for
// every read right before its use).  The rows of the next quarter are written right after the last
// reads of the current one: a wave's LDS operations complete in order, so the writes cannot pass
// those reads, and the pipeline runs through all four quarters without draining.
template <int RTN>
__device__ __forceinline__ void dft_contract_tile(float* __restrict__ sF, const f32x4 (&dk)[DFT_MAX_FIELDS],
                                                  const int (&oa)[RTN], const int (&ob)[RTN], const int (&oc)[2],
                                                  int ct1_tiles, f32x4 (&acc)[RTN][2]) {
  const int lane = threadIdx.x & 63, kq = lane >> 4;
  float4 ra[2][2], rb[2][2], rc[2][2][2];
  auto write_q = [&](int q) {
#pragma unroll
    for (int j = 0; j < DFT_MAX_FIELDS; ++j)   // rows past nbu hold zeros and are never read
      sF[(size_t)j * DFT_LDQ + lane] = dk[j][q];
  };
  auto load_ab = [&](int ks, int rt, int buf) {
    const int vb = ks * 32 + kq * 8;
    ra[buf][0] = *(const float4*)&sF[oa[rt] + vb];
    ra[buf][1] = *(const float4*)&sF[oa[rt] + vb + 4];
    rb[buf][0] = *(const float4*)&sF[ob[rt] + vb];
    rb[buf][1] = *(const float4*)&sF[ob[rt] + vb + 4];
  };
  auto load_c = [&](int ks, int buf) {
    const int vb = ks * 32 + kq * 8;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      rc[buf][ct][0] = *(const float4*)&sF[oc[ct] + vb];
      rc[buf][ct][1] = *(const float4*)&sF[oc[ct] + vb + 4];
    }
  };
  write_q(0);
  load_c(0, 0);
  load_ab(0, 0, 0);
  bf16x8 bh[2], bl[2];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int kk = 2 * q + ks;   // 32-voxel step of the tile (parity selects the rc buffer)
#pragma unroll
      for (int rt = 0; rt < RTN; ++rt) {
        const int i = kk * RTN + rt;
        __builtin_amdgcn_sched_barrier(0);
        if (rt + 1 < RTN) {
          load_ab(ks, rt + 1, (i + 1) & 1);
        } else if (ks + 1 < 2) {
          load_ab(ks + 1, 0, (i + 1) & 1);
          load_c(ks + 1, (kk + 1) & 1);
        } else if (q + 1 < 4) {
          write_q(q + 1);
          load_ab(0, 0, (i + 1) & 1);
          load_c(0, (kk + 1) & 1);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (rt == 0) {
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) {
            const float4 c0 = rc[kk & 1][ct][0], c1 = rc[kk & 1][ct][1];
            const float v[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
            split8(v, bh[ct], bl[ct]);
          }
        }
        const float4 a0 = ra[i & 1][0], a1 = ra[i & 1][1], b0 = rb[i & 1][0], b1 = rb[i & 1][1];
        const float v[8] = {a0.x * b0.x, a0.y * b0.y, a0.z * b0.z, a0.w * b0.w,
                            a1.x * b1.x, a1.y * b1.y, a1.z * b1.z, a1.w * b1.w};
        bf16x8 ah, al;
        split8(v, ah, al);
        __builtin_amdgcn_sched_barrier(0);
        // a raised wave priority while the MFMAs issue: the SIMD's other wave fills the gaps with
        // its vector work instead of holding the matrix core back
        __builtin_amdgcn_s_setprio(1);
        acc[rt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[0], acc[rt][0], 0, 0, 0);
        acc[rt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[0], acc[rt][0], 0, 0, 0);
        acc[rt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[0], acc[rt][0], 0, 0, 0);
        // fields 16..31 only for the pair row tiles that serve such a column
        if (rt < ct1_tiles) {
          acc[rt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[1], acc[rt][1], 0, 0, 0);
          acc[rt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[1], acc[rt][1], 0, 0, 0);
          acc[rt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[1], acc[rt][1], 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

template <int RTN>
__global__ __launch_bounds__(DFT_WAVES * 64) void k3_dft(Dft3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  constexpr int ROWS = DFT_MAX_FIELDS + 1;   // fields + one zero row
  // the wave index is uniform: readfirstlane lets the tile and copy loops run on scalar control
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), r16 = lane & 15;
  const int nbu = a.nbu, nfr = 2 * a.kb[nbu];
  const int M = a.M;
  v4u_t* stage = (v4u_t*)smem_raw;                                      // [nfr + 1][64], last = zeros
  float2* twf = (float2*)(stage + (size_t)(nfr + 2) * 64);              // [M] (cos, sin) of 2 pi m / M
  // synthesis schedule: sched[s][j] = hi fragment of field j at step s (lo follows it), or the zero
  // pair nfr, nfr + 1 once the field has no modes left; sched[s][DFT_MAX_FIELDS] = bit c set when
  // fields 4c .. 4c + 3 still have modes at step s
  int* sched = (int*)(twf + M);
  float* sF = (float*)(sched + DFT_MAX_STEPS * DFT_SCHED) + (size_t)wave * ROWS * DFT_LDQ;   // this wave's rows
  // the whole stage starts at zero: lane groups past a field's last mode are never copied and
  // stay zero, and fragments nfr, nfr + 1 are the zero pair
  for (int e = tid; e < (nfr + 2) * 64; e += DFT_WAVES * 64) stage[e] = v4u_t{0u, 0u, 0u, 0u};
  for (int e = tid; e < M; e += DFT_WAVES * 64) twf[e] = ((const float2*)a.W)[e];
  for (int e = tid; e < DFT_MAX_STEPS * DFT_SCHED; e += DFT_WAVES * 64) {
    const int st = e / DFT_SCHED, j = e - st * DFT_SCHED;
    int v = 0;
    if (j < DFT_MAX_FIELDS) {
      v = j < nbu && st < a.Sj[j] ? 2 * (a.kb[j] + st) : nfr;
    } else if (j == DFT_MAX_FIELDS) {
      for (int f = 0; f < nbu; ++f)
        if (st < a.Sj[f]) v |= 1 << (f >> 2);
    }
    sched[e] = v;
  }
  for (int e = lane; e < DFT_LDQ; e += 64) sF[DFT_MAX_FIELDS * DFT_LDQ + e] = 0.f;
  // per-lane contraction rows: pair (a, b) of row rt * 16 + r16 and field c = ct * 16 + r16
  int oa[RTN], ob[RTN], oc[2];
#pragma unroll
  for (int rt = 0; rt < RTN; ++rt) {
    const int p = rt * 16 + r16;
    const bool ok = p < a.npairs;
    oa[rt] = (ok ? a.pairs[2 * p] : DFT_MAX_FIELDS) * DFT_LDQ;
    ob[rt] = (ok ? a.pairs[2 * p + 1] : DFT_MAX_FIELDS) * DFT_LDQ;
  }
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int c = ct * 16 + r16;
    oc[ct] = (c < nbu ? c : DFT_MAX_FIELDS) * DFT_LDQ;
  }
  // this wave's FP64 slot (pair-tile rows only): the first flush stores the FP32 sums, later ones
  // add them with FP64 atomic adds that return nothing, so a flush never waits for memory (each
  // entry is updated only by its owning lane, in program order: the sums stay deterministic)
  double* slot = a.partial + ((size_t)blockIdx.x * DFT_WAVES + wave) * 112 * 32;
  bool first = true;
  f32x4 acc[RTN][2];
#pragma unroll
  for (int i = 0; i < RTN; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto flush = [&]() {
    // the lane index passes through an empty asm so that the addresses are formed here
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int i = 0; i < RTN; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double* d = &slot[(i * 16 + (ln >> 4) * 4 + q) * 32 + j * 16 + (ln & 15)];
          if (first) *d = (double)acc[i][j][q];
          else unsafeAtomicAdd(d, (double)acc[i][j][q]);
          acc[i][j][q] = 0.f;
        }
    first = false;
  };
  const v4u_t* Gs = (const v4u_t*)a.Gs;
  const int ntt = M >> 4;   // a multiple of 8: every wave takes ntt / DFT_WAVES tiles per group
  const int g_beg = blockIdx.x * a.groups_per_block;
  const int g_end = min(a.ngroups, g_beg + a.groups_per_block);
  // Stage fragment f = 2 kb[j] + s2 holds the hi (s2 even) or lo part of K-step s2 / 2 of field j;
  // each lane copies its 16 bytes, and lanes whose group holds no mode of the field
  // (16 (s2 / 2) + 4 (lane / 16) > H_j) copy zeros.  The copies are buffer loads into LDS over the
  // whole fragment array (byte offsets below 2^31): unlike the global form, the compiler does not
  // count them as LDS operations, so the LDS reads issued while they are in flight keep partial
  // waits.  Wave w copies the stage fragments
  // f = w (mod DFT_WAVES), reading their offsets from the copy table with scalar loads (a table in
  // LDS would make every read wait for the copies before it; per-field arguments read field by
  // field serialise their scalar loads).
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)Gs, (short)0, (int)((unsigned)a.ngroups * (unsigned)a.kb[nbu] * 2048u), BUF_DWORD3);
  // the table is read through the constant address space, so its uniform reads are scalar loads
  typedef const __attribute__((address_space(4))) int cint_t;
  cint_t* ctab = (cint_t*)(unsigned long long)a.ctab;
  auto copy_group = [&](int g) {
    // three fragments a round: their table reads go out together (indices clamped to the table)
    for (int f0 = wave; f0 < nfr; f0 += 3 * DFT_WAVES) {
      int tx[3], ty[3], tz[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int f = min(f0 + u * DFT_WAVES, nfr - 1);
        tx[u] = ctab[4 * f]; ty[u] = ctab[4 * f + 1]; tz[u] = ctab[4 * f + 2];
      }
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int f = f0 + u * DFT_WAVES;
        if (f < nfr) {
          // lanes whose modes all lie above H_j get bit 31 set in their offset (the fragment array
          // is below 2^31 bytes), which reads past the end of the resource and returns zeros: their
          // part of the stage stays zero, and the copy needs no branch
          const unsigned above = (unsigned)(tz[u] - 4 * (lane >> 4)) >> 31;
          const unsigned off = ((unsigned)(tx[u] + g * ty[u] + lane) * 16u) | (above << 31);
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)(stage + (size_t)f * 64), 16, off, 0, 0, 0);
        }
      }
    }
  };

  __syncthreads();   // the zeroed stage is complete before any copy lands in it
  if (g_beg < g_end) copy_group(g_beg);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int since = 0;
  for (int g = g_beg; g < g_end; ++g) {
    // ntt is a multiple of DFT_WAVES: every wave has ntt / DFT_WAVES tiles
    for (int tt = wave; tt < ntt; tt += DFT_WAVES) {
      // twiddle B-fragment of step s for this lane: modes q_c = 16 s + 4 (lane / 16) + c (c = 0..3) at
      // t = 16 tt + lane % 16, i.e. e^{2 pi i q_c t / M}; step 0 comes from the table and every later
      // step is the previous one times e^{2 pi i 16 t / M} (FP32 rotations, at most seven)
      const int t = 16 * tt + r16;
      float2 wv[4];
      {
        int m = (4 * (lane >> 4) * t) % M;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          wv[c] = twf[m];
          m += t;
          if (m >= M) m -= M;
        }
      }
      const float2 rot = twf[(16 * t) % M];
      f32x4 dk[DFT_MAX_FIELDS];                                   // every field's 16 x 16 tile
#pragma unroll
      for (int j = 0; j < DFT_MAX_FIELDS; ++j) dk[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < DFT_MAX_STEPS; ++s) {
        const int cm = __builtin_amdgcn_readfirstlane(sched[s * DFT_SCHED + DFT_MAX_FIELDS]);
        if (cm != 0) {
          if (s > 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const float2 w = wv[c];
              wv[c] = make_float2(w.x * rot.x - w.y * rot.y, w.x * rot.y + w.y * rot.x);
            }
          }
          // B rows (cos, -sin) per mode, split into bf16 hi and lo parts
          uint32_t hw[4], lw[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float cs = wv[c].x, sn = -wv[c].y;
            dft_split2(cs, sn, hw[c], lw[c]);
          }
          const bf16x8 wh = __builtin_bit_cast(bf16x8, v4u_t{hw[0], hw[1], hw[2], hw[3]});
          const bf16x8 wl = __builtin_bit_cast(bf16x8, v4u_t{lw[0], lw[1], lw[2], lw[3]});
#pragma unroll
          for (int c = 0; c < DFT_MAX_FIELDS / 4; ++c) {
            if ((cm >> c) & 1) {
              const int4 fo = *(const int4*)&sched[s * DFT_SCHED + 4 * c];
              const int f[4] = {fo.x, fo.y, fo.z, fo.w};
              bf16x8 gh[4], gl[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                gh[u] = __builtin_bit_cast(bf16x8, stage[(size_t)f[u] * 64 + lane]);
                gl[u] = __builtin_bit_cast(bf16x8, stage[(size_t)(f[u] + 1) * 64 + lane]);
              }
              __builtin_amdgcn_s_setprio(1);
#pragma unroll
              for (int u = 0; u < 4; ++u) dk[4 * c + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gl[u], wh, dk[4 * c + u], 0, 0, 0);
#pragma unroll
              for (int u = 0; u < 4; ++u) dk[4 * c + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gh[u], wl, dk[4 * c + u], 0, 0, 0);
#pragma unroll
              for (int u = 0; u < 4; ++u) dk[4 * c + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gh[u], wh, dk[4 * c + u], 0, 0, 0);
              __builtin_amdgcn_s_setprio(0);
            }
          }
        }
      }
      if (tt + DFT_WAVES >= ntt) {
        // the group's last synthesis on every wave: the fragments of the next group may land
        __syncthreads();
        if (g + 1 < g_end) copy_group(g + 1);
      }
      dft_contract_tile<RTN>(sF, dk, oa, ob, oc, a.ct1_tiles, acc);
      since += 256;
      if (since >= a.flush_vox) { since = 0; flush(); }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  flush();
  // sum the block's wave slots into the first one, in wave order (rows past the pair tiles stay
  // zero); the reduction over blocks then reads one slot per block
  __syncthreads();
  double* bslot = a.partial + (size_t)blockIdx.x * DFT_WAVES * 112 * 32;
  for (int e = tid; e < RTN * 16 * 32; e += DFT_WAVES * 64) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < DFT_WAVES; ++w)   // read at device scope: the adds were made at L2
      v += __hip_atomic_load(&bslot[(size_t)w * 112 * 32 + e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bslot[e] = v;
  }
}

// Sum the per-block partial sums: out[e] = sum_p partial[p][e] (fixed order, coalesced).
// Two fixed-order stages: first every group of RGROUP consecutive parts is summed into the group's
// first slot (in place), then the group sums are added in group order.
// Parts are pstride slots apart; only the first nent entries of each are summed (the rows of the
// pair tiles in use), the rest of `out` is cleared.
constexpr int RGROUP = kReduceGroup;
__global__ void k3_reduce_groups(double* __restrict__ partial, int nparts, int pstride, int nent) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  const int p0 = blockIdx.y * RGROUP, p1 = min(nparts, p0 + RGROUP);
  double s = 0.0;
  for (int p = p0; p < p1; ++p) s += partial[(size_t)p * pstride * 112 * 32 + e];
  partial[(size_t)p0 * pstride * 112 * 32 + e] = s;
}
__global__ void k3_reduce_parts(const double* __restrict__ partial, int nparts, int pstride, int nent,
                                double* __restrict__ out) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 112 * 32) return;
  double s = 0.0;
  if (e < nent)
    for (int p = 0; p < nparts; p += RGROUP) s += partial[(size_t)p * pstride * 112 * 32 + e];
  out[e] = s;
}

// --------------------------------------------------------------- finalisation
__global__ void k3_fin(Fin3Args a) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.ntri) return;
  int idx = a.tri_pair[t] * 32 + a.tri_col[t];
  double s = a.partial[idx] * a.sfac;   // partial holds the reduced sums here
  if (!a.T3D) {
    a.Ssum[t] = s;
    return;
  }
  int64_t T = a.T3D[t];
  double neff = (double)T * a.rho3;
  a.N[t] = T;
  if (a.Neff) a.Neff[t] = neff;
  a.B[t] = (T > 0 && neff > 0) ? a.norm * a.nvox * s / neff : __builtin_nan("");
}

}  // namespace

// ----------------------------------------------------------------- launchers
template <typename T>
static void set_lds(const void* f, size_t lds) {
  (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int IP>
static void launch_delay3_t(const Delay3Args& a, hipStream_t s, size_t lds) {
  set_lds<T>((const void*)k3_delay<T, IP>, lds);
  hipLaunchKernelGGL((k3_delay<T, IP>), dim3((a.g.nvb + a.NL - 1) / a.NL * a.g.nub), dim3(256), lds, s, a);
}
template <typename T>
static void launch_delay3_ip(const Delay3Args& a, hipStream_t s, size_t lds) {
  if (a.ip == 2) launch_delay3_t<T, 2>(a, s, lds);
  else if (a.ip == 4) launch_delay3_t<T, 4>(a, s, lds);
  else launch_delay3_t<T, 0>(a, s, lds);
}
void launch_delay3_f32(const Delay3Args& a, hipStream_t s, size_t lds) { launch_delay3_ip<float>(a, s, lds); }
void launch_delay3_f64(const Delay3Args& a, hipStream_t s, size_t lds) { launch_delay3_ip<double>(a, s, lds); }
template <typename T, int IP>
static void launch_pass3_t(bool upass, const Pass3Args& a, int nwork, hipStream_t s, size_t lds) {
  const void* f = upass ? (const void*)k3_upass<T, IP> : (const void*)k3_vpass<T, IP>;
  set_lds<T>(f, lds);
  if (upass) hipLaunchKernelGGL((k3_upass<T, IP>), dim3(nwork), dim3(256), lds, s, a);
  else hipLaunchKernelGGL((k3_vpass<T, IP>), dim3(nwork), dim3(256), lds, s, a);
}
template <typename T>
static void launch_pass3_ip(bool upass, const Pass3Args& a, int nwork, hipStream_t s, size_t lds) {
  if (a.ip == 2) launch_pass3_t<T, 2>(upass, a, nwork, s, lds);
  else if (a.ip == 4) launch_pass3_t<T, 4>(upass, a, nwork, s, lds);
  else launch_pass3_t<T, 0>(upass, a, nwork, s, lds);
}
void launch_vpass3(const Pass3Args& a, int nwork, bool fp64, hipStream_t s, size_t lds) {
  if (nwork <= 0) return;
  if (fp64) launch_pass3_ip<double>(false, a, nwork, s, lds);
  else launch_pass3_ip<float>(false, a, nwork, s, lds);
}
void launch_upass3(const Pass3Args& a, int nwork, bool fp64, hipStream_t s, size_t lds) {
  if (nwork <= 0) return;
  if (fp64) launch_pass3_ip<double>(true, a, nwork, s, lds);
  else launch_pass3_ip<float>(true, a, nwork, s, lds);
}
void launch_etapass3(const Pass3Args& a, int nwork, bool fp64, hipStream_t s, size_t lds) {
  if (nwork <= 0) return;
  if (fp64) { set_lds<double>((const void*)k3_etapass<double>, lds); hipLaunchKernelGGL(k3_etapass<double>, dim3(nwork), dim3(256), lds, s, a); }
  else { set_lds<float>((const void*)k3_etapass<float>, lds); hipLaunchKernelGGL(k3_etapass<float>, dim3(nwork), dim3(256), lds, s, a); }
}
void launch_contract3(const Con3Args& a, int mode, int nblocks, hipStream_t s) {
  if (mode == 0) hipLaunchKernelGGL((k3_contract<0, double>), dim3(nblocks), dim3(256), 0, s, a);
  else if (mode == 1) hipLaunchKernelGGL((k3_contract<1, float>), dim3(nblocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k3_contract<2, float>), dim3(nblocks), dim3(256), 0, s, a);
}
void launch_fin3(const Fin3Args& a, double* reduced, hipStream_t s) {
  const int groups = (a.nparts + RGROUP - 1) / RGROUP;
  const int ps = a.pstride > 0 ? a.pstride : 1, ne = a.nent > 0 ? a.nent : 112 * 32;
  hipLaunchKernelGGL(k3_reduce_groups, dim3((ne + 255) / 256, groups), dim3(256), 0, s, (double*)a.partial, a.nparts,
                     ps, ne);
  hipLaunchKernelGGL(k3_reduce_parts, dim3((112 * 32 + 255) / 256), dim3(256), 0, s, a.partial, a.nparts, ps, ne,
                     reduced);
  Fin3Args b = a;
  b.partial = reduced;
  if (a.ntri > 0) hipLaunchKernelGGL(k3_fin, dim3((a.ntri + 127) / 128), dim3(128), 0, s, b);
}
template <int RTN>
static void launch_dft3_rt(const Dft3Args& a, int nblocks, size_t lds, hipStream_t s) {
  (void)hipFuncSetAttribute((const void*)k3_dft<RTN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k3_dft<RTN>, dim3(nblocks), dim3(DFT_WAVES * 64), lds, s, a);
}
void launch_dft3(const Dft3Args& a, int nblocks, size_t lds, hipStream_t s) {
  switch ((a.npairs + 15) / 16) {
    case 1: launch_dft3_rt<1>(a, nblocks, lds, s); break;
    case 2: launch_dft3_rt<2>(a, nblocks, lds, s); break;
    case 3: launch_dft3_rt<3>(a, nblocks, lds, s); break;
    case 4: launch_dft3_rt<4>(a, nblocks, lds, s); break;
    case 5: launch_dft3_rt<5>(a, nblocks, lds, s); break;
    case 6: launch_dft3_rt<6>(a, nblocks, lds, s); break;
    default: launch_dft3_rt<7>(a, nblocks, lds, s); break;
  }
}
void launch_fused3(const Fused3Args& a, int mode, int nblocks, size_t lds, hipStream_t s) {
  if (mode == 1) {
    (void)hipFuncSetAttribute((const void*)k3_fused<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k3_fused<1>, dim3(nblocks), dim3(256), lds, s, a);
  } else {
    (void)hipFuncSetAttribute((const void*)k3_fused<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k3_fused<2>, dim3(nblocks), dim3(256), lds, s, a);
  }
}
