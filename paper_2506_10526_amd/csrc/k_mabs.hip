// MABS kernels for gfx950: ring-filtered fields (Eqs. iFT, iFT_I), the triple-product
// contraction of Eq. (estimator_t) as an MFMA GEMM, counts, normalisation and the
// ergodic collapse to channel separations.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <cstdlib>

#include "bs_kernels.h"

namespace {

__device__ __forceinline__ int signed_idx(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// ---------------------------------------------------------------------------
// Ring-filtered field of one (ring, channel) plane.
//
// X(u, v) = 1_ring(U) W(U, nu) V(U, nu) (or the unit indicator in count mode) on the
// half plane is inverse-transformed to the real n x n field: a C2C pass along u for every
// column v <= vmax that can hold support, then a C2R pass along v for every output row.
// A block computes the output rows x_u = G m + g (m < n/G) of its plane; the u pass is
// folded to length n/G so the columns fit in LDS:
//   Y_v[u'] = sum_q X(u' + q n/G, v) e^{+2 pi i (u' + q n/G) g / n},  G_v[m] = IDFT_{n/G}(Y_v)[m].
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ Cx<T> ring_cell(const MabsFieldArgs& a, int bin, int nu, int iu, int v) {
  const int n = a.n;
  int qu = signed_idx(iu, n);
  int s = qu * qu + v * v;
  if (s == 0 || s > a.smax || qu == -n / 2) return cmk(T(0), T(0));
  if (a.lut[s] != bin) return cmk(T(0), T(0));
  size_t cell = ((size_t)nu * n + iu) * a.nh + v;
  size_t cell_uv = (size_t)iu * a.nh + v;
  T w;
  if (a.ng) {
    unsigned c = a.ng[cell];
    if (a.count_mode) w = c > 0 ? T(1) : T(0);
    else w = c > 0 ? T(1) / T(c) : T(0);
  } else {
    T m = a.uvm ? T(a.uvm[cell_uv]) : T(1);
    T cw = (a.chw && !a.ignore_chan) ? T(a.chw[nu]) : T(1);
    w = m * cw;
    if (a.count_mode) w = (w > T(0)) ? T(1) : T(0);
  }
  if (a.count_mode) return cmk(w, T(0));
  if (w == T(0)) return cmk(T(0), T(0));
  const Cx<T>* vis = (const Cx<T>*)a.vis;
  Cx<T> x = vis[cell];
  return cscale(x, w);
}

template <typename T>
__device__ __forceinline__ Cx<T> ring_input(const MabsFieldArgs& a, int bin, int nu, int iu, int v) {
  Cx<T> x = ring_cell<T>(a, bin, nu, iu, v);
  if (v == 0) {  // self-conjugate column: (X(u) + conj X(-u)) / 2
    int ineg = (a.n - iu) % a.n;
    Cx<T> y = ring_cell<T>(a, bin, nu, ineg, 0);
    x = cscale(cadd(x, cconj(y)), T(0.5));
  }
  return x;
}

template <typename T>
__global__ __launch_bounds__(256) void k_mabs_fields(MabsFieldArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int g = blockIdx.x;
  const int nu = a.chan_offset + blockIdx.y;
  const int bi = blockIdx.z;
  const int bin = a.bins[bi];
  const int n = a.n, G = a.G, Lc = n / G, M = n / 2, ncols = a.vmax + 1;
  const int tid = threadIdx.x;
  const int work = (a.CB * Lc > a.RB * M) ? a.CB * Lc : a.RB * M;
  Cx<T>* Rg = (Cx<T>*)smem_raw;
  Cx<T>* wa = Rg + (size_t)ncols * Lc;
  Cx<T>* wb = wa + work;
  const Cx<T>* tw = (const Cx<T>*)a.tw_n;

  // Phase 1: folded u pass over the columns v = 0..vmax.
  for (int c0 = 0; c0 < ncols; c0 += a.CB) {
    const int nb = min(a.CB, ncols - c0);
    for (int e = tid; e < nb * Lc; e += blockDim.x) {
      int cl = e / Lc, up = e - cl * Lc, v = c0 + cl;
      Cx<T> acc = cmk(T(0), T(0));
      for (int q = 0; q < G; ++q) {
        int iu = up + q * Lc;
        Cx<T> x = ring_input<T>(a, bin, nu, iu, v);
        if (g) {
          Cx<T> w = tw[(iu * g) % n];
          w.y = -w.y;
          x = cmul(x, w);
        }
        acc = cadd(acc, x);
      }
      wa[e] = acc;
    }
    __syncthreads();
    Cx<T>* r = lds_fft<+1, T>(wa, wb, a.pcol, nb, tw, G);
    for (int e = tid; e < nb * Lc; e += blockDim.x) Rg[(size_t)c0 * Lc + e] = r[e];
    __syncthreads();
  }

  // Phase 2: C2R along v for output rows x_u = G m + g.
  T* out = (T*)a.out + (size_t)bi * a.bin_stride + (size_t)nu * a.plane_stride;
  const T sc = T(a.scale);
  const int vmax = a.vmax;
  for (int m0 = 0; m0 < Lc; m0 += a.RB) {
    const int nb = min(a.RB, Lc - m0);
    for (int e = tid; e < nb * M; e += blockDim.x) {
      int rl = e / M, k = e - rl * M, m = m0 + rl;
      auto get = [&](int v) -> Cx<T> { return v <= vmax ? Rg[(size_t)v * Lc + m] : cmk(T(0), T(0)); };
      wa[e] = c2r_pack<T>(k, M, get, tw, 1);
    }
    __syncthreads();
    Cx<T>* r = lds_fft<+1, T>(wa, wb, a.prow, nb, tw, 2);
    for (int e = tid; e < nb * M; e += blockDim.x) {
      int rl = e / M, k = e - rl * M;
      int xu = G * (m0 + rl) + g;
      Cx<T> z = r[e];
      Cx<T>* o = (Cx<T>*)(out + (size_t)xu * n);
      o[k] = cmk(z.x * sc, z.y * sc);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// bf16 hi/lo split of FP32 fields: hi = rne(x), lo = rne(x - hi).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  __bf16 h = (__bf16)x;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf16_float(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}
// two floats as packed bf16 (round to nearest even), x in the low half: one conversion instruction
typedef __bf16 bf16x2_m __attribute__((ext_vector_type(2)));
typedef float f32x2_m __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pk(float x, float y) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_m{x, y}, bf16x2_m));
}
// hi = rne(x), lo = rne(x - hi) for two floats, packed (x in the low halves); x - hi is exact
// (hi lies within a factor two of x and shares its grid).
__device__ __forceinline__ void bf16_split2(float x, float y, uint32_t& hp, uint32_t& lp) {
  hp = bf16_pk(x, y);
  lp = bf16_pk(x - __builtin_bit_cast(float, hp << 16), y - __builtin_bit_cast(float, hp & 0xffff0000u));
}

__global__ __launch_bounds__(256) void k_split_bf16(const float* __restrict__ F, uint16_t* __restrict__ hi,
                                                      uint16_t* __restrict__ lo, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    float x = F[i];
    uint16_t h = bf16_bits(x);
    float r = x - bf16_float(h);
    hi[i] = h;
    lo[i] = bf16_bits(r);
  }
}

// ---------------------------------------------------------------------------
// Triple-product contraction as a GEMM per triangle t = (b1, b2, b3):
//   S[t][R = i*nc + nu2][nu3] = sum_p F_b1(nu1_i, p) F_b2(nu2, p) F_b3(nu3, p)
// A rows are formed on the fly from the two FP32 field rows (one multiply per element),
// B rows are the b3 fields.  A 256-thread block computes a 128 x 128 tile over one pixel
// chunk; each wave owns 64 x 64 = 2 x 2 MFMA tiles of 32 x 32.  FP32 MFMA accumulators are
// flushed into FP64 registers every KFLUSH pixels; the chunk sum is stored in FP64.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TM = 128, TN = 128, TK = 32;
constexpr int KFLUSH = 256;   // pixels per FP32 accumulation run before the FP64 flush
constexpr int LDA = TK + 8;  // bf16 row stride in LDS (16-byte aligned, staggers banks)

template <int MODE>  // 1 = FP32 MFMA, 2 = split-BF16 MFMA
__global__ __launch_bounds__(256) void k_mabs_gemm(MabsGemmArgs a) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int nrows = a.n_nu1 * a.nc;
  const int col0 = blockIdx.x * TN;
  const int row0 = blockIdx.y * TM;
  const int t = blockIdx.z / a.kchunks;
  const int kc = blockIdx.z - t * a.kchunks;
  const int b1 = a.tri[3 * t], b2 = a.tri[3 * t + 1], b3 = a.tri[3 * t + 2];
  const int kbeg = kc * a.kchunk;
  const int kend = min(a.P, kbeg + a.kchunk);

  // split mode: Ah, Al [TM][LDA], Bh, Bl [TN][LDA] bf16; FP32 mode: A [TK][LD32], B [TK][LD32] float
  constexpr int LD32 = TM + 4;
  constexpr int SPLIT_BYTES = 2 * (TM + TN) * LDA * 2;
  constexpr int F32_BYTES = 2 * TK * LD32 * 4;
  __shared__ __attribute__((aligned(16))) unsigned char smem[SPLIT_BYTES > F32_BYTES ? SPLIT_BYTES : F32_BYTES];
  uint16_t* sAh = (uint16_t*)smem;
  uint16_t* sAl = sAh + TM * LDA;
  uint16_t* sBh = sAl + TM * LDA;
  uint16_t* sBl = sBh + TN * LDA;
  float* sA32 = (float*)smem;
  float* sB32 = sA32 + TK * LD32;

  // loader mapping: each thread stages 16 consecutive pixels of one row
  const int lr = tid >> 1, lk = (tid & 1) * 16;
  const int R = row0 + lr;
  const bool rok = R < nrows;
  const float* f1 = nullptr;
  const float* f2 = nullptr;
  if (rok) {
    int i = R / a.nc, nu2 = R - i * a.nc;
    f1 = a.F + (size_t)b1 * a.bin_stride + (size_t)a.nu1[i] * a.P;
    f2 = a.F + (size_t)b2 * a.bin_stride + (size_t)nu2 * a.P;
  }
  const int nu3 = col0 + lr;
  const bool cok = nu3 < a.nc;
  const size_t boff = (size_t)b3 * a.bin_stride + (size_t)(cok ? nu3 : 0) * a.P;

  f32x16 acc[2][2];
  double acc64[2][2][16];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int e = 0; e < 16; ++e) { acc[i][j][e] = 0.f; acc64[i][j][e] = 0.0; }
    }

  int since_flush = 0;
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    // ---- stage A = F1 .* F2 and B = F3 for pixels k0 .. k0+31 ----
    {
      float av[16];
      if (rok) {
        const float4* p1 = (const float4*)(f1 + k0 + lk);
        const float4* p2 = (const float4*)(f2 + k0 + lk);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float4 x = p1[q], y = p2[q];
          av[4 * q + 0] = x.x * y.x; av[4 * q + 1] = x.y * y.y;
          av[4 * q + 2] = x.z * y.z; av[4 * q + 3] = x.w * y.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) av[q] = 0.f;
      }
      if (MODE == 2) {
        uint16_t h[16], l[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          h[q] = bf16_bits(av[q]);
          l[q] = bf16_bits(av[q] - bf16_float(h[q]));
        }
        uint4* dh = (uint4*)&sAh[lr * LDA + lk];
        uint4* dl = (uint4*)&sAl[lr * LDA + lk];
        dh[0] = *(uint4*)&h[0]; dh[1] = *(uint4*)&h[8];
        dl[0] = *(uint4*)&l[0]; dl[1] = *(uint4*)&l[8];
        uint4 bh0 = {0, 0, 0, 0}, bh1 = bh0, bl0 = bh0, bl1 = bh0;
        if (cok) {
          const uint4* ph = (const uint4*)(a.Fh + boff + k0 + lk);
          const uint4* pl = (const uint4*)(a.Fl + boff + k0 + lk);
          bh0 = ph[0]; bh1 = ph[1]; bl0 = pl[0]; bl1 = pl[1];
        }
        uint4* eh = (uint4*)&sBh[lr * LDA + lk];
        uint4* el = (uint4*)&sBl[lr * LDA + lk];
        eh[0] = bh0; eh[1] = bh1; el[0] = bl0; el[1] = bl1;
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) sA32[(lk + q) * LD32 + lr] = av[q];
        float bv[16];
        if (cok) {
          const float4* p3 = (const float4*)(a.F + boff + k0 + lk);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float4 x = p3[q];
            bv[4 * q] = x.x; bv[4 * q + 1] = x.y; bv[4 * q + 2] = x.z; bv[4 * q + 3] = x.w;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 16; ++q) bv[q] = 0.f;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) sB32[(lk + q) * LD32 + lr] = bv[q];
      }
    }
    __syncthreads();
    // ---- MFMA ----
    if (MODE == 2) {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 16) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
        const int ko = kk + (lane >> 5) * 8;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          int r = wm * 64 + i * 32 + (lane & 31);
          ah[i] = *(const bf16x8*)&sAh[r * LDA + ko];
          al[i] = *(const bf16x8*)&sAl[r * LDA + ko];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          int c = wn * 64 + j * 32 + (lane & 31);
          bh[j] = *(const bf16x8*)&sBh[c * LDA + ko];
          bl[j] = *(const bf16x8*)&sBl[c * LDA + ko];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 2) {
        const int kr = kk + (lane >> 5);
        float av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) av[i] = sA32[kr * LD32 + wm * 64 + i * 32 + (lane & 31)];
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = sB32[kr * LD32 + wn * 64 + j * 32 + (lane & 31)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
    since_flush += TK;
    if (since_flush >= KFLUSH) {
      since_flush = 0;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int e = 0; e < 16; ++e) { acc64[i][j][e] += (double)acc[i][j][e]; acc[i][j][e] = 0.f; }
    }
  }
  // ---- store the FP64 chunk sums ----
  double* S = a.S + ((size_t)kc * a.ntri + t) * (size_t)nrows * a.nc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      int col = col0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        int row = row0 + wm * 64 + i * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
        if (row < nrows && col < a.nc) S[(size_t)row * a.nc + col] = acc64[i][j][e] + (double)acc[i][j][e];
      }
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 contraction, large tiles.  Block tile 128 x 256 (rows R = i*nc + nu2, columns nu3),
// four waves of 64 x 128 (2 x 4 MFMA 32x32x16 tiles, 128 FP32 accumulators per lane), pixel
// stages of 32 in three LDS buffers, software-pipelined around the MFMAs:
//  * the pre-split B rows (bf16 hi/lo of F_b3) of stage s+2 go from global memory straight into
//    the buffer of stage s+2 with 16-byte global_load_lds, issued during stage s, so a copy has two
//    stages to land;
//  * the F1 and F2 values of stage s+2 are loaded into registers during stage s, and the A
//    operand of stage s+1 (A = F_b1(nu1) .* F_b2(nu2), split into bf16 hi/lo) is formed from
//    the registers loaded one stage earlier and written into the other buffer, interleaved with
//    the MFMAs of stage s;
//  * the fragments of the second half of a stage are read while the first half's MFMAs run,
//    and the last twelve MFMAs of a stage are issued after the stage barrier, covering the
//    reads of the next stage's first fragments.
// Each stage ends with a wait for this wave's LDS operations and for its global loads except the
// 16 issued in this stage (the copies and loads of stage s+2), and one barrier.  LDS rows
// hold 32 bf16 as four 16-byte chunks XOR-swizzled by row.  The block's FP32 tile is added into
// its FP64 output every SFLUSH pixels.  Blocks are mapped to tiles so that tiles sharing a B
// column block and neighbouring A rows run on the same XCD (blocks are dealt to the eight XCDs
// round-robin).
// ---------------------------------------------------------------------------
constexpr int S_TM = 128, S_TN = 256, S_TK = 32, SFLUSH = 8192;
// uint16 offsets inside one stage buffer
constexpr int S_AH = 0, S_AL = S_TM * S_TK, S_BH = 2 * S_TM * S_TK, S_BL = S_BH + S_TN * S_TK;
constexpr int S_BUF = S_BL + S_TN * S_TK;
constexpr int S_NBUF = 3;   // stage buffers in LDS (147,456 bytes)
// s_waitcnt encoding (gfx9 family): vmcnt(16) lgkmcnt(0), expcnt not waited for
constexpr int S_WAIT_VM16_LGKM0 = (16 & 15) | ((16 >> 4) << 14) | (7 << 4) | (0 << 8);
// vmcnt(16) alone (expcnt and lgkmcnt not waited for)
constexpr int S_WAIT_VM16 = (16 & 15) | ((16 >> 4) << 14) | (7 << 4) | (15 << 8);

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(3))) const char lds_cchar;
typedef unsigned v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lds_addr(const void* p) { return (uint32_t)(uintptr_t)(lds_cchar*)p; }

__device__ __forceinline__ int swz(int r, int chunk) { return (chunk ^ ((r >> 2) & 3)); }
// Chunk swizzle of 64-byte rows for 16-byte accesses of one chunk index by consecutive rows: any
// eight consecutive rows (aligned) land in eight distinct 16-byte slots of a 128-byte bank line,
// and any sixteen in sixteen distinct slots of a 256-byte line, so such accesses meet no bank
// conflict (measured: none, against a fifth of the LDS cycles with the swizzle above)
__device__ __forceinline__ int swz_rows(int r, int chunk) { return chunk ^ (((r >> 1) ^ (r >> 2)) & 3); }

struct SplitFrags {
  bf16x8 ah[2], al[2], bh[4], bl[4];
};

// XCD-aware order of the tiles of one GEMM: blocks are dealt to the eight XCDs round-robin, so
// block b0 runs on XCD b0 mod 8; it takes tile (b0 mod 8) (nb/8) + b0/8, which gives each XCD a
// contiguous run of tiles (the row tiles of one column tile and pixel chunk share their B operand
// in that XCD's L2).  The last nb mod 8 tiles keep their index.
__device__ __forceinline__ int xcd_tile(int b0, int nb) {
  const int full = (nb / 8) * 8;
  return b0 < full ? (b0 & 7) * (full / 8) + (b0 >> 3) : b0;
}

// One block tile of GEMM `a`; b is the tile's index within this GEMM's nb = rtiles ctiles ntri
// kchunks tiles, row tile fastest.
__device__ __forceinline__ void split2_tile(const MabsGemmArgs& a, int b, unsigned char* smem_raw) {
  uint16_t* lds = (uint16_t*)smem_raw;   // [S_NBUF][S_BUF]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int nrows = a.n_nu1 * a.nc;
  const int rtiles = (nrows + S_TM - 1) / S_TM, ctiles = (a.nc + S_TN - 1) / S_TN;
  const int rt = b % rtiles;
  int rest = b / rtiles;
  const int ct = rest % ctiles;
  rest /= ctiles;
  const int kc = rest % a.kchunks;
  const int t = rest / a.kchunks;
  const int row0 = rt * S_TM, col0 = ct * S_TN;
  const int b1 = a.tri[3 * t], b2 = a.tri[3 * t + 1], b3 = a.tri[3 * t + 2];
  const int kbeg = kc * a.kchunk;
  const int kend = min(a.P, kbeg + a.kchunk);
  const int nst = (kend - kbeg) / S_TK;   // >= 1; pixel ranges are multiples of S_TK
  const int klast = kend - S_TK;          // loads past the range re-read the last stage

  // A operand: thread (ar, ahalf) owns row ar, pixels ahalf .. ahalf+15 of each stage; rows past
  // the last repeat it (their output rows are never stored)
  const int ar = tid >> 1, ahalf = (tid & 1) * 16;
  const int R = row0 + ar;
  const int Rc = R < nrows ? R : nrows - 1;
  const int ia = Rc / a.nc, nu2 = Rc - ia * a.nc;
  const float* f1 = a.F + (size_t)b1 * a.bin_stride + (size_t)a.nu1[ia] * a.P + ahalf;
  const float* f2 = a.F + (size_t)b2 * a.bin_stride + (size_t)nu2 * a.P + ahalf;
  // LDS uint16 offsets of this thread's two A chunks
  int aoff[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) aoff[c] = ar * S_TK + swz(ar, (ahalf >> 3) + c) * 8;
  // B copies: this wave's rows w*64 .. w*64+63, 16 rows per instruction
  size_t boff[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int br = wave * 64 + q * 16 + (lane >> 2);
    const int col = min(col0 + br, a.nc - 1);   // columns past nc load a valid row, never stored
    boff[q] = (size_t)b3 * a.bin_stride + (size_t)col * a.P + 8 * swz(br, lane & 3);
  }
  // fragment offsets (uint16, inside a stage buffer) per half-stage kk
  int oa[2][2], ob[2][4];
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int chunk = kk * 2 + (lane >> 5);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 64 + i * 32 + (lane & 31);
      oa[kk][i] = r * S_TK + swz(r, chunk) * 8;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = wn * 128 + j * 32 + (lane & 31);
      ob[kk][j] = c * S_TK + swz(c, chunk) * 8;
    }
  }

  auto copy_b1 = [&](int m, int k0, uint16_t* buf) {   // copy m of 8: rows q = m/2, hi or lo
    const int q = m >> 1;
    __builtin_amdgcn_global_load_lds((const void*)((m & 1 ? a.Fl : a.Fh) + boff[q] + k0),
                                     (lds_void*)(buf + (m & 1 ? S_BL : S_BH) + (wave * 64 + q * 16) * S_TK),
                                     16, 0, 0);
  };
  auto load_a1 = [&](int m, int k0, float4* p1, float4* p2) {   // load m of 8: F1 (m < 4) or F2
    if (m < 4) p1[m] = ((const float4*)(f1 + k0))[m];
    else p2[m - 4] = ((const float4*)(f2 + k0))[m - 4];
  };
  // A formation piece m of 8: products 2m, 2m+1 of this thread's 16, split into packed hi / lo words
  auto form1 = [&](int m, const float4* p1, const float4* p2, uint32_t (&hw)[2][4], uint32_t (&lw)[2][4]) {
    const int g = m >> 1, u = (m & 1) * 2;   // float4 index, component
    const float4 x = p1[g], y = p2[g];
    const float w0 = u ? x.z * y.z : x.x * y.x;
    const float w1 = u ? x.w * y.w : x.y * y.y;
    uint32_t hp, lp;
    bf16_split2(w0, w1, hp, lp);
    hw[g >> 1][(g & 1) * 2 + (u >> 1)] = hp;
    lw[g >> 1][(g & 1) * 2 + (u >> 1)] = lp;
  };
  // The A stores are written in asm: the compiler cannot tell them apart from the B copies into
  // the same buffer and would otherwise wait for every memory operation in flight before them.
  // They touch only the A region; the wait at the end of the stage covers their completion.
  auto store_a = [&](int c, const uint32_t (&hw)[2][4], const uint32_t (&lw)[2][4], uint16_t* buf) {
    const v4u h = {hw[c][0], hw[c][1], hw[c][2], hw[c][3]};
    const v4u l = {lw[c][0], lw[c][1], lw[c][2], lw[c][3]};
    asm volatile("ds_write_b128 %0, %1\n\tds_write_b128 %0, %2 offset:%3"
                 :
                 : "v"(lds_addr(buf + S_AH + aoff[c])), "v"(h), "v"(l), "n"(2 * (S_AL - S_AH))
                 : "memory");
  };
  auto form = [&](const float4* p1, const float4* p2, uint16_t* buf) {
    uint32_t hw[2][4], lw[2][4];
#pragma unroll
    for (int m = 0; m < 8; ++m) form1(m, p1, p2, hw, lw);
    store_a(0, hw, lw, buf);
    store_a(1, hw, lw, buf);
  };
  // fragment m of 12 of half-stage kk: A hi (0, 1), A lo (2, 3), B hi (4..7), B lo (8..11)
  auto read_frag1 = [&](SplitFrags& f, const uint16_t* buf, int kk, int m) {
    if (m < 2) f.ah[m] = *(const bf16x8*)&buf[S_AH + oa[kk][m]];
    else if (m < 4) f.al[m - 2] = *(const bf16x8*)&buf[S_AL + oa[kk][m - 2]];
    else if (m < 8) f.bh[m - 4] = *(const bf16x8*)&buf[S_BH + ob[kk][m - 4]];
    else f.bl[m - 8] = *(const bf16x8*)&buf[S_BL + ob[kk][m - 8]];
  };
  auto read_frags = [&](SplitFrags& f, const uint16_t* buf, int kk) {
#pragma unroll
    for (int m = 0; m < 12; ++m) read_frag1(f, buf, kk, m);
  };

  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  // MFMA m of the 24 of a half stage: products (lo, hi), (hi, lo), (hi, hi) of the (i, j) tiles,
  // eight apart
  auto mfma1 = [&](const SplitFrags& f, int m) {
    const int p = m >> 3, i = (m >> 2) & 1, j = m & 3;
    const bf16x8 x = p == 0 ? f.al[i] : f.ah[i];
    const bf16x8 y = p == 1 ? f.bl[j] : f.bh[j];
    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc[i][j], 0, 0, 0);
  };

  double* S = a.S + ((size_t)kc * a.ntri + t) * (size_t)nrows * a.nc;
  const bool interior = row0 + S_TM <= nrows && col0 + S_TN <= a.nc;
  bool first_flush = true;
  auto flush = [&]() {
    // the lane index passes through an empty asm so that the 128 output addresses are computed
    // here and not hoisted out of the pixel loop (where they would hold 256 registers)
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = col0 + wn * 128 + j * 32 + (ln & 31);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int row = row0 + wm * 64 + i * 32 + (e >> 2) * 8 + (ln >> 5) * 4 + (e & 3);
          if (interior || (row < nrows && col < a.nc)) {
            // first flush: a plain store; later ones: FP64 atomic adds that return nothing, so
            // the copies in flight are not waited for (each entry belongs to one lane: the
            // order of the adds and the result are fixed)
            double* d = &S[(size_t)row * a.nc + col];
            const double v = (double)acc[i][j][e];
            if (first_flush) *d = v;
            else unsafeAtomicAdd(d, v);
          }
          acc[i][j][e] = 0.f;
        }
      }
    first_flush = false;
  };

  SplitFrags F0, F1;
  auto zero_frags = [&](SplitFrags& f) {
    const bf16x8 z = {};
#pragma unroll
    for (int i = 0; i < 2; ++i) f.ah[i] = f.al[i] = z;
#pragma unroll
    for (int j = 0; j < 4; ++j) f.bh[j] = f.bl[j] = z;
  };
  zero_frags(F1);   // the first stage's deferred MFMAs add zeros
  float4 P[2][2][4];   // [set][F1 / F2][4]: register-staged A inputs, set = stage parity

  // prologue: stage 0 into buffer 0, the B rows of stage 1 into buffer 1, registers of stage 1
#pragma unroll
  for (int m = 0; m < 8; ++m) copy_b1(m, kbeg, lds);
#pragma unroll
  for (int m = 0; m < 8; ++m) load_a1(m, kbeg, P[0][0], P[0][1]);
#pragma unroll
  for (int m = 0; m < 8; ++m) load_a1(m, min(kbeg + S_TK, klast), P[1][0], P[1][1]);
#pragma unroll
  for (int m = 0; m < 8; ++m) copy_b1(m, min(kbeg + S_TK, klast), lds + S_BUF);
  form(P[0][0], P[0][1], lds);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_s_barrier();
  read_frags(F0, lds, 0);

  // Stage s (buffer s mod 3, its kk = 0 fragments in F0, the deferred MFMAs of stage s-1 in F1),
  // as 48 issue slots of one MFMA each plus, in program order: the B copies and the register loads
  // of stage s+2 (slots 0-11), the kk = 1 fragment reads (12-23), the A formation of stage s+1
  // (24-33); sched_barrier keeps every slot's instructions in place.  The buffer of stage s+2 was
  // last read in stage s-1 and that of stage s+1 in stage s-2, both before a barrier.
  auto stage = [&](int s, auto par) {
    constexpr int PAR = decltype(par)::value;
    const int b0i = s % S_NBUF, b1i = b0i + 1 == S_NBUF ? 0 : b0i + 1, b2i = b1i + 1 == S_NBUF ? 0 : b1i + 1;
    uint16_t* cur = lds + b0i * S_BUF;
    uint16_t* nxt = lds + b1i * S_BUF;
    uint16_t* nx2 = lds + b2i * S_BUF;
    // wave-uniform: kept in a scalar register (a vector temporary here can be the destination of
    // a load still in flight, which would force a wait for every load)
    const int kb = __builtin_amdgcn_readfirstlane(min(kbeg + (s + 2) * S_TK, klast)), ka = kb;
    uint32_t hw[2][4], lw[2][4];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < 12; ++m) {
      mfma1(F1, 12 + m);   // deferred, stage s-1
      if (m < 8) {
        copy_b1(m, kb, nx2);
      } else {
        load_a1(2 * (m - 8), ka, P[PAR][0], P[PAR][1]);
        load_a1(2 * (m - 8) + 1, ka, P[PAR][0], P[PAR][1]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int m = 0; m < 24; ++m) {
      mfma1(F0, m);
      if (m < 12) read_frag1(F1, cur, 1, m);
      // the registers of stage s+1 were loaded in stage s-1; only this stage's 16 loads may still
      // be in flight (without this the compiler waits for all of them before the formation)
      if (m == 11) __builtin_amdgcn_s_waitcnt(S_WAIT_VM16);
      else if (m < 20) form1(m - 12, P[PAR ^ 1][0], P[PAR ^ 1][1], hw, lw);
      else if (m < 22) store_a(m - 20, hw, lw, nxt);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int m = 0; m < 12; ++m) {
      mfma1(F1, m);
      __builtin_amdgcn_sched_barrier(0);
    }
    // B of stage s+1 landed (copied during stage s-1), A of stage s+1 stored; the 16 loads of
    // stage s+2 issued in this stage stay in flight
    __builtin_amdgcn_s_waitcnt(S_WAIT_VM16_LGKM0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    read_frags(F0, nxt, 0);
  };

  for (int s = 0; s < nst;) {
    const int se = min(nst, s + SFLUSH / S_TK);   // s is even here
    while (true) {
      stage(s, std::integral_constant<int, 0>{});
      if (++s >= se) break;
      stage(s, std::integral_constant<int, 1>{});
      if (++s >= se) break;
    }
#pragma unroll
    for (int m = 12; m < 24; ++m) mfma1(F1, m);
    flush();
    zero_frags(F1);
  }
  __builtin_amdgcn_s_waitcnt(0);   // no copy into LDS may outlive the block
}

__device__ __forceinline__ int split2_tiles(const MabsGemmArgs& a) {
  return ((a.n_nu1 * a.nc + S_TM - 1) / S_TM) * ((a.nc + S_TN - 1) / S_TN) * a.ntri * a.kchunks;
}

__global__ __launch_bounds__(256) void k_mabs_gemm_split2(MabsGemmArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  split2_tile(a, xcd_tile(blockIdx.x, split2_tiles(a)), smem_raw);
}

// ---------------------------------------------------------------------------
// Split-BF16 contraction, 256 x 192 tiles.  Rows are tiled as (nu1 block of m1) x (nu2 block of
// m2), m1 m2 = 256 (m1 = 16, 8 or 4): the A tile is formed from m1 + m2 loaded field rows
// (F_b1(nu1) and F_b2(nu2)) instead of one row per A row.  Four waves of 128 x 96 (4 x 3 MFMA
// 32x32x16 tiles, 192 FP32 accumulators per lane), pixel stages of 32 in two A buffers (hi/lo,
// 32 KB each), two B buffers (hi/lo, 24 KB each) and two raw buffers of the m1 + m2 FP32 rows:
//  * the B rows of stage s+1 (pre-split F_b3) and the raw rows of stage s+2 are copied from
//    global memory straight into LDS (16-byte buffer loads) at the start of stage s;
//  * the A operand of stage s+1 is formed from the raw rows of stage s+1 (products F1 F2 split
//    into bf16 hi / lo) and stored into the other A buffer during stage s;
//  * one set of fragments: each kind (A lo / hi, B hi / lo) is reloaded for the next half stage as
//    soon as its last MFMA has issued, and the last 16 MFMAs of a stage are issued at the start of
//    the next one, covering the reads of its first fragments.
// Each stage ends with a wait for all of this wave's memory operations and one barrier.  Per MFMA
// this moves about a fifth less data through LDS than 128 x 256 tiles with 64 x 128 per wave, and
// the A inputs a fifth of the bytes.  (128 x 128 per wave, 256 accumulators, does not fit the
// register file without spills.)
// ---------------------------------------------------------------------------
constexpr int T3_NJ = 3;   // 32-column MFMA tiles per wave
constexpr int T3_M = 256, T3_N = 64 * T3_NJ, T3_K = 32, T3_FLUSH = 8192;
constexpr int T3_AL = T3_M * T3_K, T3_ABUF = 2 * T3_M * T3_K;   // A stage buffer: hi rows, then lo rows (32 KB)
constexpr int T3_BL = T3_N * T3_K, T3_BBUF = 2 * T3_N * T3_K;   // B stage buffer: hi columns, then lo (24 KB)
constexpr int T3_RAWLD = 36;                   // floats per raw row: 8 data chunks + 1 pad (bank spread)
constexpr int T3_RAW = 12 * 64 * 4;             // floats per raw buffer: 12 copy instructions of 64 chunks
// the F_b1 rows rounded up to whole copy instructions, then the F_b2 rows (m1 = 4, 8, 16, 32)
constexpr int t3_raw_chunks(int m1) { return 64 * ((9 * m1 + 63) / 64) + 9 * (256 / m1); }
static_assert(t3_raw_chunks(4) <= 12 * 64 && t3_raw_chunks(8) <= 12 * 64 && t3_raw_chunks(16) <= 12 * 64 &&
              t3_raw_chunks(32) <= 12 * 64, "twelve copy instructions hold every raw row");
static_assert(2 * (size_t)(T3_ABUF + T3_BBUF) * 2 + 2 * (size_t)T3_RAW * 4 <= 160 * 1024, "stage and raw buffers fit in LDS");


__device__ __forceinline__ int t3_m1(const MabsGemmArgs& a) {
  return a.tile_m1 ? a.tile_m1 : (a.n_nu1 >= 16 ? 16 : (a.n_nu1 >= 8 ? 8 : 4));
}
__device__ __forceinline__ int split3_tiles(const MabsGemmArgs& a) {
  const int m1 = t3_m1(a), m2 = T3_M / m1;
  return ((a.n_nu1 + m1 - 1) / m1) * ((a.nc + m2 - 1) / m2) * ((a.nc + T3_N - 1) / T3_N) * a.ntri * a.kchunks;
}

// The six LDS buffers (A, B and raw rows, two of each) are separate variables, so that the compiler
// can tell the copies into one from the reads and stores of another and does not wait for every
// copy in flight before them.
__device__ __forceinline__ void split3_tile(const MabsGemmArgs& a, int b, uint16_t* abuf0, uint16_t* abuf1,
                                            uint16_t* bbuf0, uint16_t* bbuf1, float* raw0, float* raw1) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const int m1 = t3_m1(a), m2 = T3_M / m1, lm2 = __builtin_ctz(m2);
  const int r1t = (a.n_nu1 + m1 - 1) / m1, r2t = (a.nc + m2 - 1) / m2, rtiles = r1t * r2t;
  const int ctiles = (a.nc + T3_N - 1) / T3_N;
  const int rt = b % rtiles;
  int rest = b / rtiles;
  const int ct = rest % ctiles;
  rest /= ctiles;
  const int kc = rest % a.kchunks;
  const int t = rest / a.kchunks;
  const int i0 = (rt / r2t) * m1, n20 = (rt % r2t) * m2, col0 = ct * T3_N;
  const int b1 = a.tri[3 * t], b2 = a.tri[3 * t + 1], b3 = a.tri[3 * t + 2];
  const int kbeg = __builtin_amdgcn_readfirstlane(kc * a.kchunk);
  const int kend = __builtin_amdgcn_readfirstlane(min(a.P, kbeg + a.kchunk));
  const int nst = (kend - kbeg) / T3_K;   // >= 1; pixel ranges are multiples of T3_K
  const int klast = kend - T3_K;          // copies past the range re-read the last stage

  // Copies into LDS are buffer loads (the global form counts as an LDS access for the compiler,
  // which then drains every LDS read at each wait); a buffer resource covers one field plane
  // (byte offsets below 2^32, checked by the launchers).  Raw copies: 12 instructions of 64
  // 16-byte chunks a stage (three a wave), each within one plane.  Chunks from 0 hold the m1 rows
  // of F_b1 (row q = nu1[i0 + q], chunk c at 9 q + c, the ninth a pad that re-reads chunk 0), chunks
  // from R2 = 64 ceil(9 m1 / 64) the m2 rows of F_b2 (nu2 = n20 + q) the same way; rows past the
  // valid ones are clamped (their products are never stored) and chunks past a row set re-read
  // its last row into unused LDS, so the copies carry no branch.
  const int nI1 = (9 * m1 + 63) / 64, R2 = 64 * nI1;
  unsigned roff[3];
  bool rsec[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int I = wave + 4 * k;
    rsec[k] = I >= nI1;
    const int h = rsec[k] ? (I - nI1) * 64 + lane : I * 64 + lane;
    const int q = min(h / 9, (rsec[k] ? m2 : m1) - 1), c = h % 9 == 8 ? 0 : h % 9;
    const int row = rsec[k] ? min(n20 + q, a.nc - 1) : a.nu1[min(i0 + q, a.n_nu1 - 1)];
    roff[k] = (unsigned)(((size_t)row * a.P + 4 * c) * 4);
  }
  // the resources are built from values read from the first lane: every lane holds the same ones,
  // and the compiler must see them as uniform (else it loops over the lanes' distinct resources)
  const int plane4 = __builtin_amdgcn_readfirstlane((int)(unsigned)(a.bin_stride * 4));
  const int plane2 = __builtin_amdgcn_readfirstlane((int)(unsigned)(a.bin_stride * 2));
  auto rsrc = [](const void* p, int bytes) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v), hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((unsigned long long)hi << 32) | lo), (short)0, bytes, BUF_DWORD3);
  };
  const __amdgpu_buffer_rsrc_t rF1 = rsrc(a.F + (size_t)b1 * a.bin_stride, plane4);
  const __amdgpu_buffer_rsrc_t rF2 = rsrc(a.F + (size_t)b2 * a.bin_stride, plane4);
  const __amdgpu_buffer_rsrc_t rH = rsrc(a.Fh + (size_t)b3 * a.bin_stride, plane2);
  const __amdgpu_buffer_rsrc_t rL = rsrc(a.Fl + (size_t)b3 * a.bin_stride, plane2);
  // B copies: this wave's columns w*16NJ .. w*16NJ+16NJ-1, 16 per instruction, hi then lo
  unsigned boff[T3_NJ];
#pragma unroll
  for (int q = 0; q < T3_NJ; ++q) {
    const int br = wave * 16 * T3_NJ + q * 16 + (lane >> 2);
    const int col = min(col0 + br, a.nc - 1);   // columns past nc load a valid row, never stored
    boff[q] = (unsigned)(((size_t)col * a.P + 8 * swz_rows(br, lane & 3)) * 2);
  }
  // A formation: thread r = tid owns tile row r = (i1, i2), i2 = r mod m2
  const int fr = tid, fi1 = fr >> lm2, fi2 = fr & (m2 - 1);
  const int rawf1 = fi1 * T3_RAWLD, rawf2 = 4 * R2 + fi2 * T3_RAWLD;
  // fragment offsets (uint16, inside a stage buffer) per half-stage kk
  int oa[2][4], ob[2][T3_NJ];
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int chunk = kk * 2 + (lane >> 5);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 128 + i * 32 + (lane & 31);
      oa[kk][i] = r * T3_K + swz_rows(r, chunk) * 8;
    }
#pragma unroll
    for (int j = 0; j < T3_NJ; ++j) {
      const int c = wn * 32 * T3_NJ + j * 32 + (lane & 31);
      ob[kk][j] = c * T3_K + swz_rows(c, chunk) * 8;
    }
  }

  auto copy_b1 = [&](int m, int k0, uint16_t* buf) {   // copy m of 2 NJ: columns q = m/2, hi or lo
    const int q = m >> 1;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(m & 1 ? rL : rH,
                                             (lds_void*)(buf + (m & 1 ? T3_BL : 0) + (wave * 16 * T3_NJ + q * 16) * T3_K),
                                             16, boff[q], 2 * k0, 0, 0);
  };
  auto copy_raw1 = [&](int k, int k0, float* rb) {    // raw copy instruction wave + 4 k
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsec[k] ? rF2 : rF1, (lds_void*)(rb + (wave + 4 * k) * 256), 16, roff[k],
                                             4 * k0, 0, 0);
  };
  // A formation piece pc of 4 (pixels 8 pc .. 8 pc + 7 of row fr) in six steps spread over the
  // MFMA slots: the raw reads (into R[pc]), four pair products split into bf16 hi / lo words (one
  // step of eight VALU operations, about the time of one MFMA), the two LDS stores
  float4 R[4][4];
  uint32_t HW[4][4], LW[4][4];
  auto form_read = [&](int pc, const float* rb) {
    R[pc][0] = *(const float4*)&rb[rawf1 + 8 * pc];
    R[pc][1] = *(const float4*)&rb[rawf1 + 8 * pc + 4];
    R[pc][2] = *(const float4*)&rb[rawf2 + 8 * pc];
    R[pc][3] = *(const float4*)&rb[rawf2 + 8 * pc + 4];
  };
  auto form_pair = [&](int pc, int q) {   // pixels 8 pc + 2 q, 8 pc + 2 q + 1
    const float4 x = R[pc][q >> 1], y = R[pc][2 + (q >> 1)];
    if (q & 1) bf16_split2(x.z * y.z, x.w * y.w, HW[pc][q], LW[pc][q]);
    else bf16_split2(x.x * y.x, x.y * y.y, HW[pc][q], LW[pc][q]);
  };
  auto form_write = [&](int pc, uint16_t* buf) {
    const v4u h = {HW[pc][0], HW[pc][1], HW[pc][2], HW[pc][3]};
    const v4u l = {LW[pc][0], LW[pc][1], LW[pc][2], LW[pc][3]};
    *(v4u*)(buf + fr * T3_K + swz_rows(fr, pc) * 8) = h;
    *(v4u*)(buf + T3_AL + fr * T3_K + swz_rows(fr, pc) * 8) = l;
  };
  auto form_piece = [&](int pc, const float* rb, uint16_t* buf) {
    form_read(pc, rb);
#pragma unroll
    for (int q = 0; q < 4; ++q) form_pair(pc, q);
    form_write(pc, buf);
  };
  // One set of fragments (A lo / hi of four 32-row tiles, B hi / lo of NJ 32-column tiles): each
  // kind is reloaded for the next half stage as soon as its last MFMA of the current one has issued.
  bf16x8 fal[4], fah[4], fbh[T3_NJ], fbl[T3_NJ];
  // read kind w (0: A lo, 1: A hi, 2: B hi, 3: B lo) of tile i for half stage kk from buf
  auto read1 = [&](int w, int i, const uint16_t* abuf, const uint16_t* bbuf, int kk) {
    if (w == 0) fal[i] = *(const bf16x8*)&abuf[T3_AL + oa[kk][i]];
    else if (w == 1) fah[i] = *(const bf16x8*)&abuf[oa[kk][i]];
    else if (w == 2) fbh[i] = *(const bf16x8*)&bbuf[ob[kk][i]];
    else fbl[i] = *(const bf16x8*)&bbuf[T3_BL + ob[kk][i]];
  };

  f32x16 acc[4][T3_NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < T3_NJ; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  constexpr int G = 4 * T3_NJ;   // MFMAs of a product group
  // MFMA m of G of product group p (0: A lo B hi, 1: A hi B lo, 2: A hi B hi) over the 4 x NJ tiles
  auto mfma1 = [&](int p, int m) {
    const int i = m / T3_NJ, j = m % T3_NJ;
    const bf16x8 x = p == 0 ? fal[i] : fah[i];
    const bf16x8 y = p == 1 ? fbl[j] : fbh[j];
    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc[i][j], 0, 0, 0);
  };

  const int nrows = a.n_nu1 * a.nc;
  double* S = a.S + ((size_t)kc * a.ntri + t) * (size_t)nrows * a.nc;
  bool first_flush = true;
  auto flush = [&]() {
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < T3_NJ; ++j) {
        const int col = col0 + wn * 32 * T3_NJ + j * 32 + (ln & 31);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int r = wm * 128 + i * 32 + (e >> 2) * 8 + (ln >> 5) * 4 + (e & 3);
          const int ii = i0 + (r >> lm2), nu2 = n20 + (r & (m2 - 1));
          if (ii < a.n_nu1 && nu2 < a.nc && col < a.nc) {
            double* d = &S[((size_t)ii * a.nc + nu2) * a.nc + col];
            const double v = (double)acc[i][j][e];
            if (first_flush) *d = v;
            else unsafeAtomicAdd(d, v);
          }
          acc[i][j][e] = 0.f;
        }
      }
    first_flush = false;
  };

  const bf16x8 zf = {};
#pragma unroll
  for (int i = 0; i < 4; ++i) fah[i] = zf;   // the deferred group of stage -1 adds zeros
#pragma unroll
  for (int j = 0; j < T3_NJ; ++j) fbl[j] = zf;
  // prologue: B of stage 0 and raw rows of stages 0 and 1 land, A of stage 0 is formed
#pragma unroll
  for (int m = 0; m < 2 * T3_NJ; ++m) copy_b1(m, kbeg, bbuf0);
#pragma unroll
  for (int k = 0; k < 3; ++k) copy_raw1(k, kbeg, raw0);
#pragma unroll
  for (int k = 0; k < 3; ++k) copy_raw1(k, min(kbeg + T3_K, klast), raw1);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_s_barrier();
#pragma unroll
  for (int pc = 0; pc < 4; ++pc) form_piece(pc, raw0, abuf0);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_s_barrier();

  // Stage s (buffer s&1; raw rows of stage s+1 in raw buffer (s+1)&1): 72 MFMA slots in six
  // product groups of G, sched_barrier keeping every slot in place; every LDS read is issued at
  // least eight slots before its first use, and no slot holds more than about one MFMA's time of
  // other work:
  //   G0  group (A hi, B lo) of half 1 of stage s-1 (deferred); B copies of stage s+1, raw copies
  //       of stage s+2; reads of A lo, B hi of half 0
  //   G1  (A lo, B hi) half 0; reads of A hi, B lo of half 0; raw reads of formation pieces 0, 1
  //   G2  (A hi, B hi) half 0; reads of A lo of half 1; piece 0 formed; raw reads of pieces 2, 3
  //   G3  (A hi, B lo) half 0; reads of B hi of half 1; pieces 1, 2, 3 formed
  //   G4  (A lo, B hi) half 1; reads of A hi, B lo of half 1
  //   G5  (A hi, B hi) half 1
  // then the wait for this wave's memory operations and the barrier.
  auto stage = [&](int s, auto par) {
    constexpr int PAR = decltype(par)::value;
    const uint16_t* ac = PAR ? abuf1 : abuf0;   // A and B of stage s
    const uint16_t* bc = PAR ? bbuf1 : bbuf0;
    uint16_t* an = PAR ? abuf0 : abuf1;         // A and B of stage s+1
    uint16_t* bn = PAR ? bbuf0 : bbuf1;
    const float* rawc = PAR ? raw0 : raw1;   // raw rows of stage s+1
    float* rawn = PAR ? raw1 : raw0;         // raw rows of stage s+2 land here
    const int kb = __builtin_amdgcn_readfirstlane(min(kbeg + (s + 1) * T3_K, klast));
    const int kr = __builtin_amdgcn_readfirstlane(min(kbeg + (s + 2) * T3_K, klast));
    __builtin_amdgcn_sched_barrier(0);
#pragma clang loop unroll(full)
    for (int sl = 0; sl < 6 * G; ++sl) {
      const int grp = sl / G, m = sl % G;
      mfma1(grp % 3 == 0 ? 1 : (grp % 3 == 1 ? 0 : 2), m);
      // copies of stage s+1 (B) and s+2 (raw rows)
      if (sl < 2 * T3_NJ) copy_b1(sl, kb, bn);
      else if (sl < 2 * T3_NJ + 3) copy_raw1(sl - 2 * T3_NJ, kr, rawn);
      // fragments
      if (sl < 4) read1(0, sl, ac, bc, 0);
      else if (sl < 4 + T3_NJ) read1(2, sl - 4, ac, bc, 0);
      else if (sl >= 12 && sl < 16) read1(1, sl - 12, ac, bc, 0);
      else if (sl >= 16 && sl < 16 + T3_NJ) read1(3, sl - 16, ac, bc, 0);
      else if (sl >= 24 && sl < 28) read1(0, sl - 24, ac, bc, 1);
      else if (sl >= 36 && sl < 36 + T3_NJ) read1(2, sl - 36, ac, bc, 1);
      else if (sl >= 48 && sl < 52) read1(1, sl - 48, ac, bc, 1);
      else if (sl >= 52 && sl < 52 + T3_NJ) read1(3, sl - 52, ac, bc, 1);
      // A of stage s+1
      if (sl == 20) form_read(0, rawc);
      if (sl == 22) form_read(1, rawc);
      if (sl == 31) form_read(2, rawc);
      if (sl == 33) form_read(3, rawc);
      if (sl >= 28 && sl < 32) form_pair(0, sl - 28);
      if (sl == 32) form_write(0, an);
      if (sl >= 33 && sl < 37) form_pair(1, sl - 33);
      if (sl == 37) form_write(1, an);
      if (sl >= 39 && sl < 43) form_pair(2, sl - 39);
      if (sl == 43) form_write(2, an);
      if (sl >= 44 && sl < 48) form_pair(3, sl - 44);
      if (sl == 48) form_write(3, an);
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_waitcnt(0);   // B of stage s+1, raw rows of stage s+2 landed; A of stage s+1 stored
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
  };

  for (int s = 0; s < nst;) {
    const int se = min(nst, s + T3_FLUSH / T3_K);   // s is even here
    while (true) {
      stage(s, std::integral_constant<int, 0>{});
      if (++s >= se) break;
      stage(s, std::integral_constant<int, 1>{});
      if (++s >= se) break;
    }
#pragma unroll
    for (int m = 0; m < G; ++m) mfma1(1, m);   // the deferred group of the last stage
    flush();
#pragma unroll
    for (int i = 0; i < 4; ++i) fah[i] = zf;
#pragma unroll
    for (int j = 0; j < T3_NJ; ++j) fbl[j] = zf;
  }
  __builtin_amdgcn_s_waitcnt(0);   // no copy into LDS may outlive the block
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mabs_gemm_split3(MabsGemmArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t abuf0[T3_ABUF], abuf1[T3_ABUF], bbuf0[T3_BBUF], bbuf1[T3_BBUF];
  __shared__ __attribute__((aligned(16))) float raw0[T3_RAW], raw1[T3_RAW];
  split3_tile(a, xcd_tile(blockIdx.x, split3_tiles(a)), abuf0, abuf1, bbuf0, bbuf1, raw0, raw1);
}

// ---------------------------------------------------------------------------
// FP32 contraction on FP32 MFMA (v_mfma_f32_32x32x2_f32), 128 x 128 tiles laid out like the split
// kernel above: rows are an m1 x (128 / m1) block of (nu1, nu2), the A tile is formed in LDS from
// the m1 + m2 raw FP32 rows (one FP32 product per element), B is the F_b3 rows copied straight into
// LDS.  Each wave owns 64 x 64 outputs (2 x 2 MFMA tiles); 80 KB of LDS and at most 256 registers
// a lane let two blocks share a CU.  LDS rows hold 32 floats as eight
// 16-byte chunks, chunk c of row r stored at slot c ^ (r ^ r >> 3) & 7, so that 16-byte accesses
// of one chunk by 8, 16 or 32 consecutive rows meet distinct slots of a 128-, 256- or 512-byte bank
// line.  A lane's 16-byte fragment read serves four MFMA steps: step e pairs pixels 8q + e and
// 8q + 4 + e of an 8-pixel group q (lanes 0-31 and 32-63), the same pairing on both operands.
// Per 32-pixel stage a wave issues 64 MFMAs (64 cycles each); the B copies of stage s+1 and the raw
// copies of stage s+2 go out first, the A formation of stage s+1 runs between the MFMAs, and the
// next 8-pixel group's fragments are read while the current group's MFMAs run; one wait and one
// barrier per stage.  Accumulation: FP32 MFMA sums over runs of 256 pixels are added into a second
// FP32 accumulator, which goes into the FP64 output every 8192 pixels (the first time a store,
// later FP64 atomics), so no FP32 sum takes more than 256 products before it joins a larger sum.
// ---------------------------------------------------------------------------
constexpr int F4_M = 128, F4_N = 128, F4_RUN = 256, F4_FLUSH = 8192;
constexpr int F4_AB = F4_M * T3_K, F4_BB = F4_N * T3_K;   // floats per A / B stage buffer (16 KB each)
constexpr int F4_RAW = 8 * 64 * 4;                        // floats per raw buffer: 8 copy instructions
// the F_b1 rows rounded up to whole copy instructions, then the F_b2 rows (m1 = 4, 8, 16, 32)
constexpr int f4_raw_chunks(int m1) { return 64 * ((9 * m1 + 63) / 64) + 9 * (128 / m1); }
static_assert(f4_raw_chunks(4) <= 8 * 64 && f4_raw_chunks(8) <= 8 * 64 && f4_raw_chunks(16) <= 8 * 64 &&
              f4_raw_chunks(32) <= 8 * 64, "eight copy instructions hold every raw row");
__device__ __forceinline__ int f4_swz(int r, int c) { return c ^ ((r ^ (r >> 3)) & 7); }
__device__ __forceinline__ int f4_m1(const MabsGemmArgs& a) {
  return a.tile_m1 ? a.tile_m1 : (a.n_nu1 >= 16 ? 16 : (a.n_nu1 >= 8 ? 8 : 4));
}
__device__ __forceinline__ int f32t_tiles(const MabsGemmArgs& a) {
  const int m1 = f4_m1(a), m2 = F4_M / m1;
  return ((a.n_nu1 + m1 - 1) / m1) * ((a.nc + m2 - 1) / m2) * ((a.nc + F4_N - 1) / F4_N) * a.ntri * a.kchunks;
}

__device__ __forceinline__ void f32t_tile(const MabsGemmArgs& a, int b, float* abuf0, float* abuf1, float* bbuf0,
                                          float* bbuf1, float* raw0, float* raw1) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const int m1 = f4_m1(a), m2 = F4_M / m1, lm2 = __builtin_ctz(m2);
  const int r1t = (a.n_nu1 + m1 - 1) / m1, r2t = (a.nc + m2 - 1) / m2, rtiles = r1t * r2t;
  const int ctiles = (a.nc + F4_N - 1) / F4_N;
  const int rt = b % rtiles;
  int rest = b / rtiles;
  const int ct = rest % ctiles;
  rest /= ctiles;
  const int kc = rest % a.kchunks;
  const int t = rest / a.kchunks;
  const int i0 = (rt / r2t) * m1, n20 = (rt % r2t) * m2, col0 = ct * F4_N;
  const int b1 = a.tri[3 * t], b2 = a.tri[3 * t + 1], b3 = a.tri[3 * t + 2];
  const int kbeg = __builtin_amdgcn_readfirstlane(kc * a.kchunk);
  const int kend = __builtin_amdgcn_readfirstlane(min(a.P, kbeg + a.kchunk));
  const int nst = (kend - kbeg) / T3_K;   // >= 1; pixel ranges are multiples of T3_K
  const int klast = kend - T3_K;          // copies past the range re-read the last stage

  // Copies into LDS are buffer loads over one field plane each, laid out as in the split kernel:
  // raw copies are 8 instructions of 64 16-byte chunks a stage (two a wave), chunks from 0 the m1
  // rows of F_b1 (row q = nu1[i0 + q], chunk c at 9 q + c, the ninth a pad that re-reads chunk 0),
  // chunks from 64 ceil(9 m1 / 64) the m2 rows of F_b2 (nu2 = n20 + q), rows clamped to a valid
  // one (their products are never stored), chunks past a row set re-reading its last row.
  const int nI1 = (9 * m1 + 63) / 64, rbase2 = 64 * nI1;
  unsigned roff[2];
  bool rsec[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int I = wave + 4 * k;
    rsec[k] = I >= nI1;
    const int h = rsec[k] ? (I - nI1) * 64 + lane : I * 64 + lane;
    const int q = min(h / 9, (rsec[k] ? m2 : m1) - 1), c = h % 9 == 8 ? 0 : h % 9;
    const int row = rsec[k] ? min(n20 + q, a.nc - 1) : a.nu1[min(i0 + q, a.n_nu1 - 1)];
    roff[k] = (unsigned)(((size_t)row * a.P + 4 * c) * 4);
  }
  const int plane4 = __builtin_amdgcn_readfirstlane((int)(unsigned)(a.bin_stride * 4));
  auto rsrc = [](const void* p, int bytes) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v), hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((unsigned long long)hi << 32) | lo), (short)0, bytes, BUF_DWORD3);
  };
  const __amdgpu_buffer_rsrc_t rF1 = rsrc(a.F + (size_t)b1 * a.bin_stride, plane4);
  const __amdgpu_buffer_rsrc_t rF2 = rsrc(a.F + (size_t)b2 * a.bin_stride, plane4);
  const __amdgpu_buffer_rsrc_t rF3 = rsrc(a.F + (size_t)b3 * a.bin_stride, plane4);
  // B copies: this wave's columns w*32 .. w*32+31, eight a copy instruction (lane l: column l / 8,
  // LDS slot l % 8, which holds global chunk (l % 8) ^ swizzle)
  unsigned boff[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int br = wave * 32 + q * 8 + (lane >> 3);
    const int col = min(col0 + br, a.nc - 1);   // columns past nc load a valid row, never stored
    boff[q] = (unsigned)(((size_t)col * a.P + 4 * f4_swz(br, lane & 7)) * 4);
  }
  // A formation: threads 2r, 2r + 1 own tile row r = (i1, i2), i2 = r mod m2, chunks 4h .. 4h + 3
  const int fr = tid >> 1, fh = tid & 1, fi1 = fr >> lm2, fi2 = fr & (m2 - 1);
  const int rawf1 = fi1 * T3_RAWLD, rawf2 = 4 * rbase2 + fi2 * T3_RAWLD;
  // fragment offsets (floats, inside a stage buffer) per 8-pixel group q
  int oa[4][2], ob[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int chunk = 2 * q + (lane >> 5);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 64 + i * 32 + (lane & 31);
      oa[q][i] = r * T3_K + 4 * f4_swz(r, chunk);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wn * 64 + j * 32 + (lane & 31);
      ob[q][j] = c * T3_K + 4 * f4_swz(c, chunk);
    }
  }
  auto copy_b1 = [&](int q, int k0, float* buf) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rF3, (lds_void*)(buf + (wave * 32 + q * 8) * T3_K), 16, boff[q], 4 * k0, 0, 0);
  };
  auto copy_raw1 = [&](int k, int k0, float* rb) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsec[k] ? rF2 : rF1, (lds_void*)(rb + (wave + 4 * k) * 256), 16, roff[k],
                                             4 * k0, 0, 0);
  };
  float4 R1, R2;
  auto form_read = [&](int c, const float* rb) {   // chunk 4 fh + c of this thread's row
    R1 = *(const float4*)&rb[rawf1 + 4 * (4 * fh + c)];
    R2 = *(const float4*)&rb[rawf2 + 4 * (4 * fh + c)];
  };
  auto form_write = [&](int c, float* buf) {
    const float4 v = {R1.x * R2.x, R1.y * R2.y, R1.z * R2.z, R1.w * R2.w};
    *(float4*)(buf + fr * T3_K + 4 * f4_swz(fr, 4 * fh + c)) = v;
  };
  float4 fa[2][2], fb[2][2];
  auto read_frags = [&](int par, int q, const float* ab, const float* bb) {
#pragma unroll
    for (int i = 0; i < 2; ++i) fa[par][i] = *(const float4*)&ab[oa[q][i]];
#pragma unroll
    for (int j = 0; j < 2; ++j) fb[par][j] = *(const float4*)&bb[ob[q][j]];
  };

  f32x16 acc[2][2], acc2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = acc2[i][j][e] = 0.f;
  auto mfma1 = [&](int par, int m) {   // MFMA m of 16 of an 8-pixel group: step m / 4, tile m % 4
    const int e = m / 4, i = (m % 4) / 2, j = m % 2;
    const float x = e == 0 ? fa[par][i].x : (e == 1 ? fa[par][i].y : (e == 2 ? fa[par][i].z : fa[par][i].w));
    const float y = e == 0 ? fb[par][j].x : (e == 1 ? fb[par][j].y : (e == 2 ? fb[par][j].z : fb[par][j].w));
    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc[i][j], 0, 0, 0);
  };

  const int nrows = a.n_nu1 * a.nc;
  double* S = a.S + ((size_t)kc * a.ntri + t) * (size_t)nrows * a.nc;
  bool first_flush = true;
  auto fold = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) { acc2[i][j][e] += acc[i][j][e]; acc[i][j][e] = 0.f; }
  };
  auto flush = [&]() {
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = col0 + wn * 64 + j * 32 + (ln & 31);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int r = wm * 64 + i * 32 + (e >> 2) * 8 + (ln >> 5) * 4 + (e & 3);
          const int ii = i0 + (r >> lm2), nu2 = n20 + (r & (m2 - 1));
          if (ii < a.n_nu1 && nu2 < a.nc && col < a.nc) {
            double* d = &S[((size_t)ii * a.nc + nu2) * a.nc + col];
            const double v = (double)acc2[i][j][e];
            if (first_flush) *d = v;
            else unsafeAtomicAdd(d, v);
          }
          acc2[i][j][e] = 0.f;
        }
      }
    first_flush = false;
  };

  // prologue: B of stage 0 and raw rows of stages 0 and 1 land, A of stage 0 is formed
#pragma unroll
  for (int q = 0; q < 4; ++q) copy_b1(q, kbeg, bbuf0);
#pragma unroll
  for (int k = 0; k < 2; ++k) copy_raw1(k, kbeg, raw0);
#pragma unroll
  for (int k = 0; k < 2; ++k) copy_raw1(k, min(kbeg + T3_K, klast), raw1);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_s_barrier();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    form_read(c, raw0);
    form_write(c, abuf0);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_s_barrier();

  // Stage s: four 8-pixel groups of 16 MFMA slots; copies in the first six slots, the A formation
  // of stage s+1 (four chunks: a raw read, six slots later the product and its store) from slot 10
  // on, the next group's fragments read in slot 2 of each group.
  auto stage = [&](int s, auto par) {
    constexpr int PAR = decltype(par)::value;
    const float* ac = PAR ? abuf1 : abuf0;   // A and B of stage s
    const float* bc = PAR ? bbuf1 : bbuf0;
    float* an = PAR ? abuf0 : abuf1;         // A and B of stage s+1
    float* bn = PAR ? bbuf0 : bbuf1;
    const float* rawc = PAR ? raw0 : raw1;   // raw rows of stage s+1
    float* rawn = PAR ? raw1 : raw0;         // raw rows of stage s+2 land here
    const int kb = __builtin_amdgcn_readfirstlane(min(kbeg + (s + 1) * T3_K, klast));
    const int kr = __builtin_amdgcn_readfirstlane(min(kbeg + (s + 2) * T3_K, klast));
    read_frags(0, 0, ac, bc);
    __builtin_amdgcn_sched_barrier(0);
#pragma clang loop unroll(full)
    for (int sl = 0; sl < 64; ++sl) {
      const int q = sl / 16, m = sl % 16;
      mfma1(q & 1, m);
      if (sl < 4) copy_b1(sl, kb, bn);
      else if (sl < 6) copy_raw1(sl - 4, kr, rawn);
      if (q < 3 && m == 2) read_frags((q + 1) & 1, q + 1, ac, bc);
      if (sl >= 10 && sl < 10 + 4 * 12 && (sl - 10) % 12 == 0) form_read((sl - 10) / 12, rawc);
      if (sl >= 16 && sl < 16 + 4 * 12 && (sl - 16) % 12 == 0) form_write((sl - 16) / 12, an);
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_waitcnt(0);   // B of stage s+1, raw rows of stage s+2 landed; A of stage s+1 stored
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
  };

  for (int s = 0; s < nst;) {
    const int se = min(nst, s + F4_FLUSH / T3_K);   // s is a multiple of F4_RUN / T3_K here
    while (s < se) {
      const int re = min(se, s + F4_RUN / T3_K);    // s is even here
      while (true) {
        stage(s, std::integral_constant<int, 0>{});
        if (++s >= re) break;
        stage(s, std::integral_constant<int, 1>{});
        if (++s >= re) break;
      }
      fold();
    }
    flush();
  }
  __builtin_amdgcn_s_waitcnt(0);   // no copy into LDS may outlive the block
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mabs_gemm_f32t(MabsGemmArgs a) {
  __shared__ __attribute__((aligned(16))) float abuf0[F4_AB], abuf1[F4_AB], bbuf0[F4_BB], bbuf1[F4_BB];
  __shared__ __attribute__((aligned(16))) float raw0[F4_RAW], raw1[F4_RAW];
  f32t_tile(a, xcd_tile(blockIdx.x, f32t_tiles(a)), abuf0, abuf1, bbuf0, bbuf1, raw0, raw1);
}

// Several independent GEMMs (e.g. cubes of different sizes) in one launch: group g owns blocks
// [offs[g], offs[g+1]); offsets are multiples of 8 so that the XCD remap of each group holds.
__global__ __launch_bounds__(256) void k_mabs_gemm_split2_grouped(const MabsGemmArgs* __restrict__ groups,
                                                                  const int* __restrict__ offs, int ngroups) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int b = blockIdx.x;
  int g = 0;
  while (g + 1 < ngroups && offs[g + 1] <= b) ++g;
  const MabsGemmArgs a = groups[g];
  const int nb = split2_tiles(a);
  const int lb = b - offs[g];
  if (lb >= nb) return;   // alignment padding
  split2_tile(a, xcd_tile(lb, nb), smem_raw);
}

// ---------------------------------------------------------------------------
// Persistent split-BF16 contraction over many GEMMs (cubes of uneven sizes, each with its own tile
// choice): a grid of one block per CU (both tile kinds take more than half of a CU's LDS) pulls
// tiles from eight work queues, one per XCD, until every queue is empty.  Queue x holds, for each
// GEMM in the order given (largest tile cost first), the run of that GEMM's tiles that the
// XCD-aware order gives to XCD x.  A block drains the queue of its own XCD first (block b runs on
// XCD b mod 8), so tiles that share an operand mostly meet in one L2, and then takes tiles from
// the other queues, so that no CU idles while work remains.  A pull is one atomic add on the
// queue's counter (zero at launch); a block leaves after one failed pull on each of the eight
// queues, so every block exits.  Tiles write disjoint outputs, so the result does not depend on
// which block takes which tile.
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ int persist_pull(const MabsPersistArgs& p, int& x, int& q, int* pull_sh, MabsGemmArgs& a) {
  // returns the tile index inside GEMM a, or -1 when every queue is empty
  while (q < 8) {
    x = ((int)blockIdx.x + q) & 7;
    __syncthreads();   // every wave is done with the previous tile's LDS and with pull_sh
    if (threadIdx.x == 0) *pull_sh = atomicAdd(&p.counters[x], 1);
    __syncthreads();
    const int j = __builtin_amdgcn_readfirstlane(*pull_sh);
    const int* qo = p.qoff + x * (p.ngroups + 1);
    if (j >= qo[p.ngroups]) { ++q; continue; }
    int g = 0;
    while (qo[g + 1] <= j) ++g;
    g = __builtin_amdgcn_readfirstlane(g);
    a = p.groups[g];
    const int nb = KIND ? split3_tiles(a) : split2_tiles(a);
    const int per = nb / 8, lj = j - qo[g];
    return lj < per ? x * per + lj : 8 * per + x;
  }
  return -1;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mabs_gemm_persist3(MabsPersistArgs p) {
  __shared__ __attribute__((aligned(16))) uint16_t abuf0[T3_ABUF], abuf1[T3_ABUF], bbuf0[T3_BBUF], bbuf1[T3_BBUF];
  __shared__ __attribute__((aligned(16))) float raw0[T3_RAW], raw1[T3_RAW];
  __shared__ int pull_sh;
  int x = 0, q = 0;
  MabsGemmArgs a;
  for (int t; (t = persist_pull<1>(p, x, q, &pull_sh, a)) >= 0;)
    split3_tile(a, t, abuf0, abuf1, bbuf0, bbuf1, raw0, raw1);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mabs_gemm_persist2(MabsPersistArgs p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  __shared__ int pull_sh;
  int x = 0, q = 0;
  MabsGemmArgs a;
  for (int t; (t = persist_pull<0>(p, x, q, &pull_sh, a)) >= 0;) split2_tile(a, t, smem_raw);
}

__global__ void k_zero_i32(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// FP64 contraction on the vector ALUs (data in BS_FP64 mode, counts for per-cell N_g).
// 64 x 64 tile, 256 threads, 4 x 4 outputs per thread (strided by 16), K staged by 16.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mabs_gemm_f64(MabsGemmArgs a) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double sA[BK][BM + 1];
  __shared__ double sB[BK][BN + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int nrows = a.n_nu1 * a.nc;
  const int col0 = blockIdx.x * BN, row0 = blockIdx.y * BM;
  const int t = blockIdx.z / a.kchunks;
  const int kc = blockIdx.z - t * a.kchunks;
  const int b1 = a.tri[3 * t], b2 = a.tri[3 * t + 1], b3 = a.tri[3 * t + 2];
  const int kbeg = kc * a.kchunk;
  const int kend = min(a.P, kbeg + a.kchunk);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      int r = e / BK, k = e - r * BK;
      int R = row0 + r;
      double v = 0.0;
      if (R < nrows && k0 + k < kend) {
        int i = R / a.nc, nu2 = R - i * a.nc;
        v = a.F64[(size_t)b1 * a.bin_stride + (size_t)a.nu1[i] * a.P + k0 + k] *
            a.F64[(size_t)b2 * a.bin_stride + (size_t)nu2 * a.P + k0 + k];
      }
      sA[k][r] = v;
      int c = r, nu3 = col0 + c;
      double w = 0.0;
      if (nu3 < a.nc && k0 + k < kend) w = a.F64[(size_t)b3 * a.bin_stride + (size_t)nu3 * a.P + k0 + k];
      sB[k][c] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* S = a.S + ((size_t)kc * a.ntri + t) * (size_t)nrows * a.nc;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int row = row0 + ty + 16 * i, col = col0 + tx + 16 * j;
      if (row < nrows && col < a.nc) S[(size_t)row * a.nc + col] = acc[i][j];
    }
}

// Few entries (n_nu1 nc x nc <= 64, e.g. one channel): a 64 x 64 tile would be almost all padding,
// so a block per (entry, triangle, pixel chunk) sums F1 F2 F3 over its chunk, threads over pixels
// (the same fused product F1 F2 * F3 per pixel), then a fixed tree; it writes the chunk's partial
// where the tiled kernel would.
__global__ __launch_bounds__(256) void k_mabs_dot_f64(MabsGemmArgs a) {
  __shared__ double red[256];
  const int nrows = a.n_nu1 * a.nc;
  const int ent = blockIdx.x, row = ent / a.nc, col = ent - row * a.nc;
  const int t = blockIdx.z / a.kchunks, kc = blockIdx.z - t * a.kchunks;
  const int b1 = a.tri[3 * t], b2 = a.tri[3 * t + 1], b3 = a.tri[3 * t + 2];
  const int i = row / a.nc, nu2 = row - i * a.nc;
  const double* __restrict__ f1 = a.F64 + (size_t)b1 * a.bin_stride + (size_t)a.nu1[i] * a.P;
  const double* __restrict__ f2 = a.F64 + (size_t)b2 * a.bin_stride + (size_t)nu2 * a.P;
  const double* __restrict__ f3 = a.F64 + (size_t)b3 * a.bin_stride + (size_t)col * a.P;
  const int kbeg = kc * a.kchunk, kend = min(a.P, kbeg + a.kchunk);
  double s = 0.0;
  for (int k = kbeg + (int)threadIdx.x; k < kend; k += 256) s = fma(f1[k] * f2[k], f3[k], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.S[((size_t)kc * a.ntri + t) * (size_t)nrows * a.nc + ent] = red[0];
}

// ---------------------------------------------------------------------------
// Channel-independent triangle counts: Tsum[t] = npix^2 sum_p I_b1(p) I_b2(p) I_b3(p).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tperp(const double* __restrict__ I, const int* __restrict__ tri, int P,
                                                double npix2, double* __restrict__ Tsum) {
  const int t = blockIdx.x;
  const double* a = I + (size_t)tri[3 * t] * P;
  const double* b = I + (size_t)tri[3 * t + 1] * P;
  const double* c = I + (size_t)tri[3 * t + 2] * P;
  double s = 0.0;
  for (int p = threadIdx.x; p < P; p += blockDim.x) s = fma(a[p] * b[p], c[p], s);
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) Tsum[t] = npix2 * red[0];
}

// Rounds an FP64 triangle count and records |x - rint(x)| in *maxdev (bit pattern of a
// non-negative double, so integer max == floating max; NaN maps above every finite value).
__device__ __forceinline__ int64_t round_count(double x, unsigned long long* maxdev) {
  double r = rint(x);
  double d = fabs(x - r);
  if (d != d) d = __builtin_inf();
  atomicMax(maxdev, (unsigned long long)__double_as_longlong(d));
  return (int64_t)r;
}

__global__ void k_round_counts(const double* __restrict__ x, int n, int64_t* __restrict__ out,
                               unsigned long long* bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = round_count(x[i], bad);
}

__device__ __forceinline__ double sum_chunks(const double* S, int kchunks, size_t chunk_stride, size_t idx) {
  double s = 0.0;
  for (int k = 0; k < kchunks; ++k) s += S[(size_t)k * chunk_stride + idx];
  return s;
}

__device__ __forceinline__ void mabs_entry(const double* S, int kchunks, const double* Sc, int kchunks_c,
                                           const int64_t* Tperp, const float* chw, int ntri, int nrows, int nc,
                                           int t, int R, int n1, int n2, int n3, double npix, double norm,
                                           unsigned long long* bad, double& Bo, int64_t& No) {
  size_t chunk_stride = (size_t)ntri * nrows * nc;
  size_t idx = ((size_t)t * nrows + R) * nc + n3;
  double s = sum_chunks(S, kchunks, chunk_stride, idx);
  int64_t cnt;
  if (Sc) {
    double sc = sum_chunks(Sc, kchunks_c, chunk_stride, idx);
    cnt = round_count(npix * npix * sc, bad);
  } else {
    bool on = !chw || (chw[n1] > 0.f && chw[n2] > 0.f && chw[n3] > 0.f);
    cnt = on ? Tperp[t] : 0;
  }
  No = cnt;
  Bo = cnt > 0 ? norm * npix * s / (double)cnt : __builtin_nan("");
}

__global__ __launch_bounds__(256) void k_mabs_finalize(MabsFinalArgs a) {
  const int nrows = a.n_nu1 * a.nc;
  const size_t total = (size_t)a.ntri * nrows * a.nc;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    int n3 = (int)(e % a.nc);
    size_t rest = e / a.nc;
    int R = (int)(rest % nrows);
    int t = (int)(rest / nrows);
    int i = R / a.nc, n2 = R - i * a.nc;
    double b;
    int64_t c;
    mabs_entry(a.S, a.kchunks, a.Sc, a.kchunks_c, a.Tperp, a.chw, a.ntri, nrows, a.nc, t, R, a.nu1[i], n2, n3,
               a.npix, a.norm, a.bad, b, c);
    a.B[e] = b;
    a.N[e] = c;
  }
}

// Ergodic collapse over a nu1 subset (unit channel weights): Bbar[t][d1'][d2'] is the mean of
// B(nu1, nu1 - d1 + d2, nu1 - d1) over the selected nu1 for which both other channels lie in the
// band (d' = d + nc - 1); Nnu[d1'][d2'] counts them.  B = norm npix S / Tperp as for full output.
__global__ __launch_bounds__(256) void k_mabs_collapse_subset(MabsSubsetArgs a) {
  const int nc = a.nc, D = 2 * nc - 1;
  const int nrows = a.n_nu1 * nc;
  const size_t total = (size_t)a.ntri * D * D;
  const size_t chunk_stride = (size_t)a.ntri * nrows * nc;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int j2 = (int)(e % D);
    const size_t rest = e / D;
    const int j1 = (int)(rest % D);
    const int t = (int)(rest / D);
    const int d1 = j1 - (nc - 1), d2 = j2 - (nc - 1);
    double acc = 0.0;
    int cnt = 0;
    for (int i = 0; i < a.n_nu1; ++i) {
      const int n1 = a.nu1[i], n3 = n1 - d1, n2 = n3 + d2;
      if (n3 < 0 || n3 >= nc || n2 < 0 || n2 >= nc) continue;
      const size_t idx = ((size_t)t * nrows + (size_t)i * nc + n2) * nc + n3;
      acc += sum_chunks(a.S, a.kchunks, chunk_stride, idx);
      ++cnt;
    }
    const int64_t T = a.Tperp[t];
    a.B[e] = (cnt > 0 && T > 0) ? a.norm * a.npix * (acc / cnt) / (double)T : __builtin_nan("");
    if (t == 0) a.Nnu[(size_t)j1 * D + j2] = cnt;
  }
}

// Ergodic collapse: mean over valid nu3 of B(nu3 + d1, nu3 + d2, nu3) (rows R = nu1*nc + nu2).
__global__ __launch_bounds__(256) void k_mabs_collapse(MabsCollapseArgs a) {
  const int nc = a.nc;
  const int D = a.circular ? nc : 2 * nc - 1;
  const int nrows = nc * nc;
  const size_t total = (size_t)a.ntri * D * D;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    int j2 = (int)(e % D);
    size_t rest = e / D;
    int j1 = (int)(rest % D);
    int t = (int)(rest / D);
    int d1 = a.circular ? j1 : j1 - (nc - 1);
    int d2 = a.circular ? j2 : j2 - (nc - 1);
    double acc = 0.0;
    int cnt = 0;
    int64_t tot = 0;
    for (int n3 = 0; n3 < nc; ++n3) {
      int n1 = n3 + d1, n2 = n3 + d2;
      if (a.circular) { n1 %= nc; n2 %= nc; }
      else if (n1 < 0 || n1 >= nc || n2 < 0 || n2 >= nc) continue;
      double b;
      int64_t c;
      mabs_entry(a.S, a.kchunks, a.Sc, a.kchunks_c, a.Tperp, a.chw, a.ntri, nrows, nc, t, n1 * nc + n2, n1, n2,
                 n3, a.npix, a.norm, a.bad, b, c);
      if (c > 0) { acc += b; ++cnt; tot += c; }
    }
    a.B[e] = cnt ? acc / cnt : __builtin_nan("");
    a.N[e] = tot;
    a.Nnu[e] = cnt;
  }
}

}  // namespace

// ----------------------------------------------------------------- launchers
void launch_mabs_fields_f32(const MabsFieldArgs& a, int nbins, int nchan, size_t lds, hipStream_t s) {
  (void)hipFuncSetAttribute((const void*)k_mabs_fields<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_mabs_fields<float>, dim3(a.G, nchan, nbins), dim3(256), lds, s, a);
}
void launch_mabs_fields_f64(const MabsFieldArgs& a, int nbins, int nchan, size_t lds, hipStream_t s) {
  (void)hipFuncSetAttribute((const void*)k_mabs_fields<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_mabs_fields<double>, dim3(a.G, nchan, nbins), dim3(256), lds, s, a);
}
void launch_split_bf16(const float* F, uint16_t* hi, uint16_t* lo, long long n, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)blocks), dim3(256), 0, s, F, hi, lo, n);
}
static dim3 gemm_grid(const MabsGemmArgs& a, int tm, int tn) {
  int nrows = a.n_nu1 * a.nc;
  return dim3((a.nc + tn - 1) / tn, (nrows + tm - 1) / tm, a.ntri * a.kchunks);
}
void launch_mabs_gemm_split(const MabsGemmArgs& a, hipStream_t s) {
  if (getenv("BS_MABS_SMALL_TILES")) {
    hipLaunchKernelGGL(k_mabs_gemm<2>, gemm_grid(a, TM, TN), dim3(256), 0, s, a);
    return;
  }
  if (a.n_nu1 >= 4 && buffer_fits(a.bin_stride * 4) && !getenv("BS_MABS_TILE128")) {
    // 256 x 192 tiles over (nu1 block x nu2 block) rows
    MabsGemmArgs b = a;
    if (const char* e = getenv("BS_MABS_M1")) b.tile_m1 = atoi(e);   // tuning switch: 4, 8, 16 or 32
    const int m1 = b.tile_m1 ? b.tile_m1 : (b.n_nu1 >= 16 ? 16 : (b.n_nu1 >= 8 ? 8 : 4)), m2 = T3_M / m1;
    const long long nb = (long long)((a.n_nu1 + m1 - 1) / m1) * ((a.nc + m2 - 1) / m2) * ((a.nc + T3_N - 1) / T3_N) *
                         a.ntri * a.kchunks;
    hipLaunchKernelGGL(k_mabs_gemm_split3, dim3((unsigned)nb), dim3(256), 0, s, b);
    return;
  }
  const int nrows = a.n_nu1 * a.nc;
  const long long nb = (long long)((nrows + S_TM - 1) / S_TM) * ((a.nc + S_TN - 1) / S_TN) * a.ntri * a.kchunks;
  const size_t lds = S_NBUF * (size_t)S_BUF * 2;
  (void)hipFuncSetAttribute((const void*)k_mabs_gemm_split2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_mabs_gemm_split2, dim3((unsigned)nb), dim3(256), lds, s, a);
}
int mabs_split_blocks(const MabsGemmArgs& a) {
  const int nrows = a.n_nu1 * a.nc;
  return ((nrows + S_TM - 1) / S_TM) * ((a.nc + S_TN - 1) / S_TN) * a.ntri * a.kchunks;
}
void launch_mabs_gemm_split_grouped(const MabsGemmArgs* groups_dev, const int* offs_dev, int ngroups, int nblocks,
                                    hipStream_t s) {
  if (nblocks <= 0) return;
  const size_t lds = S_NBUF * (size_t)S_BUF * 2;
  (void)hipFuncSetAttribute((const void*)k_mabs_gemm_split2_grouped, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_mabs_gemm_split2_grouped, dim3((unsigned)nblocks), dim3(256), lds, s, groups_dev, offs_dev, ngroups);
}
int mabs_split3_tiles(const MabsGemmArgs& a) {
  const int m1 = a.tile_m1 ? a.tile_m1 : (a.n_nu1 >= 16 ? 16 : (a.n_nu1 >= 8 ? 8 : 4)), m2 = T3_M / m1;
  return ((a.n_nu1 + m1 - 1) / m1) * ((a.nc + m2 - 1) / m2) * ((a.nc + T3_N - 1) / T3_N) * a.ntri * a.kchunks;
}
void launch_mabs_gemm_persist(int kind, const MabsPersistArgs& p, int nblocks, hipStream_t s) {
  if (nblocks <= 0 || p.ngroups <= 0) return;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, p.counters, 8);
  if (kind) {
    hipLaunchKernelGGL(k_mabs_gemm_persist3, dim3(nblocks), dim3(256), 0, s, p);
  } else {
    const size_t lds = S_NBUF * (size_t)S_BUF * 2;
    (void)hipFuncSetAttribute((const void*)k_mabs_gemm_persist2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_mabs_gemm_persist2, dim3(nblocks), dim3(256), lds, s, p);
  }
}
void launch_mabs_gemm_f32(const MabsGemmArgs& a, hipStream_t s) {
  if (a.n_nu1 >= 4 && buffer_fits(a.bin_stride * 4) && !getenv("BS_MABS_F32_TILE128")) {
    MabsGemmArgs b = a;
    if (const char* e = getenv("BS_MABS_M1")) b.tile_m1 = atoi(e);   // tuning switch: 4, 8, 16 or 32
    const int m1 = b.tile_m1 ? b.tile_m1 : (b.n_nu1 >= 16 ? 16 : (b.n_nu1 >= 8 ? 8 : 4)), m2 = 128 / m1;
    const long long nb = (long long)((b.n_nu1 + m1 - 1) / m1) * ((b.nc + m2 - 1) / m2) * ((b.nc + 127) / 128) *
                         b.ntri * b.kchunks;
    hipLaunchKernelGGL(k_mabs_gemm_f32t, dim3((unsigned)nb), dim3(256), 0, s, b);
    return;
  }
  hipLaunchKernelGGL(k_mabs_gemm<1>, gemm_grid(a, TM, TN), dim3(256), 0, s, a);
}
void launch_mabs_gemm_f64(const MabsGemmArgs& a, hipStream_t s) {
  const long long ents = (long long)a.n_nu1 * a.nc * a.nc;
  if (ents <= 64)
    hipLaunchKernelGGL(k_mabs_dot_f64, dim3((unsigned)ents, 1, a.ntri * a.kchunks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_mabs_gemm_f64, gemm_grid(a, 64, 64), dim3(256), 0, s, a);
}
void launch_tperp(const double* I, const int* tri, int ntri, int P, double npix2, double* Tsum, hipStream_t s) {
  if (ntri > 0) hipLaunchKernelGGL(k_tperp, dim3(ntri), dim3(256), 0, s, I, tri, P, npix2, Tsum);
}
void launch_round_counts(const double* x, int n, int64_t* out, unsigned long long* bad, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_round_counts, dim3((n + 255) / 256), dim3(256), 0, s, x, n, out, bad);
}
void launch_mabs_finalize(const MabsFinalArgs& a, hipStream_t s) {
  size_t total = (size_t)a.ntri * a.n_nu1 * a.nc * a.nc;
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (total) hipLaunchKernelGGL(k_mabs_finalize, dim3((unsigned)blocks), dim3(256), 0, s, a);
}
void launch_mabs_collapse_subset(const MabsSubsetArgs& a, hipStream_t s) {
  size_t total = (size_t)a.ntri * (2 * a.nc - 1) * (2 * a.nc - 1);
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (total) hipLaunchKernelGGL(k_mabs_collapse_subset, dim3((unsigned)blocks), dim3(256), 0, s, a);
}
void launch_mabs_collapse(const MabsCollapseArgs& a, hipStream_t s) {
  int D = a.circular ? a.nc : 2 * a.nc - 1;
  size_t total = (size_t)a.ntri * D * D;
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (total) hipLaunchKernelGGL(k_mabs_collapse, dim3((unsigned)blocks), dim3(256), 0, s, a);
}
