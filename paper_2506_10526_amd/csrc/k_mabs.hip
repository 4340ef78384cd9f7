// MABS kernels for gfx950: ring-filtered fields (Eqs. iFT, iFT_I), the triple-product
// contraction of Eq. (estimator_t) as an MFMA GEMM, counts, normalisation and the
// ergodic collapse to channel separations.
#include <hip/hip_runtime.h>

#include <cstdint>
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
// stages of 32, double-buffered LDS with one barrier per stage:
//  * the pre-split B rows (bf16 hi/lo of F_b3) go from global memory straight into the next
//    LDS buffer with 16-byte global_load_lds (lane l lands at byte 16 l of the wave's window);
//  * A = F_b1(nu1) .* F_b2(nu2) is formed and split into bf16 hi/lo by the VALU from F2 values
//    prefetched into registers and, when the whole tile shares one nu1 (UNI), an F1 chunk that
//    each wave also loads straight into LDS;
//  * the MFMAs of the current stage run while those loads are in flight.
// LDS rows hold 32 bf16 as four 16-byte chunks XOR-swizzled by row.  The block's FP32 tile is
// added into its FP64 output every SFLUSH pixels.  Blocks are mapped to tiles so that tiles
// sharing a B column block and neighbouring A rows run on the same XCD (blocks are dealt to the
// eight XCDs round-robin).
// ---------------------------------------------------------------------------
constexpr int S_TM = 128, S_TN = 256, S_TK = 32, SFLUSH = 4096;
// uint16 offsets inside one stage buffer
constexpr int S_AH = 0, S_AL = S_TM * S_TK, S_BH = 2 * S_TM * S_TK, S_BL = S_BH + S_TN * S_TK;
constexpr int S_F1 = S_BL + S_TN * S_TK;           // 4 waves x 1 KB of F1 staging
constexpr int S_BUF = S_F1 + 4 * 512;

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ int swz(int r, int chunk) { return (chunk ^ ((r >> 2) & 3)); }

// One block tile of GEMM `a`; b0 is the block's index within this GEMM's nb = rtiles ctiles ntri
// kchunks blocks.
template <bool UNI>
__device__ __forceinline__ void split2_tile(const MabsGemmArgs& a, int b0, unsigned char* smem_raw) {
  uint16_t* lds = (uint16_t*)smem_raw;   // [2][S_BUF]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int nrows = a.n_nu1 * a.nc;
  const int rtiles = (nrows + S_TM - 1) / S_TM, ctiles = (a.nc + S_TN - 1) / S_TN;
  const int nb = rtiles * ctiles * a.ntri * a.kchunks;
  // XCD-aware remap of the linear block id (blocks are dealt to the eight XCDs round-robin)
  int b = b0;
  const int full = (nb / 8) * 8;
  if (b < full) b = (b & 7) * (full / 8) + (b >> 3);
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

  // A loader: row ar (16 pixels starting at ahalf)
  const int ar = tid >> 1, ahalf = (tid & 1) * 16;
  const int R = row0 + ar;
  const bool rok = R < nrows;
  const int Rc = rok ? R : nrows - 1;
  const int ia = Rc / a.nc, nu2 = Rc - ia * a.nc;
  const float* f1 = a.F + (size_t)b1 * a.bin_stride + (size_t)a.nu1[ia] * a.P + ahalf;
  const float* f2 = a.F + (size_t)b2 * a.bin_stride + (size_t)nu2 * a.P + ahalf;
  // F1 chunk for the whole tile (UNI): lanes 0..7 cover 32 floats, the others repeat chunk 7
  const float* f1u = a.F + (size_t)b1 * a.bin_stride + (size_t)a.nu1[row0 / a.nc] * a.P + 4 * min(lane, 7);
  // B DMA: this wave's rows w*64 .. w*64+63, 16 rows per instruction
  const uint16_t* bsrc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int br = wave * 64 + q * 16 + (lane >> 2);
    const int col = min(col0 + br, a.nc - 1);   // columns past nc load a valid row, never stored
    bsrc[q] = (const uint16_t*)0 + ((size_t)b3 * a.bin_stride + (size_t)col * a.P) +
              8 * swz(br, lane & 3);
  }

  float4 pa1[4], pa2[4];
  auto issue = [&](int k0, uint16_t* buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      __builtin_amdgcn_global_load_lds((const void*)(a.Fh + ((bsrc[q] - (const uint16_t*)0) + k0)),
                                       (lds_void*)(buf + S_BH + (wave * 64 + q * 16) * S_TK), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(a.Fl + ((bsrc[q] - (const uint16_t*)0) + k0)),
                                       (lds_void*)(buf + S_BL + (wave * 64 + q * 16) * S_TK), 16, 0, 0);
    }
    if (UNI) {
      __builtin_amdgcn_global_load_lds((const void*)(f1u + k0), (lds_void*)(buf + S_F1 + wave * 512), 16, 0, 0);
    } else {
      const float4* p1 = (const float4*)(f1 + k0);
#pragma unroll
      for (int q = 0; q < 4; ++q) pa1[q] = p1[q];
    }
    const float4* p2 = (const float4*)(f2 + k0);
#pragma unroll
    for (int q = 0; q < 4; ++q) pa2[q] = p2[q];
  };
  auto form = [&](uint16_t* buf) {
    uint16_t* Ah = buf + S_AH;
    uint16_t* Al = buf + S_AL;
    if (UNI) {
      const float4* fw = (const float4*)(buf + S_F1 + wave * 512) + (ahalf >> 2);
#pragma unroll
      for (int q = 0; q < 4; ++q) pa1[q] = fw[q];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint16_t h[8], l[8];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        float4 x = pa1[2 * c + q], y = pa2[2 * c + q];
        float v[4] = {x.x * y.x, x.y * y.y, x.z * y.z, x.w * y.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          float vv = rok ? v[u] : 0.f;
          h[4 * q + u] = bf16_bits(vv);
          l[4 * q + u] = bf16_bits(vv - bf16_float(h[4 * q + u]));
        }
      }
      const int pc = swz(ar, (ahalf >> 3) + c);
      *(uint4*)&Ah[ar * S_TK + pc * 8] = *(uint4*)h;
      *(uint4*)&Al[ar * S_TK + pc * 8] = *(uint4*)l;
    }
  };

  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  double* S = a.S + ((size_t)kc * a.ntri + t) * (size_t)nrows * a.nc;
  const bool interior = row0 + S_TM <= nrows && col0 + S_TN <= a.nc;
  bool first_flush = true;

  issue(kbeg, lds);
  __builtin_amdgcn_s_waitcnt(0);
  form(lds);
  __syncthreads();
  int cur = 0;
  // outer loop: FP64 flush of the block's tile every SFLUSH pixels; inner loop: stages (MFMA only)
  for (int kf = kbeg; kf < kend; kf += SFLUSH) {
    const int kfe = min(kend, kf + SFLUSH);
    for (int k0 = kf; k0 < kfe; k0 += S_TK) {
      const bool more = k0 + S_TK < kend;
      uint16_t* nxt = lds + (cur ^ 1) * S_BUF;
      if (more) issue(k0 + S_TK, nxt);
      const uint16_t* buf = lds + cur * S_BUF;
      const uint16_t* Ah = buf + S_AH;
      const uint16_t* Al = buf + S_AL;
      const uint16_t* Bh = buf + S_BH;
      const uint16_t* Bl = buf + S_BL;
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const int chunk = kk * 2 + (lane >> 5);
        bf16x8 ah[2], al[2], bh[4], bl[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int r = wm * 64 + i * 32 + (lane & 31);
          const int off = r * S_TK + swz(r, chunk) * 8;
          ah[i] = *(const bf16x8*)&Ah[off];
          al[i] = *(const bf16x8*)&Al[off];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = wn * 128 + j * 32 + (lane & 31);
          const int off = c * S_TK + swz(c, chunk) * 8;
          bh[j] = *(const bf16x8*)&Bh[off];
          bl[j] = *(const bf16x8*)&Bl[off];
        }
        // the three products of a tile are issued eight MFMAs apart (no back-to-back dependence)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
      if (more) {
        __builtin_amdgcn_s_waitcnt(0);   // this wave's DMA and register loads of the next stage
        form(nxt);
      }
      __syncthreads();
      cur ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = col0 + wn * 128 + j * 32 + (lane & 31);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int row = row0 + wm * 64 + i * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
          if (interior || (row < nrows && col < a.nc)) {
            double* d = &S[(size_t)row * a.nc + col];
            double v = (double)acc[i][j][e];
            *d = first_flush ? v : *d + v;
          }
          acc[i][j][e] = 0.f;
        }
      }
    first_flush = false;
  }
}

template <bool UNI>
__global__ __launch_bounds__(256) void k_mabs_gemm_split2(MabsGemmArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  split2_tile<UNI>(a, blockIdx.x, smem_raw);
}

// Several independent GEMMs (e.g. cubes of different sizes) in one launch: group g owns blocks
// [offs[g], offs[g+1]); offsets are multiples of 8 so that the XCD remap of each group holds.
template <bool UNI>
__global__ __launch_bounds__(256) void k_mabs_gemm_split2_grouped(const MabsGemmArgs* __restrict__ groups,
                                                                  const int* __restrict__ offs, int ngroups) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int b = blockIdx.x;
  int g = 0;
  while (g + 1 < ngroups && offs[g + 1] <= b) ++g;
  const MabsGemmArgs a = groups[g];
  const int nrows = a.n_nu1 * a.nc;
  const int nb = ((nrows + S_TM - 1) / S_TM) * ((a.nc + S_TN - 1) / S_TN) * a.ntri * a.kchunks;
  const int lb = b - offs[g];
  if (lb >= nb) return;   // alignment padding
  split2_tile<UNI>(a, lb, smem_raw);
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
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
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
  hipFuncSetAttribute((const void*)k_mabs_fields<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_mabs_fields<float>, dim3(a.G, nchan, nbins), dim3(256), lds, s, a);
}
void launch_mabs_fields_f64(const MabsFieldArgs& a, int nbins, int nchan, size_t lds, hipStream_t s) {
  hipFuncSetAttribute((const void*)k_mabs_fields<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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
  const int nrows = a.n_nu1 * a.nc;
  const long long nb = (long long)((nrows + S_TM - 1) / S_TM) * ((a.nc + S_TN - 1) / S_TN) * a.ntri * a.kchunks;
  const size_t lds = 2 * (size_t)S_BUF * 2;
  if (a.nc % S_TM == 0) {
    (void)hipFuncSetAttribute((const void*)k_mabs_gemm_split2<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_mabs_gemm_split2<true>, dim3((unsigned)nb), dim3(256), lds, s, a);
  } else {
    (void)hipFuncSetAttribute((const void*)k_mabs_gemm_split2<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_mabs_gemm_split2<false>, dim3((unsigned)nb), dim3(256), lds, s, a);
  }
}
int mabs_split_blocks(const MabsGemmArgs& a) {
  const int nrows = a.n_nu1 * a.nc;
  return ((nrows + S_TM - 1) / S_TM) * ((a.nc + S_TN - 1) / S_TN) * a.ntri * a.kchunks;
}
bool mabs_split_uni(int nc) { return nc % S_TM == 0; }
void launch_mabs_gemm_split_grouped(const MabsGemmArgs* groups_dev, const int* offs_dev, int ngroups, int nblocks,
                                    bool uni, hipStream_t s) {
  if (nblocks <= 0) return;
  const size_t lds = 2 * (size_t)S_BUF * 2;
  if (uni) {
    (void)hipFuncSetAttribute((const void*)k_mabs_gemm_split2_grouped<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_mabs_gemm_split2_grouped<true>, dim3((unsigned)nblocks), dim3(256), lds, s, groups_dev, offs_dev, ngroups);
  } else {
    (void)hipFuncSetAttribute((const void*)k_mabs_gemm_split2_grouped<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_mabs_gemm_split2_grouped<false>, dim3((unsigned)nblocks), dim3(256), lds, s, groups_dev, offs_dev, ngroups);
  }
}
void launch_mabs_gemm_f32(const MabsGemmArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_mabs_gemm<1>, gemm_grid(a, TM, TN), dim3(256), 0, s, a);
}
void launch_mabs_gemm_f64(const MabsGemmArgs& a, hipStream_t s) {
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
