// Seeded synthetic cubes on the GPU and the Monte Carlo accumulators.
//
// A realization is the quadratic non-Gaussian field of the validation set-up (Sec. 4, Eq. mb1)
// built from counter-based white noise:
//   white(i), i = (z n + x) n + y: Philox4x64-10 (Salmon et al. 2011) with key (seed, realization)
//     and counter (i / 4, 0, 0, 0); the four 64-bit outputs give 24-bit uniforms
//     u_j = ((x_j >> 40) + 1/2) 2^-24 and two Box-Muller pairs for voxels 4c .. 4c+3;
//   g = irfftn(rfftn(white) sqrt(A P(k))), P = (k^2)^(index/2), P(0) = 0, A = sigma^2 N / sum P;
//   delta = g + f (g^2 - mean g^2);  V[z] = rfft2(delta[z]) w(z)   (complex64 [nc][n][n/2+1]).
//
// Passes (every one an LDS-staged Stockham transform of a group of lines):
//   rows_fwd<WHITE>: white noise generated in registers, two real rows packed as one complex row,
//                    forward FFT along y, split into the two half spectra           -> W
//   axis<-1>       : forward C2C along x                                             (W in place)
//   axis<SPEC>     : forward C2C along z, times sqrt(A P(k)), inverse C2C along z    (W in place)
//   axis<+1>       : inverse C2C along x                                             (W in place)
//   rows_c2r       : two half spectra packed as one complex row, inverse FFT along y -> g, sum g^2
//   mean           : mean g^2 (fixed-order reduction)
//   rows_fwd<QUAD> : delta from g on load, forward FFT along y                       -> W
//   axis<CHAN>     : forward C2C along x, times w(z)                                 (W in place)
// W is the caller's output cube, so a realization needs only the real field g as scratch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bs_gen.h"
#include "fft_lds.h"

namespace {

typedef Cx<float> C;

// ---------------------------------------------------------------- Philox4x64-10
struct U4 {
  unsigned long long v[4];
};

__device__ __forceinline__ U4 philox4x64_10(unsigned long long c0, unsigned long long k0, unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  unsigned long long x0 = c0, x1 = 0, x2 = 0, x3 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const unsigned long long h0 = __umul64hi(x0, M0), l0 = x0 * M0;
    const unsigned long long h1 = __umul64hi(x2, M1), l1 = x2 * M1;
    x0 = h1 ^ x1 ^ k0;
    x1 = l1;
    x2 = h0 ^ x3 ^ k1;
    x3 = l0;
  }
  U4 o;
  o.v[0] = x0; o.v[1] = x1; o.v[2] = x2; o.v[3] = x3;
  return o;
}

__device__ __forceinline__ float u24(unsigned long long x) {
  return ((float)(unsigned)(x >> 40) + 0.5f) * 5.9604644775390625e-8f;  // 2^-24
}

// Four standard normals of voxels 4c .. 4c+3.
__device__ __forceinline__ void normals4(unsigned long long c, unsigned long long seed, unsigned long long real,
                                         float* z) {
  U4 x = philox4x64_10(c, seed, real);
  const float r01 = sqrtf(-2.0f * logf(u24(x.v[0])));
  const float r23 = sqrtf(-2.0f * logf(u24(x.v[2])));
  float s, co;
  sincospif(2.0f * u24(x.v[1]), &s, &co);
  z[0] = r01 * co;
  z[1] = r01 * s;
  sincospif(2.0f * u24(x.v[3]), &s, &co);
  z[2] = r23 * co;
  z[3] = r23 * s;
}

__device__ __forceinline__ int signed_idx(int i, int m) { return i < (m + 1) / 2 ? i : i - m; }

// sqrt(A P(k)) for k^2 (float); P(0) = 0.
__device__ __forceinline__ float spec_amp(float k2, float sqrtA, float e4, int m2) {
  if (k2 <= 0.f) return 0.f;
  return m2 ? sqrtA / sqrtf(k2) : sqrtA * powf(k2, e4);
}

// ---------------------------------------------------------------- sum of P over the full grid
__global__ __launch_bounds__(256) void k_gen_psum(GenArgs a) {
  const int z = blockIdx.x;
  const double kz = a.cz * (double)signed_idx(z, a.nc);
  double s = 0.0;
  for (int t = threadIdx.x; t < a.n * a.n; t += 256) {
    const int x = t / a.n, y = t - x * a.n;
    const double kx = a.cxy * (double)signed_idx(x, a.n), ky = a.cxy * (double)signed_idx(y, a.n);
    const double k2 = kz * kz + kx * kx + ky * ky;
    if (k2 > 0.0) s += a.m2 ? 1.0 / k2 : pow(k2, 0.5 * a.index);
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[z] = red[0];
}

// sqrtA = sqrt(sigma^2 N / sum P), summed over the nc partials in a fixed order.
__global__ void k_gen_amp(GenArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int z = 0; z < a.nc; ++z) s += a.part[z];
  const double nvox = (double)a.nc * a.n * a.n;
  a.stat[0] = s > 0.0 ? sqrt(a.sigma * a.sigma * nvox / s) : 0.0;
}

// ---------------------------------------------------------------- rows along y
// Block: NL row pairs (rows 2p, 2p+1, p = blockIdx.x NL + l).  MODE 0: white noise; 1: delta(g).
template <int MODE, int IP>   // IP: in-place FFT bound (butterflies per thread), 0 = two buffers
__global__ __launch_bounds__(256) void k_gen_rows_fwd(GenArgs a) {
  extern __shared__ unsigned char smem[];
  const int n = a.n, nh = a.nh, ld = n + 1, NL = a.NL;
  C* bufA = (C*)smem;
  C* bufB = bufA + (size_t)NL * ld;
  const long long npairs = (long long)a.nc * n / 2;
  const long long p0 = (long long)blockIdx.x * NL;
  const int nl = (int)((npairs - p0) < NL ? (npairs - p0) : NL);
  float* fa = (float*)bufA;
  if (MODE == 0) {
    const unsigned long long seed = a.state[0], real = a.state[1];
    const int chunks = n / 4;
    for (int t = threadIdx.x; t < nl * 2 * chunks; t += 256) {
      const int l = t / (2 * chunks), rem = t - l * 2 * chunks, rsel = rem / chunks, ch = rem - rsel * chunks;
      const long long row = 2 * (p0 + l) + rsel;
      const unsigned long long c = (unsigned long long)((row * n) / 4 + ch);
      float z[4];
      normals4(c, seed, real, z);
#pragma unroll
      for (int q = 0; q < 4; ++q) fa[2 * ((size_t)l * ld + 4 * ch + q) + rsel] = z[q];
    }
  } else {
    const float f = (float)a.fng;
    const float m = (float)a.stat[1];
    for (int t = threadIdx.x; t < nl * 2 * n; t += 256) {
      const int l = t / (2 * n), rem = t - l * 2 * n, rsel = rem / n, y = rem - rsel * n;
      const long long row = 2 * (p0 + l) + rsel;
      const float gv = a.g[row * n + y];
      fa[2 * ((size_t)l * ld + y) + rsel] = gv + f * (gv * gv - m);
    }
  }
  __syncthreads();
  C* R = bufA;
  if constexpr (IP > 0) lds_fft_ip<-1, float, IP>(bufA, a.pn, nl, (const C*)a.tw_n, 1, ld);
  else R = lds_fft<-1, float>(bufA, bufB, a.pn, nl, (const C*)a.tw_n, 1, ld);
  // split Z = X0 + i X1 into the two real rows' half spectra
  for (int t = threadIdx.x; t < nl * nh; t += 256) {
    const int l = t / nh, k = t - l * nh;
    const C zk = R[(size_t)l * ld + k];
    const C zm = R[(size_t)l * ld + ((n - k) % n)];
    C x0, x1;
    x0.x = 0.5f * (zk.x + zm.x);
    x0.y = 0.5f * (zk.y - zm.y);
    x1.x = 0.5f * (zk.y + zm.y);
    x1.y = -0.5f * (zk.x - zm.x);
    const long long row = 2 * (p0 + l);
    a.W[row * nh + k] = x0;
    a.W[(row + 1) * nh + k] = x1;
  }
}

// Inverse along y of two half spectra at once; writes g and per-block partial sums of g^2.
template <int IP>
__global__ __launch_bounds__(256) void k_gen_rows_c2r(GenArgs a) {
  extern __shared__ unsigned char smem[];
  const int n = a.n, nh = a.nh, ld = n + 1, NL = a.NL;
  C* bufA = (C*)smem;
  C* bufB = bufA + (size_t)NL * ld;
  const long long npairs = (long long)a.nc * n / 2;
  const long long p0 = (long long)blockIdx.x * NL;
  const int nl = (int)((npairs - p0) < NL ? (npairs - p0) : NL);
  for (int t = threadIdx.x; t < nl * n; t += 256) {
    const int l = t / n, k = t - l * n;
    const long long row = 2 * (p0 + l);
    const int kk = k < nh ? k : n - k;
    C x0 = a.W[row * nh + kk], x1 = a.W[(row + 1) * nh + kk];
    if (k == 0 || 2 * k == n) { x0.y = 0.f; x1.y = 0.f; }  // self-conjugate terms are real
    if (k >= nh) { x0.y = -x0.y; x1.y = -x1.y; }           // Hermitian extension
    C z;
    z.x = x0.x - x1.y;
    z.y = x0.y + x1.x;
    bufA[(size_t)l * ld + k] = z;
  }
  __syncthreads();
  C* R = bufA;
  if constexpr (IP > 0) lds_fft_ip<1, float, IP>(bufA, a.pn, nl, (const C*)a.tw_n, 1, ld);
  else R = lds_fft<1, float>(bufA, bufB, a.pn, nl, (const C*)a.tw_n, 1, ld);
  const float sc = (float)(1.0 / ((double)a.nc * n * n));
  double s2 = 0.0;
  for (int t = threadIdx.x; t < nl * n; t += 256) {
    const int l = t / n, y = t - l * n;
    const long long row = 2 * (p0 + l);
    const C z = R[(size_t)l * ld + y];
    const float g0 = z.x * sc, g1 = z.y * sc;
    a.g[row * n + y] = g0;
    a.g[(row + 1) * n + y] = g1;
    s2 += (double)g0 * g0 + (double)g1 * g1;
  }
  __shared__ double red[256];
  __syncthreads();
  red[threadIdx.x] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[blockIdx.x] = red[0];
}

// stat[1] = mean g^2 over the nparts block sums (fixed order).
__global__ __launch_bounds__(256) void k_gen_mean(GenArgs a, int nparts) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += a.part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.stat[1] = red[0] / ((double)a.nc * a.n * a.n);
}

// ---------------------------------------------------------------- C2C along a strided axis
// Lines: the W elements (o, l, b) with l the transform index; o in [0, outer), b in [0, inner),
// address (o L + l) inner + b.  A block takes NL consecutive lines of the flattened (o, b) order,
// so consecutive lines are consecutive addresses.
// OP 0: forward; 1: inverse; 2: forward, times sqrt(A P), inverse (z axis, outer = 1);
// 3: forward, times w(o) (x axis, o = z).
// IP > 0: in-place FFT with at most IP butterflies per thread (one line buffer), else two buffers.
template <int OP, int IP>
__global__ __launch_bounds__(256) void k_gen_axis(GenArgs a, int L, int outer, int inner, int NL) {
  extern __shared__ unsigned char smem[];
  const int ld = L + 1;
  C* bufA = (C*)smem;
  C* bufB = bufA + (size_t)NL * ld;
  long long* base = (long long*)(bufA + (size_t)NL * ld * (IP > 0 ? 1 : 2));
  const long long nlines = (long long)outer * inner;
  const long long g0 = (long long)blockIdx.x * NL;
  const int nl = (int)((nlines - g0) < NL ? (nlines - g0) : NL);
  if ((int)threadIdx.x < nl) {
    const long long gl = g0 + threadIdx.x;
    const long long o = gl / inner, b = gl - o * inner;
    base[threadIdx.x] = o * (long long)L * inner + b;
  }
  __syncthreads();
  // eight loads in flight per thread before their LDS stores
  for (int t0 = threadIdx.x; t0 < L * NL; t0 += 8 * 256) {
    C v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * 256, l = t / NL, bl = t - l * NL;
      if (t < L * NL && bl < nl) v[u] = a.W[base[bl] + (long long)l * inner];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * 256, l = t / NL, bl = t - l * NL;
      if (t < L * NL && bl < nl) bufA[(size_t)bl * ld + l] = v[u];
    }
  }
  __syncthreads();
  const C* tw = (const C*)(L == a.n ? a.tw_n : a.tw_nc);
  const FftPlan& pl = (L == a.n) ? a.pn : a.pnc;
  C* R = bufA;
  if constexpr (IP > 0) {
    if (OP == 1) lds_fft_ip<1, float, IP>(bufA, pl, nl, tw, 1, ld);
    else lds_fft_ip<-1, float, IP>(bufA, pl, nl, tw, 1, ld);
  } else if (OP == 1) {
    R = lds_fft<1, float>(bufA, bufB, pl, nl, tw, 1, ld);
  } else {
    R = lds_fft<-1, float>(bufA, bufB, pl, nl, tw, 1, ld);
  }
  if (OP == 2) {
    const float sqrtA = (float)a.stat[0];
    const float e4 = (float)(0.25 * a.index);
    for (int t = threadIdx.x; t < L * nl; t += 256) {
      const int bl = t / L, l = t - bl * L;
      const long long gl = g0 + bl;             // outer == 1: line = x nh + y
      const int x = (int)(gl / a.nh), y = (int)(gl - (long long)x * a.nh);
      const float kz = (float)(a.cz * signed_idx(l, a.nc));
      const float kx = (float)(a.cxy * signed_idx(x, a.n));
      const float ky = (float)(a.cxy * y);
      const float s = spec_amp(kz * kz + kx * kx + ky * ky, sqrtA, e4, a.m2);
      R[(size_t)bl * ld + l] = cscale(R[(size_t)bl * ld + l], s);
    }
    __syncthreads();
    if constexpr (IP > 0) {
      lds_fft_ip<1, float, IP>(R, pl, nl, tw, 1, ld);
    } else {
      C* other = (R == bufA) ? bufB : bufA;
      R = lds_fft<1, float>(R, other, pl, nl, tw, 1, ld);
    }
  }
  for (int t = threadIdx.x; t < L * NL; t += 256) {
    const int l = t / NL, bl = t - l * NL;
    if (bl < nl) {
      C v = R[(size_t)bl * ld + l];
      if (OP == 3 && a.chw) {
        const long long o = base[bl] / ((long long)L * inner);
        v = cscale(v, a.chw[o]);
      }
      a.W[base[bl] + (long long)l * inner] = v;
    }
  }
}

// ---------------------------------------------------------------- Monte Carlo accumulators
// Welford update of the per-triangle mean and M2 with one realization's B (NaN entries skipped),
// then the realization counter of the generator state advances by one.
__global__ __launch_bounds__(256) void k_mc_accumulate(const double* __restrict__ B, int ntri,
                                                      long long* __restrict__ cnt, double* __restrict__ mean,
                                                      double* __restrict__ m2, unsigned long long* state) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < ntri) {
    const double b = B[t];
    if (b == b) {
      const long long k = cnt[t] + 1;
      const double d = b - mean[t];
      const double mu = mean[t] + d / (double)k;
      m2[t] += d * (b - mu);
      mean[t] = mu;
      cnt[t] = k;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) state[1] += 1ULL;
}

__global__ void k_mc_zero(long long* cnt, double* mean, double* m2, int ntri) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < ntri) { cnt[t] = 0; mean[t] = 0.0; m2[t] = 0.0; }
}

__global__ void k_gen_set_state(unsigned long long* state, unsigned long long seed, unsigned long long real) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { state[0] = seed; state[1] = real; }
}

template <typename K>
void set_lds(K k, size_t lds) {
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace

// ---------------------------------------------------------------- launchers
void launch_gen_amp(const GenArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_psum, dim3(a.nc), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_gen_amp, dim3(1), dim3(64), 0, s, a);
}

void launch_gen_set_state(unsigned long long* state, unsigned long long seed, unsigned long long real, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_set_state, dim3(1), dim3(64), 0, s, state, seed, real);
}

template <int OP>
static void launch_axis(const GenArgs& a, int ip, int nb, size_t lds, hipStream_t s, int L, int outer, int inner, int NL) {
  if (ip == 2) { set_lds(k_gen_axis<OP, 2>, lds); hipLaunchKernelGGL((k_gen_axis<OP, 2>), dim3(nb), dim3(256), lds, s, a, L, outer, inner, NL); }
  else if (ip == 4) { set_lds(k_gen_axis<OP, 4>, lds); hipLaunchKernelGGL((k_gen_axis<OP, 4>), dim3(nb), dim3(256), lds, s, a, L, outer, inner, NL); }
  else { set_lds(k_gen_axis<OP, 0>, lds); hipLaunchKernelGGL((k_gen_axis<OP, 0>), dim3(nb), dim3(256), lds, s, a, L, outer, inner, NL); }
}

int gen_row_blocks(const GenArgs& a) {
  const long long npairs = (long long)a.nc * a.n / 2;
  return (int)((npairs + a.NL - 1) / a.NL);
}

template <int IP>
static void launch_rows(const GenArgs& a, int which, int rb, size_t lds, hipStream_t s) {
  if (which == 0) { set_lds(k_gen_rows_fwd<0, IP>, lds); hipLaunchKernelGGL((k_gen_rows_fwd<0, IP>), dim3(rb), dim3(256), lds, s, a); }
  else if (which == 1) { set_lds(k_gen_rows_fwd<1, IP>, lds); hipLaunchKernelGGL((k_gen_rows_fwd<1, IP>), dim3(rb), dim3(256), lds, s, a); }
  else { set_lds(k_gen_rows_c2r<IP>, lds); hipLaunchKernelGGL((k_gen_rows_c2r<IP>), dim3(rb), dim3(256), lds, s, a); }
}
// which: 0 = forward rows from white noise, 1 = forward rows of delta, 2 = inverse rows (C2R)
static void launch_rows_ip(const GenArgs& a, int which, int rb, size_t lds, hipStream_t s) {
  if (a.ipx == 2) launch_rows<2>(a, which, rb, lds, s);
  else if (a.ipx == 4) launch_rows<4>(a, which, rb, lds, s);
  else launch_rows<0>(a, which, rb, lds, s);
}

void launch_gen_cube(const GenArgs& a, hipStream_t s) {
  // the rows use the plan and line count of the x passes (a.NL == a.NLx), hence a.ipx
  const size_t lds_rows = (a.ipx ? 1 : 2) * (size_t)a.NL * (a.n + 1) * sizeof(C);
  const int rb = gen_row_blocks(a);
  // axis passes: x (L = n, outer = nc, inner = nh), z (L = nc, outer = 1, inner = n nh)
  const int NLx = a.NLx, NLz = a.NLz;
  const size_t lds_x = (a.ipx ? 1 : 2) * (size_t)NLx * (a.n + 1) * sizeof(C) + (size_t)NLx * 8;
  const size_t lds_z = (a.ipz ? 1 : 2) * (size_t)NLz * (a.nc + 1) * sizeof(C) + (size_t)NLz * 8;
  const long long lx = (long long)a.nc * a.nh, lz = (long long)a.n * a.nh;
  const int bx = (int)((lx + NLx - 1) / NLx), bz = (int)((lz + NLz - 1) / NLz);
  launch_rows_ip(a, 0, rb, lds_rows, s);
  launch_axis<0>(a, a.ipx, bx, lds_x, s, a.n, a.nc, a.nh, NLx);
  launch_axis<2>(a, a.ipz, bz, lds_z, s, a.nc, 1, a.n * a.nh, NLz);
  launch_axis<1>(a, a.ipx, bx, lds_x, s, a.n, a.nc, a.nh, NLx);
  launch_rows_ip(a, 2, rb, lds_rows, s);
  hipLaunchKernelGGL(k_gen_mean, dim3(1), dim3(256), 0, s, a, rb);
  launch_rows_ip(a, 1, rb, lds_rows, s);
  launch_axis<3>(a, a.ipx, bx, lds_x, s, a.n, a.nc, a.nh, NLx);
}

void launch_mc_accumulate(const double* B, int ntri, long long* cnt, double* mean, double* m2,
                          unsigned long long* state, hipStream_t s) {
  hipLaunchKernelGGL(k_mc_accumulate, dim3((ntri + 255) / 256), dim3(256), 0, s, B, ntri, cnt, mean, m2, state);
}

void launch_mc_zero(long long* cnt, double* mean, double* m2, int ntri, hipStream_t s) {
  if (ntri > 0) hipLaunchKernelGGL(k_mc_zero, dim3((ntri + 255) / 256), dim3(256), 0, s, cnt, mean, m2, ntri);
}
