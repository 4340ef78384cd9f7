// Eq. (dft): the 2D DFT that takes the ergodically collapsed MABS over the channel separations
// (dnu1, dnu2) = (n, m) channels to the cylindrical 3D bispectrum at (k_par1 a, k_par2 b).
// The sum runs over n, m in the half-open range [-L/2, L/2) (one period: the printed limits
// would count the end separation twice), i.e. a length-L DFT of the window laid out by residue,
// so each axis is one FP64 LDS FFT.  The input is real, hence the output is Hermitian: the pass
// along n keeps the half spectrum a < H = L/2 + 1 and the pass along m writes row L - a as the
// mirror of row a, so that the output leaves in whole contiguous rows.
#include <hip/hip_runtime.h>

#include "bs_kernels.h"

namespace {

using C = Cx<double>;
constexpr int MDFT_THREADS = 512;   // largest block; the host picks 256 or 512
constexpr int MDFT_NB = 8;          // loads in flight per thread

// array index of separation d in [-h, h]: non-circular collapse at d + L - 1, circular at d mod L
__device__ __forceinline__ int sep_index(const MdftArgs& a, int d) { return a.circ ? (d < 0 ? d + a.L : d) : d + a.L - 1; }

__device__ __forceinline__ double nan0(double v) { return v == v ? v : 0.0; }

// Window entry at residues (r, c): separations n = r and m = c below L - h, else r - L and c - L,
// so that n, m run over [-h, L - 1 - h], one period with each separation once.
__device__ __forceinline__ double window_at(const MdftArgs& a, const double* __restrict__ Bt, int r, int c) {
  const int lim = a.L - 1 - a.h;
  const int rm = sep_index(a, r <= lim ? r : r - a.L), cm = sep_index(a, c <= lim ? c : c - a.L);
  return nan0(Bt[(long long)rm * a.S + cm]);
}

// Both passes loop over work groups (triangle, block of lines) so that each block copies the
// twiddle table into LDS once.  Blocks take groups in a strided order: the groups in flight at any
// time are neighbours, which keeps the HBM accesses of the whole grid on a narrow band of pages.
//
// Pass n: W = 2 CB window columns (residues) c0 .. c0 + W - 1 per group, columns 2q and 2q + 1 packed
// into complex line q (z = x0 + i x1), transformed along n; the half spectra a < H of both columns
// go to Y[t][a][c] (runs of W contiguous entries per a).
template <int BM>
__global__ __launch_bounds__(MDFT_THREADS) void k_mdft_n(MdftArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  C* tw = reinterpret_cast<C*>(smem);
  C* A = tw + a.L;
  double* Ad = reinterpret_cast<double*>(A);
  const int L = a.L, H = a.H, CB = a.nl, lg = a.lgnl + 1, ld = a.ld;
  const int W = 2 * CB;
  const C* __restrict__ twg = static_cast<const C*>(a.tw);
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = twg[i];
  const int gx = (L + W - 1) / W;
  const int total = W * L;
  for (int g = blockIdx.x; g < a.nt * gx; g += gridDim.x) {
    const int t = g / gx;
    const int c0 = (g - t * gx) * W;
    const double* __restrict__ Bt = a.B + (long long)t * a.S * a.S;
    // consecutive threads take consecutive columns of one row (W * 8 contiguous bytes); the first
    // chunk is loaded by every thread before the barrier that frees the previous group's lines
    auto load = [&](int base, double* v) {
#pragma unroll
      for (int u = 0; u < MDFT_NB; ++u) {
        const int i = base + u * blockDim.x;
        const int c = c0 + (i & (W - 1));
        v[u] = i < total && c < L ? window_at(a, Bt, i >> lg, c) : 0.0;
      }
    };
    auto store = [&](int base, const double* v) {
#pragma unroll
      for (int u = 0; u < MDFT_NB; ++u) {
        const int i = base + u * blockDim.x;
        const int k = i & (W - 1);
        if (i < total) Ad[2 * ((k >> 1) * ld + (i >> lg)) + (k & 1)] = v[u];
      }
    };
    double v[MDFT_NB];
    load(threadIdx.x, v);
    __syncthreads();
    store(threadIdx.x, v);
    for (int base = threadIdx.x + MDFT_NB * blockDim.x; base < total; base += MDFT_NB * blockDim.x) {
      load(base, v);
      store(base, v);
    }
    __syncthreads();
    lds_fft_ip<-1, double, BM>(A, a.plan, CB, tw, 1, ld);
    // z = x0 + i x1 transformed: X0[a] = (Z[a] + conj Z[-a]) / 2, X1[a] = (Z[a] - conj Z[-a]) / (2i)
    C* __restrict__ Y = static_cast<C*>(a.X) + (long long)t * H * L;
    for (int i = threadIdx.x; i < W * H; i += blockDim.x) {
      const int k = i & (W - 1), e = i >> lg;
      const int c = c0 + k;
      if (c >= L) continue;
      const C* line = A + (k >> 1) * ld;
      const C z = line[e];
      const C zm = cconj(line[e ? L - e : 0]);
      C y;
      if (k & 1) {
        const C d = csub(z, zm);
        y = cmk(0.5 * d.y, -0.5 * d.x);
      } else {
        y = cscale(cadd(z, zm), 0.5);
      }
      Y[(long long)e * L + c] = y;
    }
  }
}

// Pass m: NL rows a < H of Y per group, transformed along m, scaled; row a of the output and its
// Hermitian mirror, row L - a, are written whole.
template <int BM>
__global__ __launch_bounds__(MDFT_THREADS) void k_mdft_m(MdftArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  C* tw = reinterpret_cast<C*>(smem);
  C* A = tw + a.L;
  const int L = a.L, H = a.H, NL = a.nl;
  const C* __restrict__ twg = static_cast<const C*>(a.tw);
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = twg[i];
  const float rL = 1.0f / (float)L;
  const int gx = (H + NL - 1) / NL;
  const int total = NL * L;
  const double sc = a.scale;
  for (int g = blockIdx.x; g < a.nt * gx; g += gridDim.x) {
    const int t = g / gx;
    const int e0 = (g - t * gx) * NL;
    const C* __restrict__ Y = static_cast<const C*>(a.X) + (long long)t * H * L;
    auto load = [&](int base, C* v) {
#pragma unroll
      for (int u = 0; u < MDFT_NB; ++u) {
        const int i = base + u * blockDim.x;
        int p, c;
        fdivmod(i, L, rL, p, c);
        v[u] = i < total && e0 + p < H ? Y[(long long)(e0 + p) * L + c] : cmk(0.0, 0.0);
      }
    };
    auto store = [&](int base, const C* v) {
#pragma unroll
      for (int u = 0; u < MDFT_NB; ++u) {
        const int i = base + u * blockDim.x;
        if (i < total) A[i] = v[u];
      }
    };
    C v[MDFT_NB];
    load(threadIdx.x, v);
    __syncthreads();
    store(threadIdx.x, v);
    for (int base = threadIdx.x + MDFT_NB * blockDim.x; base < total; base += MDFT_NB * blockDim.x) {
      load(base, v);
      store(base, v);
    }
    __syncthreads();
    lds_fft_ip<-1, double, BM>(A, a.plan, NL, tw, 1, L);
    C* __restrict__ out = static_cast<C*>(a.out) + (long long)t * L * L;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
      int p, b;
      fdivmod(i, L, rL, p, b);
      const int e = e0 + p;
      if (e >= H) continue;
      const C val = cscale(A[i], sc);
      out[(long long)e * L + b] = val;
      // real input: out(-a, -b) = conj out(a, b) fills the rows a >= H
      if (e >= 1 && L - e >= H) out[(long long)(L - e) * L + (b ? L - b : 0)] = cconj(val);
    }
  }
}

void launch_mdft(void (*k)(MdftArgs), int groups, size_t lds, const MdftArgs& a, hipStream_t s) {
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(a.grid < groups ? a.grid : groups), dim3(a.threads), lds, s, a);
}

}  // namespace

void launch_mdft_n(const MdftArgs& a, size_t lds, hipStream_t s) {
  const int groups = a.nt * ((a.L + 2 * a.nl - 1) / (2 * a.nl));
  launch_mdft(a.bm == 2 ? k_mdft_n<2> : k_mdft_n<4>, groups, lds, a, s);
}

void launch_mdft_m(const MdftArgs& a, size_t lds, hipStream_t s) {
  const int groups = a.nt * ((a.H + a.nl - 1) / a.nl);
  launch_mdft(a.bm == 2 ? k_mdft_m<2> : k_mdft_m<4>, groups, lds, a, s);
}
