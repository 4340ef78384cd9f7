// Eq. (dft): the 2D DFT that takes the ergodically collapsed MABS over the channel separations
// (dnu1, dnu2) = (n, m) channels to the cylindrical 3D bispectrum at (k_par1 a, k_par2 b).
// The sum runs over n, m in [-h, h], h = L / 2, both ends included; it is a length-L DFT of the
// window folded by residue (for even L the two ends n = +-h share a residue), so each axis is one
// FP64 LDS FFT.  The input is real, hence the output is Hermitian: the row pass keeps the half
// spectrum b < H = L/2 + 1 and the column pass writes column L - b as the mirror of column b.
#include <hip/hip_runtime.h>

#include "bs_kernels.h"

namespace {

using C = Cx<double>;
constexpr int MDFT_THREADS = 512;   // largest block; the host picks 256 or 512

// array index of separation d in [-h, h]: non-circular collapse at d + L - 1, circular at d mod L
__device__ __forceinline__ int sep_index(const MdftArgs& a, int d) { return a.circ ? (d < 0 ? d + a.L : d) : d + a.L - 1; }

__device__ __forceinline__ double nan0(double v) { return v == v ? v : 0.0; }

// Folded window entry at residues (r, c): the separations n = r or r - L and m = c or c - L that lie
// in [-h, h].  Every residue has one such separation; for even L the residue h has two (n = +-h).
__device__ __forceinline__ double fold_at(const MdftArgs& a, const double* __restrict__ Bt, int r, int c) {
  const int L = a.L, h = a.h;
  const long long S = a.S;
  const int rm = sep_index(a, r <= h ? r : r - L), cm = sep_index(a, c <= h ? c : c - L);
  double s = nan0(Bt[rm * S + cm]);
  const bool er = (L & 1) == 0 && r == h, ec = (L & 1) == 0 && c == h;
  if (er | ec) {   // the second end of the range: rows / columns n = -h
    const int rx = sep_index(a, -h), cx = sep_index(a, -h);
    if (er) s += nan0(Bt[rx * S + cm]);
    if (ec) s += nan0(Bt[rm * S + cx]);
    if (er && ec) s += nan0(Bt[rx * S + cx]);
  }
  return s;
}

constexpr int MDFT_NB = 8;   // loads in flight per thread

// Both passes loop over work groups (triangle, block of lines) so that each block copies the
// twiddle table into LDS once.
template <int BM>
__global__ __launch_bounds__(MDFT_THREADS) void k_mdft_rows(MdftArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  C* tw = reinterpret_cast<C*>(smem);
  C* A = tw + a.L;
  const int L = a.L, H = a.H, NL = a.nl;
  const C* __restrict__ twg = static_cast<const C*>(a.tw);
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = twg[i];
  const float rL = 1.0f / (float)L, rH = 1.0f / (float)H;
  const int gx = (L + 2 * NL - 1) / (2 * NL);
  const int total = NL * L;
  for (int g = blockIdx.x; g < a.nt * gx; g += gridDim.x) {
    const int t = g / gx;
    const int r0 = (g - t * gx) * 2 * NL;
    const double* __restrict__ Bt = a.B + (long long)t * a.S * a.S;
    // both rows of a line pair in registers for MDFT_NB elements before they go to LDS; the first
    // chunk is loaded by every thread before the barrier that frees the previous group's lines
    auto load = [&](int base, double* v0, double* v1) {
#pragma unroll
      for (int u = 0; u < MDFT_NB; ++u) {
        const int i = base + u * blockDim.x;
        v0[u] = 0.0;
        v1[u] = 0.0;
        if (i < total) {
          int p, c;
          fdivmod(i, L, rL, p, c);
          const int r = r0 + 2 * p;
          if (r < L) v0[u] = fold_at(a, Bt, r, c);
          if (r + 1 < L) v1[u] = fold_at(a, Bt, r + 1, c);
        }
      }
    };
    auto store = [&](int base, const double* v0, const double* v1) {
#pragma unroll
      for (int u = 0; u < MDFT_NB; ++u) {
        const int i = base + u * blockDim.x;
        if (i < total) A[i] = cmk(v0[u], v1[u]);
      }
    };
    double v0[MDFT_NB], v1[MDFT_NB];
    load(threadIdx.x, v0, v1);
    __syncthreads();
    store(threadIdx.x, v0, v1);
    for (int base = threadIdx.x + MDFT_NB * blockDim.x; base < total; base += MDFT_NB * blockDim.x) {
      load(base, v0, v1);
      store(base, v0, v1);
    }
    __syncthreads();
    lds_fft_ip<-1, double, BM>(A, a.plan, NL, tw, 1, L);
    // z = x0 + i x1 transformed: X0[b] = (Z[b] + conj Z[-b]) / 2, X1[b] = (Z[b] - conj Z[-b]) / (2i)
    C* __restrict__ X = static_cast<C*>(a.X) + (long long)t * L * H;
    for (int i = threadIdx.x; i < NL * H; i += blockDim.x) {
      int p, b;
      fdivmod(i, H, rH, p, b);
      const C z = A[p * L + b];
      const C zm = cconj(A[p * L + (b ? L - b : 0)]);
      const int r = r0 + 2 * p;
      if (r < L) X[(long long)r * H + b] = cscale(cadd(z, zm), 0.5);
      if (r + 1 < L) {
        const C d = csub(z, zm);
        X[(long long)(r + 1) * H + b] = cmk(0.5 * d.y, -0.5 * d.x);
      }
    }
  }
}

template <int BM>
__global__ __launch_bounds__(MDFT_THREADS) void k_mdft_cols(MdftArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  C* tw = reinterpret_cast<C*>(smem);
  C* A = tw + a.L;
  const int L = a.L, H = a.H, CB = a.nl, lg = a.lgnl, ld = a.ld;
  const C* __restrict__ twg = static_cast<const C*>(a.tw);
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = twg[i];
  const int gx = (H + CB - 1) / CB;
  const int total = CB * L;
  const double sc = a.scale;
  for (int g = blockIdx.x; g < a.nt * gx; g += gridDim.x) {
    const int t = g / gx;
    const int b0 = (g - t * gx) * CB;
    const C* __restrict__ X = static_cast<const C*>(a.X) + (long long)t * L * H;
    // consecutive threads take consecutive columns of one row: CB * 16 contiguous bytes per row;
    // the first chunk is loaded by every thread before the barrier that frees the previous lines
    auto load = [&](int base, C* v) {
#pragma unroll
      for (int u = 0; u < MDFT_NB; ++u) {
        const int i = base + u * blockDim.x;
        const int b = b0 + (i & (CB - 1));
        v[u] = i < total && b < H ? X[(long long)(i >> lg) * H + b] : cmk(0.0, 0.0);
      }
    };
    auto store = [&](int base, const C* v) {
#pragma unroll
      for (int u = 0; u < MDFT_NB; ++u) {
        const int i = base + u * blockDim.x;
        if (i < total) A[(i & (CB - 1)) * ld + (i >> lg)] = v[u];
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
    lds_fft_ip<-1, double, BM>(A, a.plan, CB, tw, 1, ld);
    C* __restrict__ out = static_cast<C*>(a.out) + (long long)t * L * L;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
      const int j = i & (CB - 1), k = i >> lg;
      const int b = b0 + j;
      if (b >= H) continue;
      const C v = cscale(A[j * ld + k], sc);
      out[(long long)k * L + b] = v;
      // real input: out(-a, -b) = conj out(a, b) fills the columns b >= H
      if (b >= 1 && L - b >= H) out[(long long)(k ? L - k : 0) * L + (L - b)] = cconj(v);
    }
  }
}

void launch_mdft(void (*k)(MdftArgs), int groups, size_t lds, const MdftArgs& a, hipStream_t s) {
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(a.grid < groups ? a.grid : groups), dim3(a.threads), lds, s, a);
}

}  // namespace

void launch_mdft_rows(const MdftArgs& a, size_t lds, hipStream_t s) {
  const int groups = a.nt * ((a.L + 2 * a.nl - 1) / (2 * a.nl));
  launch_mdft(a.bm == 2 ? k_mdft_rows<2> : k_mdft_rows<4>, groups, lds, a, s);
}

void launch_mdft_cols(const MdftArgs& a, size_t lds, hipStream_t s) {
  const int groups = a.nt * ((a.H + a.nl - 1) / a.nl);
  launch_mdft(a.bm == 2 ? k_mdft_cols<2> : k_mdft_cols<4>, groups, lds, a, s);
}
