// Monopole of the cylindrical 3D bispectrum (Sec. 2.2 Eq. shape, Sec. 5): every cell (t, a, b) of
// the output of Eq. (dft) is a triangle with sides k_i = sqrt(kperp_i^2 + kpar_i^2), kpar_1,2 the
// line-of-sight wave numbers of a and b and kpar_3 = -(kpar_1 + kpar_2).  Ordered k1 >= k2 >= k3,
// its shape is t = k2 / k1 and mu = -k1.k2 / (k1 k2) = (k1^2 + k2^2 - k3^2) / (2 k1 k2) (closure),
// both clamped to [0.5, 1]; Re B of the cell goes to its (k1, mu, t) bin and the bin's mean is the
// monopole.  The bin decision is made in FP64 with every operation rounded on its own (no fused
// multiply-add), so that it is the same decision as a plain IEEE evaluation of the same formula.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bs_kernels.h"

namespace {

constexpr int MONO_THREADS = 256;

// number of shape edges 0.6 .. 0.9 at or below x in [0.5, 1]: the half-open bin, last bin closed
__device__ __forceinline__ int shape_bin(double x) {
  return (x >= 0.6) + (x >= 0.7) + (x >= 0.8) + (x >= 0.9);
}

// (k1, mu, t) of one cell; returns the bin index, or -1 when k1 lies outside the edges
__device__ int cell_bin(const double* __restrict__ k1e, int nk, double kq0, double kq1, double kq2, double kp1,
                        double kp2) {
#pragma clang fp contract(off)
  const double kp3 = -(kp1 + kp2);
  const double s0 = kq0 * kq0 + kp1 * kp1;
  const double s1 = kq1 * kq1 + kp2 * kp2;
  const double s2 = kq2 * kq2 + kp3 * kp3;
  // the three squared sides in descending order (exact selections)
  const double hi = fmax(s0, fmax(s1, s2)), lo = fmin(s0, fmin(s1, s2));
  const double mid = fmax(fmin(s0, s1), fmin(fmax(s0, s1), s2));
  const double k1 = sqrt(hi), k2 = sqrt(mid);
  double mu = ((hi + mid) - lo) / (2.0 * (k1 * k2));
  double t = k2 / k1;
  mu = fmin(fmax(mu, 0.5), 1.0);
  t = fmin(fmax(t, 0.5), 1.0);
  int j = -1;
  for (int e = 0; e <= nk; ++e) j += k1 >= k1e[e];
  if (j < 0 || j >= nk) return -1;
  return j * 25 + shape_bin(mu) * 5 + shape_bin(t);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Rows (t, a) in a strided order over the grid, threads over b.  Lanes of a wave that fall in the
// same bin are summed first (one LDS atomic per bin and wave); each block writes its partial bins.
__global__ __launch_bounds__(MONO_THREADS) void k_mono_bin(MonoArgs a) {
  __shared__ double ssum[MONO_MAX_K1 * 25];
  __shared__ int scnt[MONO_MAX_K1 * 25];
  __shared__ double k1e[MONO_MAX_K1 + 1];
  const int nb = a.nk * 25;
  for (int i = threadIdx.x; i < nb; i += MONO_THREADS) {
    ssum[i] = 0.0;
    scnt[i] = 0;
  }
  for (int i = threadIdx.x; i <= a.nk; i += MONO_THREADS) k1e[i] = a.k1e[i];
  __syncthreads();
  const int nc = a.nc, lane = threadIdx.x & 63;
  for (int row = blockIdx.x; row < a.nt * nc; row += gridDim.x) {
    const int t = row / nc, ai = row - t * nc;
    const double kq0 = a.kperp[3 * t], kq1 = a.kperp[3 * t + 1], kq2 = a.kperp[3 * t + 2];
    const double kp1 = a.kpar_unit * (double)(2 * ai < nc ? ai : ai - nc);
    const double* __restrict__ rowp = a.B + 2 * (long long)row * nc;
    for (int b0 = 0; b0 < nc; b0 += MONO_THREADS) {   // the same trip count for every lane
      const int b = b0 + threadIdx.x;
      int bin = -1;
      double v = 0.0;
      if (b < nc) {
        bin = cell_bin(k1e, a.nk, kq0, kq1, kq2, kp1, a.kpar_unit * (double)(2 * b < nc ? b : b - nc));
        v = rowp[2 * b];
      }
      unsigned long long m = __ballot(bin >= 0);
      while (m) {
        const int leader = __ffsll((long long)m) - 1;
        const int lb = __shfl(bin, leader);
        const bool mine = bin == lb;
        const unsigned long long mm = __ballot(mine);
        const double x = wave_sum(mine ? v : 0.0);
        if (lane == leader) {
          atomicAdd(&ssum[lb], x);
          atomicAdd(&scnt[lb], (int)__popcll(mm));
        }
        m &= ~mm;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += MONO_THREADS) {
    a.psum[(long long)blockIdx.x * nb + i] = ssum[i];
    a.pcnt[(long long)blockIdx.x * nb + i] = scnt[i];
  }
}

__global__ void k_mono_fin(MonoArgs a, int nblocks, double* __restrict__ mean, int64_t* __restrict__ count) {
  const int nb = a.nk * 25;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  double s = 0.0;
  long long c = 0;
  for (int k = 0; k < nblocks; ++k) {
    s += a.psum[(long long)k * nb + i];
    c += a.pcnt[(long long)k * nb + i];
  }
  mean[i] = c > 0 ? s / (double)c : __builtin_nan("");
  count[i] = c;
}

}  // namespace

void launch_mono_bin(const MonoArgs& a, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_mono_bin, dim3(nblocks), dim3(MONO_THREADS), 0, s, a);
}

void launch_mono_fin(const MonoArgs& a, int nblocks, double* mean, int64_t* count, hipStream_t s) {
  const int nb = a.nk * 25;
  hipLaunchKernelGGL(k_mono_fin, dim3((nb + 255) / 256), dim3(256), 0, s, a, nblocks, mean, count);
}
