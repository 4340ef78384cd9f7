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
constexpr int MONO_NB = 4;   // cells of a row per thread and step (loads in flight)

// number of shape edges 0.6 .. 0.9 at or below x in [0.5, 1]: the half-open bin, last bin closed
__device__ __forceinline__ int shape_bin(double x) {
  return (x >= 0.6) + (x >= 0.7) + (x >= 0.8) + (x >= 0.9);
}

// (k1, mu, t) of one cell; returns the bin index, or -1 when k1 lies outside the edges.  lo2 / hi2
// bound the squared largest side from outside the edges with a relative margin of 2^-20 on k1, far above
// rounding: a cell beyond them is dropped without the square roots, the rest take the exact path.
__device__ int cell_bin(const double* __restrict__ k1e, int nk, double lo2, double hi2, double kq0, double kq1,
                        double kq2, double kp1, double kp2) {
#pragma clang fp contract(off)
  const double kp3 = -(kp1 + kp2);
  const double s0 = kq0 * kq0 + kp1 * kp1;
  const double s1 = kq1 * kq1 + kp2 * kp2;
  const double s2 = kq2 * kq2 + kp3 * kp3;
  // the three squared sides in descending order (exact selections)
  const double hi = fmax(s0, fmax(s1, s2)), lo = fmin(s0, fmin(s1, s2));
  if (hi < lo2 || hi > hi2) return -1;
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
  const double elo = k1e[0] * (1.0 - 0x1p-20), ehi = k1e[a.nk] * (1.0 + 0x1p-20);
  const double lo2 = elo * elo, hi2 = ehi * ehi;
  const int nc = a.nc, lane = threadIdx.x & 63;
  for (int row = blockIdx.x; row < a.nt * nc; row += gridDim.x) {
    const int t = row / nc, ai = row - t * nc;
    const double kq0 = a.kperp[3 * t], kq1 = a.kperp[3 * t + 1], kq2 = a.kperp[3 * t + 2];
    const double kp1 = a.kpar_unit * (double)(2 * ai < nc ? ai : ai - nc);
    const double* __restrict__ rowp = a.B + 2 * (long long)row * nc;
    for (int b0 = 0; b0 < nc; b0 += MONO_NB * MONO_THREADS) {   // the same trip count for every lane
      // the row's values first (MONO_NB loads in flight), then their bins
      double v[MONO_NB];
      int bin[MONO_NB];
#pragma unroll
      for (int u = 0; u < MONO_NB; ++u) {
        const int b = b0 + u * MONO_THREADS + threadIdx.x;
        v[u] = b < nc ? rowp[2 * b] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < MONO_NB; ++u) {
        const int b = b0 + u * MONO_THREADS + threadIdx.x;
        bin[u] = b < nc ? cell_bin(k1e, a.nk, lo2, hi2, kq0, kq1, kq2, kp1,
                                   a.kpar_unit * (double)(2 * b < nc ? b : b - nc))
                        : -1;
      }
#pragma unroll
      for (int u = 0; u < MONO_NB; ++u) {
        unsigned long long m = __ballot(bin[u] >= 0);
        while (m) {
          const int leader = __ffsll((long long)m) - 1;
          const int lb = __shfl(bin[u], leader);
          const bool mine = bin[u] == lb;
          const unsigned long long mm = __ballot(mine);
          const double x = wave_sum(mine ? v[u] : 0.0);
          if (lane == leader) {
            atomicAdd(&ssum[lb], x);
            atomicAdd(&scnt[lb], (int)__popcll(mm));
          }
          m &= ~mm;
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += MONO_THREADS) {
    a.psum[(long long)blockIdx.x * nb + i] = ssum[i];
    a.pcnt[(long long)blockIdx.x * nb + i] = scnt[i];
  }
}

// One block per bin: thread k adds the partials of blocks k, k + 256, ... in order, then a fixed
// tree in LDS; the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_mono_fin(MonoArgs a, int nblocks, double* __restrict__ mean,
                                                  int64_t* __restrict__ count) {
  __shared__ double ss[256];
  __shared__ long long sc[256];
  const int nb = a.nk * 25, i = blockIdx.x;
  double s = 0.0;
  long long c = 0;
  for (int k = threadIdx.x; k < nblocks; k += 256) {
    s += a.psum[(long long)k * nb + i];
    c += a.pcnt[(long long)k * nb + i];
  }
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      ss[threadIdx.x] += ss[threadIdx.x + o];
      sc[threadIdx.x] += sc[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mean[i] = sc[0] > 0 ? ss[0] / (double)sc[0] : __builtin_nan("");
    count[i] = sc[0];
  }
}

}  // namespace

void launch_mono_bin(const MonoArgs& a, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_mono_bin, dim3(nblocks), dim3(MONO_THREADS), 0, s, a);
}

void launch_mono_fin(const MonoArgs& a, int nblocks, double* mean, int64_t* count, hipStream_t s) {
  hipLaunchKernelGGL(k_mono_fin, dim3(a.nk * 25), dim3(256), 0, s, a, nblocks, mean, count);
}
