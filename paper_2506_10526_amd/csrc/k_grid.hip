// Eq. (vg): every visibility goes to the grid point nearest its baseline, q = rint(U / du) per
// axis, with the flag factor F; the grid is the half plane q_v >= 0 (a point with q_v < 0 stands
// for (-q_u, -q_v), the visibility conjugated; a point on the line q_v = 0, which the half plane
// stores whole, also enters at (-q_u, 0) conjugated), and chan_avg consecutive channels are gridded
// together.  A thread per visibility sums its channel group in registers and adds the group to the
// FP64 cell sums and the integer counts with atomics; the cell sums are then written in the output
// precision.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bs_kernels.h"

namespace {

constexpr int GRID_THREADS = 256;

__global__ void k_grid_zero(GridArgs a) {
  const long long cells = (long long)a.nco * a.n * (a.n / 2 + 1);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cells; i += (long long)gridDim.x * blockDim.x) {
    a.acc[2 * i] = 0.0;
    a.acc[2 * i + 1] = 0.0;
    a.cnt[i] = 0;
  }
}

// blockIdx.x: visibilities; blockIdx.y: output channels o = blockIdx.y, blockIdx.y + gridDim.y, ...
__global__ __launch_bounds__(GRID_THREADS) void k_grid_scatter(GridArgs a) {
  const long long i = blockIdx.x * (long long)GRID_THREADS + threadIdx.x;
  if (i >= a.nvis) return;
  const int n = a.n, nh = n / 2 + 1, half = n / 2;
  double qu = rint(a.uv[2 * i] / a.du), qv = rint(a.uv[2 * i + 1] / a.du);
  const bool neg = qv < 0.0;
  if (neg) {
    qu = -qu;
    qv = -qv;
  }
  if (!(fabs(qu) < (double)half && fabs(qv) < (double)half)) return;
  const int iu = (int)qu, iv = (int)qv;
  const long long cell = (long long)(iu < 0 ? iu + n : iu) * nh + iv;
  const long long cell_m = (long long)(iu > 0 ? n - iu : -iu) * nh;   // (-q_u mod n, 0)
  const long long plane = (long long)n * nh;
  const float2* __restrict__ vis = reinterpret_cast<const float2*>(a.vis);
  for (int o = blockIdx.y; o < a.nco; o += gridDim.y) {
    double re = 0.0, im = 0.0;
    int c = 0;
    for (int k = 0; k < a.chan_avg; ++k) {
      const long long j = (long long)(o * a.chan_avg + k) * a.nvis + i;
      if (a.flags && a.flags[j]) continue;
      const float2 v = vis[j];
      re += (double)v.x;
      im += neg ? -(double)v.y : (double)v.y;
      ++c;
    }
    if (c) {
      double* d = a.acc + 2 * (o * plane + cell);
      unsafeAtomicAdd(d, re);
      unsafeAtomicAdd(d + 1, im);
      atomicAdd(a.cnt + o * plane + cell, c);
      if (iv == 0) {   // the mirror baseline on the stored line q_v = 0: (-q_u, 0), conjugated
        double* e = a.acc + 2 * (o * plane + cell_m);
        unsafeAtomicAdd(e, re);
        unsafeAtomicAdd(e + 1, -im);
        atomicAdd(a.cnt + o * plane + cell_m, c);
      }
    }
  }
}

template <typename T>
__global__ void k_grid_fin(GridArgs a, T* __restrict__ out, int32_t* __restrict__ ng) {
  const long long cells = (long long)a.nco * a.n * (a.n / 2 + 1);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cells; i += (long long)gridDim.x * blockDim.x) {
    out[2 * i] = (T)__hip_atomic_load(a.acc + 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    out[2 * i + 1] = (T)__hip_atomic_load(a.acc + 2 * i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ng[i] = __hip_atomic_load(a.cnt + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

void launch_grid_zero(const GridArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_grid_zero, dim3(1024), dim3(256), 0, s, a);
}

void launch_grid_scatter(const GridArgs& a, hipStream_t s) {
  const unsigned bx = (unsigned)((a.nvis + GRID_THREADS - 1) / GRID_THREADS);
  const unsigned by = (unsigned)(a.nco < 64 ? a.nco : 64);
  hipLaunchKernelGGL(k_grid_scatter, dim3(bx, by), dim3(GRID_THREADS), 0, s, a);
}

void launch_grid_fin(const GridArgs& a, bool fp64, void* out, int32_t* ng, hipStream_t s) {
  if (fp64) hipLaunchKernelGGL(k_grid_fin<double>, dim3(1024), dim3(256), 0, s, a, static_cast<double*>(out), ng);
  else hipLaunchKernelGGL(k_grid_fin<float>, dim3(1024), dim3(256), 0, s, a, static_cast<float*>(out), ng);
}
