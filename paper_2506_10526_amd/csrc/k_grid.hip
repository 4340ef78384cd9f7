// Eq. (vg): every visibility goes to the grid point nearest its baseline, q = rint(U / du) per
// axis, with the flag factor F; the grid is the half plane q_v >= 0 (a point with q_v < 0 stands
// for (-q_u, -q_v), the visibility conjugated; a point on the line q_v = 0, which the half plane
// stores whole, also enters at (-q_u, 0) conjugated), and chan_avg consecutive channels are gridded
// together.  A thread sums the channel group of each of its visibilities in registers and adds it to
// the FP64 cell sums and the integer counts with atomics (through LDS for the crowded cells around
// the origin); the cell sums are then written in the output precision.
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

// Short baselines crowd into the cells around the origin, so the cells |q_u| < GRID_HOT,
// q_v < GRID_HOT of a block's visibilities are summed in LDS, stored whole as the block's partials
// per channel group and added over blocks in block order (k_grid_hot); the other cells take global
// atomics directly.  Large blocks of visibilities (GRID_VPB) give the LDS cells many samples to
// combine.

__device__ __forceinline__ void cell_add(const GridArgs& a, long long o, long long cell, double re, double im, int c) {
  const long long plane = (long long)a.n * (a.n / 2 + 1);
  double* d = a.acc + 2 * (o * plane + cell);
  unsafeAtomicAdd(d, re);
  unsafeAtomicAdd(d + 1, im);
  atomicAdd(a.cnt + o * plane + cell, c);
}

// blockIdx.x: GRID_VPB visibilities; blockIdx.y: output channels o = blockIdx.y, blockIdx.y +
// gridDim.y, ...  The grid point of a visibility is recomputed for every channel group.
__global__ __launch_bounds__(GRID_THREADS) void k_grid_scatter(GridArgs a) {
  __shared__ double hre[GRID_NHOT], him[GRID_NHOT];
  __shared__ int hc[GRID_NHOT];
  const int n = a.n, nh = n / 2 + 1, half = n / 2;
  const long long vb = (long long)blockIdx.x * GRID_VPB;
  const long long ve = vb + GRID_VPB < a.nvis ? vb + GRID_VPB : a.nvis;
  const float2* __restrict__ vis = reinterpret_cast<const float2*>(a.vis);
  for (int o = blockIdx.y; o < a.nco; o += gridDim.y) {
    for (int h = threadIdx.x; h < GRID_NHOT; h += GRID_THREADS) {
      hre[h] = 0.0;
      him[h] = 0.0;
      hc[h] = 0;
    }
    __syncthreads();
    for (long long i = vb + threadIdx.x; i < ve; i += GRID_THREADS) {
      const double U = a.uv[2 * i], Vb = a.uv[2 * i + 1];
      double qu = rint(U / a.du), qv = rint(Vb / a.du);
      const double du_off = U - a.du * qu, dv_off = Vb - a.du * qv;   // offset from the grid point
      const bool neg = qv < 0.0;
      if (neg) {
        qu = -qu;
        qv = -qv;
      }
      if (!(fabs(qu) < (double)half && fabs(qv) < (double)half)) continue;
      const int iu = (int)qu, iv = (int)qv;
      double re = 0.0, im = 0.0;
      int c = 0;
      if (a.knode) {   // phase mode: exp(i k_o . delta), conjugated for a reversed baseline
        double sn, cs;
        sincos(a.knode[2 * o] * du_off + a.knode[2 * o + 1] * dv_off, &sn, &cs);
        re = cs;
        im = neg ? -sn : sn;
        c = 1;
      }
      for (int k = 0; !a.knode && k < a.chan_avg; ++k) {
        const long long j = (long long)(o * a.chan_avg + k) * a.nvis + i;
        if (a.flags && a.flags[j]) continue;
        const float2 v = vis[j];
        re += (double)v.x;
        im += neg ? -(double)v.y : (double)v.y;
        ++c;
      }
      if (!c) continue;
      if (iu > -GRID_HOT && iu < GRID_HOT && iv < GRID_HOT) {
        const int h = (iu + GRID_HOT - 1) * GRID_HOT + iv;
        atomicAdd(&hre[h], re);
        atomicAdd(&him[h], im);
        atomicAdd(&hc[h], c);
        if (iv == 0) {   // the mirror baseline on the stored line q_v = 0: (-q_u, 0), conjugated
          const int hm = (-iu + GRID_HOT - 1) * GRID_HOT;
          atomicAdd(&hre[hm], re);
          atomicAdd(&him[hm], -im);
          atomicAdd(&hc[hm], c);
        }
      } else {
        cell_add(a, o, (long long)(iu < 0 ? iu + n : iu) * nh + iv, re, im, c);
        if (iv == 0) cell_add(a, o, (long long)(iu > 0 ? n - iu : -iu) * nh, re, -im, c);
      }
    }
    __syncthreads();
    // the block's partials of every LDS cell, stored whole (no atomics; added over blocks later)
    const long long base = ((long long)o * gridDim.x + blockIdx.x) * GRID_NHOT;
    for (int h = threadIdx.x; h < GRID_NHOT; h += GRID_THREADS) {
      a.hot_v[2 * (base + h)] = hre[h];
      a.hot_v[2 * (base + h) + 1] = him[h];
      a.hot_c[base + h] = hc[h];
    }
    __syncthreads();
  }
}

// The LDS cells: their block partials added in block order, one plain store per cell and output
// channel (no other path writes these cells: a far baseline's mirror on the line q_v = 0 is far too).
__global__ __launch_bounds__(256) void k_grid_hot(GridArgs a, int nbx) {
  const int h = blockIdx.x * 256 + threadIdx.x, o = blockIdx.y;
  if (h >= GRID_NHOT) return;
  const int iu = h / GRID_HOT - (GRID_HOT - 1), iv = h - (h / GRID_HOT) * GRID_HOT;
  if (iu <= -a.n / 2 || iu >= a.n / 2 || iv >= a.n / 2) return;   // beyond a small grid
  double re = 0.0, im = 0.0;
  int c = 0;
  for (int b = 0; b < nbx; ++b) {
    const long long k = ((long long)o * nbx + b) * GRID_NHOT + h;
    re += a.hot_v[2 * k];
    im += a.hot_v[2 * k + 1];
    c += a.hot_c[k];
  }
  const long long cell = (long long)o * a.n * (a.n / 2 + 1) + (long long)(iu < 0 ? iu + a.n : iu) * (a.n / 2 + 1) + iv;
  a.acc[2 * cell] = re;
  a.acc[2 * cell + 1] = im;
  a.cnt[cell] = c;
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
  const unsigned bx = (unsigned)((a.nvis + GRID_VPB - 1) / GRID_VPB);
  const unsigned by = (unsigned)(a.nco < 64 ? a.nco : 64);
  hipLaunchKernelGGL(k_grid_scatter, dim3(bx, by), dim3(GRID_THREADS), 0, s, a);
}

void launch_grid_hot(const GridArgs& a, hipStream_t s) {
  const int nbx = (int)grid_blocks(a.nvis);
  hipLaunchKernelGGL(k_grid_hot, dim3((GRID_NHOT + 255) / 256, a.nco), dim3(256), 0, s, a, nbx);
}

void launch_grid_fin(const GridArgs& a, bool fp64, void* out, int32_t* ng, hipStream_t s) {
  if (fp64) hipLaunchKernelGGL(k_grid_fin<double>, dim3(1024), dim3(256), 0, s, a, static_cast<double*>(out), ng);
  else hipLaunchKernelGGL(k_grid_fin<float>, dim3(1024), dim3(256), 0, s, a, static_cast<float*>(out), ng);
}
