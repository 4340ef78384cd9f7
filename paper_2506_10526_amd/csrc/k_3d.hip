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

// --------------------------------------------------------------- delay transform
// Vt(eta, U) = sum_nu w(nu) m(U) V(U, nu) e^{-2 pi i eta nu / nc}, with the v = 0 column
// symmetrised per channel.  Block: NL consecutive qv of one qu row, all channels.
template <typename T>
__global__ __launch_bounds__(256) void k3_delay(Delay3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Shell3Geom& g = a.g;
  const int nc = g.nc, n = g.n, nh = g.nh;
  const int ub = blockIdx.y;
  const int qu = ub - g.vmax;
  const int iu = wrap(qu, n), iun = wrap(-qu, n);
  const int v0 = blockIdx.x * a.NL;
  const int nl = min(a.NL, g.nvb - v0);
  const int ld = nc + 1;
  Cx<T>* A = (Cx<T>*)smem_raw;
  Cx<T>* Bf = A + (size_t)a.NL * ld;
  const Cx<T>* vis = (const Cx<T>*)a.vis;
  for (int e = threadIdx.x; e < nl * nc; e += blockDim.x) {
    int nu = e / nl, l = e - nu * nl, v = v0 + l;
    T cw = a.chw ? T(a.chw[nu]) : T(1);
    T m = g.uvm ? T(g.uvm[(size_t)iu * nh + v]) : T(1);
    Cx<T> x = cscale(vis[((size_t)nu * n + iu) * nh + v], cw * m);
    if (v == 0) {
      T mn = g.uvm ? T(g.uvm[(size_t)iun * nh]) : T(1);
      Cx<T> y = cscale(vis[((size_t)nu * n + iun) * nh], cw * mn);
      x = cscale(cadd(x, cconj(y)), T(0.5));
    }
    A[(size_t)l * ld + nu] = x;
  }
  __syncthreads();
  Cx<T>* r = lds_fft<-1, T>(A, Bf, a.plan, nl, (const Cx<T>*)a.tw, 1, ld);
  Cx<T>* out = (Cx<T>*)a.out;
  const int ne = 2 * g.H + 1;
  for (int e = threadIdx.x; e < ne * nl; e += blockDim.x) {
    int ec = e / nl, l = e - ec * nl;
    int eta = ec - g.H;
    int idx = eta < 0 ? eta + nc : eta;
    out[((size_t)ec * g.nub + ub) * g.nvb + v0 + l] = r[(size_t)l * ld + idx];
  }
}

// --------------------------------------------------------------- v pass
// Input value of shell j at (eta >= 0, qu, qv): data Vt or the unit indicator.
template <typename T>
__device__ __forceinline__ Cx<T> shell_value(const Pass3Args& a, int shell, int eta, int qu, int qv) {
  const Shell3Geom& g = a.g;
  if (qv > g.vmax || qv < -g.vmax) return cmk(T(0), T(0));
  int s = qu * qu + qv * qv;
  if (s < 1 || s > g.smax) return cmk(T(0), T(0));
  if (g.lut[(size_t)eta * g.S1 + s] != shell) return cmk(T(0), T(0));
  int hu = qv >= 0 ? qu : -qu, hv = qv >= 0 ? qv : -qv;  // stored half-plane cell
  if (g.uvm && !g.uvm[(size_t)wrap(hu, g.n) * g.nh + hv]) return cmk(T(0), T(0));
  if (a.indicator) return cmk(T(1), T(0));
  const Cx<T>* D = (const Cx<T>*)a.in;
  if (qv >= 0) return D[((size_t)(eta + g.H) * g.nub + (qu + g.vmax)) * g.nvb + qv];
  return cconj(D[((size_t)(g.H - eta) * g.nub + (-qu + g.vmax)) * g.nvb + (-qv)]);
}

template <typename T>
__global__ __launch_bounds__(256) void k3_vpass(Pass3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Shell3Geom& g = a.g;
  const Work3 w = a.work[blockIdx.x];
  const int shell = a.shell_of_block[w.j];
  const int n = g.n;
  const int nl = min(a.NL, g.nub - w.start);
  Cx<T>* A = (Cx<T>*)smem_raw;
  Cx<T>* Bf = A + (size_t)a.NL * n;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int l = e / n, i = e - l * n;
    int qu = w.start + l - g.vmax;
    A[e] = shell_value<T>(a, shell, w.eta, qu, sidx(i, n));
  }
  __syncthreads();
  Cx<T>* r = lds_fft<+1, T>(A, Bf, a.plan, nl, (const Cx<T>*)a.tw, 1);
  Cx<T>* out = (Cx<T>*)a.out + a.off_out[w.j] + ((size_t)w.eta * g.nub + w.start) * n;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) out[e] = r[e];
}

// --------------------------------------------------------------- u pass
template <typename T>
__global__ __launch_bounds__(256) void k3_upass(Pass3Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Shell3Geom& g = a.g;
  const Work3 w = a.work[blockIdx.x];
  const int n = g.n;
  const int nl = min(a.NL, n - w.start);
  const int ld = n + 1;
  Cx<T>* A = (Cx<T>*)smem_raw;
  Cx<T>* Bf = A + (size_t)a.NL * ld;
  const Cx<T>* in = (const Cx<T>*)a.in + a.off_in[w.j] + (size_t)w.eta * g.nub * n + w.start;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int i = e / nl, l = e - i * nl;
    int qu = sidx(i, n);
    Cx<T> x = cmk(T(0), T(0));
    if (qu >= -g.vmax && qu <= g.vmax) x = in[(size_t)(qu + g.vmax) * n + l];
    A[(size_t)l * ld + i] = x;
  }
  __syncthreads();
  Cx<T>* r = lds_fft<+1, T>(A, Bf, a.plan, nl, (const Cx<T>*)a.tw, 1, ld);
  Cx<T>* out = (Cx<T>*)a.out + a.off_out[w.j] + (size_t)w.eta * n * n + w.start;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    int i = e / nl, l = e - i * nl;
    out[(size_t)i * n + l] = r[(size_t)l * ld + i];
  }
}

// --------------------------------------------------------------- eta pass (C2R)
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
  const Cx<T>* in = (const Cx<T>*)a.in + a.off_in[w.j] + w.start;
  const Cx<T>* tw = (const Cx<T>*)a.tw;  // table of length M
  for (int e = threadIdx.x; e < nl * Mh; e += blockDim.x) {
    int k = e / nl, l = e - k * nl;
    auto get = [&](int eta) -> Cx<T> { return eta <= Hj ? in[(size_t)eta * n2 + l] : cmk(T(0), T(0)); };
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

__device__ __forceinline__ uint16_t bfbits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bffloat(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

__device__ __forceinline__ void split8(const float* v, bf16x8& h, bf16x8& l) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    uint16_t hb = bfbits(v[q]);
    uint16_t lb = bfbits(v[q] - bffloat(hb));
    h[q] = __builtin_bit_cast(__bf16, hb);
    l[q] = __builtin_bit_cast(__bf16, lb);
  }
}

template <int MODE, typename T>  // MODE 0: FP64 MFMA, 1: FP32 MFMA, 2: split-BF16 MFMA
__global__ __launch_bounds__(256) void k3_contract(Con3Args a) {
  __shared__ T sF[32 * C3_LDS];
  __shared__ int sp[2 * 112];
  __shared__ double red[112 * 32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  for (int e = tid; e < 2 * 112; e += 256) sp[e] = e < 2 * a.npairs ? a.pairs[e] : -1;
  for (int e = tid; e < 112 * 32; e += 256) red[e] = 0.0;
  const int RT = (a.npairs + 15) / 16, CT = (a.nbu + 15) / 16;
  typedef typename std::conditional<MODE == 0, f64x4, f32x4>::type accv;
  accv acc[C3_RT][C3_CT];
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
    for (int e = a.nbu * C3_SLAB + tid; e < 32 * C3_SLAB; e += 256) {
      int j = e / C3_SLAB, v = e - j * C3_SLAB;
      sF[j * C3_LDS + v] = T(0);
    }
    __syncthreads();
    const int vw = wave * 32;
    if constexpr (MODE == 2) {
      const int vb = vw + kq * 8;
      bf16x8 bh[C3_CT], bl[C3_CT];
#pragma unroll
      for (int ct = 0; ct < C3_CT; ++ct) {
        float v[8];
        const T* src = &sF[(ct * 16 + r16) * C3_LDS + vb];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (float)src[q];
        split8(v, bh[ct], bl[ct]);
      }
#pragma unroll
      for (int rt = 0; rt < C3_RT; ++rt) {
        if (rt < RT) {
          int p = rt * 16 + r16;
          int pa = sp[2 * p], pb = sp[2 * p + 1];
          float v[8];
          if (pa >= 0) {
            const T* sa = &sF[pa * C3_LDS + vb];
            const T* sb = &sF[pb * C3_LDS + vb];
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
        const int vx = vw + ks * 4 + kq;
        T bv[C3_CT];
#pragma unroll
        for (int ct = 0; ct < C3_CT; ++ct) bv[ct] = sF[(ct * 16 + r16) * C3_LDS + vx];
#pragma unroll
        for (int rt = 0; rt < C3_RT; ++rt) {
          if (rt < RT) {
            int p = rt * 16 + r16;
            int pa = sp[2 * p], pb = sp[2 * p + 1];
            T av = pa >= 0 ? sF[pa * C3_LDS + vx] * sF[pb * C3_LDS + vx] : T(0);
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
    __syncthreads();
    since += C3_SLAB;
    if (MODE != 0 && since >= 512) {
      since = 0;
#pragma unroll
      for (int i = 0; i < C3_RT; ++i)
#pragma unroll
        for (int j = 0; j < C3_CT; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) { acc64[i][j][q] += (double)acc[i][j][q]; acc[i][j][q] = 0; }
    }
  }
  // reduce the four waves in a fixed order, then store this block's partial sums
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
  double* out = a.partial + (size_t)blockIdx.x * 112 * 32;
  for (int e = tid; e < 112 * 32; e += 256) out[e] = red[e];
}

// --------------------------------------------------------------- finalisation
__global__ void k3_fin(Fin3Args a) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.ntri) return;
  int idx = a.tri_pair[t] * 32 + a.tri_col[t];
  double s = 0.0;
  for (int p = 0; p < a.nparts; ++p) s += a.partial[(size_t)p * 112 * 32 + idx];
  s *= a.sfac;
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

void launch_delay3_f32(const Delay3Args& a, hipStream_t s, size_t lds) {
  set_lds<float>((const void*)k3_delay<float>, lds);
  hipLaunchKernelGGL(k3_delay<float>, dim3((a.g.nvb + a.NL - 1) / a.NL, a.g.nub), dim3(256), lds, s, a);
}
void launch_delay3_f64(const Delay3Args& a, hipStream_t s, size_t lds) {
  set_lds<double>((const void*)k3_delay<double>, lds);
  hipLaunchKernelGGL(k3_delay<double>, dim3((a.g.nvb + a.NL - 1) / a.NL, a.g.nub), dim3(256), lds, s, a);
}
void launch_vpass3(const Pass3Args& a, int nwork, bool fp64, hipStream_t s, size_t lds) {
  if (nwork <= 0) return;
  if (fp64) { set_lds<double>((const void*)k3_vpass<double>, lds); hipLaunchKernelGGL(k3_vpass<double>, dim3(nwork), dim3(256), lds, s, a); }
  else { set_lds<float>((const void*)k3_vpass<float>, lds); hipLaunchKernelGGL(k3_vpass<float>, dim3(nwork), dim3(256), lds, s, a); }
}
void launch_upass3(const Pass3Args& a, int nwork, bool fp64, hipStream_t s, size_t lds) {
  if (nwork <= 0) return;
  if (fp64) { set_lds<double>((const void*)k3_upass<double>, lds); hipLaunchKernelGGL(k3_upass<double>, dim3(nwork), dim3(256), lds, s, a); }
  else { set_lds<float>((const void*)k3_upass<float>, lds); hipLaunchKernelGGL(k3_upass<float>, dim3(nwork), dim3(256), lds, s, a); }
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
void launch_fin3(const Fin3Args& a, hipStream_t s) {
  if (a.ntri > 0) hipLaunchKernelGGL(k3_fin, dim3((a.ntri + 127) / 128), dim3(128), 0, s, a);
}
