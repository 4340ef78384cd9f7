// Kernels of the learned variance surrogate: a 4 -> 256 -> 256 -> 256 -> 1 MLP with SiLU hidden
// units, trained in FP32 (forward, backward, Adam) and evaluated in FP32 or BF16 (MFMA).
//
// Parameter vector (row-major, 133,121 floats): W1 [256][4], b1, W2 [256][256], b2, W3 [256][256],
// b3, w4 [1][256], b4; followed in the state buffer by the normalisation mu_x[4], s_x[4], mu_t, s_t.
// Layer l: z = h W^T + b, h' = silu(z) = z / (1 + e^-z).  Loss: mean (y' - t')^2 over the batch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bs_mlp_k.h"

namespace {

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------- FP32 GEMM
// C[M][N] = op(A)[M][K] op(B)[K][N]; op(A)(m,k) = TA ? A[k lda + m] : A[m lda + k],
// op(B)(k,n) = TB ? B[n ldb + k] : B[k ldb + n].  64 x 64 block tile, K staged by 16 through LDS,
// 4 x 4 outputs per thread (rows ty + 16 i, columns tx + 16 j).  blockIdx.z = K split: with
// ksplit > 1 the raw sums go to part[z][M][N] and k_gemm_reduce finishes them.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kc = g.kchunk;
  const int kb = blockIdx.z * kc;
  const int ke = min(g.K, kb + kc);
  float acc[4][4] = {};
  for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int idx = tid + 256 * r;
      int m, k;
      if (TA) { k = idx >> 6; m = idx & 63; } else { m = idx >> 4; k = idx & 15; }
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < g.M && gk < ke) v = TA ? g.A[(size_t)gk * g.lda + gm] : g.A[(size_t)gm * g.lda + gk];
      As[k][m] = v;
      int n, kk;
      if (TB) { n = idx >> 4; kk = idx & 15; } else { kk = idx >> 6; n = idx & 63; }
      const int gn = n0 + n, gk2 = k0 + kk;
      float w = 0.f;
      if (gn < g.N && gk2 < ke) w = TB ? g.B[(size_t)gn * g.ldb + gk2] : g.B[(size_t)gk2 * g.ldb + gn];
      Bs[kk][n] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty + 16 * i;
    if (m >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx + 16 * j;
      if (n >= g.N) continue;
      float v = acc[i][j];
      if (gridDim.z > 1) {
        g.part[((size_t)blockIdx.z * g.M + m) * g.N + n] = v;
        continue;
      }
      const size_t o = (size_t)m * g.ldc + n;
      if (EPI == EPI_BIAS_SILU) {
        const float z = v + g.bias[n];
        g.Z[o] = z;
        g.C[o] = silu(z);
      } else if (EPI == EPI_DSILU) {
        g.C[o] = v * dsilu(g.Zin[o]);
      } else if (EPI == EPI_BIAS) {
        g.C[o] = v + g.bias[n];
      } else {
        g.C[o] = v;
      }
    }
  }
}

// C[m][n] = sum over splits of part[s][m][n] (fixed order).
__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g, int splits) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long tot = (long long)g.M * g.N;
  if (e >= tot) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += g.part[(size_t)z * tot + e];
  const int m = (int)(e / g.N), n = (int)(e - (long long)m * g.N);
  g.C[(size_t)m * g.ldc + n] = s;
}

// out[c] = sum_r X[r][c] for each column (bias gradients).
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ X, int rows, int cols, float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += X[(size_t)r * cols + c];
  out[c] = s;
}

// dy = 2 (y - t) / B, loss = mean (y - t)^2 (FP64 sum, one block).
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t, int B,
                                              float* __restrict__ dy, double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < B; i += 256) {
    const float r = y[i] - t[i];
    dy[i] = 2.0f * r / (float)B;
    s += (double)r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (double)B;
}

// Adam with bias correction at step k = ts->step + 1 and learning rate
// lr_k = lr (1 + cos(pi local / K)) / 2 (cosine) or lr.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int n, const TrainState* __restrict__ ts) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int k = ts->step + 1;
  float lr = ts->lr;
  if (ts->cosine) lr *= 0.5f * (1.0f + cosf(3.14159265358979f * (float)ts->local / (float)ts->K));
  const float b1 = ts->b1, b2 = ts->b2;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)k));
  const float vh = vi / (1.0f - powf(b2, (float)k));
  p[i] -= lr * mh / (sqrtf(vh) + ts->eps);
}

__global__ void k_train_advance(TrainState* ts) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { ts->step += 1; ts->local += 1; }
}

__global__ void k_train_set(TrainState* ts, float lr, int K, int cosine, int reset_step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ts->lr = lr; ts->K = K; ts->cosine = cosine; ts->local = 0;
    if (reset_step) ts->step = 0;
    ts->b1 = 0.9f; ts->b2 = 0.999f; ts->eps = 1e-8f;
  }
}

// ---------------------------------------------------------------- data and initialisation
// Normalisation of (X, t): per-column mean and population standard deviation (1 if zero),
// written to norm[0..9] = mu_x[4], s_x[4], mu_t, s_t.  One block, FP64 sums.
__global__ __launch_bounds__(256) void k_fit_norm(const float* __restrict__ X, const float* __restrict__ t, int n,
                                                  float* __restrict__ norm) {
  __shared__ double red[256];
  for (int c = 0; c < 5; ++c) {
    double s = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
      const double x = c < 4 ? (double)X[(size_t)i * 4 + c] : (double)t[i];
      s += x;
      s2 += x * x;
    }
    double mean, var;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    mean = red[0] / n;
    __syncthreads();
    // second pass for the variance (sum of squared deviations)
    s2 = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
      const double x = c < 4 ? (double)X[(size_t)i * 4 + c] : (double)t[i];
      s2 += (x - mean) * (x - mean);
    }
    red[threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    var = red[0] / n;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double sd = sqrt(var);
      if (c < 4) { norm[c] = (float)mean; norm[4 + c] = sd > 0 ? (float)sd : 1.0f; }
      else { norm[8] = (float)mean; norm[9] = sd > 0 ? (float)sd : 1.0f; }
    }
  }
}

// Xn = (X - mu_x) / s_x; tn = (t - mu_t) / s_t (t may be NULL).
__global__ __launch_bounds__(256) void k_normalise(const float* __restrict__ X, const float* __restrict__ t, int n,
                                                   const float* __restrict__ norm, float* __restrict__ Xn,
                                                   float* __restrict__ tn) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 4; ++c) Xn[(size_t)i * 4 + c] = (X[(size_t)i * 4 + c] - norm[c]) / norm[4 + c];
  if (t && tn) tn[i] = (t[i] - norm[8]) / norm[9];
}

// y = mu_t + s_t y'
__global__ __launch_bounds__(256) void k_denorm(const float* __restrict__ yn, int n, const float* __restrict__ norm,
                                                float* __restrict__ y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = norm[8] + norm[9] * yn[i];
}

// theta_j = a_j (2 u_j - 1), u_j the 24-bit uniform of word j % 4 of Philox4x64-10 block j / 4 under
// key (seed, 0x4D4C50), a_j = 1 / sqrt(fan_in) of the layer of parameter j.
__device__ __forceinline__ void philox4x64_10(unsigned long long* x, unsigned long long k0, unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const unsigned long long h0 = __umul64hi(x[0], M0), l0 = x[0] * M0;
    const unsigned long long h1 = __umul64hi(x[2], M1), l1 = x[2] * M1;
    const unsigned long long y0 = h1 ^ x[1] ^ k0, y2 = h0 ^ x[3] ^ k1;
    x[0] = y0; x[1] = l1; x[2] = y2; x[3] = l0;
  }
}

__global__ __launch_bounds__(256) void k_mlp_init(float* __restrict__ p, unsigned long long seed) {
  const int blk = blockIdx.x * 256 + threadIdx.x;
  if (4 * blk >= MLP_NPARAM) return;
  unsigned long long x[4] = {(unsigned long long)blk, 0, 0, 0};
  philox4x64_10(x, seed, 0x4D4C50ULL);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 4 * blk + q;
    if (j >= MLP_NPARAM) break;
    const double u = ((double)(x[q] >> 40) + 0.5) * 5.9604644775390625e-8;
    const double a = j < MLP_OFF_B1 ? 0.5 : (j < MLP_OFF_W2 ? 0.5 : 0.0625);  // 1/sqrt(4), 1/sqrt(256)
    p[j] = (float)(a * (2.0 * u - 1.0));
  }
}

// ---------------------------------------------------------------- BF16 inference
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ x, __bf16* __restrict__ y, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = (__bf16)x[i];
}

// First layer in FP32 from normalised inputs: H1 = bf16(silu(Xn W1^T + b1)).
__global__ __launch_bounds__(256) void k_bf16_layer1(const float* __restrict__ Xn, int n, const float* __restrict__ p,
                                                     __bf16* __restrict__ H) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)n * MLP_HID) return;
  const int r = (int)(e / MLP_HID), u = (int)(e - (long long)r * MLP_HID);
  float z = p[MLP_OFF_B1 + u];
#pragma unroll
  for (int k = 0; k < 4; ++k) z = fmaf(p[MLP_OFF_W1 + u * 4 + k], Xn[(size_t)r * 4 + k], z);
  H[e] = (__bf16)silu(z);
}

// Hidden layer on MFMA: Hout = bf16(silu(Hin Wb^T + b)), Hin [n][256] bf16, Wb [256][256] bf16.
// One wave per 32 x 32 output tile, K = 256 in 16 steps of mfma_f32_32x32x16_bf16.
__global__ __launch_bounds__(64) void k_bf16_hidden(const __bf16* __restrict__ Hin, int n, const __bf16* __restrict__ Wb,
                                                    const float* __restrict__ bias, __bf16* __restrict__ Hout) {
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int ra = r0 + (lane & 31), cb = c0 + (lane & 31), ks = (lane >> 5) * 8;
  f32x16 acc = {};
  const bf16x8 zero = {};
#pragma unroll 4
  for (int kk = 0; kk < MLP_HID; kk += 16) {
    const bf16x8 a = ra < n ? *(const bf16x8*)&Hin[(size_t)ra * MLP_HID + kk + ks] : zero;
    const bf16x8 b = *(const bf16x8*)&Wb[(size_t)cb * MLP_HID + kk + ks];
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = r0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    const int c = c0 + (lane & 31);
    if (r < n) Hout[(size_t)r * MLP_HID + c] = (__bf16)silu(acc[i] + bias[c]);
  }
}

// Output layer: y = mu_t + s_t (sum_u H3[u] w4[u] + b4), bf16 operands, FP32 sum.
__global__ __launch_bounds__(256) void k_bf16_out(const __bf16* __restrict__ H, int n, const __bf16* __restrict__ w4,
                                                  const float* __restrict__ p, const float* __restrict__ norm,
                                                  float* __restrict__ y) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  float s = 0.f;
  for (int u = 0; u < MLP_HID; ++u) s = fmaf((float)H[(size_t)r * MLP_HID + u], (float)w4[u], s);
  y[r] = norm[8] + norm[9] * (s + p[MLP_OFF_B4]);
}


// ---------------------------------------------------------------------------
// Gaussian flag proxy of the variance surrogate: the channel-domain cube whose delay transform is
// the window-convolved power P_w(k_perp, eta) = sum_q |w~(q)|^2 / nc^2 P(k_perp, eta - q).  By the
// convolution theorem its inverse DFT along eta is a(nu) xi_s(nu), with xi_s = IDFT_eta P (real:
// P is even in eta) and a(nu) = (1/nc) sum_mu w(mu) w(mu + nu) the window's autocorrelation.
// xi depends on the cell only through s = q_u^2 + q_v^2, so it is tabulated once per s.
// ---------------------------------------------------------------------------
// xi[s][nu] = (1/nc) sum_i P(s, i) cos(2 pi i nu / nc), P(s, i) = (cperp2 s + cpar2 eta_i^2)^(pk/2),
// eta_i the signed index of i; one block per s, threads over nu, P(s, .) and cos(2 pi m / nc) in LDS.
__global__ __launch_bounds__(256) void k_var_xi(int nc, double cperp2, double cpar2, double half_pk, double* xi) {
  extern __shared__ double sh[];   // [nc] P then [nc] cos table
  double* Ps = sh;
  double* ct = sh + nc;
  const int sidx = blockIdx.x;
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const int e = i < (nc + 1) / 2 ? i : i - nc;
    const double k2 = cperp2 * sidx + cpar2 * (double)e * e;
    Ps[i] = k2 > 0.0 ? pow(k2, half_pk) : 0.0;
    ct[i] = cos(2.0 * M_PI * (double)i / nc);
  }
  __syncthreads();
  for (int nu = threadIdx.x; nu < nc; nu += blockDim.x) {
    double acc = 0.0;
    int m = 0;   // i * nu mod nc
    for (int i = 0; i < nc; ++i) {
      acc = fma(Ps[i], ct[m], acc);
      m += nu;
      if (m >= nc) m -= nc;
    }
    xi[(size_t)sidx * nc + nu] = acc / nc;
  }
}

// V[nu][u][v] = a(nu) xi[s][nu] (complex128, imaginary part 0) on support cells 1 <= s <= smax.
__global__ __launch_bounds__(256) void k_var_cube(int n, int nh, int nc, int smax, const double* a, const double* xi,
                                                  double2* V) {
  const size_t total = (size_t)nc * n * nh;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int v = (int)(e % nh);
    const size_t r = e / nh;
    const int u = (int)(r % n);
    const int nu = (int)(r / n);
    const int qu = u < (n + 1) / 2 ? u : u - n;
    const int s = qu * qu + v * v;
    double x = 0.0;
    if (s >= 1 && s <= smax) x = a[nu] * xi[(size_t)s * nc + nu];
    V[e] = make_double2(x, 0.0);
  }
}
}  // namespace

// ---------------------------------------------------------------- launchers
void launch_gemm(const GemmArgs& g0, bool ta, bool tb, int epi, int splits, hipStream_t s) {
  GemmArgs g = g0;
  if (splits < 1) splits = 1;
  g.kchunk = ((g.K + splits - 1) / splits + 15) / 16 * 16;
  splits = (g.K + g.kchunk - 1) / g.kchunk;
  if (splits < 1) splits = 1;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
#define GEMM_CASE(TA_, TB_, E_) \
  if (ta == TA_ && tb == TB_ && epi == E_) { hipLaunchKernelGGL((k_gemm<TA_, TB_, E_>), grid, dim3(256), 0, s, g); }
  GEMM_CASE(false, true, EPI_BIAS_SILU)
  GEMM_CASE(false, true, EPI_BIAS)
  GEMM_CASE(false, false, EPI_DSILU)
  GEMM_CASE(true, false, EPI_NONE)
  GEMM_CASE(false, true, EPI_NONE)
#undef GEMM_CASE
  if (splits > 1) {
    const long long tot = (long long)g.M * g.N;
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g, splits);
  }
}

void launch_colsum(const float* X, int rows, int cols, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256), dim3(256), 0, s, X, rows, cols, out);
}
void launch_loss(const float* y, const float* t, int B, float* dy, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, y, t, B, dy, loss);
}
void launch_adam(float* p, const float* g, float* m, float* v, int n, const TrainState* ts, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, ts);
  hipLaunchKernelGGL(k_train_advance, dim3(1), dim3(64), 0, s, (TrainState*)ts);
}
void launch_train_set(TrainState* ts, float lr, int K, int cosine, int reset_step, hipStream_t s) {
  hipLaunchKernelGGL(k_train_set, dim3(1), dim3(64), 0, s, ts, lr, K, cosine, reset_step);
}
void launch_fit_norm(const float* X, const float* t, int n, float* norm, hipStream_t s) {
  hipLaunchKernelGGL(k_fit_norm, dim3(1), dim3(256), 0, s, X, t, n, norm);
}
void launch_normalise(const float* X, const float* t, int n, const float* norm, float* Xn, float* tn, hipStream_t s) {
  hipLaunchKernelGGL(k_normalise, dim3((n + 255) / 256), dim3(256), 0, s, X, t, n, norm, Xn, tn);
}
void launch_denorm(const float* yn, int n, const float* norm, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_denorm, dim3((n + 255) / 256), dim3(256), 0, s, yn, n, norm, y);
}
void launch_mlp_init(float* p, unsigned long long seed, hipStream_t s) {
  const int nblk = (MLP_NPARAM + 3) / 4;
  hipLaunchKernelGGL(k_mlp_init, dim3((nblk + 255) / 256), dim3(256), 0, s, p, seed);
}
void launch_to_bf16(const float* x, void* y, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, s, x, (__bf16*)y, n);
}
void launch_bf16_forward(const float* Xn, int n, const float* p, const float* norm, const void* W2b, const void* W3b,
                         const void* w4b, void* H1, void* H2, float* y, hipStream_t s) {
  const long long e = (long long)n * MLP_HID;
  hipLaunchKernelGGL(k_bf16_layer1, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, Xn, n, p, (__bf16*)H1);
  dim3 grid((n + 31) / 32, MLP_HID / 32);
  hipLaunchKernelGGL(k_bf16_hidden, grid, dim3(64), 0, s, (const __bf16*)H1, n, (const __bf16*)W2b, p + MLP_OFF_B2,
                     (__bf16*)H2);
  hipLaunchKernelGGL(k_bf16_hidden, grid, dim3(64), 0, s, (const __bf16*)H2, n, (const __bf16*)W3b, p + MLP_OFF_B3,
                     (__bf16*)H1);
  hipLaunchKernelGGL(k_bf16_out, dim3((n + 255) / 256), dim3(256), 0, s, (const __bf16*)H1, n, (const __bf16*)w4b, p,
                     norm, y);
}

void launch_var_xi(int nc, int nsmax, double cperp2, double cpar2, double pk_index, double* xi, hipStream_t s) {
  const size_t lds = 2 * (size_t)nc * sizeof(double);
  hipLaunchKernelGGL(k_var_xi, dim3(nsmax + 1), dim3(256), lds, s, nc, cperp2, cpar2, 0.5 * pk_index, xi);
}
void launch_var_cube(int n, int nh, int nc, int smax, const double* a, const double* xi, void* V, hipStream_t s) {
  const size_t total = (size_t)nc * n * nh;
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_var_cube, dim3((unsigned)blocks), dim3(256), 0, s, n, nh, nc, smax, a, xi, (double2*)V);
}
