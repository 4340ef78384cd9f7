// Argument blocks and launchers of the variance-surrogate MLP kernels.
#pragma once
#include <hip/hip_runtime.h>

constexpr int MLP_IN = 4, MLP_HID = 256;
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_HID * MLP_IN;    // 1024
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_HID;             // 1280
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_HID * MLP_HID;   // 66816
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_HID;             // 67072
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_HID * MLP_HID;   // 132608
constexpr int MLP_OFF_W4 = MLP_OFF_B3 + MLP_HID;             // 132864
constexpr int MLP_OFF_B4 = MLP_OFF_W4 + MLP_HID;             // 133120
constexpr int MLP_NPARAM = MLP_OFF_B4 + 1;                   // 133121
constexpr int MLP_NSTATE = MLP_NPARAM + 10;                  // + mu_x[4], s_x[4], mu_t, s_t

enum { EPI_NONE = 0, EPI_BIAS_SILU = 1, EPI_DSILU = 2, EPI_BIAS = 3 };

struct GemmArgs {
  const float* A;
  const float* B;
  float* C;
  int M, N, K, lda, ldb, ldc;
  const float* bias;   // EPI_BIAS_SILU / EPI_BIAS: [N]
  float* Z;            // EPI_BIAS_SILU: pre-activation output (ldc)
  const float* Zin;    // EPI_DSILU: pre-activation input (ldc)
  float* part;         // split-K partial sums [splits][M][N]
  int kchunk;          // set by the launcher
};

// Device-resident training state read by the Adam kernel (so a captured step can be replayed).
struct TrainState {
  int step;     // Adam steps taken so far (bias correction uses step + 1)
  int local;    // steps taken in the current run (cosine schedule position)
  int K;        // steps of the current run
  int cosine;
  float lr, b1, b2, eps;
};

void launch_gemm(const GemmArgs& g, bool ta, bool tb, int epi, int splits, hipStream_t s);
void launch_colsum(const float* X, int rows, int cols, float* out, hipStream_t s);
void launch_loss(const float* y, const float* t, int B, float* dy, double* loss, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int n, const TrainState* ts, hipStream_t s);
void launch_train_set(TrainState* ts, float lr, int K, int cosine, int reset_step, hipStream_t s);
void launch_fit_norm(const float* X, const float* t, int n, float* norm, hipStream_t s);
void launch_normalise(const float* X, const float* t, int n, const float* norm, float* Xn, float* tn, hipStream_t s);
void launch_denorm(const float* yn, int n, const float* norm, float* y, hipStream_t s);
void launch_mlp_init(float* p, unsigned long long seed, hipStream_t s);
void launch_to_bf16(const float* x, void* y, int n, hipStream_t s);
void launch_bf16_forward(const float* Xn, int n, const float* p, const float* norm, const void* W2b, const void* W3b,
                         const void* w4b, void* H1, void* H2, float* y, hipStream_t s);
// Gaussian flag proxy: xi[s][nu] for s = 0..nsmax (device float64 [nsmax+1][nc]) and the cube
// V[nu][u][v] = a(nu) xi[q_u^2 + q_v^2][nu] on support cells (complex128 [nc][n][n/2+1]).
void launch_var_xi(int nc, int nsmax, double cperp2, double cpar2, double pk_index, double* xi, hipStream_t s);
void launch_var_cube(int n, int nh, int nc, int smax, const double* a, const double* xi, void* V, hipStream_t s);
