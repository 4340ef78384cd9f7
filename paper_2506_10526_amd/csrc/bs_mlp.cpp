// C ABI: the learned variance surrogate (a 4 -> 256 -> 256 -> 256 -> 1 MLP), trained on the GPU by
// hand-written FP32 forward / backward / Adam kernels from a captured training step, evaluated in
// FP32 or BF16 (MFMA).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "bs_ctx.h"
#include "bs_mlp_k.h"

#define HIPCHK(ctx, call)                                                                         \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return ctx_fail(ctx, BS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define LAUNCHCHK(ctx, what)                                                                      \
  do {                                                                                            \
    hipError_t e_ = hipGetLastError();                                                            \
    if (e_ != hipSuccess) return ctx_fail(ctx, BS_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

static_assert(MLP_NPARAM == BS_MLP_NPARAM, "parameter count");
static_assert(MLP_NSTATE == BS_MLP_NSTATE, "state size");

struct bs_mlp {
  bs_ctx* c = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int cap = 0;
  std::vector<void*> owned;
  float* state = nullptr;   // params then normalisation
  float* grad = nullptr;
  float* am = nullptr;
  float* av = nullptr;
  TrainState* ts = nullptr;
  float *Xn = nullptr, *tn = nullptr;
  int n = 0;
  float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Z3 = nullptr, *H3 = nullptr;
  float *yv = nullptr, *dy = nullptr, *dZ3 = nullptr, *dZ2 = nullptr, *dZ1 = nullptr;
  float* part = nullptr;
  size_t part_len = 0;
  double* loss = nullptr;
  float* Xp = nullptr;
  void *W2b = nullptr, *W3b = nullptr, *w4b = nullptr, *Hb1 = nullptr, *Hb2 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void* alloc(bs_mlp* m, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  m->owned.push_back(p);
  return p;
}

int splits_for(int K) { return std::max(1, std::min(16, (K + 255) / 256)); }

GemmArgs gemm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N, int K) {
  GemmArgs g{};
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.M = M; g.N = N; g.K = K;
  return g;
}

// Forward pass of the FP32 network on normalised inputs X (n rows); output y' in y.
void forward(bs_mlp* m, const float* X, int n, float* y, hipStream_t s) {
  const float* p = m->state;
  GemmArgs g = gemm(X, 4, p + MLP_OFF_W1, 4, m->H1, MLP_HID, n, MLP_HID, 4);
  g.bias = p + MLP_OFF_B1; g.Z = m->Z1;
  launch_gemm(g, false, true, EPI_BIAS_SILU, 1, s);
  g = gemm(m->H1, MLP_HID, p + MLP_OFF_W2, MLP_HID, m->H2, MLP_HID, n, MLP_HID, MLP_HID);
  g.bias = p + MLP_OFF_B2; g.Z = m->Z2;
  launch_gemm(g, false, true, EPI_BIAS_SILU, 1, s);
  g = gemm(m->H2, MLP_HID, p + MLP_OFF_W3, MLP_HID, m->H3, MLP_HID, n, MLP_HID, MLP_HID);
  g.bias = p + MLP_OFF_B3; g.Z = m->Z3;
  launch_gemm(g, false, true, EPI_BIAS_SILU, 1, s);
  g = gemm(m->H3, MLP_HID, p + MLP_OFF_W4, MLP_HID, y, 1, n, 1, MLP_HID);
  g.bias = p + MLP_OFF_B4;
  launch_gemm(g, false, true, EPI_BIAS, 1, s);
}

// Loss and gradient of the training data (forward included).
void loss_grad(bs_mlp* m, hipStream_t s) {
  const int n = m->n;
  const float* p = m->state;
  float* gr = m->grad;
  forward(m, m->Xn, n, m->yv, s);
  launch_loss(m->yv, m->tn, n, m->dy, m->loss, s);
  const int sp = splits_for(n);
  // output layer
  GemmArgs g = gemm(m->dy, 1, m->H3, MLP_HID, gr + MLP_OFF_W4, MLP_HID, 1, MLP_HID, n);
  g.part = m->part;
  launch_gemm(g, true, false, EPI_NONE, sp, s);
  launch_colsum(m->dy, n, 1, gr + MLP_OFF_B4, s);
  g = gemm(m->dy, 1, p + MLP_OFF_W4, MLP_HID, m->dZ3, MLP_HID, n, MLP_HID, 1);
  g.Zin = m->Z3;
  launch_gemm(g, false, false, EPI_DSILU, 1, s);
  // layer 3
  g = gemm(m->dZ3, MLP_HID, m->H2, MLP_HID, gr + MLP_OFF_W3, MLP_HID, MLP_HID, MLP_HID, n);
  g.part = m->part;
  launch_gemm(g, true, false, EPI_NONE, sp, s);
  launch_colsum(m->dZ3, n, MLP_HID, gr + MLP_OFF_B3, s);
  g = gemm(m->dZ3, MLP_HID, p + MLP_OFF_W3, MLP_HID, m->dZ2, MLP_HID, n, MLP_HID, MLP_HID);
  g.Zin = m->Z2;
  launch_gemm(g, false, false, EPI_DSILU, 1, s);
  // layer 2
  g = gemm(m->dZ2, MLP_HID, m->H1, MLP_HID, gr + MLP_OFF_W2, MLP_HID, MLP_HID, MLP_HID, n);
  g.part = m->part;
  launch_gemm(g, true, false, EPI_NONE, sp, s);
  launch_colsum(m->dZ2, n, MLP_HID, gr + MLP_OFF_B2, s);
  g = gemm(m->dZ2, MLP_HID, p + MLP_OFF_W2, MLP_HID, m->dZ1, MLP_HID, n, MLP_HID, MLP_HID);
  g.Zin = m->Z1;
  launch_gemm(g, false, false, EPI_DSILU, 1, s);
  // layer 1
  g = gemm(m->dZ1, MLP_HID, m->Xn, 4, gr + MLP_OFF_W1, 4, MLP_HID, 4, n);
  g.part = m->part;
  launch_gemm(g, true, false, EPI_NONE, sp, s);
  launch_colsum(m->dZ1, n, MLP_HID, gr + MLP_OFF_B1, s);
}

void train_step(bs_mlp* m, hipStream_t s) {
  loss_grad(m, s);
  launch_adam(m->state, m->grad, m->am, m->av, MLP_NPARAM, m->ts, s);
}

template <typename F>
int on_stream(bs_mlp* m, F f) {
  bs_ctx* c = m->c;
  if (hipEventRecord(m->ev_in, c->stream) != hipSuccess || hipStreamWaitEvent(m->s, m->ev_in, 0) != hipSuccess)
    return ctx_fail(c, BS_EHIP, "stream ordering");
  int rc = f(m->s);
  if (hipEventRecord(m->ev_out, m->s) != hipSuccess || hipStreamWaitEvent(c->stream, m->ev_out, 0) != hipSuccess)
    return ctx_fail(c, BS_EHIP, "stream ordering");
  return rc;
}

void drop_graph(bs_mlp* m) {
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->exec = nullptr;
  m->graph = nullptr;
}

}  // namespace

extern "C" int bs_mlp_create(bs_ctx* c, uint64_t seed, int32_t max_batch, bs_mlp** out) {
  if (!c || !out) return BS_EINVAL;
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1 << 20)) return ctx_fail(c, BS_EINVAL, "max_batch must be in [1, 2^20]");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  bs_mlp* m = new bs_mlp();
  m->c = c;
  m->cap = max_batch;
  auto fail = [&](int code, const char* msg) { bs_mlp_destroy(m); return ctx_fail(c, code, msg); };
  if (hipStreamCreateWithFlags(&m->s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BS_EHIP, "stream/event creation");
  }
  const size_t cap = (size_t)max_batch, H = (size_t)MLP_HID;
  m->state = (float*)alloc(m, MLP_NSTATE * 4);
  m->grad = (float*)alloc(m, MLP_NPARAM * 4);
  m->am = (float*)alloc(m, MLP_NPARAM * 4);
  m->av = (float*)alloc(m, MLP_NPARAM * 4);
  m->ts = (TrainState*)alloc(m, sizeof(TrainState));
  m->Xn = (float*)alloc(m, cap * 16);
  m->tn = (float*)alloc(m, cap * 4);
  m->Xp = (float*)alloc(m, cap * 16);
  m->Z1 = (float*)alloc(m, cap * H * 4); m->H1 = (float*)alloc(m, cap * H * 4);
  m->Z2 = (float*)alloc(m, cap * H * 4); m->H2 = (float*)alloc(m, cap * H * 4);
  m->Z3 = (float*)alloc(m, cap * H * 4); m->H3 = (float*)alloc(m, cap * H * 4);
  m->dZ1 = (float*)alloc(m, cap * H * 4); m->dZ2 = (float*)alloc(m, cap * H * 4);
  m->dZ3 = (float*)alloc(m, cap * H * 4);
  m->yv = (float*)alloc(m, cap * 4);
  m->dy = (float*)alloc(m, cap * 4);
  m->part_len = (size_t)16 * H * H;
  m->part = (float*)alloc(m, m->part_len * 4);
  m->loss = (double*)alloc(m, 16);
  m->W2b = alloc(m, H * H * 2);
  m->W3b = alloc(m, H * H * 2);
  m->w4b = alloc(m, H * 2);
  m->Hb1 = alloc(m, cap * H * 2);
  m->Hb2 = alloc(m, cap * H * 2);
  const void* need[] = {m->state, m->grad, m->am, m->av, m->ts, m->Xn, m->tn, m->Xp, m->Z1, m->H1, m->Z2, m->H2,
                        m->Z3, m->H3, m->dZ1, m->dZ2, m->dZ3, m->yv, m->dy, m->part, m->loss, m->W2b, m->W3b,
                        m->w4b, m->Hb1, m->Hb2};
  for (const void* p : need)
    if (!p) return fail(BS_ENOMEM, "surrogate buffers");
  const float norm0[10] = {0, 0, 0, 0, 1, 1, 1, 1, 0, 1};
  if (hipMemsetAsync(m->am, 0, MLP_NPARAM * 4, m->s) != hipSuccess ||
      hipMemsetAsync(m->av, 0, MLP_NPARAM * 4, m->s) != hipSuccess ||
      hipMemcpyAsync(m->state + MLP_NPARAM, norm0, sizeof norm0, hipMemcpyHostToDevice, m->s) != hipSuccess)
    return fail(BS_EHIP, "surrogate set-up");
  launch_mlp_init(m->state, seed, m->s);
  launch_train_set(m->ts, 1e-3f, 1, 0, 1, m->s);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(m->s) != hipSuccess) return fail(BS_EHIP, "surrogate init");
  *out = m;
  return BS_OK;
}

extern "C" void bs_mlp_destroy(bs_mlp* m) {
  if (!m) return;
  drop_graph(m);
  if (m->s) (void)hipStreamSynchronize(m->s);
  for (void* p : m->owned)
    if (p) (void)hipFree(p);
  if (m->ev_in) (void)hipEventDestroy(m->ev_in);
  if (m->ev_out) (void)hipEventDestroy(m->ev_out);
  if (m->s) (void)hipStreamDestroy(m->s);
  (void)hipGetLastError();
  delete m;
}

extern "C" int bs_mlp_read_state(bs_mlp* m, float* state_host) {
  if (!m || !state_host) return BS_EINVAL;
  bs_ctx* c = m->c;
  HIPCHK(c, hipStreamSynchronize(m->s));
  HIPCHK(c, hipMemcpy(state_host, m->state, MLP_NSTATE * 4, hipMemcpyDeviceToHost));
  return BS_OK;
}

extern "C" int bs_mlp_write_state(bs_mlp* m, const float* state_host) {
  if (!m || !state_host) return BS_EINVAL;
  bs_ctx* c = m->c;
  HIPCHK(c, hipStreamSynchronize(m->s));
  HIPCHK(c, hipMemcpy(m->state, state_host, MLP_NSTATE * 4, hipMemcpyHostToDevice));
  return BS_OK;
}

extern "C" int bs_mlp_set_data(bs_mlp* m, const float* X, const float* t, int32_t n) {
  if (!m) return BS_EINVAL;
  bs_ctx* c = m->c;
  if (!X || !t) return ctx_fail(c, BS_EINVAL, "X and t must be non-NULL");
  if (n < 2 || n > m->cap) return ctx_fail(c, BS_EINVAL, "training set size must be in [2, max_batch]");
  if (n != m->n) drop_graph(m);
  m->n = n;
  return on_stream(m, [&](hipStream_t s) {
    launch_fit_norm(X, t, n, m->state + MLP_NPARAM, s);
    launch_normalise(X, t, n, m->state + MLP_NPARAM, m->Xn, m->tn, s);
    LAUNCHCHK(c, "normalise");
    return BS_OK;
  });
}

extern "C" int bs_mlp_loss_grad(bs_mlp* m, float* grad, double* loss_host) {
  if (!m) return BS_EINVAL;
  bs_ctx* c = m->c;
  if (m->n < 2) return ctx_fail(c, BS_EINVAL, "no training data (bs_mlp_set_data)");
  int rc = on_stream(m, [&](hipStream_t s) {
    loss_grad(m, s);
    LAUNCHCHK(c, "loss/gradient");
    if (grad) HIPCHK(c, hipMemcpyAsync(grad, m->grad, MLP_NPARAM * 4, hipMemcpyDeviceToDevice, s));
    return BS_OK;
  });
  if (rc) return rc;
  if (loss_host) {
    HIPCHK(c, hipStreamSynchronize(m->s));
    HIPCHK(c, hipMemcpy(loss_host, m->loss, 8, hipMemcpyDeviceToHost));
  }
  return BS_OK;
}

extern "C" int bs_mlp_train(bs_mlp* m, int32_t steps, double lr, int32_t cosine, double* loss_host) {
  if (!m) return BS_EINVAL;
  bs_ctx* c = m->c;
  if (m->n < 2) return ctx_fail(c, BS_EINVAL, "no training data (bs_mlp_set_data)");
  if (steps < 0 || !(lr > 0)) return ctx_fail(c, BS_EINVAL, "steps >= 0 and lr > 0 required");
  int rc = on_stream(m, [&](hipStream_t s) {
    launch_train_set(m->ts, (float)lr, std::max(steps, 1), cosine ? 1 : 0, 0, s);
    LAUNCHCHK(c, "train set-up");
    if (steps == 0) return BS_OK;
    if (!m->exec) {
      HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      train_step(m, s);
      hipError_t le = hipGetLastError();
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(s, &g);
      if (le != hipSuccess || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return ctx_fail(c, BS_EHIP, "training step capture failed");
      }
      m->graph = g;
      HIPCHK(c, hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0));
    }
    for (int i = 0; i < steps; ++i) HIPCHK(c, hipGraphLaunch(m->exec, s));
    return BS_OK;
  });
  if (rc) return rc;
  if (loss_host) {
    HIPCHK(c, hipStreamSynchronize(m->s));
    HIPCHK(c, hipMemcpy(loss_host, m->loss, 8, hipMemcpyDeviceToHost));
  }
  return BS_OK;
}

extern "C" int bs_mlp_predict(bs_mlp* m, const float* X, int32_t n, int32_t bf16, float* y) {
  if (!m) return BS_EINVAL;
  bs_ctx* c = m->c;
  if (!X || !y) return ctx_fail(c, BS_EINVAL, "X and y must be non-NULL");
  if (n < 1 || n > m->cap) return ctx_fail(c, BS_EINVAL, "prediction batch must be in [1, max_batch]");
  const float* norm = m->state + MLP_NPARAM;
  return on_stream(m, [&](hipStream_t s) {
    launch_normalise(X, nullptr, n, norm, m->Xp, nullptr, s);
    if (!bf16) {
      forward(m, m->Xp, n, m->dy, s);
      launch_denorm(m->dy, n, norm, y, s);
    } else {
      launch_to_bf16(m->state + MLP_OFF_W2, m->W2b, MLP_HID * MLP_HID, s);
      launch_to_bf16(m->state + MLP_OFF_W3, m->W3b, MLP_HID * MLP_HID, s);
      launch_to_bf16(m->state + MLP_OFF_W4, m->w4b, MLP_HID, s);
      launch_bf16_forward(m->Xp, n, m->state, norm, m->W2b, m->W3b, m->w4b, m->Hb1, m->Hb2, y, s);
    }
    LAUNCHCHK(c, "predict");
    return BS_OK;
  });
}

// ------------------------------------------------------------------ features (host)
extern "C" int bs_var_features(const bs_bins* b, const int64_t* T3D_host, double pk_index, double rho,
                               float* X_host, double* base_host) {
  if (!b || !X_host) return BS_EINVAL;
  const auto& P = b->P;
  const int nt = (int)(P.tri.size() / 3);
  const double nvox = (double)P.nc * P.n * P.n;
  std::vector<double> lc(P.nbins);
  for (int j = 0; j < P.nbins; ++j) lc[j] = 0.5 * (std::log(P.edges[j]) + std::log(P.edges[j + 1]));
  for (int t = 0; t < nt; ++t) {
    double s = 0;
    for (int i = 0; i < 3; ++i) {
      X_host[4 * t + i] = (float)lc[P.tri[3 * t + i]];
      s += lc[P.tri[3 * t + i]];
    }
    X_host[4 * t + 3] = (float)rho;
    if (base_host) {
      const double T = T3D_host ? (double)T3D_host[t] : 0.0;
      base_host[t] = T > 0 ? std::log(nvox / T) + pk_index * s : -INFINITY;
    }
  }
  return BS_OK;
}

// ---- Gaussian flag proxy and flag-aware features (Sec. 4 error bars; Sec. 2.2 shells) ----
extern "C" int bs_var_flag_proxy(bs_ctx* c, const bs_bins* b, double pk_index, const float* chan_w_host,
                                 double* G_host) {
  if (!c || !b || !G_host) return BS_EINVAL;
  const auto& P = b->P;
  if (P.kind != BS_SHELL_K || !b->d_lut) return ctx_fail(c, BS_EINVAL, "bs_var_flag_proxy needs device 3D shell bins");
  if (!std::isfinite(pk_index)) return ctx_fail(c, BS_EINVAL, "bad power-law index");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  const int n = P.n, nc = P.nc, nh = n / 2 + 1;
  // window autocorrelation a(nu) = (1/nc) sum_mu w(mu) w(mu + nu mod nc)
  std::vector<double> w(nc, 1.0), a(nc, 0.0);
  if (chan_w_host)
    for (int i = 0; i < nc; ++i) {
      if (!std::isfinite(chan_w_host[i]) || chan_w_host[i] < 0.f) return ctx_fail(c, BS_EINVAL, "channel weights must be finite and >= 0");
      w[i] = chan_w_host[i];
    }
  for (int nu = 0; nu < nc; ++nu) {
    double acc = 0.0;
    for (int mu = 0; mu < nc; ++mu) acc += w[mu] * w[(mu + nu) % nc];
    a[nu] = acc / nc;
  }
  if (!(a[0] > 0.0)) return ctx_fail(c, BS_EINVAL, "every channel is flagged");
  const int ncand = (int)(P.tri.size() / 3);
  double* d_a = (double*)ctx_ws(c, "varp_a", (size_t)nc * 8);
  double* d_xi = (double*)ctx_ws(c, "varp_xi", (size_t)(P.smax + 1) * nc * 8);
  void* d_V = ctx_ws(c, "varp_V", (size_t)nc * n * nh * 16);
  double* d_B = (double*)ctx_ws(c, "varp_B", (size_t)std::max(ncand, 1) * 8);
  int64_t* d_N = (int64_t*)ctx_ws(c, "varp_N", (size_t)std::max(ncand, 1) * 8);
  if (!d_a || !d_xi || !d_V || !d_B || !d_N) return ctx_fail(c, BS_ENOMEM, "flag proxy workspace");
  HIPCHK(c, hipMemcpyAsync(d_a, a.data(), (size_t)nc * 8, hipMemcpyHostToDevice, c->stream));
  launch_var_xi(nc, P.smax, P.cperp * P.cperp, P.cpar * P.cpar, pk_index, d_xi, c->stream);
  launch_var_cube(n, nh, nc, P.smax, d_a, d_xi, d_V, c->stream);
  LAUNCHCHK(c, "flag proxy cube");
  // the FP64 estimator with unit weights: B = N_vox S_D / T3D = mean over closed triangles of
  // P_w1 P_w2 P_w3 / N_vox
  const int rc = bs_estimate_3d(c, b, d_V, nullptr, BS_FP64, 1.0, d_B, d_N, nullptr);
  if (rc) return rc;
  std::vector<double> hb(ncand);
  HIPCHK(c, hipMemcpyAsync(hb.data(), d_B, (size_t)ncand * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double nvox = (double)nc * n * n;
  for (int t = 0; t < ncand; ++t) G_host[t] = hb[t] * nvox;   // NaN where N_tri = 0 stays NaN
  return BS_OK;
}

extern "C" int bs_var_features_flag(const bs_bins* b, const int64_t* T3D_host, const double* G_host,
                                    const double* G1_host, double rho3, float* X_host, double* base_host) {
  if (!b || !X_host || !G_host || !G1_host || !(rho3 > 0.0)) return BS_EINVAL;
  const auto& P = b->P;
  const int nt = (int)(P.tri.size() / 3);
  const double nvox = (double)P.nc * P.n * P.n;
  std::vector<double> lc(P.nbins);
  for (int j = 0; j < P.nbins; ++j) lc[j] = 0.5 * (std::log(P.edges[j]) + std::log(P.edges[j + 1]));
  for (int t = 0; t < nt; ++t) {
    for (int i = 0; i < 3; ++i) X_host[4 * t + i] = (float)lc[P.tri[3 * t + i]];
    const bool ok = G_host[t] > 0.0 && G1_host[t] > 0.0;
    X_host[4 * t + 3] = ok ? (float)(std::log(G_host[t] / G1_host[t]) - 2.0 * std::log(rho3)) : NAN;
    if (base_host) {
      const double T = T3D_host ? (double)T3D_host[t] : 0.0;
      base_host[t] = (T > 0 && ok) ? std::log(nvox / T) + std::log(G_host[t]) - 2.0 * std::log(rho3) : -INFINITY;
    }
  }
  return BS_OK;
}
