// C ABI: seeded synthetic cubes on the GPU and Monte Carlo runs of the 3D estimator
// (generator -> delay transform -> shell fields -> contraction -> normalisation -> FP64
// accumulators), replayed from a captured hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include <cmath>
#include <string>
#include <vector>

#include "bs_ctx.h"
#include "bs_est3.h"
#include "bs_gen.h"

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

namespace {

int check_field_desc(bs_ctx* c, const bs_field_desc* d) {
  if (!d) return ctx_fail(c, BS_EINVAL, "field description is NULL");
  if (d->n < 8 || d->n % 4 || !fft_len_ok(d->n) || d->n > 1024)
    return ctx_fail(c, BS_EINVAL, "generator: n must be a multiple of 4, 2^a 3^b, 8 <= n <= 1024");
  if (d->nc < 2 || d->nc % 2 || !fft_len_ok(d->nc) || d->nc > 1536)
    return ctx_fail(c, BS_EINVAL, "generator: nc must be even, 2^a 3^b, <= 1536");
  if (d->kind != BS_K_CUBIC && d->kind != BS_K_PHYSICAL) return ctx_fail(c, BS_EINVAL, "generator: bad kind");
  if (d->kind == BS_K_PHYSICAL && !(d->du_lambda > 0 && d->r_mpc > 0 && d->rprime_mpc_per_mhz > 0 && d->dnu_mhz > 0))
    return ctx_fail(c, BS_EINVAL, "generator: physical constants must be positive");
  if (!(d->sigma >= 0) || !std::isfinite(d->f_ng) || !std::isfinite(d->pk_index))
    return ctx_fail(c, BS_EINVAL, "generator: bad sigma, f or index");
  return BS_OK;
}

// Fills everything but the device pointers.
GenArgs gen_args(bs_ctx* c, const bs_field_desc* d, int& rc) {
  GenArgs a{};
  rc = BS_OK;
  a.n = d->n; a.nc = d->nc; a.nh = d->n / 2 + 1;
  const double tp = 6.283185307179586476925286766559;
  if (d->kind == BS_K_CUBIC) { a.cz = tp / d->nc; a.cxy = tp / d->n; }
  else { a.cz = tp / (d->rprime_mpc_per_mhz * d->nc * d->dnu_mhz); a.cxy = tp * d->du_lambda / d->r_mpc; }
  a.index = d->pk_index;
  a.m2 = d->pk_index == -2.0 ? 1 : 0;
  a.sigma = d->sigma;
  a.fng = d->f_ng;
  a.tw_n = ctx_twiddle(c, d->n, false);
  a.tw_nc = ctx_twiddle(c, d->nc, false);
  if (!a.tw_n || !a.tw_nc) rc = ctx_fail(c, BS_ENOMEM, "twiddle tables");
  a.pn = make_fft_plan(d->n);
  a.pnc = make_fft_plan(d->nc);
  // smallest radices first (first-pass LDS writes spread over more banks; the same DFT)
  if (!getenv("BS_GEN_RADIX_DESC")) {
    std::reverse(a.pn.rad, a.pn.rad + a.pn.nr);
    std::reverse(a.pnc.rad, a.pnc.rad + a.pnc.nr);
  }
  a.NL = d->n <= 256 ? 16 : (d->n <= 512 ? 8 : 4);
  a.NLx = a.NL;
  auto ip_of = [](const FftPlan& p, int nl) { return fft_ip_fits(p, nl, 256, 2) ? 2 : fft_ip_fits(p, nl, 256, 4) ? 4 : 0; };
  a.ipx = ip_of(a.pn, a.NLx);
  // z pass: the most lines that transform in place within 32 KB of LDS (several blocks per CU),
  // else two buffers within 100 KB
  a.ipz = 0;
  for (int nl = 16; nl >= 1 && !a.ipz; nl /= 2)
    if ((size_t)nl * (d->nc + 1) * 8 + (size_t)nl * 8 <= 32 * 1024 && ip_of(a.pnc, nl)) { a.NLz = nl; a.ipz = ip_of(a.pnc, nl); }
  if (!a.ipz) {
    a.NLz = 16;
    while (a.NLz > 1 && 2 * (size_t)a.NLz * (d->nc + 1) * 8 + (size_t)a.NLz * 8 > 100 * 1024) a.NLz /= 2;
  }
  return a;
}

size_t part_len(const GenArgs& a) { return (size_t)std::max(a.nc, gen_row_blocks(a)); }

}  // namespace

int gen_prepare(bs_ctx* c, const bs_field_desc* d, GenArgs& a) {
  int rc = check_field_desc(c, d);
  if (rc) return rc;
  a = gen_args(c, d, rc);
  return rc;
}

extern "C" int bs_generate_cube(bs_ctx* c, const bs_field_desc* d, uint64_t seed, uint64_t realization,
                                const float* chan_w, void* vis) {
  if (!c) return BS_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  int rc = check_field_desc(c, d);
  if (rc) return rc;
  if (!vis) return ctx_fail(c, BS_EINVAL, "vis is NULL");
  GenArgs a = gen_args(c, d, rc);
  if (rc) return rc;
  a.state = (unsigned long long*)ctx_ws(c, "gen_state", 64);
  a.stat = (double*)ctx_ws(c, "gen_stat", 64);
  a.part = (double*)ctx_ws(c, "gen_part", part_len(a) * 8);
  a.g = (float*)ctx_ws(c, "gen_g", (size_t)d->nc * d->n * d->n * 4);
  if (!a.state || !a.stat || !a.part || !a.g) return ctx_fail(c, BS_ENOMEM, "generator workspace");
  a.chw = chan_w;
  a.W = (Cx<float>*)vis;
  launch_gen_set_state((unsigned long long*)a.state, seed, realization, c->stream);
  launch_gen_amp(a, c->stream);
  launch_gen_cube(a, c->stream);
  LAUNCHCHK(c, "generator");
  return BS_OK;
}

// ------------------------------------------------------------------ Monte Carlo object
struct bs_mc {
  bs_ctx* c = nullptr;
  const bs_bins* b = nullptr;
  bs_weights w{};
  double norm = 1.0;
  Est3 e;
  GenArgs ga{};
  hipStream_t s = nullptr;     // own stream (graph capture cannot use the null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<void*> owned;    // device allocations of this object
  unsigned long long* state = nullptr;
  double* B = nullptr;
  int64_t* N = nullptr;
  long long* cnt = nullptr;
  double* mean = nullptr;
  double* m2 = nullptr;
  int ntri = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void* mc_alloc(bs_mc* m, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  m->owned.push_back(p);
  return p;
}

// Runs f with the context's stream temporarily set to the object's own stream.
template <typename F>
int on_mc_stream(bs_mc* m, F f) {
  bs_ctx* c = m->c;
  hipStream_t saved = c->stream;
  const bool timing = c->timing;
  c->stream = m->s;
  c->timing = false;
  int rc = f();
  c->stream = saved;
  c->timing = timing;
  return rc;
}

// One realization: generate, estimate, accumulate (launches only).
int mc_enqueue_one(bs_mc* m) {
  bs_ctx* c = m->c;
  launch_gen_cube(m->ga, c->stream);
  LAUNCHCHK(c, "generator");
  int rc = est3_enqueue(c, m->b, m->ga.W, &m->w, m->e, m->norm, m->B, m->N, nullptr);
  if (rc) return rc;
  launch_mc_accumulate(m->B, m->ntri, m->cnt, m->mean, m->m2, m->state, c->stream);
  LAUNCHCHK(c, "accumulate");
  return BS_OK;
}

void mc_free(bs_mc* m) {
  if (!m) return;
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  if (m->s) (void)hipStreamSynchronize(m->s);
  for (void* p : m->owned) (void)hipFree(p);
  if (m->c && !m->e.tag.empty()) {  // private workspace slots of this object
    for (auto it = m->c->ws.begin(); it != m->c->ws.end();) {
      if (it->first.compare(0, m->e.tag.size(), m->e.tag) == 0) {
        (void)hipFree(it->second.p);
        it = m->c->ws.erase(it);
      } else {
        ++it;
      }
    }
  }
  if (m->ev_in) (void)hipEventDestroy(m->ev_in);
  if (m->ev_out) (void)hipEventDestroy(m->ev_out);
  if (m->s) (void)hipStreamDestroy(m->s);
  (void)hipGetLastError();
  delete m;
}

}  // namespace

extern "C" int bs_mc_create(bs_ctx* c, const bs_bins* b, const bs_field_desc* d, const bs_weights* w,
                            int32_t precision, double norm, bs_mc** out) {
  if (!c || !out) return BS_EINVAL;
  *out = nullptr;
  if (!b || !b->d_lut) return ctx_fail(c, BS_EINVAL, "bs_mc_create: host-only or NULL bins");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  int rc = check_field_desc(c, d);
  if (rc) return rc;
  if (b->P.kind != BS_SHELL_K) return ctx_fail(c, BS_EINVAL, "Monte Carlo runs need BS_SHELL_K bins");
  if (b->P.n != d->n || b->P.nc != d->nc) return ctx_fail(c, BS_EINVAL, "bins and field description differ in size");
  if (precision != BS_FP32 && precision != BS_SPLIT_BF16)
    return ctx_fail(c, BS_EINVAL, "Monte Carlo runs use BS_FP32 or BS_SPLIT_BF16");
  bs_mc* m = new bs_mc();
  m->c = c;
  m->b = b;
  if (w) m->w = *w;
  m->norm = norm;
  if (hipStreamCreateWithFlags(&m->s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    mc_free(m);
    return ctx_fail(c, BS_EHIP, "stream/event creation");
  }
  char tag[48];
  snprintf(tag, sizeof tag, "mc%p_", (void*)m);
  rc = on_mc_stream(m, [&]() { return est3_prepare(c, b, &m->w, precision, tag, m->e); });
  if (rc) { mc_free(m); return rc; }
  m->ntri = m->e.ntri;
  m->ga = gen_args(c, d, rc);
  if (rc) { mc_free(m); return rc; }
  const size_t cube = (size_t)d->nc * d->n * (d->n / 2 + 1) * 8;
  m->state = (unsigned long long*)mc_alloc(m, 64);
  m->ga.state = m->state;
  m->ga.stat = (double*)mc_alloc(m, 64);
  m->ga.part = (double*)mc_alloc(m, part_len(m->ga) * 8);
  m->ga.g = (float*)mc_alloc(m, (size_t)d->nc * d->n * d->n * 4);
  m->ga.W = (Cx<float>*)mc_alloc(m, cube);
  m->ga.chw = m->w.chan_w;
  const size_t nt = (size_t)std::max(m->ntri, 1);
  m->B = (double*)mc_alloc(m, nt * 8);
  m->N = (int64_t*)mc_alloc(m, nt * 8);
  m->cnt = (long long*)mc_alloc(m, nt * 8);
  m->mean = (double*)mc_alloc(m, nt * 8);
  m->m2 = (double*)mc_alloc(m, nt * 8);
  if (!m->state || !m->ga.stat || !m->ga.part || !m->ga.g || !m->ga.W || !m->B || !m->N || !m->cnt || !m->mean || !m->m2) {
    mc_free(m);
    return ctx_fail(c, BS_ENOMEM, "Monte Carlo buffers");
  }
  rc = on_mc_stream(m, [&]() {
    launch_gen_set_state(m->state, 0, 0, c->stream);
    launch_gen_amp(m->ga, c->stream);
    launch_mc_zero(m->cnt, m->mean, m->m2, m->ntri, c->stream);
    LAUNCHCHK(c, "Monte Carlo set-up");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return BS_OK;
  });
  if (rc) { mc_free(m); return rc; }
  *out = m;
  return BS_OK;
}

extern "C" int bs_mc_run(bs_mc* m, uint64_t seed, uint64_t first, int32_t count, int32_t use_graph) {
  if (!m) return BS_EINVAL;
  bs_ctx* c = m->c;
  if (count < 0) return ctx_fail(c, BS_EINVAL, "count must be >= 0");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  if (c->timing) (void)hipEventRecord(c->ev[0], c->stream);
  // order after earlier work on the context's stream
  HIPCHK(c, hipEventRecord(m->ev_in, c->stream));
  HIPCHK(c, hipStreamWaitEvent(m->s, m->ev_in, 0));
  int rc = on_mc_stream(m, [&]() -> int {
    launch_gen_set_state(m->state, seed, first, c->stream);
    LAUNCHCHK(c, "generator state");
    if (count == 0) return BS_OK;
    if (!use_graph) {
      for (int i = 0; i < count; ++i) {
        int r = mc_enqueue_one(m);
        if (r) return r;
      }
      return BS_OK;
    }
    if (!m->exec) {
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      int r = mc_enqueue_one(m);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->stream, &g);
      if (r) { if (g) (void)hipGraphDestroy(g); return r; }
      if (e != hipSuccess || !g) return ctx_fail(c, BS_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
      m->graph = g;
      HIPCHK(c, hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0));
    }
    for (int i = 0; i < count; ++i) HIPCHK(c, hipGraphLaunch(m->exec, c->stream));
    return BS_OK;
  });
  if (rc) return rc;
  HIPCHK(c, hipEventRecord(m->ev_out, m->s));
  HIPCHK(c, hipStreamWaitEvent(c->stream, m->ev_out, 0));
  if (c->timing) {
    (void)hipEventRecord(c->ev[1], c->stream);
    // contraction / fields split is not recorded for Monte Carlo runs
    (void)hipEventRecord(c->ev[2], c->stream); (void)hipEventRecord(c->ev[3], c->stream);
    (void)hipEventRecord(c->ev[4], c->stream); (void)hipEventRecord(c->ev[5], c->stream);
    c->have_timing = true;
  }
  return BS_OK;
}

extern "C" int bs_mc_stats(bs_mc* m, int64_t* n_host, double* mean_host, double* var_host) {
  if (!m) return BS_EINVAL;
  bs_ctx* c = m->c;
  const int nt = m->ntri;
  std::vector<long long> cn(nt);
  std::vector<double> mu(nt), q(nt);
  HIPCHK(c, hipStreamSynchronize(m->s));
  if (nt) {
    HIPCHK(c, hipMemcpy(cn.data(), m->cnt, nt * 8, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(mu.data(), m->mean, nt * 8, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(q.data(), m->m2, nt * 8, hipMemcpyDeviceToHost));
  }
  for (int t = 0; t < nt; ++t) {
    if (n_host) n_host[t] = cn[t];
    if (mean_host) mean_host[t] = cn[t] > 0 ? mu[t] : NAN;
    if (var_host) var_host[t] = cn[t] > 1 ? q[t] / (double)(cn[t] - 1) : NAN;
  }
  return BS_OK;
}

extern "C" int bs_mc_last(bs_mc* m, double* B_host, int64_t* N_host) {
  if (!m) return BS_EINVAL;
  bs_ctx* c = m->c;
  HIPCHK(c, hipStreamSynchronize(m->s));
  if (m->ntri && B_host) HIPCHK(c, hipMemcpy(B_host, m->B, (size_t)m->ntri * 8, hipMemcpyDeviceToHost));
  if (m->ntri && N_host) HIPCHK(c, hipMemcpy(N_host, m->N, (size_t)m->ntri * 8, hipMemcpyDeviceToHost));
  return BS_OK;
}

extern "C" int bs_mc_reset(bs_mc* m) {
  if (!m) return BS_EINVAL;
  bs_ctx* c = m->c;
  HIPCHK(c, hipEventRecord(m->ev_in, c->stream));
  HIPCHK(c, hipStreamWaitEvent(m->s, m->ev_in, 0));
  launch_mc_zero(m->cnt, m->mean, m->m2, m->ntri, m->s);
  LAUNCHCHK(c, "reset");
  HIPCHK(c, hipEventRecord(m->ev_out, m->s));
  HIPCHK(c, hipStreamWaitEvent(c->stream, m->ev_out, 0));
  return BS_OK;
}

extern "C" void bs_mc_destroy(bs_mc* m) { mc_free(m); }
