// C ABI of libbs: context, workspace, bin plans, and the MABS estimator pipeline.
// The 3D estimator lives in bs_api3d.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "bs_ctx.h"
#include "bs_kernels.h"

// ------------------------------------------------------------------ helpers
int ctx_fail(bs_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

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

void* ctx_ws(bs_ctx* c, const char* name, size_t bytes) {
  DevBuf& b = c->ws[name];
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return b.p;
  if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
  b.mirror.clear();
  ++c->ws_gen;
  if (getenv("BS_FORCE_ENOMEM")) return nullptr;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  b.p = p;
  b.bytes = bytes;
  return p;
}

bool fft_len_ok(int L) {
  if (L < 2) return false;
  while (L % 2 == 0) L /= 2;
  while (L % 3 == 0) L /= 3;
  return L == 1;
}

FftPlan make_fft_plan(int L) {
  FftPlan p{};
  p.L = L;
  int m = L, nr = 0;
  while (m % 8 == 0 && nr < 13) { p.rad[nr++] = 8; m /= 8; }
  if (m % 4 == 0) { p.rad[nr++] = 4; m /= 4; }
  if (m % 2 == 0) { p.rad[nr++] = 2; m /= 2; }
  while (m % 3 == 0 && nr < 14) { p.rad[nr++] = 3; m /= 3; }
  p.nr = nr;
  return p;
}

bool fft_ip_fits(const FftPlan& p, int nl, int threads, int bmax) {
  for (int s = 0; s < p.nr; ++s) {
    const int R = p.rad[s];
    const int bm = R == 8 ? std::max(1, bmax / 2) : bmax;
    if ((long long)nl * (p.L / R) > (long long)bm * threads) return false;
  }
  return true;
}

const void* ctx_twiddle(bs_ctx* c, int L, bool fp64) {
  auto& mp = fp64 ? c->tw64 : c->tw32;
  auto it = mp.find(L);
  if (it != mp.end()) return it->second;
  std::vector<double> w(2 * (size_t)L);
  for (int m = 0; m < L; ++m) {
    // exp(-2 pi i m / L), reduced to the first octant-free form via exact symmetric angles
    long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)L;
    w[2 * m] = (double)cosl(ang);
    w[2 * m + 1] = (double)sinl(ang);
  }
  void* d = nullptr;
  size_t bytes = fp64 ? 16 * (size_t)L : 8 * (size_t)L;
  if (hipMalloc(&d, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  if (fp64) {
    if (hipMemcpy(d, w.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  } else {
    std::vector<float> f(2 * (size_t)L);
    for (size_t i = 0; i < f.size(); ++i) f[i] = (float)w[i];
    if (hipMemcpy(d, f.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  }
  mp[L] = d;
  return d;
}

// ------------------------------------------------------------------ context
extern "C" int bs_create(int device, void* hip_stream, bs_ctx** out) {
  if (!out) return BS_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) { (void)hipGetLastError(); return BS_EHIP; }
  if (device < 0 || device >= ndev) return BS_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return BS_EHIP;
  if (noalloc_scratch_init(device) != BS_OK) return BS_EHIP;
  bs_ctx* c = new bs_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  for (auto& e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) { delete c; return BS_EHIP; }
  }
  *out = c;
  return BS_OK;
}

extern "C" void bs_destroy(bs_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : c->ws) if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto& kv : c->tw32) (void)hipFree(kv.second);
  for (auto& kv : c->tw64) (void)hipFree(kv.second);
  for (auto& kv : c->dftw) (void)hipFree(kv.second);
  for (auto& kv : c->counts) if (kv.second.d_counts) (void)hipFree(kv.second.d_counts);
  for (auto& e : c->ev) if (e) (void)hipEventDestroy(e);
  delete c;
}

extern "C" const char* bs_last_error(const bs_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" int bs_last_count_dev(const bs_ctx* c, double* dev) {
  if (!c || !dev) return BS_EINVAL;
  *dev = c->last_count_dev;
  return BS_OK;
}

extern "C" int bs_last_count_bound(const bs_ctx* c, double* bound) {
  if (!c || !bound) return BS_EINVAL;
  *bound = c->last_count_bound;
  return BS_OK;
}

extern "C" int bs_set_stream(bs_ctx* c, void* s) {
  if (!c) return BS_EINVAL;
  c->stream = (hipStream_t)s;
  return BS_OK;
}

extern "C" int bs_set_timing(bs_ctx* c, int32_t enable) {
  if (!c) return BS_EINVAL;
  c->timing = enable != 0;
  c->have_timing = false;
  return BS_OK;
}

extern "C" int bs_last_timing(const bs_ctx* cc, double* out, int32_t n) {
  bs_ctx* c = const_cast<bs_ctx*>(cc);
  if (!c || !out || !c->timing || !c->have_timing) return BS_EINVAL;
  // events: 0 start, 1 end, 2/3 contraction, 4/5 fields
  float ms = 0.f;
  if (hipEventSynchronize(c->ev[1]) != hipSuccess) return BS_EHIP;
  double v[6] = {0, 0, 0, (double)c->last_grid_M, c->last_flops_vox, c->last_vox};
  if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) v[0] = ms;
  if (hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess) v[1] = ms;
  if (hipEventElapsedTime(&ms, c->ev[4], c->ev[5]) == hipSuccess) v[2] = ms;
  (void)hipGetLastError();
  for (int i = 0; i < n && i < 6; ++i) out[i] = v[i];
  return BS_OK;
}

// ------------------------------------------------------------------ bins
extern "C" int bs_make_bins(bs_ctx* c, const bs_bins_desc* d, bs_bins** out, int32_t* ncand) {
  if (!d || !out) return ctx_fail(c, BS_EINVAL, "bs_make_bins: NULL argument");
  *out = nullptr;
  if (d->kind == BS_SHELL_K && !fft_len_ok(d->nc)) return ctx_fail(c, BS_EINVAL, "nc must be 2^a 3^b");
  if (d->kind == BS_RING_U && !fft_len_ok(d->n)) return ctx_fail(c, BS_EINVAL, "n must be 2^a 3^b");
  bs_bins* b = new bs_bins();
  std::string e = bsplan::build_plan(d->kind, d->n, d->nc, d->nbins, d->edges_host, d->umax, d->du_lambda,
                                     d->r_mpc, d->rprime_mpc_per_mhz, d->dnu_mhz, b->P);
  if (!e.empty()) { delete b; return ctx_fail(c, BS_EINVAL, "bs_make_bins: " + e); }
  if (!fft_len_ok(d->n)) { delete b; return ctx_fail(c, BS_EINVAL, "n must be 2^a 3^b"); }
  b->ctx = c;
  if (!c) {  // host-only plan: triangle lists and mode counts, no device LUT
    *out = b;
    if (ncand) *ncand = (int32_t)(b->P.tri.size() / 3);
    return BS_OK;
  }
  if (hipSetDevice(c->device) != hipSuccess) { delete b; return ctx_fail(c, BS_EHIP, "hipSetDevice"); }
  size_t bytes = b->P.lut.size();
  if (hipMalloc(&b->d_lut, bytes) != hipSuccess) { (void)hipGetLastError(); delete b; return ctx_fail(c, BS_ENOMEM, "lut"); }
  if (hipMemcpy(b->d_lut, b->P.lut.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(b->d_lut); delete b; return ctx_fail(c, BS_EHIP, "lut copy");
  }
  *out = b;
  if (ncand) *ncand = (int32_t)(b->P.tri.size() / 3);
  return BS_OK;
}

extern "C" int bs_bins_triangles(const bs_bins* b, int32_t* tri, int64_t* modes) {
  if (!b) return BS_EINVAL;
  if (tri) std::memcpy(tri, b->P.tri.data(), b->P.tri.size() * sizeof(int32_t));
  if (modes) std::memcpy(modes, b->P.modes.data(), b->P.modes.size() * sizeof(int64_t));
  return BS_OK;
}

extern "C" int bs_bins_info(const bs_bins* b, int32_t* eta_max, int32_t* true_closure) {
  if (!b) return BS_EINVAL;
  if (eta_max) *eta_max = b->P.eta_max;
  if (true_closure) *true_closure = b->P.true_closure ? 1 : 0;
  return BS_OK;
}

extern "C" void bs_free_bins(bs_bins* b) {
  if (!b) return;
  if (b->d_lut) (void)hipFree(b->d_lut);
  delete b;
}

// ------------------------------------------------------------------ ring fields
namespace {

struct RingFieldLaunch {
  int G, CB, RB;
  size_t lds;
};

RingFieldLaunch ring_field_geometry(int n, int vmax, size_t esz) {
  const int ncols = vmax + 1, M = n / 2;
  RingFieldLaunch r{};
  for (int G = 1; G <= n / 4; G *= 2) {
    if (n % G) break;
    int Lc = n / G;
    int CB = std::max(1, std::min(ncols, 2048 / Lc));
    int RB = std::max(1, std::min(Lc, 2048 / M));
    size_t work = std::max((size_t)CB * Lc, (size_t)RB * M);
    size_t lds = esz * ((size_t)ncols * Lc + 2 * work);
    r = {G, CB, RB, lds};
    if (lds <= 128 * 1024) return r;
  }
  return r;
}

}  // namespace

// Arguments of the ring-field kernel for ring ids already on the device (no upload, no launch).
int ring_fields_prepare(bs_ctx* c, const bs_bins* b, const bs_weights* w, bool fp64, bool count_mode,
                        bool ignore_chan, const int* d_bins, void* out, long long bin_stride, MabsFieldArgs& a,
                        size_t& lds) {
  const auto& P = b->P;
  const int n = P.n;
  const void* tw = ctx_twiddle(c, n, fp64);
  if (!tw) return ctx_fail(c, BS_ENOMEM, "twiddle table");
  RingFieldLaunch g = ring_field_geometry(n, P.vmax, fp64 ? 16 : 8);
  if (g.lds > 160 * 1024) return ctx_fail(c, BS_EUNSUPPORTED, "ring field transform does not fit in LDS");
  a = MabsFieldArgs{};
  a.vis = nullptr;
  a.ng = w ? w->ng : nullptr;
  a.uvm = w ? w->uv_mask : nullptr;
  a.chw = w ? w->chan_w : nullptr;
  a.lut = b->d_lut;
  a.smax = P.smax;
  a.bins = d_bins;
  a.n = n; a.nh = P.nh; a.nc = P.nc; a.vmax = P.vmax;
  a.G = g.G; a.CB = g.CB; a.RB = g.RB;
  a.count_mode = count_mode ? 1 : 0;
  a.ignore_chan = ignore_chan ? 1 : 0;
  a.out = out;
  a.plane_stride = (long long)n * n;
  a.bin_stride = bin_stride;
  a.tw_n = tw;
  a.pcol = make_fft_plan(n / g.G);
  a.prow = make_fft_plan(n / 2);
  // smallest radices first (first-pass LDS writes spread over more banks; the same DFT)
  if (!getenv("BS_MABS_RADIX_DESC")) {
    std::reverse(a.pcol.rad, a.pcol.rad + a.pcol.nr);
    std::reverse(a.prow.rad, a.prow.rad + a.prow.nr);
  }
  a.scale = 1.0 / ((double)n * (double)n);
  lds = g.lds;
  return BS_OK;
}

// Launches the ring-field kernel over `nblocks` rings and channels [0, nch) (grid.y <= 65535 each).
void ring_fields_launch(MabsFieldArgs a, bool fp64, int nblocks, int nch, size_t lds, hipStream_t s) {
  for (int c0 = 0; c0 < nch; c0 += 65535) {
    a.chan_offset = c0;
    int cn = std::min(65535, nch - c0);
    if (fp64) launch_mabs_fields_f64(a, nblocks, cn, lds, s);
    else launch_mabs_fields_f32(a, nblocks, cn, lds, s);
  }
}

namespace {

// Launch ring-filtered fields for `blocks` (ring ids) over channels [0, nch) of `vis`.
int run_ring_fields(bs_ctx* c, const bs_bins* b, const void* vis, const bs_weights* w, bool fp64,
                    bool count_mode, bool ignore_chan, int nch, const std::vector<int>& blocks,
                    void* out, long long bin_stride) {
  if (blocks.empty()) return BS_OK;
  int* d_bins = (int*)ctx_ws(c, count_mode ? "ring_bins_c" : "ring_bins_d", blocks.size() * sizeof(int));
  if (!d_bins) return ctx_fail(c, BS_ENOMEM, "workspace (ring ids)");
  HIPCHK(c, hipMemcpyAsync(d_bins, blocks.data(), blocks.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  MabsFieldArgs a;
  size_t lds = 0;
  int rc = ring_fields_prepare(c, b, w, fp64, count_mode, ignore_chan, d_bins, out, bin_stride, a, lds);
  if (rc) return rc;
  a.vis = vis;
  ring_fields_launch(a, fp64, (int)blocks.size(), nch, lds, c->stream);
  LAUNCHCHK(c, "ring field kernel");
  return BS_OK;
}

int check_weights(bs_ctx* c, const bs_weights* w) {
  if (!w) return BS_OK;
  if (w->ng && (w->uv_mask || w->chan_w)) return ctx_fail(c, BS_EINVAL, "weights: give either ng or (uv_mask, chan_w)");
  return BS_OK;
}

uint64_t hash_bytes(uint64_t h, const void* p, size_t n) {
  const unsigned char* q = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) { h ^= q[i]; h *= 1099511628211ULL; }
  return h;
}

}  // namespace

extern "C" int bs_filter_fields(bs_ctx* c, const bs_bins* b, const void* vis, const bs_weights* w,
                                int32_t three_d, int32_t precision, void* fields, double* count_fields);
int filter_fields_3d(bs_ctx* c, const bs_bins* b, const void* vis, const bs_weights* w, int32_t precision,
                     void* fields, double* count_fields);

extern "C" int bs_filter_fields(bs_ctx* c, const bs_bins* b, const void* vis, const bs_weights* w,
                                int32_t three_d, int32_t precision, void* fields, double* count_fields) {
  if (!c || !b || !b->d_lut) return ctx_fail(c, BS_EINVAL, "bs_filter_fields: NULL context or host-only bins");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  int rc = check_weights(c, w);
  if (rc) return rc;
  if (precision < 0 || precision > 2) return ctx_fail(c, BS_EINVAL, "bad precision");
  if (three_d) return filter_fields_3d(c, b, vis, w, precision, fields, count_fields);
  if (b->P.kind != BS_RING_U) return ctx_fail(c, BS_EINVAL, "three_d == 0 needs BS_RING_U bins");
  if (!vis && fields) return ctx_fail(c, BS_EINVAL, "vis is NULL");
  const auto& P = b->P;
  const long long plane = (long long)P.n * P.n;
  std::vector<int> blocks(P.nbins);
  for (int i = 0; i < P.nbins; ++i) blocks[i] = i;
  if (fields) {
    rc = run_ring_fields(c, b, vis, w, precision == BS_FP64, false, false, P.nc, blocks, fields, plane * P.nc);
    if (rc) return rc;
  }
  if (count_fields) {
    rc = run_ring_fields(c, b, vis, w, true, true, false, P.nc, blocks, count_fields, plane * P.nc);
    if (rc) return rc;
  }
  return BS_OK;
}

// ------------------------------------------------------------------ Eq. (dft)
extern "C" int bs_mabs_dft(bs_ctx* c, int32_t nc, int32_t n_tri, int32_t circular, const double* Bbar, double scale,
                           void* out) {
  if (!c) return BS_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  if (nc > 4096 || !fft_len_ok(nc)) return ctx_fail(c, BS_EINVAL, "bs_mabs_dft: nc must be 2^a 3^b in [2, 4096]");
  if (n_tri < 0 || n_tri > 65535) return ctx_fail(c, BS_EINVAL, "bs_mabs_dft: n_tri must be in [0, 65535]");
  if (n_tri == 0) return BS_OK;
  if (!Bbar || !out) return ctx_fail(c, BS_EINVAL, "bs_mabs_dft: Bbar and out must be non-NULL");
  MdftArgs a{};
  a.plan = make_fft_plan(nc);
  // smallest radices first: the first pass writes with a lane stride of R elements, and radix 3
  // spreads those writes over the LDS banks better than radix 8 (any order gives the same DFT)
  if (!getenv("BS_MDFT_RADIX_DESC")) std::reverse(a.plan.rad, a.plan.rad + a.plan.nr);
  a.tw = ctx_twiddle(c, nc, true);
  if (!a.tw) return ctx_fail(c, BS_ENOMEM, "twiddle table");
  a.B = Bbar;
  a.out = out;
  a.L = nc;
  a.H = nc / 2 + 1;
  a.h = nc / 2;
  a.S = circular ? nc : 2 * nc - 1;
  a.circ = circular ? 1 : 0;
  a.nt = n_tri;
  a.scale = scale;
  constexpr size_t kLdsMax = 160 * 1024;
  auto knob = [](const char* name, int def) {
    const char* e = getenv(name);
    return e ? atoi(e) : def;
  };
  // Pass n: column pairs per group (at most BS_MDFT_NCOLS, default 4), line stride 4 mod 16
  // elements (BS_MDFT_LDMOD) so that the transposing store spreads over the LDS banks.  Pass m: rows per
  // group (at most BS_MDFT_MROWS, default 2).  A block of 256 threads is tried first where asked
  // for (512 threads fit every length up to 4096); each pass takes the fewest butterflies per
  // thread (2 or 4) that its in-place FFT fits.
  const int nwant = std::max(1, std::min(8, knob("BS_MDFT_NCOLS", 4)));
  const int mwant = std::max(1, std::min(4, knob("BS_MDFT_MROWS", 2)));
  const int ldr = knob("BS_MDFT_LDMOD", 4) & 15;
  const int ld = nc + (16 + ldr - nc % 16) % 16;
  int nnl = 0, mnl = 0, nthreads = 0, mthreads = 0, nbm = 0, mbm = 0;
  for (int th : {knob("BS_MDFT_NCOLS_THREADS", 512) > 256 ? 512 : 256, 512})
    for (int nl : {8, 4, 2, 1})
      for (int bm : {2, 4})
        if (!nnl && nl <= nwant && fft_ip_fits(a.plan, nl, th, bm) && (size_t)(nc + nl * ld) * 16 <= kLdsMax) {
          nnl = nl;
          nthreads = th;
          nbm = bm;
        }
  for (int th : {knob("BS_MDFT_MROWS_THREADS", 256) > 256 ? 512 : 256, 512})
    for (int nl : {4, 2, 1})
      for (int bm : {2, 4})
        if (!mnl && nl <= mwant && fft_ip_fits(a.plan, nl, th, bm) && (size_t)(nl + 1) * nc * 16 <= kLdsMax) {
          mnl = nl;
          mthreads = th;
          mbm = bm;
        }
  if (!nnl || !mnl) return ctx_fail(c, BS_EUNSUPPORTED, "bs_mabs_dft: no in-place FFT layout for this nc");
  a.grid = std::max(1, knob("BS_MDFT_GRID", 4096));
  a.X = ctx_ws(c, "mdft_half", (size_t)n_tri * nc * a.H * 16);
  if (!a.X) return ctx_fail(c, BS_ENOMEM, "bs_mabs_dft workspace");
  if (c->timing) { (void)hipEventRecord(c->ev[0], c->stream); (void)hipEventRecord(c->ev[4], c->stream); }
  a.nl = nnl;
  a.lgnl = nnl == 8 ? 3 : nnl == 4 ? 2 : nnl == 2 ? 1 : 0;
  a.ld = ld;
  a.threads = nthreads;
  a.bm = nbm;
  launch_mdft_n(a, (size_t)(nc + nnl * ld) * 16, c->stream);
  if (c->timing) { (void)hipEventRecord(c->ev[5], c->stream); (void)hipEventRecord(c->ev[2], c->stream); }
  a.nl = mnl;
  a.threads = mthreads;
  a.bm = mbm;
  launch_mdft_m(a, (size_t)(mnl + 1) * nc * 16, c->stream);
  if (c->timing) {
    (void)hipEventRecord(c->ev[3], c->stream);
    (void)hipEventRecord(c->ev[1], c->stream);
    c->have_timing = true;
  }
  if (hipGetLastError() != hipSuccess) return ctx_fail(c, BS_EHIP, "bs_mabs_dft launch");
  return BS_OK;
}

// ------------------------------------------------------------------ monopole B(k1, mu, t)
extern "C" int bs_monopole(bs_ctx* c, int32_t nc, int32_t n_tri, const double* kperp_host, double kpar_unit,
                           const void* Bcyl, int32_t n_k1, const double* k1_edges_host, double* mean,
                           int64_t* count) {
  if (!c) return BS_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  if (nc < 1 || nc > 65536) return ctx_fail(c, BS_EINVAL, "bs_monopole: nc must be in [1, 65536]");
  if (n_tri < 0 || (long long)n_tri * nc > (1LL << 31) - 1)
    return ctx_fail(c, BS_EINVAL, "bs_monopole: n_tri * nc must be in [0, 2^31)");
  if (n_k1 < 1 || n_k1 > MONO_MAX_K1) return ctx_fail(c, BS_EINVAL, "bs_monopole: n_k1 must be in [1, 64]");
  if (!k1_edges_host || !mean || !count) return ctx_fail(c, BS_EINVAL, "bs_monopole: NULL edges or outputs");
  for (int i = 0; i < n_k1; ++i)
    if (!(k1_edges_host[i + 1] > k1_edges_host[i]) || !(k1_edges_host[i] >= 0.0))
      return ctx_fail(c, BS_EINVAL, "bs_monopole: k1 edges must be non-negative and increasing");
  if (!(kpar_unit > 0.0) || !std::isfinite(kpar_unit)) return ctx_fail(c, BS_EINVAL, "bs_monopole: kpar_unit must be > 0");
  if (n_tri > 0 && (!kperp_host || !Bcyl)) return ctx_fail(c, BS_EINVAL, "bs_monopole: NULL kperp or Bcyl");
  for (long long i = 0; i < 3LL * n_tri; ++i)
    if (!(kperp_host[i] > 0.0) || !std::isfinite(kperp_host[i]))
      return ctx_fail(c, BS_EINVAL, "bs_monopole: kperp must be positive and finite");
  const int nb = n_k1 * 25;
  // a wave per row, blocks of four rows, at most 2048 blocks (eight waves per SIMD on 256 CUs, to hide
  // the latency of each row's loads): partial bins then a fixed-order reduction
  const long long rows = (long long)n_tri * nc;
  const int nblocks = (int)std::max(1LL, std::min(2048LL, (rows + 3) / 4));
  MonoArgs a{};
  double* dk = static_cast<double*>(ctx_ws(c, "mono_k", (size_t)(3 * std::max(n_tri, 1) + n_k1 + 1) * sizeof(double)));
  a.psum = static_cast<double*>(ctx_ws(c, "mono_psum", (size_t)nblocks * nb * sizeof(double)));
  a.pcnt = static_cast<int*>(ctx_ws(c, "mono_pcnt", (size_t)nblocks * nb * sizeof(int)));
  a.stage_s = static_cast<double*>(ctx_ws(c, "mono_stage_s", (size_t)part_groups(nblocks) * nb * sizeof(double)));
  a.stage_c = static_cast<long long*>(ctx_ws(c, "mono_stage_c", (size_t)part_groups(nblocks) * nb * sizeof(long long)));
  if (!dk || !a.psum || !a.pcnt || !a.stage_s || !a.stage_c) return ctx_fail(c, BS_ENOMEM, "bs_monopole workspace");
  std::vector<double> hk((size_t)3 * n_tri + n_k1 + 1);
  for (long long i = 0; i < 3LL * n_tri; ++i) hk[i] = kperp_host[i];
  for (int i = 0; i <= n_k1; ++i) hk[(size_t)3 * n_tri + i] = k1_edges_host[i];
  HIPCHK(c, hipMemcpyAsync(dk, hk.data(), hk.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  a.B = static_cast<const double*>(Bcyl);
  a.kperp = dk;
  a.k1e = dk + 3 * (size_t)n_tri;
  a.kpar_unit = kpar_unit;
  a.nc = nc;
  a.nt = n_tri;
  a.nk = n_k1;
  if (c->timing) { (void)hipEventRecord(c->ev[0], c->stream); (void)hipEventRecord(c->ev[2], c->stream); }
  launch_mono_bin(a, nblocks, c->stream);
  if (c->timing) { (void)hipEventRecord(c->ev[3], c->stream); (void)hipEventRecord(c->ev[4], c->stream); }
  launch_mono_fin(a, nblocks, mean, count, c->stream);
  if (c->timing) {
    (void)hipEventRecord(c->ev[5], c->stream);
    (void)hipEventRecord(c->ev[1], c->stream);
    c->have_timing = true;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));   // the host staging of the tables is released on return
  if (hipGetLastError() != hipSuccess) return ctx_fail(c, BS_EHIP, "bs_monopole launch");
  return BS_OK;
}

// ------------------------------------------------------------------ (k_par1, k_par2) grid (Sec. 5, Fig. 4)
extern "C" int bs_kpar_grid(bs_ctx* c, int32_t nc, int32_t n_tri, double kpar_unit, const void* Bcyl, int32_t n_e,
                            const double* edges_host, double* mean, int64_t* count) {
  if (!c) return BS_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  if (nc < 1 || nc > 65536) return ctx_fail(c, BS_EINVAL, "bs_kpar_grid: nc must be in [1, 65536]");
  if (n_tri < 0 || (long long)n_tri * nc > (1LL << 31) - 1)
    return ctx_fail(c, BS_EINVAL, "bs_kpar_grid: n_tri * nc must be in [0, 2^31)");
  if (n_e < 1 || n_e > KPAR_MAX_BINS) return ctx_fail(c, BS_EINVAL, "bs_kpar_grid: n_e must be in [1, 64]");
  if (!edges_host || !mean || !count || (n_tri > 0 && !Bcyl)) return ctx_fail(c, BS_EINVAL, "bs_kpar_grid: NULL pointer");
  for (int i = 0; i <= n_e; ++i)
    if (!std::isfinite(edges_host[i]) || (i > 0 && !(edges_host[i] > edges_host[i - 1])))
      return ctx_fail(c, BS_EINVAL, "bs_kpar_grid: edges must be finite and increasing");
  if (!(kpar_unit > 0.0) || !std::isfinite(kpar_unit)) return ctx_fail(c, BS_EINVAL, "bs_kpar_grid: kpar_unit must be > 0");
  // bin of every index on either axis, decided here once: k = kpar_unit a' in float64, the number of
  // edges at or below it minus one, the top edge closing the last bin
  std::vector<int> bin1(nc);
  std::vector<long long> h(n_e, 0);
  for (int x = 0; x < nc; ++x) {
    const double k = kpar_unit * (double)(2 * x < nc ? x : x - nc);
    int i = -1;
    for (int e = 0; e <= n_e; ++e) i += edges_host[e] <= k;
    if (k == edges_host[n_e]) i = n_e - 1;
    bin1[x] = (i >= 0 && i < n_e) ? i : -1;
    if (bin1[x] >= 0) ++h[bin1[x]];
  }
  std::vector<int64_t> cnt((size_t)n_e * n_e);
  for (int i = 0; i < n_e; ++i)
    for (int j = 0; j < n_e; ++j) cnt[(size_t)i * n_e + j] = h[i] * h[j];
  KparArgs a{};
  a.nc = nc;
  a.nt = n_tri;
  a.ne = n_e;
  // the signed indices inside the edges form one interval (k_par grows with a', the bins with k_par)
  a.jlo = 1;
  a.jhi = 0;
  for (int j = -(nc / 2); j <= (nc - 1) / 2; ++j) {
    if (bin1[j < 0 ? j + nc : j] < 0) continue;
    if (a.jlo > a.jhi) a.jlo = j;
    a.jhi = j;
  }
  const int L = std::max(0, a.jhi - a.jlo + 1);
  // row slabs of that interval so that about a thousand blocks run
  a.slabs = std::max(1, std::min(std::max(L, 1), (1024 + std::max(n_tri, 1) - 1) / std::max(n_tri, 1)));
  int* dbin = static_cast<int*>(ctx_ws(c, "kpar_bin", (size_t)nc * sizeof(int)));
  a.psum = static_cast<double*>(ctx_ws(c, "kpar_psum", (size_t)std::max(n_tri, 1) * a.slabs * n_e * n_e * sizeof(double)));
  if (!dbin || !a.psum) return ctx_fail(c, BS_ENOMEM, "bs_kpar_grid workspace");
  HIPCHK(c, hipMemcpyAsync(dbin, bin1.data(), bin1.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(count, cnt.data(), cnt.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  a.B = static_cast<const double*>(Bcyl);
  a.bin1 = dbin;
  a.count = count;
  if (c->timing) { (void)hipEventRecord(c->ev[0], c->stream); (void)hipEventRecord(c->ev[2], c->stream); }
  if (n_tri > 0 && L > 0) launch_kpar_bin(a, c->stream);
  if (c->timing) { (void)hipEventRecord(c->ev[3], c->stream); (void)hipEventRecord(c->ev[4], c->stream); }
  if (n_tri > 0) launch_kpar_fin(a, mean, c->stream);
  if (c->timing) {
    (void)hipEventRecord(c->ev[5], c->stream);
    (void)hipEventRecord(c->ev[1], c->stream);
    c->have_timing = true;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));   // the host staging of the tables is released on return
  if (hipGetLastError() != hipSuccess) return ctx_fail(c, BS_EHIP, "bs_kpar_grid launch");
  return BS_OK;
}

// ------------------------------------------------------------------ multipoles (Eqs. orient, bs_lm)
extern "C" int bs_multipoles(bs_ctx* c, int32_t nc, int32_t n_tri, const double* kperp_host, double kpar_unit,
                             const void* Bcyl, int32_t n_k1, const double* k1_edges_host, int32_t lmax,
                             double* moments, int64_t* count) {
  if (!c) return BS_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  if (lmax < 0 || lmax > MULTI_MAX_LMAX) return ctx_fail(c, BS_EINVAL, "bs_multipoles: lmax must be in [0, 4]");
  const int nlm = (lmax + 1) * (lmax + 2) / 2;
  if (nc < 1 || nc > 65536) return ctx_fail(c, BS_EINVAL, "bs_multipoles: nc must be in [1, 65536]");
  if (n_tri < 0 || (long long)n_tri * nc > (1LL << 31) - 1)
    return ctx_fail(c, BS_EINVAL, "bs_multipoles: n_tri * nc must be in [0, 2^31)");
  if (n_k1 < 1 || n_k1 > MONO_MAX_K1 || n_k1 * 25 * nlm > MULTI_MAX_BINVALS)
    return ctx_fail(c, BS_EINVAL, "bs_multipoles: n_k1 must be in [1, 64] with 25 n_k1 (lmax+1)(lmax+2)/2 <= 6400");
  if (!k1_edges_host || !moments || !count) return ctx_fail(c, BS_EINVAL, "bs_multipoles: NULL edges or outputs");
  for (int i = 0; i < n_k1; ++i)
    if (!(k1_edges_host[i + 1] > k1_edges_host[i]) || !(k1_edges_host[i] >= 0.0))
      return ctx_fail(c, BS_EINVAL, "bs_multipoles: k1 edges must be non-negative and increasing");
  if (!(kpar_unit > 0.0) || !std::isfinite(kpar_unit)) return ctx_fail(c, BS_EINVAL, "bs_multipoles: kpar_unit must be > 0");
  if (n_tri > 0 && (!kperp_host || !Bcyl)) return ctx_fail(c, BS_EINVAL, "bs_multipoles: NULL kperp or Bcyl");
  for (long long i = 0; i < 3LL * n_tri; ++i)
    if (!(kperp_host[i] > 0.0) || !std::isfinite(kperp_host[i]))
      return ctx_fail(c, BS_EINVAL, "bs_multipoles: kperp must be positive and finite");
  const int nb = n_k1 * 25;
  const long long rows = (long long)n_tri * nc;
  // a wave per row: blocks of eight rows, at most 512 blocks
  const int nblocks = (int)std::max(1LL, std::min(512LL, (rows + 7) / 8));
  MultiArgs a{};
  double* dk = static_cast<double*>(ctx_ws(c, "multi_k", (size_t)(3 * std::max(n_tri, 1) + n_k1 + 1) * sizeof(double)));
  a.m.psum = static_cast<double*>(ctx_ws(c, "multi_psum", (size_t)nblocks * nb * nlm * sizeof(double)));
  a.m.pcnt = static_cast<int*>(ctx_ws(c, "multi_pcnt", (size_t)nblocks * nb * sizeof(int)));
  a.m.stage_s = static_cast<double*>(ctx_ws(c, "multi_stage_s", (size_t)part_groups(nblocks) * nb * nlm * sizeof(double)));
  a.m.stage_c = static_cast<long long*>(ctx_ws(c, "multi_stage_c", (size_t)part_groups(nblocks) * nb * sizeof(long long)));
  if (!dk || !a.m.psum || !a.m.pcnt || !a.m.stage_s || !a.m.stage_c)
    return ctx_fail(c, BS_ENOMEM, "bs_multipoles workspace");
  std::vector<double> hk((size_t)3 * n_tri + n_k1 + 1);
  for (long long i = 0; i < 3LL * n_tri; ++i) hk[i] = kperp_host[i];
  for (int i = 0; i <= n_k1; ++i) hk[(size_t)3 * n_tri + i] = k1_edges_host[i];
  HIPCHK(c, hipMemcpyAsync(dk, hk.data(), hk.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  a.m.B = static_cast<const double*>(Bcyl);
  a.m.kperp = dk;
  a.m.k1e = dk + 3 * (size_t)n_tri;
  a.m.kpar_unit = kpar_unit;
  a.m.nc = nc;
  a.m.nt = n_tri;
  a.m.nk = n_k1;
  a.lmax = lmax;
  a.nlm = nlm;
  // (2l + 1) sqrt((l - m)! / (l + m)!): sqrt(4 pi (2l + 1)) times the normalisation of Y_l^m
  for (int l = 0; l <= lmax; ++l)
    for (int m = 0; m <= l; ++m) {
      double r = 1.0;
      for (int k = l - m + 1; k <= l + m; ++k) r /= (double)k;
      a.lm_norm[l * (l + 1) / 2 + m] = (2.0 * l + 1.0) * std::sqrt(r);
    }
  if (c->timing) { (void)hipEventRecord(c->ev[0], c->stream); (void)hipEventRecord(c->ev[2], c->stream); }
  launch_multi_bin(a, nblocks, c->stream);
  if (c->timing) { (void)hipEventRecord(c->ev[3], c->stream); (void)hipEventRecord(c->ev[4], c->stream); }
  launch_multi_fin(a, nblocks, moments, count, c->stream);
  if (c->timing) {
    (void)hipEventRecord(c->ev[5], c->stream);
    (void)hipEventRecord(c->ev[1], c->stream);
    c->have_timing = true;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));   // the host staging of the tables is released on return
  if (hipGetLastError() != hipSuccess) return ctx_fail(c, BS_EHIP, "bs_multipoles launch");
  return BS_OK;
}

// ------------------------------------------------------------------ Eq. (vg) gridding
extern "C" int bs_grid_visibilities(bs_ctx* c, int32_t n, int32_t nc, double du_lambda, int64_t n_vis,
                                    const double* uv, const void* vis, const uint8_t* flags, int32_t chan_avg,
                                    int32_t out_precision, void* Vg, int32_t* Ng) {
  if (!c) return BS_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  if (n < 2 || n > 4096 || n % 2) return ctx_fail(c, BS_EINVAL, "bs_grid_visibilities: n must be even in [2, 4096]");
  if (chan_avg < 1 || nc < chan_avg || nc % chan_avg)
    return ctx_fail(c, BS_EINVAL, "bs_grid_visibilities: nc must be a positive multiple of chan_avg");
  if (!(du_lambda > 0.0) || !std::isfinite(du_lambda)) return ctx_fail(c, BS_EINVAL, "bs_grid_visibilities: du must be > 0");
  // the scatter launch has n_vis / 8 work-items along x, which must stay below 2^32
  if (n_vis < 0 || n_vis > (1LL << 34)) return ctx_fail(c, BS_EINVAL, "bs_grid_visibilities: n_vis must be in [0, 2^34]");
  if (out_precision < 0 || out_precision > 2) return ctx_fail(c, BS_EINVAL, "bad precision");
  if (!Vg || !Ng || (n_vis > 0 && (!uv || !vis))) return ctx_fail(c, BS_EINVAL, "bs_grid_visibilities: NULL pointer");
  GridArgs a{};
  a.uv = uv;
  a.vis = static_cast<const float*>(vis);
  a.flags = flags;
  a.nvis = n_vis;
  a.n = n;
  a.nc = nc;
  a.chan_avg = chan_avg;
  a.nco = nc / chan_avg;
  a.du = du_lambda;
  const size_t cells = (size_t)a.nco * n * (n / 2 + 1);
  a.acc = static_cast<double*>(ctx_ws(c, "grid_acc", cells * 2 * sizeof(double)));
  a.cnt = static_cast<int*>(ctx_ws(c, "grid_cnt", cells * sizeof(int)));
  const size_t hot = (size_t)a.nco * (size_t)std::max(1LL, grid_blocks(n_vis)) * GRID_NHOT;
  a.hot_v = static_cast<double*>(ctx_ws(c, "grid_hot_v", hot * 2 * sizeof(double)));
  a.hot_c = static_cast<int*>(ctx_ws(c, "grid_hot_c", hot * sizeof(int)));
  if (!a.acc || !a.cnt || !a.hot_v || !a.hot_c) return ctx_fail(c, BS_ENOMEM, "bs_grid_visibilities workspace");
  if (c->timing) (void)hipEventRecord(c->ev[0], c->stream);
  launch_grid_zero(a, c->stream);
  if (c->timing) (void)hipEventRecord(c->ev[2], c->stream);
  if (n_vis > 0) {
    launch_grid_scatter(a, c->stream);
    launch_grid_hot(a, c->stream);
  }
  if (c->timing) { (void)hipEventRecord(c->ev[3], c->stream); (void)hipEventRecord(c->ev[4], c->stream); }
  launch_grid_fin(a, out_precision == BS_FP64, Vg, Ng, c->stream);
  if (c->timing) {
    (void)hipEventRecord(c->ev[5], c->stream);
    (void)hipEventRecord(c->ev[1], c->stream);
    c->have_timing = true;
  }
  if (hipGetLastError() != hipSuccess) return ctx_fail(c, BS_EHIP, "bs_grid_visibilities launch");
  return BS_OK;
}

// ------------------------------------------------------------------ Eq. (S3) decorrelation
// Nodes z and weights w of the Q-point Gauss rule for the standard normal weight (probabilists'
// Hermite), from the eigen-decomposition of the symmetric tridiagonal Jacobi matrix of the
// recurrence x He_k = He_{k+1} + k He_{k-1} (off-diagonal sqrt(k)): the nodes are its eigenvalues,
// the weights the squared first components of its unit eigenvectors (Golub and Welsch 1969).
// Cyclic Jacobi rotations on the dense Q x Q matrix; Q <= 32.
static void gauss_normal_rule(int Q, std::vector<double>& z, std::vector<double>& w) {
  std::vector<double> A((size_t)Q * Q, 0.0), V((size_t)Q * Q, 0.0);
  for (int i = 0; i < Q; ++i) V[(size_t)i * Q + i] = 1.0;
  for (int k = 1; k < Q; ++k) A[(size_t)(k - 1) * Q + k] = A[(size_t)k * Q + (k - 1)] = std::sqrt((double)k);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < Q; ++p)
      for (int q = p + 1; q < Q; ++q) off += A[(size_t)p * Q + q] * A[(size_t)p * Q + q];
    if (off < 1e-34) break;
    for (int p = 0; p < Q; ++p)
      for (int q = p + 1; q < Q; ++q) {
        const double apq = A[(size_t)p * Q + q];
        if (apq == 0.0) continue;
        const double th = (A[(size_t)q * Q + q] - A[(size_t)p * Q + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < Q; ++k) {   // A <- A J (columns p, q)
          const double akp = A[(size_t)k * Q + p], akq = A[(size_t)k * Q + q];
          A[(size_t)k * Q + p] = c * akp - sn * akq;
          A[(size_t)k * Q + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < Q; ++k) {   // A <- J^T A (rows p, q)
          const double apk = A[(size_t)p * Q + k], aqk = A[(size_t)q * Q + k];
          A[(size_t)p * Q + k] = c * apk - sn * aqk;
          A[(size_t)q * Q + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < Q; ++k) {   // V <- V J
          const double vkp = V[(size_t)k * Q + p], vkq = V[(size_t)k * Q + q];
          V[(size_t)k * Q + p] = c * vkp - sn * vkq;
          V[(size_t)k * Q + q] = sn * vkp + c * vkq;
        }
      }
  }
  z.resize(Q);
  w.resize(Q);
  double ws = 0.0;
  for (int i = 0; i < Q; ++i) {
    z[i] = A[(size_t)i * Q + i];
    w[i] = V[(size_t)i] * V[(size_t)i];   // first component of eigenvector i
    ws += w[i];
  }
  for (int i = 0; i < Q; ++i) w[i] /= ws;
}

extern "C" int bs_decorrelation(bs_ctx* c, const bs_bins* rings, int64_t n_vis, const double* uv, double du_lambda,
                                double theta0_rad, int32_t n_nodes, double* D_host) {
  if (!c) return BS_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  if (!rings || rings->P.kind != BS_RING_U) return ctx_fail(c, BS_EINVAL, "bs_decorrelation: ring bins required");
  if (!D_host) return ctx_fail(c, BS_EINVAL, "bs_decorrelation: D_host is NULL");
  if (n_vis < 0 || n_vis > (1LL << 34) || (n_vis > 0 && !uv)) return ctx_fail(c, BS_EINVAL, "bs_decorrelation: bad baselines");
  if (!(du_lambda > 0.0) || !std::isfinite(du_lambda)) return ctx_fail(c, BS_EINVAL, "bs_decorrelation: du must be > 0");
  if (!(theta0_rad > 0.0) || !std::isfinite(theta0_rad)) return ctx_fail(c, BS_EINVAL, "bs_decorrelation: theta0 must be > 0");
  if (n_nodes < 2 || n_nodes > 32 || n_nodes % 2) return ctx_fail(c, BS_EINVAL, "bs_decorrelation: n_nodes must be even in [2, 32]");
  const bsplan::Plan& P = rings->P;
  const int n = P.n, nh = n / 2 + 1, ncand = (int)(P.tri.size() / 3);
  // exp(-a |dU|^2) = E_z[exp(i sqrt(2a) z . dU)] over a standard normal z in 2D; z -> -z conjugates
  // every cell value and leaves the (real) triangle averages unchanged, so the nodes with z_x > 0
  // carry twice their weight
  const double a = M_PI * M_PI * theta0_rad * theta0_rad / 3.0, t = std::sqrt(2.0 * a);
  std::vector<double> z, w;
  gauss_normal_rule(n_nodes, z, w);
  std::vector<double> kn, wn;
  for (int i = 0; i < n_nodes; ++i) {
    if (!(z[i] > 0.0)) continue;
    for (int j = 0; j < n_nodes; ++j) {
      kn.push_back(t * z[i]);
      kn.push_back(t * z[j]);
      wn.push_back(2.0 * w[i] * w[j]);
    }
  }
  const int nk = (int)wn.size();
  // per-node cell averages phi_g(k) = mean over the cell's baselines of exp(i k . delta) (Eq. vg,
  // phase mode of the gridding kernel), and the counts N_g
  const size_t plane = (size_t)n * nh;
  GridArgs g{};
  g.uv = uv;
  g.nvis = n_vis;
  g.n = n;
  g.nc = nk;
  g.chan_avg = 1;
  g.nco = nk;
  g.du = du_lambda;
  double* dk = static_cast<double*>(ctx_ws(c, "dec_k", (size_t)nk * 2 * sizeof(double)));
  g.acc = static_cast<double*>(ctx_ws(c, "grid_acc", (size_t)nk * plane * 2 * sizeof(double)));
  g.cnt = static_cast<int*>(ctx_ws(c, "grid_cnt", (size_t)nk * plane * sizeof(int)));
  const size_t ghot = (size_t)nk * (size_t)std::max(1LL, grid_blocks(n_vis)) * GRID_NHOT;
  g.hot_v = static_cast<double*>(ctx_ws(c, "grid_hot_v", ghot * 2 * sizeof(double)));
  g.hot_c = static_cast<int*>(ctx_ws(c, "grid_hot_c", ghot * sizeof(int)));
  void* phi = ctx_ws(c, "dec_phi", (size_t)nk * plane * 2 * sizeof(double));
  int32_t* ng32 = static_cast<int32_t*>(ctx_ws(c, "dec_ng32", (size_t)nk * plane * sizeof(int32_t)));
  uint16_t* ng16 = static_cast<uint16_t*>(ctx_ws(c, "dec_ng16", plane * sizeof(uint16_t)));
  double* dB = static_cast<double*>(ctx_ws(c, "dec_B", (size_t)std::max(ncand, 1) * sizeof(double)));
  int64_t* dN = static_cast<int64_t*>(ctx_ws(c, "dec_N", (size_t)std::max(ncand, 1) * sizeof(int64_t)));
  if (!dk || !g.acc || !g.cnt || !g.hot_v || !g.hot_c || !phi || !ng32 || !ng16 || !dB || !dN)
    return ctx_fail(c, BS_ENOMEM, "bs_decorrelation workspace");
  g.knode = dk;
  HIPCHK(c, hipMemcpyAsync(dk, kn.data(), kn.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  launch_grid_zero(g, c->stream);
  if (n_vis > 0) {
    launch_grid_scatter(g, c->stream);
    launch_grid_hot(g, c->stream);
  }
  launch_grid_fin(g, true, phi, ng32, c->stream);
  if (hipGetLastError() != hipSuccess) return ctx_fail(c, BS_EHIP, "bs_decorrelation gridding");
  // the counts do not depend on the node: N_g of node 0 as the per-cell weights (uint16)
  std::vector<int32_t> hn(plane);
  HIPCHK(c, hipMemcpyAsync(hn.data(), ng32, plane * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<uint16_t> h16(plane);
  for (size_t i = 0; i < plane; ++i) {
    if (hn[i] > 65535) return ctx_fail(c, BS_EINVAL, "bs_decorrelation: more than 65535 baselines in one grid cell");
    h16[i] = (uint16_t)hn[i];
  }
  HIPCHK(c, hipMemcpyAsync(ng16, h16.data(), plane * sizeof(uint16_t), hipMemcpyHostToDevice, c->stream));
  // one-channel ring bins of the same geometry
  bs_bins_desc d{};
  d.kind = BS_RING_U;
  d.n = n;
  d.nc = 1;
  d.nbins = P.nbins;
  d.edges_host = P.edges.data();
  d.umax = P.umax;
  bs_bins* b1 = nullptr;
  int32_t nc1 = 0;
  int rc = bs_make_bins(c, &d, &b1, &nc1);
  if (rc) return rc;
  std::vector<double> acc(ncand, 0.0), hb(ncand);
  bs_weights wt{ng16, nullptr, nullptr};
  for (int q = 0; q < nk && !rc; ++q) {
    // mean over the closed grid triangles of prod phi (norm n^2: the estimator's B is that mean / n^2)
    rc = bs_estimate_mabs(c, b1, static_cast<const char*>(phi) + (size_t)q * plane * 2 * sizeof(double), &wt, nullptr,
                          BS_FP64, (double)n * (double)n, dB, dN, nullptr);
    if (!rc && hipMemcpyAsync(hb.data(), dB, (size_t)ncand * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      rc = ctx_fail(c, BS_EHIP, "bs_decorrelation copy");
    if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = ctx_fail(c, BS_EHIP, "bs_decorrelation sync");
    for (int tt = 0; !rc && tt < ncand; ++tt) acc[tt] += wn[q] * hb[tt];   // NaN (no triangle) propagates
  }
  bs_free_bins(b1);
  if (rc) return rc;
  for (int tt = 0; tt < ncand; ++tt) D_host[tt] = acc[tt];
  return BS_OK;
}

// ------------------------------------------------------------------ MABS
// Certified rounding bound (bsplan::count_error_bound) of the FP64 ring counts of triangles `tri`
// ([n][3] bins): ring fields from a folded C2C along u and a C2R along v, two normalisations, and
// a summation whose longest chain of roundings is `depth`.
double ring_count_bound(const bsplan::Plan& P, const std::vector<int>& tri, double depth) {
  const double eps = bsplan::field_error_units(2 * bsplan::fft_stage_units(P.n) + 2, 2);
  double bound = 0.0;
  for (size_t t = 0; t + 2 < tri.size(); t += 3)
    bound = std::max(bound, bsplan::count_error_bound((double)P.modes[tri[t]], (double)P.modes[tri[t + 1]],
                                                      (double)P.modes[tri[t + 2]], eps, depth));
  return bound;
}

extern "C" int bs_estimate_mabs(bs_ctx* c, const bs_bins* b, const void* vis, const bs_weights* w,
                                const bs_mabs_sel* sel, int32_t precision, double norm, double* B,
                                int64_t* N_tri, int32_t* N_nu) {
  if (!c || !b || !b->d_lut) return ctx_fail(c, BS_EINVAL, "bs_estimate_mabs: NULL context or host-only bins");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  const auto& P = b->P;
  if (P.kind != BS_RING_U) return ctx_fail(c, BS_EINVAL, "MABS needs BS_RING_U bins");
  if (!vis || !B || !N_tri) return ctx_fail(c, BS_EINVAL, "vis, B and N_tri must be non-NULL");
  if (precision < 0 || precision > 2) return ctx_fail(c, BS_EINVAL, "bad precision");
  int rc = check_weights(c, w);
  if (rc) return rc;
  const int nc = P.nc, n = P.n;
  const int Ppix = n * n;
  if (precision != BS_FP64 && n % 8)
    return ctx_fail(c, BS_EUNSUPPORTED, "MFMA contraction needs n % 8 == 0 (pixel rows in 64-element blocks)");
  // ---- selection ----
  std::vector<int> tri;
  if (sel && sel->tri3_host) {
    if (sel->n_tri < 0) return ctx_fail(c, BS_EINVAL, "n_tri < 0");
    tri.assign(sel->tri3_host, sel->tri3_host + 3 * (size_t)sel->n_tri);
    for (int x : tri) if (x < 0 || x >= P.nbins) return ctx_fail(c, BS_EINVAL, "triangle bin out of range");
  } else {
    tri.assign(P.tri.begin(), P.tri.end());
  }
  const int ntri = (int)(tri.size() / 3);
  const int collapse = sel ? sel->collapse : 0;
  if (collapse < 0 || collapse > 2) return ctx_fail(c, BS_EINVAL, "collapse must be 0, 1 or 2");
  std::vector<int> nu1;
  if (sel && sel->nu1_host) {
    if (collapse) return ctx_fail(c, BS_EINVAL, "collapse needs all channels as nu1");
    if (sel->n_nu1 <= 0) return ctx_fail(c, BS_EINVAL, "n_nu1 must be positive");
    nu1.assign(sel->nu1_host, sel->nu1_host + sel->n_nu1);
    for (int x : nu1) if (x < 0 || x >= nc) return ctx_fail(c, BS_EINVAL, "nu1 out of range");
  } else {
    nu1.resize(nc);
    for (int i = 0; i < nc; ++i) nu1[i] = i;
  }
  if (collapse && !N_nu) return ctx_fail(c, BS_EINVAL, "collapse needs N_nu");
  if (ntri == 0) return BS_OK;
  const int n_nu1 = (int)nu1.size();
  const bool separable = !(w && w->ng);
  const bool fp64 = precision == BS_FP64;
  if (c->timing) { (void)hipEventRecord(c->ev[0], c->stream); (void)hipEventRecord(c->ev[4], c->stream); }

  // ---- ring blocks used by the selection ----
  std::map<int, int> blk;
  for (int x : tri) blk.emplace(x, 0);
  std::vector<int> blocks;
  for (auto& kv : blk) { kv.second = (int)blocks.size(); blocks.push_back(kv.first); }
  std::vector<int> tri_blk(tri.size());
  for (size_t i = 0; i < tri.size(); ++i) tri_blk[i] = blk[tri[i]];
  const int nbu = (int)blocks.size();
  const long long bstride = (long long)nc * Ppix;

  // ---- data fields ----
  size_t esz = fp64 ? 8 : 4;
  void* F = ctx_ws(c, "mabs_F", (size_t)nbu * bstride * esz);
  if (!F) return ctx_fail(c, BS_ENOMEM, "workspace (fields)");
  rc = run_ring_fields(c, b, vis, w, fp64, false, false, nc, blocks, F, bstride);
  if (rc) return rc;
  uint16_t *Fh = nullptr, *Fl = nullptr;
  if (precision == BS_SPLIT_BF16) {
    Fh = (uint16_t*)ctx_ws(c, "mabs_Fh", (size_t)nbu * bstride * 2);
    Fl = (uint16_t*)ctx_ws(c, "mabs_Fl", (size_t)nbu * bstride * 2);
    if (!Fh || !Fl) return ctx_fail(c, BS_ENOMEM, "workspace (split fields)");
    launch_split_bf16((const float*)F, Fh, Fl, (long long)nbu * bstride, c->stream);
    LAUNCHCHK(c, "split kernel");
  }
  if (c->timing) (void)hipEventRecord(c->ev[5], c->stream);

  unsigned long long* bad = (unsigned long long*)ctx_ws(c, "count_dev", 256);
  if (!bad) return ctx_fail(c, BS_ENOMEM, "workspace (flag)");
  HIPCHK(c, hipMemsetAsync(bad, 0, sizeof(unsigned long long), c->stream));

  // ---- counts ----
  int* d_tri = (int*)ctx_ws(c, "mabs_tri", tri_blk.size() * sizeof(int) + 16);
  if (!d_tri) return ctx_fail(c, BS_ENOMEM, "workspace (triangles)");
  HIPCHK(c, hipMemcpyAsync(d_tri, tri_blk.data(), tri_blk.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  int64_t* d_tperp = nullptr;
  double* I64 = nullptr;
  if (separable) {
    // channel-independent count fields and n^4 sum_p I1 I2 I3 per triangle (cached per geometry)
    uint64_t key = P.hash ^ 0x9e3779b97f4a7c15ULL;
    std::vector<uint8_t> hm;
    if (w && w->uv_mask) {
      hm.resize((size_t)n * P.nh);
      HIPCHK(c, hipMemcpyAsync(hm.data(), w->uv_mask, hm.size(), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      key = hash_bytes(key, hm.data(), hm.size());
    }
    key = hash_bytes(key, tri.data(), tri.size() * sizeof(int));
    auto it = c->counts.find(key);
    if (it == c->counts.end()) {
      // ring count fields: C2C along u (folded), C2R along v; the triple sum is 256 strided
      // chains of Ppix / 256 fused multiply-adds and an 8-level tree
      const double bound = ring_count_bound(P, tri, (double)((Ppix + 255) / 256) + 8.0);
      c->last_count_bound = bound;
      if (!(bound < 0.5))
        return ctx_fail(c, BS_ECOUNT, "triangle counts cannot be certified at this size (FP64 error bound " +
                                          std::to_string(bound) + " >= 1/2)");
      double* Ic = (double*)ctx_ws(c, "mabs_Iperp", (size_t)nbu * Ppix * 8);
      double* Ts = (double*)ctx_ws(c, "mabs_Tsum", (size_t)ntri * 8 + 16);
      if (!Ic || !Ts) return ctx_fail(c, BS_ENOMEM, "workspace (counts)");
      bs_weights wu{nullptr, w ? w->uv_mask : nullptr, nullptr};
      rc = run_ring_fields(c, b, nullptr, &wu, true, true, true, 1, blocks, Ic, Ppix);
      if (rc) return rc;
      launch_tperp(Ic, d_tri, ntri, Ppix, (double)Ppix * (double)Ppix, Ts, c->stream);
      LAUNCHCHK(c, "count contraction");
      CountCache cc;
      cc.tri.assign(tri.begin(), tri.end());
      if (hipMalloc(&cc.d_counts, (size_t)ntri * 8) != hipSuccess) { (void)hipGetLastError(); return ctx_fail(c, BS_ENOMEM, "count cache"); }
      launch_round_counts(Ts, ntri, cc.d_counts, bad, c->stream);
      LAUNCHCHK(c, "count rounding");
      double dev = 0.0;
      HIPCHK(c, hipMemcpyAsync(&dev, bad, sizeof(dev), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      c->last_count_dev = dev;
      if (!(dev <= bound)) {
        (void)hipFree(cc.d_counts);
        return ctx_fail(c, BS_ECOUNT, "triangle count off an integer by " + std::to_string(dev) + ", beyond its error bound " +
                                          std::to_string(bound));
      }
      cc.dev = dev;
      cc.bound = bound;
      it = c->counts.emplace(key, std::move(cc)).first;
    }
    d_tperp = it->second.d_counts;
    c->last_count_dev = it->second.dev;
    c->last_count_bound = it->second.bound;
  } else {
    I64 = (double*)ctx_ws(c, "mabs_I64", (size_t)nbu * bstride * 8);
    if (!I64) return ctx_fail(c, BS_ENOMEM, "workspace (count fields)");
    rc = run_ring_fields(c, b, nullptr, w, true, true, false, nc, blocks, I64, bstride);
    if (rc) return rc;
  }

  // ---- contraction + finalisation, batched over triangles to bound the workspace ----
  int* d_nu1 = (int*)ctx_ws(c, "mabs_nu1", nu1.size() * sizeof(int) + 16);
  if (!d_nu1) return ctx_fail(c, BS_ENOMEM, "workspace (nu1)");
  HIPCHK(c, hipMemcpyAsync(d_nu1, nu1.data(), nu1.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  const long long nrows = (long long)n_nu1 * nc;
  const size_t per_tri = (size_t)nrows * nc * 8;
  // number of pixel chunks: enough blocks to fill the chip, chunks of >= 1024 pixels
  const int tm = fp64 ? 64 : 128, tn = fp64 ? 64 : 128;
  long long tiles_per_tri = ((nrows + tm - 1) / tm) * ((nc + tn - 1) / tn);
  const size_t budget = (size_t)8 << 30;
  int tb = (int)std::max<size_t>(1, std::min<size_t>(ntri, budget / std::max<size_t>(per_tri, 1)));
  long long blocks_batch = tiles_per_tri * tb;
  int kchunks = 1;
  while (blocks_batch * kchunks < 2048 && Ppix / (kchunks * 2) >= 1024 && (Ppix / (kchunks * 2)) % 32 == 0) kchunks *= 2;
  // BS_MABS_KCHUNKS (tests): a fixed pixel-chunk count, so that small GEMMs run the long chunks of
  // large ones (used only if it splits the pixels into multiples of 32)
  if (const char* ek = getenv("BS_MABS_KCHUNKS")) {
    const int k = atoi(ek);
    if (k >= 1 && Ppix % k == 0 && (Ppix / k) % 32 == 0) kchunks = k;
  }
  int kchunk = Ppix / kchunks;
  if (!separable) {
    // per-channel count fields, FP64 GEMM: chains of kchunk products, then the chunk sums
    c->last_count_bound = ring_count_bound(P, tri, (double)kchunk + (double)kchunks + 4.0);
    if (!(c->last_count_bound < 0.5))
      return ctx_fail(c, BS_ECOUNT, "triangle counts cannot be certified at this size (FP64 error bound " +
                                        std::to_string(c->last_count_bound) + " >= 1/2)");
  }
  // the batch must hold kchunks partial copies
  tb = (int)std::max<size_t>(1, std::min<size_t>(ntri, budget / std::max<size_t>(per_tri * kchunks, 1)));
  double* S = (double*)ctx_ws(c, "mabs_S", per_tri * kchunks * tb);
  double* Sc = nullptr;
  if (!separable) Sc = (double*)ctx_ws(c, "mabs_Sc", per_tri * kchunks * tb);
  if (!S || (!separable && !Sc)) return ctx_fail(c, BS_ENOMEM, "workspace (partial sums)");
  const int D = collapse == 1 ? 2 * nc - 1 : nc;
  const size_t out_per_tri = collapse ? (size_t)D * D : (size_t)nrows * nc;
  bool first_gemm = true;
  for (int t0 = 0; t0 < ntri; t0 += tb) {
    const int nt = std::min(tb, ntri - t0);
    MabsGemmArgs g{};
    g.F = fp64 ? nullptr : (const float*)F;
    g.Fh = Fh; g.Fl = Fl;
    g.F64 = fp64 ? (const double*)F : nullptr;
    g.tri = d_tri + 3 * t0;
    g.nu1 = d_nu1;
    g.nc = nc; g.n_nu1 = n_nu1; g.P = Ppix; g.ntri = nt;
    g.kchunk = kchunk; g.kchunks = kchunks;
    g.bin_stride = bstride;
    g.S = S;
    if (c->timing && first_gemm) (void)hipEventRecord(c->ev[2], c->stream);
    if (precision == BS_SPLIT_BF16) launch_mabs_gemm_split(g, c->stream);
    else if (precision == BS_FP32) launch_mabs_gemm_f32(g, c->stream);
    else launch_mabs_gemm_f64(g, c->stream);
    LAUNCHCHK(c, "contraction kernel");
    if (c->timing && t0 + nt >= ntri) (void)hipEventRecord(c->ev[3], c->stream);
    first_gemm = false;
    if (!separable) {
      MabsGemmArgs gc = g;
      gc.F = nullptr; gc.Fh = gc.Fl = nullptr;
      gc.F64 = I64;
      gc.S = Sc;
      launch_mabs_gemm_f64(gc, c->stream);
      LAUNCHCHK(c, "count contraction kernel");
    }
    if (!collapse) {
      MabsFinalArgs f{};
      f.S = S; f.kchunks = kchunks;
      f.Sc = Sc; f.kchunks_c = kchunks;
      f.Tperp = d_tperp ? d_tperp + t0 : nullptr;
      f.chw = separable && w ? w->chan_w : nullptr;
      f.nu1 = d_nu1;
      f.nc = nc; f.n_nu1 = n_nu1; f.ntri = nt;
      f.npix = (double)Ppix; f.norm = norm;
      f.B = B + (size_t)t0 * out_per_tri;
      f.N = N_tri + (size_t)t0 * out_per_tri;
      f.bad = bad;
      launch_mabs_finalize(f, c->stream);
      LAUNCHCHK(c, "finalize kernel");
    } else {
      MabsCollapseArgs f{};
      f.S = S; f.kchunks = kchunks;
      f.Sc = Sc; f.kchunks_c = kchunks;
      f.Tperp = d_tperp ? d_tperp + t0 : nullptr;
      f.chw = separable && w ? w->chan_w : nullptr;
      f.nc = nc; f.ntri = nt; f.circular = collapse == 2;
      f.npix = (double)Ppix; f.norm = norm;
      f.B = B + (size_t)t0 * out_per_tri;
      f.N = N_tri + (size_t)t0 * out_per_tri;
      f.Nnu = N_nu + (size_t)t0 * out_per_tri;
      f.bad = bad;
      launch_mabs_collapse(f, c->stream);
      LAUNCHCHK(c, "collapse kernel");
    }
  }
  if (c->timing) { (void)hipEventRecord(c->ev[1], c->stream); c->have_timing = true; }
  if (!separable) {
    double dev = 0.0;
    HIPCHK(c, hipMemcpyAsync(&dev, bad, sizeof(dev), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->last_count_dev = dev;
    if (!(dev <= c->last_count_bound))
      return ctx_fail(c, BS_ECOUNT, "triangle count off an integer by " + std::to_string(dev) + ", beyond its error bound " +
                                        std::to_string(c->last_count_bound));
  }
  return BS_OK;
}
