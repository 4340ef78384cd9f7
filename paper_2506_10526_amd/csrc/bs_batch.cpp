// C ABI: a batch of seeded cubes of uneven sizes through the MABS estimator (split-BF16 MFMA
// contraction), captured once into a hipGraph and replayed with one launch.
//
// Per cube: ring bins geomspace(1, umax + 1, nrings + 1) (umax = floor((n - 1) / 3)), every
// candidate triangle, a nu1 subset with all (nu2, nu3), unit weights.  The output per cube is the
// ergodic collapse over the nu1 subset (mean over the selected nu1 of B(nu1, nu1 - d1 + d2, nu1 - d1),
// Sec. 3.2 and Sec. 5), so that it stays O(nc^2) per triangle.
// Cubes are packed into waves whose workspaces fit a memory budget; the contraction of a wave is
// one persistent launch per tile kind in use (one block per CU pulling the tiles of all its cubes
// from per-XCD work queues, largest tiles first).  The tile shape and the pixel-chunk count (split
// K) of each cube shape class are picked by timing the candidates on the device the first time the
// class is seen in a context (or set beforehand with bs_tune_set), and cached in the context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "bs_ctx.h"
#include "bs_gen.h"
#include "bs_kernels.h"

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

struct BCube {
  int n = 0, nc = 0, nh = 0;
  uint64_t seed = 0, real = 0;
  bs_bins* bins = nullptr;
  std::vector<int> nu1, tri, blocks;   // tri: candidate ring ids; blocks: rings in use
  int ntri = 0, nbu = 0, n_nu1 = 0, kchunks = 1, wave = 0, valid = 0;
  int kind = 1, m1 = 16;   // tile: 0 = 128 x 256, 1 = 256 x 192 over m1 x 256/m1 (nu1, nu2) row blocks
  int *d_nu1 = nullptr, *d_tri = nullptr, *d_blocks = nullptr;
  int64_t* d_tperp = nullptr;
  std::vector<int64_t> tperp;
  GenArgs ga{};
  MabsFieldArgs fa{};
  size_t flds = 0;
  size_t off_vis = 0, off_g = 0, off_F = 0, off_Fh = 0, off_Fl = 0, off_S = 0;   // arena offsets
  double* Bbar = nullptr;
  int32_t* Nnu = nullptr;
  long long products = 0;
  size_t bytes_fields() const { return (size_t)nbu * nc * (size_t)n * n; }
  size_t footprint(int kc) const {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al((size_t)nc * n * nh * 8) + al((size_t)nc * n * n * 4) + al(bytes_fields() * 4) + 2 * al(bytes_fields() * 2) +
           al((size_t)kc * ntri * n_nu1 * nc * (size_t)nc * 8);
  }
};

}  // namespace

struct bs_batch {
  bs_ctx* c = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<BCube> cubes;
  std::vector<void*> owned;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int nwaves = 0;
  struct PLaunch {
    int wave, kind;
    MabsPersistArgs args;
  };
  std::vector<PLaunch> launches;   // persistent contraction launches, by wave
  int grid = 0;                    // blocks of a persistent launch (one per CU)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void* balloc(bs_batch* b, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  b->owned.push_back(p);
  return p;
}

template <typename T>
T* upload(bs_batch* b, const std::vector<T>& v) {
  T* d = (T*)balloc(b, std::max<size_t>(v.size() * sizeof(T), 16));
  if (d && !v.empty() && hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return d;
}

MabsGemmArgs gemm_args(const BCube& q, char* arena, int kchunks) {
  MabsGemmArgs g{};
  g.F = (const float*)(arena + q.off_F);
  g.Fh = (const uint16_t*)(arena + q.off_Fh);
  g.Fl = (const uint16_t*)(arena + q.off_Fl);
  g.tri = q.d_tri;
  g.nu1 = q.d_nu1;
  g.nc = q.nc; g.n_nu1 = q.n_nu1; g.P = q.n * q.n; g.ntri = q.ntri;
  g.kchunks = kchunks;
  g.kchunk = g.P / kchunks;
  g.bin_stride = (long long)q.nc * g.P;
  g.S = (double*)(arena + q.off_S);
  g.tile_m1 = q.kind ? q.m1 : 0;
  return g;
}

int tiles_of(int kind, const MabsGemmArgs& g) { return kind ? mabs_split3_tiles(g) : mabs_split_blocks(g); }

// Per-XCD queue prefixes [8][ngroups + 1] of the persistent launch over `gs` (in that order).
std::vector<int> queue_offsets(int kind, const std::vector<MabsGemmArgs>& gs) {
  const int ng = (int)gs.size();
  std::vector<int> q(8 * (ng + 1), 0);
  for (int g = 0; g < ng; ++g) {
    const int nb = tiles_of(kind, gs[g]), per = nb / 8, rem = nb - 8 * per;
    for (int x = 0; x < 8; ++x) q[x * (ng + 1) + g + 1] = q[x * (ng + 1) + g] + per + (x < rem ? 1 : 0);
  }
  return q;
}

int cu_count(int device) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    n = 256;
  }
  return std::max(8, n / 8 * 8);
}

std::string tile_key(int n, int nc, int n_nu1, int nrings) {
  char key[96];
  snprintf(key, sizeof key, "mabs_split_tile:%d:%d:%d:%d", n, nc, n_nu1, nrings);
  return key;
}
int tile_code(int kind, int m1, int kchunks) { return kind | (m1 << 4) | (kchunks << 12); }
void tile_decode(int code, int& kind, int& m1, int& kchunks) {
  kind = code & 15; m1 = (code >> 4) & 255; kchunks = code >> 12;
}
// whether (kind, m1, kchunks) can run a GEMM of this class
bool tile_ok(int kind, int m1, int kchunks, int n, int nc, int n_nu1) {
  const int P = n * n;
  if (kchunks < 1 || kchunks > 8 || (kchunks & (kchunks - 1)) || P % (32 * kchunks) || P / kchunks < 1024) return false;
  if (kind == 0) return m1 == 0;
  return kind == 1 && n_nu1 >= 4 && (m1 == 4 || m1 == 8 || m1 == 16 || m1 == 32) && (m1 == 4 || m1 <= n_nu1) &&
         buffer_fits((long long)nc * P * 4);
}

// Generator, ring fields and split of one cube into the arena slots (launches only).
void enqueue_front(const BCube& q, char* arena, hipStream_t s) {
  GenArgs ga = q.ga;
  ga.W = (Cx<float>*)(arena + q.off_vis);
  ga.g = (float*)(arena + q.off_g);
  launch_gen_set_state(const_cast<unsigned long long*>(ga.state), q.seed, q.real, s);
  launch_gen_cube(ga, s);
  MabsFieldArgs fa = q.fa;
  fa.vis = arena + q.off_vis;
  fa.out = arena + q.off_F;
  ring_fields_launch(fa, false, q.nbu, q.nc, q.flds, s);
  launch_split_bf16((const float*)(arena + q.off_F), (uint16_t*)(arena + q.off_Fh), (uint16_t*)(arena + q.off_Fl),
                    (long long)q.bytes_fields(), s);
}

// Device-side tables of a one-GEMM persistent launch (autotuner timing runs).
struct TuneLaunch {
  MabsGemmArgs* dg = nullptr;
  int* dq = nullptr;
  int* dcnt = nullptr;
  bool alloc() {
    if (hipMalloc(&dg, sizeof(MabsGemmArgs)) != hipSuccess || hipMalloc(&dq, 16 * sizeof(int)) != hipSuccess ||
        hipMalloc(&dcnt, 8 * sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return true;
  }
  void release() {
    if (dg) (void)hipFree(dg);
    if (dq) (void)hipFree(dq);
    if (dcnt) (void)hipFree(dcnt);
  }
  // mean time of `reps` launches after one warm-up
  float time(int kind, const MabsGemmArgs& g, int grid, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const std::vector<MabsGemmArgs> gs{g};
    const std::vector<int> q = queue_offsets(kind, gs);
    (void)hipMemcpyAsync(dg, &g, sizeof g, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dq, q.data(), q.size() * sizeof(int), hipMemcpyHostToDevice, s);
    MabsPersistArgs pa{dg, dq, 1, dcnt};
    float ms = 0.f, tot = 0.f;
    for (int rep = 0; rep <= reps; ++rep) {
      (void)hipEventRecord(e0, s);
      launch_mabs_gemm_persist(kind, pa, grid, s);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep) tot += ms;
    }
    return tot / reps;
  }
};

// Tile shape and pixel-chunk count of one cube shape class (n, nc, n_nu1, nrings): cached in the
// context, else timed on this cube's own fields.  Tile shapes are compared on a leading subset of
// the triangles with about eight tiles per CU (rate = products / time); the pixel-chunk count is
// then timed on the whole GEMM when it has fewer than 4096 tiles unsplit (below that a split can
// help to fill the chip).
int pick_tile(bs_ctx* c, bs_batch* bt, BCube& q, int nrings, hipStream_t s) {
  const std::string key = tile_key(q.n, q.nc, q.n_nu1, nrings);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    tile_decode(it->second, q.kind, q.m1, q.kchunks);
    if (!tile_ok(q.kind, q.m1, q.kchunks, q.n, q.nc, q.n_nu1))
      return ctx_fail(c, BS_EINVAL, "the tile set for this cube shape cannot run it");
    return BS_OK;
  }
  std::vector<std::pair<int, int>> tiles{{0, 0}};
  for (int m1 : {4, 8, 16, 32})
    if (tile_ok(1, m1, 1, q.n, q.nc, q.n_nu1)) tiles.push_back({1, m1});
  std::vector<int> ks;
  for (int k = 1; k <= 8; k *= 2)
    if (tile_ok(0, 0, k, q.n, q.nc, q.n_nu1)) ks.push_back(k);
  if (ks.empty()) return ctx_fail(c, BS_EINVAL, "batch cube too small for the split-BF16 contraction");
  // temporary slots for one cube at the largest pixel-chunk count
  BCube t = q;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
  t.off_vis = take((size_t)q.nc * q.n * q.nh * 8);
  t.off_g = take((size_t)q.nc * q.n * q.n * 4);
  t.off_F = take(q.bytes_fields() * 4);
  t.off_Fh = take(q.bytes_fields() * 2);
  t.off_Fl = take(q.bytes_fields() * 2);
  t.off_S = take((size_t)ks.back() * q.ntri * q.n_nu1 * q.nc * (size_t)q.nc * 8);
  char* tmp = nullptr;
  if (hipMalloc(&tmp, off) != hipSuccess) { (void)hipGetLastError(); return ctx_fail(c, BS_ENOMEM, "autotuner workspace"); }
  TuneLaunch tl;
  if (!tl.alloc()) { tl.release(); (void)hipFree(tmp); return ctx_fail(c, BS_ENOMEM, "autotuner tables"); }
  enqueue_front(t, tmp, s);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // 1. tile shape
  double best_rate = -1.0;
  for (auto [kind, m1] : tiles) {
    t.kind = kind; t.m1 = m1;
    MabsGemmArgs g = gemm_args(t, tmp, 1);
    g.ntri = 1;
    const int per_tri = tiles_of(kind, g);
    g.ntri = std::min(q.ntri, std::max(1, (8 * bt->grid + per_tri - 1) / per_tri));
    const float ms = tl.time(kind, g, bt->grid, 2, s, e0, e1);
    const double rate = (double)g.ntri * g.n_nu1 * (double)g.nc * g.nc * g.P / std::max(ms, 1e-6f);
    if (rate > best_rate) { best_rate = rate; q.kind = kind; q.m1 = m1; }
  }
  // 2. pixel chunks for that tile
  t.kind = q.kind; t.m1 = q.m1;   // m1 = 0 for 128 x 256 tiles
  q.kchunks = 1;
  if (tiles_of(q.kind, gemm_args(t, tmp, 1)) < 4096 && ks.size() > 1) {
    float best = 1e30f;
    for (int k : ks) {
      const float ms = tl.time(q.kind, gemm_args(t, tmp, k), bt->grid, 2, s, e0, e1);
      if (ms < best) { best = ms; q.kchunks = k; }
    }
  }
  hipError_t err = hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(tmp);
  tl.release();
  if (err != hipSuccess) return ctx_fail(c, BS_EHIP, std::string("autotuner: ") + hipGetErrorString(err));
  c->tuned[key] = tile_code(q.kind, q.m1, q.kchunks);
  return BS_OK;
}

void batch_free(bs_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->s) (void)hipStreamSynchronize(b->s);
  for (auto& q : b->cubes)
    if (q.bins) bs_free_bins(q.bins);
  for (void* p : b->owned)
    if (p) (void)hipFree(p);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->s) (void)hipStreamDestroy(b->s);
  (void)hipGetLastError();
  delete b;
}

}  // namespace

extern "C" int bs_batch_create(bs_ctx* c, const bs_batch_cube* cubes, int32_t ncubes, int32_t nrings,
                               const bs_field_desc* field, double budget_gib, bs_batch** out) {
  if (!c || !out) return BS_EINVAL;
  *out = nullptr;
  if (!cubes || ncubes <= 0 || !field) return ctx_fail(c, BS_EINVAL, "bs_batch_create: no cubes or no field description");
  if (nrings < 1 || nrings > 64) return ctx_fail(c, BS_EINVAL, "nrings must be in [1, 64]");
  if (!(budget_gib > 0)) return ctx_fail(c, BS_EINVAL, "memory budget must be positive");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  bs_batch* b = new bs_batch();
  b->c = c;
  auto fail = [&](int rc) { batch_free(b); return rc; };
  if (hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx_fail(c, BS_EHIP, "stream/event creation"));
  }
  b->grid = cu_count(c->device);
  hipStream_t saved = c->stream;
  c->stream = b->s;   // eager set-up work (counts, tuning) runs on the batch stream
  auto restore_fail = [&](int rc) { c->stream = saved; return fail(rc); };
  b->cubes.resize(ncubes);
  for (int i = 0; i < ncubes; ++i) {
    BCube& q = b->cubes[i];
    const bs_batch_cube& d = cubes[i];
    q.n = d.n; q.nc = d.nc; q.nh = d.n / 2 + 1; q.seed = d.seed; q.real = d.realization;
    bs_field_desc fd = *field;
    fd.n = d.n; fd.nc = d.nc;
    if (d.n % 8 || d.n < 16) return restore_fail(ctx_fail(c, BS_EINVAL, "batch cubes need n % 8 == 0 and n >= 16"));
    // bins: log rings in cells up to umax
    const int umax = (d.n - 1) / 3;
    std::vector<double> edges(nrings + 1);
    for (int j = 0; j <= nrings; ++j) edges[j] = std::exp(std::log(umax + 1.0) * j / nrings);
    bs_bins_desc bd{};
    bd.kind = BS_RING_U; bd.n = d.n; bd.nc = d.nc; bd.nbins = nrings; bd.edges_host = edges.data();
    int32_t ncand = 0;
    int rc = bs_make_bins(c, &bd, &q.bins, &ncand);
    if (rc) return restore_fail(rc);
    q.tri.assign(q.bins->P.tri.begin(), q.bins->P.tri.end());
    q.ntri = ncand;
    if (q.ntri == 0) return restore_fail(ctx_fail(c, BS_EINVAL, "a batch cube has no candidate triangle"));
    std::map<int, int> blk;
    for (int x : q.tri) blk.emplace(x, 0);
    for (auto& kv : blk) { kv.second = (int)q.blocks.size(); q.blocks.push_back(kv.first); }
    q.nbu = (int)q.blocks.size();
    std::vector<int> tri_blk(q.tri.size());
    for (size_t k = 0; k < q.tri.size(); ++k) tri_blk[k] = blk[q.tri[k]];
    if (d.nu1_host) {
      if (d.n_nu1 <= 0) return restore_fail(ctx_fail(c, BS_EINVAL, "n_nu1 must be positive"));
      q.nu1.assign(d.nu1_host, d.nu1_host + d.n_nu1);
      for (int x : q.nu1) if (x < 0 || x >= d.nc) return restore_fail(ctx_fail(c, BS_EINVAL, "nu1 out of range"));
    } else {
      for (int x = 0; x < d.nc; ++x) q.nu1.push_back(x);
    }
    q.n_nu1 = (int)q.nu1.size();
    q.d_nu1 = upload(b, q.nu1);
    q.d_tri = upload(b, tri_blk);
    q.d_blocks = upload(b, q.blocks);
    if (!q.d_nu1 || !q.d_tri || !q.d_blocks) return restore_fail(ctx_fail(c, BS_ENOMEM, "batch tables"));
    // generator
    q.ga = GenArgs{};
    rc = gen_prepare(c, &fd, q.ga);   // checks the sizes
    if (rc) return restore_fail(rc);
    q.ga.state = (unsigned long long*)balloc(b, 64);
    q.ga.stat = (double*)balloc(b, 64);
    q.ga.part = (double*)balloc(b, (size_t)std::max(q.nc, gen_row_blocks(q.ga)) * 8);
    if (!q.ga.state || !q.ga.stat || !q.ga.part) return restore_fail(ctx_fail(c, BS_ENOMEM, "generator buffers"));
    launch_gen_amp(q.ga, c->stream);
    // ring-field kernel arguments (data), unit weights
    rc = ring_fields_prepare(c, q.bins, nullptr, false, false, false, q.d_blocks, nullptr, (long long)q.nc * q.n * q.n,
                             q.fa, q.flds);
    if (rc) return restore_fail(rc);
    // channel-independent counts T_perp = n^4 sum_p I1 I2 I3, certified like the MABS counts
    const double bound = ring_count_bound(q.bins->P, q.tri, (double)((q.n * q.n + 255) / 256) + 8.0);
    if (!(bound < 0.5)) return restore_fail(ctx_fail(c, BS_ECOUNT, "batch triangle counts cannot be certified at this size"));
    double* Ic = nullptr;
    double* Ts = nullptr;
    unsigned long long* bad = nullptr;
    if (hipMalloc(&Ic, (size_t)q.nbu * q.n * q.n * 8) != hipSuccess || hipMalloc(&Ts, (size_t)q.ntri * 8) != hipSuccess ||
        hipMalloc(&bad, 8) != hipSuccess) {
      (void)hipGetLastError(); (void)hipFree(Ic); (void)hipFree(Ts);
      return restore_fail(ctx_fail(c, BS_ENOMEM, "count workspace"));
    }
    MabsFieldArgs ca;
    size_t clds = 0;
    rc = ring_fields_prepare(c, q.bins, nullptr, true, true, true, q.d_blocks, Ic, (long long)q.n * q.n, ca, clds);
    if (!rc) {
      ring_fields_launch(ca, true, q.nbu, 1, clds, c->stream);
      const double P2 = (double)q.n * q.n * (double)q.n * q.n;
      launch_tperp(Ic, q.d_tri, q.ntri, q.n * q.n, P2, Ts, c->stream);
      q.d_tperp = (int64_t*)balloc(b, (size_t)q.ntri * 8);
      (void)hipMemsetAsync(bad, 0, 8, c->stream);
      if (q.d_tperp) launch_round_counts(Ts, q.ntri, q.d_tperp, bad, c->stream);
    }
    double dev = 0.0;
    hipError_t e = hipGetLastError();
    if (!rc && e == hipSuccess) e = hipMemcpyAsync(&dev, bad, 8, hipMemcpyDeviceToHost, c->stream);
    if (!rc && e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(Ic); (void)hipFree(Ts); (void)hipFree(bad);
    if (rc) return restore_fail(rc);
    if (e != hipSuccess || !q.d_tperp) return restore_fail(ctx_fail(c, BS_EHIP, "batch counts"));
    if (!(dev <= bound)) return restore_fail(ctx_fail(c, BS_ECOUNT, "batch triangle count off an integer beyond its error bound"));
    q.tperp.resize(q.ntri);
    HIPCHK(c, hipMemcpy(q.tperp.data(), q.d_tperp, (size_t)q.ntri * 8, hipMemcpyDeviceToHost));
    for (int t = 0; t < q.ntri; ++t)
      if (q.tperp[t] > 0) ++q.valid;
    q.products = (long long)q.valid * q.n_nu1 * q.nc * (long long)q.nc * q.n * q.n;
    const int D = 2 * q.nc - 1;
    q.Bbar = (double*)balloc(b, (size_t)q.ntri * D * D * 8);
    q.Nnu = (int32_t*)balloc(b, (size_t)D * D * 4);
    if (!q.Bbar || !q.Nnu) return restore_fail(ctx_fail(c, BS_ENOMEM, "batch outputs"));
    int rc2 = pick_tile(c, b, q, nrings, c->stream);
    if (rc2) return restore_fail(rc2);
  }
  // ---- waves under the memory budget ----
  const size_t budget = (size_t)(budget_gib * (double)(1ull << 30));
  size_t cur = 0, maxw = 0;
  int w = 0;
  for (auto& q : b->cubes) {
    const size_t f = q.footprint(q.kchunks);
    if (cur > 0 && cur + f > budget) { ++w; cur = 0; }
    q.wave = w;
    size_t off = cur;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    q.off_vis = take((size_t)q.nc * q.n * q.nh * 8);
    q.off_g = take((size_t)q.nc * q.n * q.n * 4);
    q.off_F = take(q.bytes_fields() * 4);
    q.off_Fh = take(q.bytes_fields() * 2);
    q.off_Fl = take(q.bytes_fields() * 2);
    q.off_S = take((size_t)q.kchunks * q.ntri * q.n_nu1 * q.nc * (size_t)q.nc * 8);
    cur = off;
    maxw = std::max(maxw, cur);
  }
  b->nwaves = w + 1;
  b->arena = (char*)balloc(b, maxw);
  b->arena_bytes = maxw;
  if (!b->arena) return restore_fail(ctx_fail(c, BS_ENOMEM, "batch arena (lower the budget)"));
  // ---- persistent launch tables: per wave and tile kind, cubes by tile cost (largest first) ----
  for (int wv = 0; wv < b->nwaves; ++wv) {
    for (int kind = 1; kind >= 0; --kind) {
      std::vector<const BCube*> cs;
      for (auto& q : b->cubes)
        if (q.wave == wv && q.kind == kind) cs.push_back(&q);
      if (cs.empty()) continue;
      // tile cost: MACs of one tile = tile area x pixels of one chunk (the area is the same for all
      // cubes of one kind)
      std::stable_sort(cs.begin(), cs.end(), [](const BCube* x, const BCube* y) {
        return (long long)x->n * x->n / x->kchunks > (long long)y->n * y->n / y->kchunks;
      });
      std::vector<MabsGemmArgs> gs;
      for (const BCube* q : cs) gs.push_back(gemm_args(*q, b->arena, q->kchunks));
      const std::vector<int> qo = queue_offsets(kind, gs);
      bs_batch::PLaunch L{wv, kind, {}};
      L.args.groups = upload(b, gs);
      L.args.qoff = upload(b, qo);
      L.args.ngroups = (int)gs.size();
      L.args.counters = (int*)balloc(b, 8 * sizeof(int));
      if (!L.args.groups || !L.args.qoff || !L.args.counters) return restore_fail(ctx_fail(c, BS_ENOMEM, "queue tables"));
      b->launches.push_back(L);
    }
  }
  HIPCHK(c, hipStreamSynchronize(b->s));
  // ---- capture the whole batch ----
  if (hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return restore_fail(ctx_fail(c, BS_EHIP, "begin capture"));
  for (int wv = 0; wv < b->nwaves; ++wv) {
    for (auto& q : b->cubes)
      if (q.wave == wv) enqueue_front(q, b->arena, b->s);
    for (const auto& L : b->launches)
      if (L.wave == wv) launch_mabs_gemm_persist(L.kind, L.args, b->grid, b->s);
    for (auto& q : b->cubes) {
      if (q.wave != wv) continue;
      MabsSubsetArgs a{};
      a.S = (const double*)(b->arena + q.off_S); a.kchunks = q.kchunks;
      a.Tperp = q.d_tperp; a.nu1 = q.d_nu1; a.n_nu1 = q.n_nu1; a.nc = q.nc; a.ntri = q.ntri;
      a.npix = (double)q.n * q.n; a.norm = 1.0;
      a.B = q.Bbar; a.Nnu = q.Nnu;
      launch_mabs_collapse_subset(a, b->s);
    }
  }
  hipError_t le = hipGetLastError();
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(b->s, &g);
  if (le != hipSuccess || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return restore_fail(ctx_fail(c, BS_EHIP, "batch capture failed"));
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
    return restore_fail(ctx_fail(c, BS_EHIP, "graph instantiate"));
  c->stream = saved;
  *out = b;
  return BS_OK;
}

extern "C" int bs_batch_run(bs_batch* b) {
  if (!b) return BS_EINVAL;
  bs_ctx* c = b->c;
  if (c->timing) (void)hipEventRecord(c->ev[0], c->stream);
  HIPCHK(c, hipEventRecord(b->ev_in, c->stream));
  HIPCHK(c, hipStreamWaitEvent(b->s, b->ev_in, 0));
  HIPCHK(c, hipGraphLaunch(b->exec, b->s));
  HIPCHK(c, hipEventRecord(b->ev_out, b->s));
  HIPCHK(c, hipStreamWaitEvent(c->stream, b->ev_out, 0));
  if (c->timing) {
    (void)hipEventRecord(c->ev[1], c->stream);
    for (int k = 2; k < 6; ++k) (void)hipEventRecord(c->ev[k], c->stream);
    c->have_timing = true;
  }
  return BS_OK;
}

extern "C" int bs_batch_info(const bs_batch* b, int32_t cube, int32_t* n_cand, int32_t* wave, int32_t* kchunks,
                             int64_t* products) {
  if (!b || cube < 0 || cube >= (int)b->cubes.size()) return BS_EINVAL;
  const BCube& q = b->cubes[cube];
  if (n_cand) *n_cand = q.ntri;
  if (wave) *wave = q.wave;
  if (kchunks) *kchunks = q.kchunks;
  if (products) *products = q.products;
  return BS_OK;
}

extern "C" int bs_batch_tile(const bs_batch* b, int32_t cube, int32_t* tile_m, int32_t* tile_n, int32_t* m1,
                             int32_t* kchunks) {
  if (!b || cube < 0 || cube >= (int)b->cubes.size()) return BS_EINVAL;
  const BCube& q = b->cubes[cube];
  if (tile_m) *tile_m = q.kind ? 256 : 128;
  if (tile_n) *tile_n = q.kind ? 192 : 256;
  if (m1) *m1 = q.kind ? q.m1 : 0;
  if (kchunks) *kchunks = q.kchunks;
  return BS_OK;
}

extern "C" int bs_tune_set(bs_ctx* c, int32_t n, int32_t nc, int32_t n_nu1, int32_t nrings, int32_t tile_m, int32_t m1,
                           int32_t kchunks) {
  if (!c) return BS_EINVAL;
  const int kind = tile_m == 256 ? 1 : (tile_m == 128 ? 0 : -1);
  if (kind < 0 || n < 16 || n % 8 || nc < 1 || n_nu1 < 1 || n_nu1 > nc || nrings < 1 || nrings > 64 ||
      !tile_ok(kind, kind ? m1 : 0, kchunks, n, nc, n_nu1))
    return ctx_fail(c, BS_EINVAL, "bs_tune_set: this tile cannot run the cube shape");
  c->tuned[tile_key(n, nc, n_nu1, nrings)] = tile_code(kind, kind ? m1 : 0, kchunks);
  return BS_OK;
}

extern "C" int bs_tune_get(bs_ctx* c, int32_t n, int32_t nc, int32_t n_nu1, int32_t nrings, int32_t* tile_m,
                           int32_t* tile_n, int32_t* m1, int32_t* kchunks) {
  if (!c) return BS_EINVAL;
  int kind = -1, mm = 0, k = 0;
  auto it = c->tuned.find(tile_key(n, nc, n_nu1, nrings));
  if (it != c->tuned.end()) tile_decode(it->second, kind, mm, k);
  if (tile_m) *tile_m = kind < 0 ? 0 : (kind ? 256 : 128);
  if (tile_n) *tile_n = kind < 0 ? 0 : (kind ? 192 : 256);
  if (m1) *m1 = kind == 1 ? mm : 0;
  if (kchunks) *kchunks = kind < 0 ? 0 : k;
  return BS_OK;
}

extern "C" int bs_batch_result(bs_batch* b, int32_t cube, double* Bbar_host, int32_t* Nnu_host, int64_t* tperp_host,
                               int32_t* tri3_host) {
  if (!b || cube < 0 || cube >= (int)b->cubes.size()) return BS_EINVAL;
  bs_ctx* c = b->c;
  const BCube& q = b->cubes[cube];
  const size_t D = 2 * (size_t)q.nc - 1;
  HIPCHK(c, hipStreamSynchronize(b->s));
  if (Bbar_host) HIPCHK(c, hipMemcpy(Bbar_host, q.Bbar, (size_t)q.ntri * D * D * 8, hipMemcpyDeviceToHost));
  if (Nnu_host) HIPCHK(c, hipMemcpy(Nnu_host, q.Nnu, D * D * 4, hipMemcpyDeviceToHost));
  if (tperp_host) std::copy(q.tperp.begin(), q.tperp.end(), tperp_host);
  if (tri3_host) std::copy(q.tri.begin(), q.tri.end(), tri3_host);
  return BS_OK;
}

extern "C" void bs_batch_destroy(bs_batch* b) { batch_free(b); }
