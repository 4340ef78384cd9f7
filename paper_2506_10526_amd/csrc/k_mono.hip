// Monopole of the cylindrical 3D bispectrum (Sec. 2.2 Eq. shape, Sec. 5): every cell (t, a, b) of
// the output of Eq. (dft) is a triangle with sides k_i = sqrt(kperp_i^2 + kpar_i^2), kpar_1,2 the
// line-of-sight wave numbers of a and b and kpar_3 = -(kpar_1 + kpar_2).  Ordered k1 >= k2 >= k3,
// its shape is t = k2 / k1 and mu = -k1.k2 / (k1 k2) = (k1^2 + k2^2 - k3^2) / (2 k1 k2) (closure),
// both clamped to [0.5, 1]; Re B of the cell goes to its (k1, mu, t) bin and the bin's mean is the
// monopole.  The bin decision is made in FP64 with every operation rounded on its own (no fused
// multiply-add), so that it is the same decision as a plain IEEE evaluation of the same formula.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "bs_kernels.h"

namespace {

constexpr int MONO_THREADS = 256;
constexpr int MONO_NB = 4;   // cells of a row per thread and step (loads in flight)

// number of shape edges 0.6 .. 0.9 at or below x in [0.5, 1]: the half-open bin, last bin closed
__device__ __forceinline__ int shape_bin(double x) {
  return (x >= 0.6) + (x >= 0.7) + (x >= 0.8) + (x >= 0.9);
}

// Number of edges k1e[0..nk] at or below k1, minus one: the k1 bin, or -1 / nk outside (edges
// strictly increasing, nk <= 64, so a seven-step binary search finds the same count as a linear scan).
__device__ __forceinline__ int k1_bin(const double* __restrict__ k1e, int nk, double k1) {
  int c = 0;
#pragma unroll
  for (int step = 64; step > 0; step >>= 1)
    if (c + step <= nk + 1 && k1e[c + step - 1] <= k1) c += step;
  return c - 1;
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
  const int j = k1_bin(k1e, nk, k1);
  if (j < 0 || j >= nk) return -1;
  return j * 25 + shape_bin(mu) * 5 + shape_bin(t);
}

// The first test of cell_bin alone: false exactly when cell_bin drops the cell before its square
// roots, so that a cell that fails it needs neither its value nor the rest of the decision.
__device__ __forceinline__ bool cell_may_bin(double lo2, double hi2, double kq0, double kq1, double kq2, double kp1,
                                             double kp2) {
#pragma clang fp contract(off)
  const double kp3 = -(kp1 + kp2);
  const double s0 = kq0 * kq0 + kp1 * kp1;
  const double s1 = kq1 * kq1 + kp2 * kp2;
  const double s2 = kq2 * kq2 + kp3 * kp3;
  const double hi = fmax(s0, fmax(s1, s2));
  return !(hi < lo2 || hi > hi2);
}

// The largest squared side of every cell of row (t, a) is at least kperp_1^2 + kpar_1^2, the same
// rounded value cell_bin forms: above hi2 no cell of the row is binned.
__device__ __forceinline__ bool row_above_edges(double hi2, double kq0, double kp1) {
#pragma clang fp contract(off)
  return kq0 * kq0 + kp1 * kp1 > hi2;
}

// Signed line-of-sight indices j (kpar_2 = j unit; b = j for 2b < nc, else j + nc) of row (t, a) that can
// pass the first test of cell_bin: |kpar_2| <= sqrt(hi2 - kperp_2^2) and |kpar_1 + kpar_2| <= sqrt(hi2 -
// kperp_3^2), widened by two cells for rounding.  A superset: every cell in [jlo, jhi] still takes the
// exact test, and none outside it can pass (both bounds are far looser than a rounding error).
__device__ __forceinline__ void row_span(double hi2, double kq1, double kq2, double kp1, double unit, int nc,
                                         int& jlo, int& jhi) {
  const double r1 = sqrt(fmax(hi2 - kq1 * kq1, 0.0)), r2 = sqrt(fmax(hi2 - kq2 * kq2, 0.0));
  const double lo = fmax(-r1, -r2 - kp1) / unit - 2.0, hi = fmin(r1, r2 - kp1) / unit + 2.0;
  jlo = (int)fmax(ceil(lo), (double)(-(nc / 2)));   // NaN-safe: fmax / fmin return the bound
  jhi = (int)fmin(floor(hi), (double)((nc - 1) / 2));
}

// Rows (t, a) one per wave, in a strided order over the grid; lanes over the row's span of j (only
// there can a cell be binned, and only binned cells are read).  Every binned lane adds its value
// into the block's LDS bins with its own atomic (neighbouring cells share bins, but the LDS
// serialises those adds faster than a wave reduction per bin could combine them); each block
// writes its partial bins.
__global__ __launch_bounds__(MONO_THREADS) void k_mono_bin(MonoArgs a) {
  __shared__ double ssum[MONO_MAX_K1 * 25];
  __shared__ int scnt[MONO_MAX_K1 * 25];
  __shared__ double k1e[MONO_MAX_K1 + 1];
  constexpr int WPB = MONO_THREADS / 64;
  const int nb = a.nk * 25;
  for (int i = threadIdx.x; i < nb; i += MONO_THREADS) {
    ssum[i] = 0.0;
    scnt[i] = 0;
  }
  for (int i = threadIdx.x; i <= a.nk; i += MONO_THREADS) k1e[i] = a.k1e[i];
  __syncthreads();
  const double elo = k1e[0] * (1.0 - 0x1p-20), ehi = k1e[a.nk] * (1.0 + 0x1p-20);
  const double lo2 = elo * elo, hi2 = ehi * ehi;
  const int nc = a.nc, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int row = blockIdx.x * WPB + wave; row < a.nt * nc; row += gridDim.x * WPB) {
    const int t = row / nc, ai = row - t * nc;
    const double kq0 = a.kperp[3 * t], kq1 = a.kperp[3 * t + 1], kq2 = a.kperp[3 * t + 2];
    const double kp1 = a.kpar_unit * (double)(2 * ai < nc ? ai : ai - nc);
    if (row_above_edges(hi2, kq0, kp1)) continue;   // wave-uniform
    int jlo, jhi;
    row_span(hi2, kq1, kq2, kp1, a.kpar_unit, nc, jlo, jhi);
    const double* __restrict__ rowp = a.B + 2 * (long long)row * nc;
    for (int j0 = jlo; j0 <= jhi; j0 += MONO_NB * 64) {   // the same trip count for every lane
      // the bins first (they need no memory), then the values of the binned cells only (MONO_NB loads
      // in flight)
      double v[MONO_NB];
      int bin[MONO_NB];
#pragma unroll
      for (int u = 0; u < MONO_NB; ++u) {
        const int j = j0 + u * 64 + lane;
        bin[u] = j <= jhi ? cell_bin(k1e, a.nk, lo2, hi2, kq0, kq1, kq2, kp1, a.kpar_unit * (double)j) : -1;
      }
#pragma unroll
      for (int u = 0; u < MONO_NB; ++u) {
        const int j = j0 + u * 64 + lane;
        v[u] = bin[u] >= 0 ? rowp[2 * (j < 0 ? j + nc : j)] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < MONO_NB; ++u) {
        if (bin[u] >= 0) {
          atomicAdd(&ssum[bin[u]], v[u]);
          atomicAdd(&scnt[bin[u]], 1);
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

// Stage 1 of the reduction of the block partials: group y adds blocks y PART_KC .. y PART_KC + PART_KC - 1
// in order, entries over the lanes (each block's row of partials is read coalesced): sums of the E
// entries, counts of the C bins.
__global__ __launch_bounds__(64) void k_part_stage(const double* __restrict__ psum, const int* __restrict__ pcnt,
                                                   int nblocks, int E, int C, double* __restrict__ ss,
                                                   long long* __restrict__ sc) {
  const int e = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y;
  const int k0 = y * PART_KC, n = min(nblocks - k0, PART_KC);
  // all of the group's loads in flight first, then the sums in block order (a missing block adds 0)
  if (e < E) {
    double v[PART_KC];
#pragma unroll
    for (int i = 0; i < PART_KC; ++i) v[i] = i < n ? psum[(long long)(k0 + i) * E + e] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < PART_KC; ++i) s += v[i];
    ss[(long long)y * E + e] = s;
  }
  if (e < C) {
    int v[PART_KC];
#pragma unroll
    for (int i = 0; i < PART_KC; ++i) v[i] = i < n ? pcnt[(long long)(k0 + i) * C + e] : 0;
    long long c = 0;
#pragma unroll
    for (int i = 0; i < PART_KC; ++i) c += v[i];
    sc[(long long)y * C + e] = c;
  }
}

// Stage 2: entry e adds the G groups in order and divides by its bin's count (bin e mod C; NaN where
// the bin is empty); the first C entries also store the counts.
__global__ __launch_bounds__(256) void k_part_fin(const double* __restrict__ ss, const long long* __restrict__ sc,
                                                  int G, int E, int C, double* __restrict__ out,
                                                  int64_t* __restrict__ count) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= E) return;
  const int bin = e % C;
  double s = 0.0;
  long long c = 0;
  for (int y0 = 0; y0 < G; y0 += 16) {   // sixteen groups' loads in flight, then their sums in order
    double v[16];
    long long w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      v[i] = y0 + i < G ? ss[(long long)(y0 + i) * E + e] : 0.0;
      w[i] = y0 + i < G ? sc[(long long)(y0 + i) * C + bin] : 0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      s += v[i];
      c += w[i];
    }
  }
  out[e] = c > 0 ? s / (double)c : __builtin_nan("");
  if (e < C) count[e] = c;
}

void launch_part_fin(const double* psum, const int* pcnt, int nblocks, int E, int C, double* ss, long long* sc,
                     double* out, int64_t* count, hipStream_t s) {
  const int G = part_groups(nblocks);
  hipLaunchKernelGGL(k_part_stage, dim3((std::max(E, C) + 63) / 64, G), dim3(64), 0, s, psum, pcnt, nblocks, E, C,
                     ss, sc);
  hipLaunchKernelGGL(k_part_fin, dim3((E + 255) / 256), dim3(256), 0, s, ss, sc, G, E, C, out, count);
}

// ---------------------------------------------------------------------------
// Multipole moments (Eqs. orient, bs_lm).  A cell's triangle is binned exactly as for the monopole;
// its sides sorted with ties kept in index order (k_1 the largest, k_2 the next), the line of sight
// in the triangle's frame is p_z = kpar(k_1) / k1, p_x = (mu_2 + mu p_z) / sqrt(1 - mu^2) (mu_2 =
// kpar(k_2) / k2, mu the clamped shape parameter), |p_x| <= sqrt(1 - p_z^2), p_y = sqrt(1 - p_z^2 -
// p_x^2) >= 0.  Weight of moment (l, m): lm_norm P_l^m(p_z) cos(m phi), written as Q_l^m(p_z)
// Re((p_x + i p_y)^m) with Q_l^m = P_l^m / (1 - x^2)^(m/2) (Condon-Shortley phase), so that no
// division by sin(theta) occurs; sides collinear to within mu > 1 - 1e-9 leave the azimuth undefined
// and add 0 to m > 0.  The bin decision is the monopole's (FP64, no contraction).
constexpr double MULTI_COLLINEAR_TOL = 1e-9;

__device__ int cell_bin_orient(const double* __restrict__ k1e, int nk, double lo2, double hi2, double kq0,
                               double kq1, double kq2, double kp1, double kp2, double& pz, double& px, double& py,
                               bool& azimuth) {
#pragma clang fp contract(off)
  const double kp3 = -(kp1 + kp2);
  const double s0 = kq0 * kq0 + kp1 * kp1;
  const double s1 = kq1 * kq1 + kp2 * kp2;
  const double s2 = kq2 * kq2 + kp3 * kp3;
  const double hi = fmax(s0, fmax(s1, s2)), lo = fmin(s0, fmin(s1, s2));
  if (hi < lo2 || hi > hi2) return -1;
  const double mid = fmax(fmin(s0, s1), fmin(fmax(s0, s1), s2));
  const double k1 = sqrt(hi), k2 = sqrt(mid);
  double mu = ((hi + mid) - lo) / (2.0 * (k1 * k2));
  double t = k2 / k1;
  mu = fmin(fmax(mu, 0.5), 1.0);
  t = fmin(fmax(t, 0.5), 1.0);
  const int j = k1_bin(k1e, nk, k1);
  if (j < 0 || j >= nk) return -1;
  // kpar of the largest and the second side, ties in index order (a stable descending sort)
  int i1 = 0;
  if (s1 > s0) i1 = 1;
  if (s2 > (i1 == 0 ? s0 : s1)) i1 = 2;
  int i2;
  if (i1 == 0) i2 = s2 > s1 ? 2 : 1;
  else if (i1 == 1) i2 = s2 > s0 ? 2 : 0;
  else i2 = s1 > s0 ? 1 : 0;
  const double kpa = i1 == 0 ? kp1 : (i1 == 1 ? kp2 : kp3);
  const double kpb = i2 == 0 ? kp1 : (i2 == 1 ? kp2 : kp3);
  pz = kpa / k1;
  const double mu2 = kpb / k2;
  azimuth = mu <= 1.0 - MULTI_COLLINEAR_TOL;
  px = azimuth ? (mu2 + mu * pz) / sqrt(fmax(1.0 - mu * mu, 0.0)) : 0.0;
  const double sn2 = 1.0 - pz * pz;   // sin^2 of the polar angle
  double py2 = sn2 - px * px;
  if (py2 < 0.0) {                    // |p_x| above sin theta by rounding: p_x = +-sin theta, p_y = 0
    px = copysign(sqrt(fmax(sn2, 0.0)), px);
    py2 = 0.0;
  }
  py = sqrt(py2);
  return j * 25 + shape_bin(mu) * 5 + shape_bin(t);
}

// w[i] for i in lm order: lm_norm[i] Q_l^m(x) Re((px + i py)^m), with m > 0 zero without azimuth and
// every l > lmax zero.  The loops run to the largest lmax with constant bounds, so that the
// recurrence's coefficients, 1 / (l - m) among them, are constants.
__device__ __forceinline__ void multi_weights(const double* __restrict__ norm, int lmax, double x, double px,
                                              double py, bool azimuth, double* w) {
  double cr = 1.0, ci = 0.0;   // Re, Im of (px + i py)^m
  double qmm = 1.0;            // Q_m^m = (-1)^m (2m - 1)!!
#pragma unroll
  for (int m = 0; m <= MULTI_MAX_LMAX; ++m) {
    if (m > 0) {
      const double r = cr * px - ci * py;
      ci = cr * py + ci * px;
      cr = r;
      qmm *= -(2.0 * m - 1.0);
    }
    const double c = (m == 0 || azimuth) ? cr : 0.0;
    double q2 = 0.0, q1 = qmm;   // Q_{l-2}^m, Q_{l-1}^m
#pragma unroll
    for (int l = m; l <= MULTI_MAX_LMAX; ++l) {
      double q;
      if (l == m) q = qmm;
      else if (l == m + 1) q = x * (2.0 * m + 1.0) * qmm;
      else q = ((2.0 * l - 1.0) * x * q1 - (l + m - 1.0) * q2) * (1.0 / (double)(l - m));
      if (l > m) { q2 = q1; q1 = q; }
      const int i = l * (l + 1) / 2 + m;
      w[i] = l <= lmax ? norm[i] * q * c : 0.0;
    }
  }
}

// Queue of a wave: the cells that pass the cheap first test, in the order met (ring of MQ_CAP
// entries: triangle, a << 16 | b, value).  A batch is MQ_R consecutive entries per lane.
constexpr int MULTI_THREADS = 512;   // eight waves share the block's bins
constexpr int MQ_R = 2, MQ_NB = 2, MQ_BATCH = 64 * MQ_R, MQ_CAP = 256;
static_assert(MQ_CAP >= MQ_BATCH + 64 * MQ_NB, "a scan step must fit behind an unprocessed batch");

struct MultiRun {   // a lane's running sums over consecutive cells of one bin
  int cur = -1, cnt = 0;
  double acc[MULTI_MAX_NLM];
};

__device__ __forceinline__ void multi_flush(MultiRun& r, double* ssum, int* scnt, int nb, int nlm) {
#pragma unroll
  for (int i = 0; i < MULTI_MAX_NLM; ++i)   // constant indices keep acc in registers
    if (i < nlm) atomicAdd(&ssum[i * nb + r.cur], r.acc[i]);
  atomicAdd(&scnt[r.cur], r.cnt);
}

// Lane j takes entries start + j MQ_R + r, r < MQ_R, of the n queued: the exact bin decision, the
// orientation and the weights, all lanes busy; sums stay in registers while the bin does not change.
__device__ __forceinline__ void multi_batch(const MultiArgs& a, const double* k1e, double lo2, double hi2,
                                            const int* qt, const unsigned* qab, const double* qv, int start,
                                            int n, MultiRun& run, double* ssum, int* scnt, int nb, int lane) {
  const int nc = a.m.nc;
#pragma unroll 1
  for (int r = 0; r < MQ_R; ++r) {
    const int idx = lane * MQ_R + r;
    if (idx >= n) break;
    const int e = (start + idx) & (MQ_CAP - 1);
    const int t = qt[e];
    const unsigned ab = qab[e];
    const double v = qv[e];
    const int ai = (int)(ab >> 16), b = (int)(ab & 0xffffu);
    double pz = 0.0, px = 0.0, py = 0.0;
    bool az = false;
    const int bin = cell_bin_orient(k1e, a.m.nk, lo2, hi2, a.m.kperp[3 * t], a.m.kperp[3 * t + 1],
                                    a.m.kperp[3 * t + 2], a.m.kpar_unit * (double)(2 * ai < nc ? ai : ai - nc),
                                    a.m.kpar_unit * (double)(2 * b < nc ? b : b - nc), pz, px, py, az);
    if (bin < 0) continue;
    if (bin != run.cur) {
      if (run.cur >= 0) multi_flush(run, ssum, scnt, nb, a.nlm);
      run.cur = bin;
      run.cnt = 0;
#pragma unroll
      for (int i = 0; i < MULTI_MAX_NLM; ++i) run.acc[i] = 0.0;
    }
    double w[MULTI_MAX_NLM];
    multi_weights(a.lm_norm, a.lmax, pz, px, py, az, w);
#pragma unroll
    for (int i = 0; i < MULTI_MAX_NLM; ++i) run.acc[i] += w[i] * v;
    ++run.cnt;
  }
}

// Rows (t, a) one per wave.  A scan over the row's span of j, lanes over j, applies the cheap first test
// and reads the values of the surviving cells only (about one cell in twenty at the usual k1 edges);
// those are queued, and whenever a batch is full it is binned, oriented and weighted with every lane
// busy (a lane per cell would leave most lanes idle through the costly part).
__global__ __launch_bounds__(MULTI_THREADS) void k_multi_bin(MultiArgs a) {
  extern __shared__ double ssum[];            // [nlm][nb] sums, then nb counts
  __shared__ double k1e[MONO_MAX_K1 + 1];
  constexpr int WPB = MULTI_THREADS / 64;
  __shared__ int sqt[WPB][MQ_CAP];
  __shared__ unsigned sqab[WPB][MQ_CAP];
  __shared__ double sqv[WPB][MQ_CAP];
  const int nb = a.m.nk * 25, nlm = a.nlm;
  int* scnt = reinterpret_cast<int*>(ssum + nb * nlm);
  for (int i = threadIdx.x; i < nb * nlm; i += MULTI_THREADS) ssum[i] = 0.0;
  for (int i = threadIdx.x; i < nb; i += MULTI_THREADS) scnt[i] = 0;
  for (int i = threadIdx.x; i <= a.m.nk; i += MULTI_THREADS) k1e[i] = a.m.k1e[i];
  __syncthreads();
  const double elo = k1e[0] * (1.0 - 0x1p-20), ehi = k1e[a.m.nk] * (1.0 + 0x1p-20);
  const double lo2 = elo * elo, hi2 = ehi * ehi;
  const int nc = a.m.nc, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int* qt = sqt[wave];
  unsigned* qab = sqab[wave];
  double* qv = sqv[wave];
  int head = 0, tail = 0;   // wave-uniform queue positions (mod MQ_CAP on use)
  MultiRun run;
  for (int row = blockIdx.x * WPB + wave; row < a.m.nt * nc; row += gridDim.x * WPB) {
    const int t = row / nc, ai = row - t * nc;
    const double kq0 = a.m.kperp[3 * t], kq1 = a.m.kperp[3 * t + 1], kq2 = a.m.kperp[3 * t + 2];
    const double kp1 = a.m.kpar_unit * (double)(2 * ai < nc ? ai : ai - nc);
    if (row_above_edges(hi2, kq0, kp1)) continue;   // wave-uniform
    int jlo, jhi;
    row_span(hi2, kq1, kq2, kp1, a.m.kpar_unit, nc, jlo, jhi);
    const double* __restrict__ rowp = a.m.B + 2 * (long long)row * nc;
    for (int j0 = jlo; j0 <= jhi; j0 += 64 * MQ_NB) {
      bool in[MQ_NB];
      double v[MQ_NB];
#pragma unroll
      for (int u = 0; u < MQ_NB; ++u) {
        const int j = j0 + u * 64 + lane;
        in[u] = j <= jhi && cell_may_bin(lo2, hi2, kq0, kq1, kq2, kp1, a.m.kpar_unit * (double)j);
      }
#pragma unroll
      for (int u = 0; u < MQ_NB; ++u) {
        const int j = j0 + u * 64 + lane;
        v[u] = in[u] ? rowp[2 * (j < 0 ? j + nc : j)] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < MQ_NB; ++u) {
        const unsigned long long m = __ballot(in[u]);
        if (in[u]) {
          const int j = j0 + u * 64 + lane;
          const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
          const int e = (tail + below) & (MQ_CAP - 1);
          qt[e] = t;
          qab[e] = ((unsigned)ai << 16) | (unsigned)(j < 0 ? j + nc : j);
          qv[e] = v[u];
        }
        tail += (int)__popcll(m);
      }
      if (tail - head >= MQ_BATCH) {
        __builtin_amdgcn_wave_barrier();   // a wave's LDS accesses stay in program order
        multi_batch(a, k1e, lo2, hi2, qt, qab, qv, head, MQ_BATCH, run, ssum, scnt, nb, lane);
        __builtin_amdgcn_wave_barrier();
        head += MQ_BATCH;
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (tail > head) multi_batch(a, k1e, lo2, hi2, qt, qab, qv, head, tail - head, run, ssum, scnt, nb, lane);
  if (run.cur >= 0) multi_flush(run, ssum, scnt, nb, nlm);
  __syncthreads();
  for (int i = threadIdx.x; i < nb * nlm; i += MULTI_THREADS) a.m.psum[(long long)blockIdx.x * nb * nlm + i] = ssum[i];
  for (int i = threadIdx.x; i < nb; i += MULTI_THREADS) a.m.pcnt[(long long)blockIdx.x * nb + i] = scnt[i];
}

// ---------------------------------------------------------------------------
// (k_par1, k_par2) grid.  Only the signed indices jlo..jhi lie inside the edges, on both axes: a
// wave per row j1 of the block's slab of that interval (its bin i1 is the row's), lanes over j2 in
// it with their bins from the table, each adding its value into the block's LDS bins.
__global__ __launch_bounds__(256) void k_kpar_bin(KparArgs a) {
  extern __shared__ double ks[];   // [ne * ne]
  const int nb = a.ne * a.ne, nc = a.nc;
  const int t = blockIdx.x / a.slabs, sl = blockIdx.x - t * a.slabs;
  for (int i = threadIdx.x; i < nb; i += 256) ks[i] = 0.0;
  __syncthreads();
  const int L = a.jhi - a.jlo + 1;
  const int r0 = (int)((long long)sl * L / a.slabs), r1 = (int)((long long)(sl + 1) * L / a.slabs);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = r0 + wave; r < r1; r += 4) {
    const int j1 = a.jlo + r, row = j1 < 0 ? j1 + nc : j1;
    const int i1 = a.bin1[row];   // wave-uniform, inside the edges
    const double* __restrict__ rowp = a.B + 2 * ((long long)t * nc + row) * nc;
    for (int q0 = 0; q0 < L; q0 += 4 * 64) {
      int bin[4], col[4];
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * 64 + lane, j2 = a.jlo + q;
        col[u] = j2 < 0 ? j2 + nc : j2;
        bin[u] = q < L ? a.bin1[col[u]] : -1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = bin[u] >= 0 ? rowp[2 * col[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (bin[u] >= 0) atomicAdd(&ks[i1 * a.ne + bin[u]], v[u]);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += 256) a.psum[(long long)blockIdx.x * nb + i] = ks[i];
}

// (triangle, bin) per thread: the slabs in order, divided by the bin's count (NaN where empty)
__global__ __launch_bounds__(256) void k_kpar_fin(KparArgs a, double* __restrict__ mean) {
  const int nb = a.ne * a.ne;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)a.nt * nb) return;
  const int t = (int)(e / nb), k = (int)(e - (long long)t * nb);
  const long long c = a.count[k];
  if (c <= 0) {   // no cell in the bin (no partial was written for it when no index is inside)
    mean[e] = __builtin_nan("");
    return;
  }
  double s = 0.0;
  for (int sl = 0; sl < a.slabs; ++sl) s += a.psum[((long long)t * a.slabs + sl) * nb + k];
  mean[e] = s / (double)c;
}

}  // namespace

void launch_mono_bin(const MonoArgs& a, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_mono_bin, dim3(nblocks), dim3(MONO_THREADS), 0, s, a);
}

void launch_mono_fin(const MonoArgs& a, int nblocks, double* mean, int64_t* count, hipStream_t s) {
  launch_part_fin(a.psum, a.pcnt, nblocks, a.nk * 25, a.nk * 25, a.stage_s, a.stage_c, mean, count, s);
}

void launch_multi_bin(const MultiArgs& a, int nblocks, hipStream_t s) {
  const size_t lds = (size_t)a.m.nk * 25 * (a.nlm * sizeof(double) + sizeof(int));
  (void)hipFuncSetAttribute((const void*)k_multi_bin, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_multi_bin, dim3(nblocks), dim3(MULTI_THREADS), lds, s, a);
}

void launch_multi_fin(const MultiArgs& a, int nblocks, double* moments, int64_t* count, hipStream_t s) {
  launch_part_fin(a.m.psum, a.m.pcnt, nblocks, a.m.nk * 25 * a.nlm, a.m.nk * 25, a.m.stage_s, a.m.stage_c, moments,
                  count, s);
}

void launch_kpar_bin(const KparArgs& a, hipStream_t s) {
  const size_t lds = (size_t)a.ne * a.ne * sizeof(double);
  hipLaunchKernelGGL(k_kpar_bin, dim3(a.nt * a.slabs), dim3(256), lds, s, a);
}

void launch_kpar_fin(const KparArgs& a, double* mean, hipStream_t s) {
  const long long n = (long long)a.nt * a.ne * a.ne;
  hipLaunchKernelGGL(k_kpar_fin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, mean);
}
