// LDS-staged mixed-radix Stockham FFT for gfx950 work-groups.
//
// A work-group transforms `nl` lines of length L that sit contiguously in LDS
// (line i at a + i*L).  Each radix-R pass reads from one LDS buffer and writes
// the self-sorting (Stockham) permutation into the other, so no bit reversal
// is needed.  Twiddles come from a float64-accurate table exp(-2 pi i m / Lt)
// held in global memory (L2-resident); the L-point transform reads entry
// m * (Lt / L).  Radices 2, 3, 4 and 8 cover every length 2^a 3^b used by the
// estimator (uv grids 64..1024, channel axes up to 1536).
//
// Conventions: SIGN = -1 computes X[q] = sum_r x[r] exp(-2 pi i r q / L)
// (forward), SIGN = +1 the unnormalised inverse.
#pragma once
#include <hip/hip_runtime.h>

template <typename T>
struct Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmk(T x, T y) { Cx<T> r; r.x = x; r.y = y; return r; }
template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return cmk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return cmk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) { return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename T>
__device__ __forceinline__ Cx<T> cconj(Cx<T> a) { return cmk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ Cx<T> cscale(Cx<T> a, T s) { return cmk(a.x * s, a.y * s); }
// multiply by SIGN * i
template <int SIGN, typename T>
__device__ __forceinline__ Cx<T> cmul_si(Cx<T> a) { return SIGN > 0 ? cmk(-a.y, a.x) : cmk(a.y, -a.x); }

// Exact q = t / d, r = t % d for 0 <= t < 2^18 and 1 <= d <= 4096 from a float reciprocal
// rd = 1/d (one correction step; checked exhaustively over that range).
__device__ __forceinline__ void fdivmod(int t, int d, float rd, int& q, int& r) {
  q = (int)((float)t * rd);
  r = t - q * d;
  if (r < 0) { --q; r += d; }
  if (r >= d) { ++q; r -= d; }
}

struct FftPlan {
  int L;        // transform length
  int nr;       // number of radix passes
  int rad[14];  // radices, product == L
};

template <int SIGN, typename T>
__device__ __forceinline__ void dft2(Cx<T>* v) {
  Cx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft3(Cx<T>* v) {
  const T c = T(-0.5);
  const T s = T(SIGN) * T(0.86602540378443864676);  // sin(2 pi / 3)
  Cx<T> t1 = cadd(v[1], v[2]);
  Cx<T> t2 = csub(v[1], v[2]);
  Cx<T> m = cadd(v[0], cscale(t1, c));
  Cx<T> is = cmk(-s * t2.y, s * t2.x);  // i * s * t2
  v[0] = cadd(v[0], t1);
  v[1] = cadd(m, is);
  v[2] = csub(m, is);
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft4(Cx<T>* v) {
  Cx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  Cx<T> c = cadd(v[1], v[3]), d = cmul_si<SIGN>(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft8(Cx<T>* v) {
  const T h = T(0.70710678118654752440);
  Cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  Cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<SIGN>(e);
  dft4<SIGN>(o);
  // w^q = exp(SIGN 2 pi i q / 8), q = 0..3
  Cx<T> w1 = cmk(h, T(SIGN) * h);
  Cx<T> w3 = cmk(-h, T(SIGN) * h);
  Cx<T> t0 = o[0];
  Cx<T> t1 = cmul(o[1], w1);
  Cx<T> t2 = cmul_si<SIGN>(o[2]);
  Cx<T> t3 = cmul(o[3], w3);
  v[0] = cadd(e[0], t0); v[4] = csub(e[0], t0);
  v[1] = cadd(e[1], t1); v[5] = csub(e[1], t1);
  v[2] = cadd(e[2], t2); v[6] = csub(e[2], t2);
  v[3] = cadd(e[3], t3); v[7] = csub(e[3], t3);
}

// LDS position of element i of a line in a padded intermediate buffer: one spare slot after every
// 16 elements, which spreads the stride-R writes of the early Stockham passes over the banks
// (radix-8 first pass: 12-way -> 3-way conflicts on 32 four-byte banks).
__device__ __forceinline__ int fft_pad(int i) { return i + (i >> 4); }

// One Stockham pass of radix R over nl lines, butterflies spread over the work-group.
// PIN / POUT: the source / destination lines use the padded layout fft_pad().
template <int SIGN, int R, typename T, bool PIN = false, bool POUT = false>
__device__ __forceinline__ void stockham_pass(const Cx<T>* __restrict__ src, Cx<T>* __restrict__ dst, int L,
                                              int Ns, int nl, int ld, const Cx<T>* __restrict__ tw, int tws) {
  const int nbf = L / R;
  const int total = nl * nbf;
  const int tstep = (L / (Ns * R)) * tws;  // table stride of the unit angle 2 pi / (Ns R)
  const float rnbf = 1.0f / (float)nbf, rns = 1.0f / (float)Ns;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int line, j, jq, k;
    fdivmod(t, nbf, rnbf, line, j);
    fdivmod(j, Ns, rns, jq, k);
    const Cx<T>* in = src + (size_t)line * ld;
    Cx<T>* out = dst + (size_t)line * ld;
    Cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = j + r * nbf;
      v[r] = in[PIN ? fft_pad(i) : i];
    }
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        Cx<T> w = tw[k * r * tstep];
        if (SIGN > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    if (R == 2) dft2<SIGN>(v);
    else if (R == 3) dft3<SIGN>(v);
    else if (R == 4) dft4<SIGN>(v);
    else dft8<SIGN>(v);
    int o = jq * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = o + r * Ns;
      out[POUT ? fft_pad(i) : i] = v[r];
    }
  }
}

template <int SIGN, typename T, bool PIN, bool POUT>
__device__ __forceinline__ void stockham_any(int R, const Cx<T>* src, Cx<T>* dst, int L, int Ns, int nl, int ld,
                                             const Cx<T>* __restrict__ tw, int tws) {
  if (R == 8) stockham_pass<SIGN, 8, T, PIN, POUT>(src, dst, L, Ns, nl, ld, tw, tws);
  else if (R == 4) stockham_pass<SIGN, 4, T, PIN, POUT>(src, dst, L, Ns, nl, ld, tw, tws);
  else if (R == 3) stockham_pass<SIGN, 3, T, PIN, POUT>(src, dst, L, Ns, nl, ld, tw, tws);
  else stockham_pass<SIGN, 2, T, PIN, POUT>(src, dst, L, Ns, nl, ld, tw, tws);
}

// In-place Stockham pass: every thread first gathers, twiddles and transforms all of its
// butterflies (at most BM of them, held in registers), then, after a barrier, writes them back
// over the same buffer.  Needs nl * L / R <= BM * blockDim.x.
template <int BMAX, int R>
constexpr int fft_ip_bm() { return R == 8 ? (BMAX > 1 ? BMAX / 2 : 1) : BMAX; }   // radix 8: half the butterflies
template <int SIGN, int R, int BM, typename T>
__device__ __forceinline__ void stockham_pass_ip(Cx<T>* buf, int L, int Ns, int nl, int ld,
                                                 const Cx<T>* __restrict__ tw, int tws) {
  const int nbf = L / R;
  const int total = nl * nbf;
  const int tstep = (L / (Ns * R)) * tws;
  const float rnbf = 1.0f / (float)nbf, rns = 1.0f / (float)Ns;
  Cx<T> v[BM][R];
  int o[BM];
#pragma unroll
  for (int b = 0; b < BM; ++b) {
    const int t = threadIdx.x + b * blockDim.x;
    o[b] = -1;
    if (t < total) {
      int line, j, jq, k;
      fdivmod(t, nbf, rnbf, line, j);
      fdivmod(j, Ns, rns, jq, k);
      const Cx<T>* in = buf + (size_t)line * ld;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = in[j + r * nbf];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> w = tw[k * r * tstep];
          if (SIGN > 0) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      if (R == 2) dft2<SIGN>(v[b]);
      else if (R == 3) dft3<SIGN>(v[b]);
      else if (R == 4) dft4<SIGN>(v[b]);
      else dft8<SIGN>(v[b]);
      o[b] = line * ld + jq * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BM; ++b) {
    if (o[b] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[o[b] + r * Ns] = v[b][r];
    }
  }
}

// In-place transform of nl lines held in `a` (line i at a + i*ld): one buffer instead of two.
// Every pass must satisfy nl * L / R <= fft_ip_bm<BMAX, R>() * blockDim.x (the host checks
// this with fft_ip_fits).  Ends with a barrier.
template <int SIGN, typename T, int BMAX>
__device__ void lds_fft_ip(Cx<T>* a, const FftPlan& p, int nl, const Cx<T>* __restrict__ tw, int tws, int ld) {
  int Ns = 1;
  for (int s = 0; s < p.nr; ++s) {
    const int R = p.rad[s];
    if (R == 8) stockham_pass_ip<SIGN, 8, fft_ip_bm<BMAX, 8>(), T>(a, p.L, Ns, nl, ld, tw, tws);
    else if (R == 4) stockham_pass_ip<SIGN, 4, fft_ip_bm<BMAX, 4>(), T>(a, p.L, Ns, nl, ld, tw, tws);
    else if (R == 3) stockham_pass_ip<SIGN, 3, fft_ip_bm<BMAX, 3>(), T>(a, p.L, Ns, nl, ld, tw, tws);
    else stockham_pass_ip<SIGN, 2, fft_ip_bm<BMAX, 2>(), T>(a, p.L, Ns, nl, ld, tw, tws);
    __syncthreads();
    Ns *= R;
  }
}

// Transform nl lines held in `a` (line i at a + i*ld, ld >= L; ld = L when omitted).
// `b` is scratch of the same size.  Returns the buffer holding the result (a or b).
// Ends with a barrier.  PAD: intermediate passes use the padded layout fft_pad() (input and
// result keep the plain layout); needs ld >= L + L/16.
template <int SIGN, typename T, bool PAD = false>
__device__ Cx<T>* lds_fft(Cx<T>* a, Cx<T>* b, const FftPlan& p, int nl, const Cx<T>* __restrict__ tw, int tws,
                          int ld = 0) {
  if (ld <= 0) ld = p.L;
  int Ns = 1;
  Cx<T>* src = a;
  Cx<T>* dst = b;
  for (int s = 0; s < p.nr; ++s) {
    const int R = p.rad[s];
    const bool first = s == 0, last = s == p.nr - 1;
    if (!PAD || (first && last)) stockham_any<SIGN, T, false, false>(R, src, dst, p.L, Ns, nl, ld, tw, tws);
    else if (first) stockham_any<SIGN, T, false, true>(R, src, dst, p.L, Ns, nl, ld, tw, tws);
    else if (last) stockham_any<SIGN, T, true, false>(R, src, dst, p.L, Ns, nl, ld, tw, tws);
    else stockham_any<SIGN, T, true, true>(R, src, dst, p.L, Ns, nl, ld, tw, tws);
    __syncthreads();
    Cx<T>* t = src; src = dst; dst = t;
    Ns *= R;
  }
  return src;
}

// Pack a Hermitian half spectrum H[0..M] (M = L/2, values read through `get`) into the
// M-point complex sequence Z whose inverse DFT z gives the real inverse transform
// x[2m] = Re z[m], x[2m+1] = Im z[m] of length L:
//   Z[k] = (H[k] + conj H[M-k]) + i e^{+2 pi i k / L} (H[k] - conj H[M-k]),
// with the imaginary parts of H[0] and H[M] dropped (the self-conjugate terms).
// twL is the table exp(-2 pi i m / (L * twsL)).
template <typename T, typename Get>
__device__ __forceinline__ Cx<T> c2r_pack(int k, int M, Get get, const Cx<T>* __restrict__ twL, int twsL) {
  Cx<T> hk = get(k);
  Cx<T> hm = get(M - k);
  if (k == 0) { hk.y = T(0); hm.y = T(0); }
  Cx<T> e = cadd(hk, cconj(hm));
  Cx<T> d = csub(hk, cconj(hm));
  Cx<T> w = twL[k * twsL];
  w.y = -w.y;  // e^{+2 pi i k / L}
  Cx<T> o = cmul(d, w);
  return cmk(e.x - o.y, e.y + o.x);  // e + i o
}
