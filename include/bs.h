/*
 * bs.h -- C ABI of libbs, a gfx950 (MI355X) implementation of the FFT-accelerated
 * binned bispectrum estimator on gridded radio-interferometric visibilities of
 * Gill & Bharadwaj 2025 (arXiv:2506.10526), "A Visibility-based 21 cm Bispectrum
 * Estimator for Radio-interferometric Data".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns an int status, BS_OK (0) on success or a
 *   negative BS_E* code.  No C++ exception crosses this boundary.  The message
 *   of the last failure on a context is returned by bs_last_error().
 * Memory: array arguments are DEVICE pointers (hipMalloc'd, or a PyTorch tensor's
 *   data_ptr()) unless the parameter name ends in _host.  They are borrowed for
 *   the duration of the call only.  Outputs go to caller-allocated buffers.  All
 *   device work is enqueued on the context's HIP stream; a call returns after the
 *   work is enqueued and the small host-visible results (if any) are ready, so the
 *   caller must synchronise the stream before reading device outputs.
 *   The library owns its scratch memory (workspace, plans, count caches) until
 *   bs_destroy(); it grows on demand with hipMalloc and is never shrunk.
 * Layout of the visibility cube (Sec. 3.2, Eq. vg): V[nc][n][n/2+1], channel-major,
 *   the Hermitian half plane v >= 0 of an n x n uv grid with signed FFT indices
 *   (q = i for i < n/2, i - n otherwise).  complex64 (interleaved float re,im) for
 *   BS_FP32 and BS_SPLIT_BF16, complex128 for BS_FP64.  Self-conjugate columns
 *   (v = 0, v = n/2) are symmetrised as (X(u) + conj X(-u)) / 2 after weighting.
 * Discrete conventions: unnormalised forward DFTs, inverse transforms carry 1/N
 *   (N = pixels for the MABS, voxels for the 3D estimator).  B is in grid units
 *   times `norm` (pass 1/A with A = pi theta_0^2 Q^3 / 3 for the physical units of
 *   Eq. estimator_t).
 * Threads: a context must not be used by two host threads at the same time.
 */
#ifndef BS_H
#define BS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define BS_OK 0
#define BS_EINVAL (-1)        /* bad argument: shapes, edges, pointers, unsupported combination of inputs */
#define BS_ENOMEM (-2)        /* device allocation failed */
#define BS_EHIP (-3)          /* a HIP runtime call or kernel launch failed */
#define BS_ECOUNT (-4)        /* FP64 triangle counts could not be certified exact (bs_last_count_bound) */
#define BS_EUNSUPPORTED (-5)  /* valid request the library does not implement (e.g. 3D with per-cell N_g) */

typedef struct bs_ctx bs_ctx;
typedef struct bs_bins bs_bins;

/* ---- context ----
 * bs_create: bind a context to HIP device `device` and stream `hip_stream`
 *   (a hipStream_t; NULL = the device's null stream).  *out receives the context.
 * bs_destroy: frees all library-owned device memory of the context.  NULL is a no-op.
 * bs_last_error: message of the last failing call on `ctx` ("" if none). */
int bs_create(int device, void* hip_stream, bs_ctx** out);
void bs_destroy(bs_ctx* ctx);
const char* bs_last_error(const bs_ctx* ctx);
/* Rebind the stream work is enqueued on (same device). */
int bs_set_stream(bs_ctx* ctx, void* hip_stream);

/* ---- binning (Sec. 3.2 and Fig. 1: annular rings of the uv plane; 3D |k| shells) ----
 * BS_RING_U: rings in |U| = sqrt(q_u^2 + q_v^2), in grid cells, for the MABS.
 * BS_SHELL_K: shells in |k| = sqrt(k_perp^2 + k_par^2) in Mpc^-1 for the 3D estimator, with
 *   k_perp = 2 pi du_lambda |U| / r_mpc (Sec. 2.1: l = 2 pi U = r k_perp) and
 *   k_par = 2 pi q_eta / (rprime_mpc_per_mhz * nc * dnu_mhz) (Eq. dft: k_par,a = 2 pi a / (r' B_bw)),
 *   evaluated in float64 as sqrt(cperp*cperp*(qu*qu+qv*qv) + cpar*cpar*qeta*qeta) with
 *   cperp = 2 pi du / r and cpar = 2 pi / (r' nc dnu).
 * Bins are half open, e_j <= x < e_{j+1}.  The uv support is 1 <= |U| <= umax cells
 * (umax <= 0 selects floor((n-1)/3), which makes closure mod n true closure) and never
 * contains Nyquist rows/columns; the Nyquist delay plane is excluded as well.
 * Candidate triangles are the sorted bin triples b1 >= b2 >= b3 over non-empty bins
 * (ordering k1 >= k2 >= k3 of Sec. 2.2, Eq. shape); when closure is true closure, triples
 * with e_{b1} >= e_{b2+1} + e_{b3+1} cannot close and are dropped.  A candidate is valid
 * when its triangle count is non-zero. */
typedef enum { BS_RING_U = 0, BS_SHELL_K = 1 } bs_bin_kind;

typedef struct {
  int32_t kind;             /* bs_bin_kind */
  int32_t n;                /* uv grid is n x n (n even, 8 <= n <= 1024) */
  int32_t nc;               /* channels (2^a 3^b, 2 <= nc <= 1536) */
  int32_t nbins;            /* number of bins, 1 <= nbins <= 120 */
  const double* edges_host; /* nbins+1 strictly increasing finite edges: cells (RING_U) or Mpc^-1 (SHELL_K) */
  double umax;              /* uv support radius in cells; <= 0 for the default floor((n-1)/3) */
  double du_lambda;         /* SHELL_K only: uv cell size in wavelengths (dU_g of Sec. 3.2) */
  double r_mpc;             /* SHELL_K only: comoving distance r */
  double rprime_mpc_per_mhz;/* SHELL_K only: r' = dr/dnu */
  double dnu_mhz;           /* SHELL_K only: channel width */
} bs_bins_desc;

/* Build the bin plan.  *out receives a plan owned by the caller (free with bs_free_bins);
 * *n_candidates receives the number of candidate triangles.  Device LUTs live on the
 * context's device.  ctx == NULL gives a host-only plan (triangles, modes, info; no
 * estimates).  Errors: BS_EINVAL for bad descriptors. */
int bs_make_bins(bs_ctx* ctx, const bs_bins_desc* desc, bs_bins** out, int32_t* n_candidates);
/* Copy the candidate list (int32 [n_candidates][3], b1 >= b2 >= b3) and the per-bin mode
 * counts over the full Fourier grid (int64 [nbins]) to host buffers; either may be NULL. */
int bs_bins_triangles(const bs_bins* bins, int32_t* tri3_host, int64_t* modes_per_bin_host);
/* Largest |q_eta| inside any shell (SHELL_K) and whether closure mod the grid is true closure. */
int bs_bins_info(const bs_bins* bins, int32_t* eta_max, int32_t* true_closure);
void bs_free_bins(bs_bins* bins);

/* ---- weights (Sec. 3.2, Eq. vg and the weights below Eq. iFT) ----
 * Exactly one form:
 *  - per-cell counts: ng != NULL, uint16 [nc][n][n/2+1]; data weight W_g = 1/N_g on filled
 *    cells and 0 on empty ones, unit weight [N_g > 0] (Eq. iFT_I).  The v = 0 column must be
 *    Hermitian-consistent (N_g(-u,0) == N_g(u,0)).
 *  - separable: ng == NULL; uv_mask uint8 [n][n/2+1] occupancy (NULL = all ones) times
 *    chan_w float [nc] with values in {0,1} (flagged channels, NULL = all ones).  The library
 *    multiplies V by W_g itself; the uv_mask v = 0 column must be Hermitian-consistent. */
typedef struct {
  const uint16_t* ng;
  const uint8_t* uv_mask;
  const float* chan_w;
} bs_weights;

typedef enum { BS_FP64 = 0, BS_FP32 = 1, BS_SPLIT_BF16 = 2 } bs_precision;

/* ---- filtered fields (Eqs. iFT and iFT_I) ----
 * three_d == 0 (RING_U bins): fields[nbins][nc][n][n] real, D(l_m, nu, theta) = inverse 2D FT
 *   of W_g V_g restricted to ring m, per channel (NumPy normalisation, 1/n^2).
 * three_d == 1 (SHELL_K bins): fields[nbins][nc][n][n] real, the inverse 3D FT over
 *   (delay, u, v) of the delay-transformed weighted cube restricted to shell m (1/(nc n^2)).
 * count_fields (nullable): same shape, float64, from the unit-weight indicator (Eq. iFT_I).
 * `fields` is float32 for BS_FP32 / BS_SPLIT_BF16 and float64 for BS_FP64 (precision argument).
 * Empty bins give all-zero fields. */
int bs_filter_fields(bs_ctx* ctx, const bs_bins* bins, const void* vis, const bs_weights* w,
                     int32_t three_d, int32_t precision, void* fields, double* count_fields);

/* ---- gridding of visibilities (Sec. 3.2, Eq. vg) ----
 * Visibility i has baseline uv[i] = (U, V) in wavelengths (device float64 [n_vis][2], the same in
 * every channel) and values vis[nu][i] (device complex64 [nc][n_vis]); flags (device uint8
 * [nc][n_vis], nonzero = flagged, NULL = none) give F = 0 or 1.  Its grid point is
 * q = rint(U / du_lambda) per axis (round half to even); a point with q_v < 0 stands for
 * (-q_u, -q_v) with the visibility conjugated (V(-U) = V*(U), a real sky), so that the grid is
 * the half plane q_v >= 0 of the library's visibility layout; that layout stores both halves of
 * the line q_v = 0, so a visibility on it also enters at (-q_u, 0) conjugated (as its mirror
 * baseline would; N_g stays symmetric on the line).  Points with |q_u| or |q_v| >= n/2 are dropped.  chan_avg consecutive channels are gridded into one (the channel collapse of
 * Sec. 4): V_g = sum of F V, N_g = sum of F over the visibilities and channels of a cell.
 * Outputs (device): Vg [nc/chan_avg][n][n/2+1] complex64 (out_precision BS_FP32 / BS_SPLIT_BF16)
 * or complex128 (BS_FP64), in the layout bs_estimate_mabs and bs_estimate_3d take; Ng int32 of
 * the same shape, the per-cell counts of bs_weights (W_g = 1/N_g; bs_weights takes them as uint16).  Sums are
 * accumulated in float64 (atomics: the order of additions, hence the last bits of a float64
 * result, may vary between calls); counts are exact.  Scratch: 20 bytes a cell of context
 * workspace.  bs_last_timing reports [0] the call, [1] the scatter kernel, [2] the output pass.
 * Errors: BS_EINVAL (n odd or outside [2, 4096], nc not a multiple of chan_avg, du <= 0,
 * n_vis outside [0, 2^34], NULL pointers), BS_ENOMEM, BS_EHIP. */
int bs_grid_visibilities(bs_ctx* ctx, int32_t n, int32_t nc, double du_lambda, int64_t n_vis, const double* uv,
                         const void* vis, const uint8_t* flags, int32_t chan_avg, int32_t out_precision, void* Vg,
                         int32_t* Ng);

/* ---- primary-beam decorrelation of the gridded estimator (Sec. 3.1 Eq. S3, Sec. 3.2 Eq. vg) ----
 * Eq. S3: the correlation of three baselines whose sum is dU instead of zero is the closed one times
 * exp(-a |dU|^2), a = pi^2 theta_0^2 / 3 (theta_0 = 0.6 theta_F).  Gridding (Eq. vg, as
 * bs_grid_visibilities: nearest point, reversed baselines for q_v < 0, the line q_v = 0 stored whole)
 * makes a closed grid triangle correlate baseline triplets that do not close: with offsets
 * delta = U - U_g from their grid points, dU = delta_1 + delta_2 + delta_3.  With the cell-average
 * weight W_g = 1/N_g the expected estimate of each ring triangle is the true MABS times
 *   D = mean over its closed grid triangles (all cells sampled) of the mean over the baseline
 *       triplets of the three cells of exp(-a |dU|^2);
 * dividing an estimate by D removes this bias (largest for the smallest rings).
 * Computed as D = sum over nodes k of w_k * (mean over closed grid triangles of prod_j phi_gj(k)),
 * phi_g(k) = mean over cell g of exp(i k . delta), using exp(-a |dU|^2) = E[exp(i sqrt(2a) z . dU)]
 * for a 2D standard normal z and the n_nodes-point Gauss rule per axis (Golub-Welsch); each node's
 * triangle average is the FP64 MABS of the phi grid with the N_g weights (bs_estimate_mabs).  The
 * rule is exact to 4e-14 at n_nodes = 12 for the offsets of a cell of dU_g = sqrt(ln 2)/(pi theta_0).
 * rings: BS_RING_U bins (their n, edges and umax are used); uv: device float64 [n_vis][2] baselines in
 * wavelengths, the same in every channel, no flags.  D_host: host float64 [n_candidates], NaN where
 * no closed grid triangle has all three cells sampled.  Synchronises the context's stream.
 * Scratch: about (n_nodes^2 / 2) n (n/2+1) 40 bytes of context workspace.
 * Errors: BS_EINVAL (not ring bins, n_nodes not even in [2, 32], du or theta0 not positive, more than
 * 65535 baselines in one cell, bad pointers), BS_ENOMEM, BS_EHIP, and those of bs_estimate_mabs. */
int bs_decorrelation(bs_ctx* ctx, const bs_bins* rings, int64_t n_vis, const double* uv, double du_lambda,
                     double theta0_rad, int32_t n_nodes, double* D_host);

/* ---- MABS estimator (Sec. 3.2, Eq. estimator_t; ergodic collapse described before Eq. dft) ----
 * For each selected triangle t = (b1,b2,b3) and channels (nu1,nu2,nu3):
 *   S_D = sum_theta D_b1(nu1) D_b2(nu2) D_b3(nu3),  N_tri = n^4 sum_theta I_b1 I_b2 I_b3 (exact int),
 *   B = norm * n^2 * S_D / N_tri, and NaN where N_tri == 0.
 * Selection: tri3_host (int32 [n_tri][3], any order of the three bins; NULL = all candidates)
 *   and nu1_host (int32 [n_nu1]; NULL = all channels).
 * collapse == 0: B, N_tri are [n_tri][n_nu1][nc][nc] indexed [t][i][nu2][nu3] with nu1 = nu1_host[i];
 *   N_nu unused (may be NULL).
 * collapse == 1 (non-circular) / 2 (circular channels): requires all channels as nu1 (nu1_host NULL);
 *   B[t][d1'][d2'] is the mean over valid nu3 of B(nu3+d1, nu3+d2, nu3) with d' = d + nc - 1 and
 *   size 2nc-1 (non-circular) or d' = d mod nc and size nc (circular); N_tri sums the counts of the
 *   averaged triplets; N_nu (int32, same shape) counts them (Sec. 5, Fig. 2).
 * The contraction runs in `precision`: BS_FP64 (vis complex128), BS_FP32 (FP32 MFMA) or
 * BS_SPLIT_BF16 (three-product hi/lo bfloat16 MFMA with FP32 accumulation); partial sums across
 * pixel chunks and the final division are float64 in every mode.  Counts always use float64 fields.
 * Errors: BS_EINVAL (shapes, selection), BS_ECOUNT, BS_ENOMEM, BS_EHIP. */
typedef struct {
  int32_t n_tri;
  const int32_t* tri3_host;
  int32_t n_nu1;
  const int32_t* nu1_host;
  int32_t collapse;
} bs_mabs_sel;

int bs_estimate_mabs(bs_ctx* ctx, const bs_bins* bins, const void* vis, const bs_weights* w,
                     const bs_mabs_sel* sel, int32_t precision, double norm,
                     double* B, int64_t* N_tri, int32_t* N_nu);

/* ---- collapsed MABS -> cylindrical 3D bispectrum (Sec. 3.2, Eq. dft) ----
 * out[t][a][b] = scale * sum_{n,m} exp(-2 pi i (n a + m b) / nc) Bbar_t(n, m) for a, b in [0, nc):
 * a 2D DFT of the ergodically collapsed MABS over the channel separations (dnu1, dnu2) =
 * (n dnu_c, m dnu_c), with n and m over the half-open range [-nc/2, nc/2), i.e. -h .. nc-1-h for
 * h = nc / 2 (one period, each separation once; the printed limits would count +-nc/2 twice).
 * a and b index k_par = 2 pi a / (r' B_bw) (a >= nc/2: the negative frequencies a - nc);
 * scale is the caller's (r^2 r' dnu_c)^2 (1 for grid units).
 * Bbar (device float64): the output of bs_estimate_mabs with collapse == 1, [n_tri][2nc-1][2nc-1]
 *   with separation d at index d + nc - 1 (circular == 0), or with collapse == 2, [n_tri][nc][nc]
 *   with d at d mod nc (circular == 1).  Only separations in the range are read.  NaN (no sampled
 *   triplet, N_nu == 0) contributes zero.
 * out (device): complex128 [n_tri][nc][nc], interleaved (re, im); the caller owns both buffers.
 * Runs on the context's stream as two FP64 FFT passes; scratch: n_tri nc (nc/2 + 1) 16 bytes of
 * context workspace.  bs_last_timing then reports [0] the call, [1] the pass along m (which writes
 * the output), [2] the pass along n (which reads Bbar).
 * Errors: BS_EINVAL (nc not 2^a 3^b in [2, 4096], n_tri outside [0, 65535], NULL pointers with
 * n_tri > 0), BS_ENOMEM, BS_EHIP.  n_tri == 0 returns BS_OK without touching the GPU buffers. */
int bs_mabs_dft(bs_ctx* ctx, int32_t nc, int32_t n_tri, int32_t circular, const double* Bbar, double scale,
                void* out);

/* ---- monopole B(k1, mu, t) of the cylindrical 3D bispectrum (Sec. 2.2 Eq. shape, Sec. 5) ----
 * Every cell (t, a, b) of a cylindrical BS (the output of bs_mabs_dft) is a triangle with sides
 * k_i = sqrt(kperp_i^2 + kpar_i^2): kperp_host[t][0..2] (the three rings' k_perp, > 0),
 * kpar_1 = kpar_unit a', kpar_2 = kpar_unit b' (a' = a for 2a < nc, else a - nc; kpar_unit =
 * 2 pi / (r' B_bw)) and kpar_3 = -(kpar_1 + kpar_2).  Ordered k1 >= k2 >= k3 its shape is
 * t = k2 / k1 and mu = (k1^2 + k2^2 - k3^2) / (2 k1 k2) (Eq. shape with closure), both clamped to
 * [0.5, 1].  Bins: k1 half-open on k1_edges_host[0..n_k1] (increasing; cells outside are dropped),
 * mu and t in 5 linear bins over [0.5, 1] (half-open, the last closed).  Without redshift-space
 * distortion the BS does not depend on orientation, so the monopole of a bin is the mean of Re B
 * over the cells in it.
 * Bcyl (device): complex128 [n_tri][nc][nc].  Outputs (device): mean float64 [n_k1][5][5] (NaN
 * where empty), count int64 [n_k1][5][5] (cells per bin).  The bin of every cell is decided in
 * FP64 with each operation rounded separately, as a plain IEEE evaluation of the formula above.
 * Synchronises the context's stream before returning.  bs_last_timing reports [0] the call,
 * [1] the binning kernel, [2] the reduction.
 * Errors: BS_EINVAL (n_k1 outside [1, 64], edges not increasing, kperp not positive, kpar_unit
 * not positive, n_tri nc >= 2^31, NULL pointers), BS_ENOMEM, BS_EHIP. */
int bs_monopole(bs_ctx* ctx, int32_t nc, int32_t n_tri, const double* kperp_host, double kpar_unit,
                const void* Bcyl, int32_t n_k1, const double* k1_edges_host, double* mean, int64_t* count);

/* ---- multipole moments B_l^m(k1, mu, t) of the cylindrical 3D bispectrum (Sec. 2.2 Eqs. orient, bs_lm) ----
 * The cells and bins of bs_monopole; each cell's triangle, its sides sorted k1 >= k2 >= k3 (ties in the
 * order kperp_1, kperp_2, kperp_3), also fixes the line of sight p in the triangle's frame (k_1 along z,
 * k_2 in the x-z plane, Eq. orient): p_z = kpar(k_1) / k1, p_x = (mu_2 + mu p_z) / sqrt(1 - mu^2) with
 * mu_2 = kpar(k_2) / k2 and mu the clamped shape parameter, |p_x| <= sqrt(1 - p_z^2), p_y = +sqrt(1 -
 * p_z^2 - p_x^2) (the mirror image p_y -> -p_y is the same triangle).  Eq. bs_lm's integral over the
 * orientations is taken as 4 pi times the mean over the bin's cells:
 *   moment (l, m) = (2l + 1) sqrt((l - m)! / (l + m)!) mean over cells of P_l^m(p_z) cos(m phi) Re B,
 * P_l^m with the Condon-Shortley phase, phi the azimuth of (p_x, p_y); m < 0 follows from
 * B_l^-m = (-1)^m B_l^m, and (0, 0) is the monopole.  Cells whose sides are collinear (mu > 1 - 1e-9,
 * azimuth undefined) add 0 to m > 0.  lmax in [0, 4]; moments are ordered l = 0 .. lmax, m = 0 .. l.
 * Outputs (device): moments float64 [(lmax+1)(lmax+2)/2][n_k1][5][5] (NaN where the bin is empty),
 * count int64 [n_k1][5][5].  Needs 25 n_k1 (lmax+1)(lmax+2)/2 <= 6400.  Synchronises the context's
 * stream; bs_last_timing reports [0] the call, [1] the binning kernel, [2] the reduction.
 * Errors: those of bs_monopole, and BS_EINVAL for lmax outside [0, 4] or too many bin values. */
int bs_multipoles(bs_ctx* ctx, int32_t nc, int32_t n_tri, const double* kperp_host, double kpar_unit,
                  const void* Bcyl, int32_t n_k1, const double* k1_edges_host, int32_t lmax, double* moments,
                  int64_t* count);

/* ---- the cylindrical 3D BS on a (k_par1, k_par2) grid (Sec. 5; the binning of Fig. 4) ----
 * mean[t][i][j] = mean of Re Bcyl[t][a][b] over the cells whose k_par1 = kpar_unit a' lies in bin i
 * and k_par2 = kpar_unit b' in bin j (a' = a for 2a < nc, else a - nc; b' likewise); the same
 * n_e + 1 increasing edges bin both axes, half-open [e_i, e_i+1) with the last bin closed at its
 * top edge, and cells outside them are dropped; NaN where a bin is empty.
 * Bcyl: device complex128 [n_tri][nc][nc] (the output of bs_mabs_dft); edges_host: host float64
 * [n_e + 1]; mean: device float64 [n_tri][n_e][n_e]; count: device int64 [n_e][n_e], the cells of
 * each bin (the same for every triangle).  The bin of every index is decided on the host in
 * float64.  Synchronises the context's stream; bs_last_timing reports [0] the call, [1] the
 * binning kernel, [2] the reduction.
 * Errors: BS_EINVAL (nc outside [1, 65536], n_tri * nc >= 2^31, n_e outside [1, 64], edges not
 * finite and increasing, kpar_unit not positive, NULL pointers), BS_ENOMEM, BS_EHIP. */
int bs_kpar_grid(bs_ctx* ctx, int32_t nc, int32_t n_tri, double kpar_unit, const void* Bcyl, int32_t n_e,
                 const double* edges_host, double* mean, int64_t* count);

/* ---- allocation-free monopole ----
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): bs_monopole with the same inputs, outputs, binning and
 * results (up to the order of the float64 additions: fewer blocks may share the cells), except
 *  - kperp [n_tri][3] and k1_edges [n_k1 + 1] are DEVICE float64 arrays (not checked on the host:
 *    kperp must be positive and the edges non-negative and increasing, as for bs_monopole);
 *  - the call only enqueues work on the context's stream: no host staging, no synchronisation,
 *    no bs_last_timing figures;
 *  - the per-block partial bins and their group sums live in a fixed 8 MiB device array of the
 *    library, one per GPU, held until the process ends (at most (8 MiB - 1 KiB) / (25 n_k1 * 13
 *    bytes) blocks, 403 at n_k1 = 64).
 * Calls on one GPU share that array: calls that overlap on one GPU (two streams, two contexts)
 * race.  Every block and group writes all of its slots before they are read, so nothing has to be
 * cleared between calls.  It allocates nothing: no hipMalloc, hipFree or allocating library call.
 * Errors: BS_EINVAL (n_k1 outside [1, 64], nc outside [1, 65536], n_tri * nc >= 2^31, kpar_unit not
 * positive, NULL pointers), BS_EHIP (launch failure, or the scratch address of the device unknown). */
int bs_monopole_noalloc(bs_ctx* ctx, int32_t nc, int32_t n_tri, const double* kperp, double kpar_unit,
                        const void* Bcyl, int32_t n_k1, const double* k1_edges, double* mean, int64_t* count);

/* ---- 3D bispectrum (delay transform along frequency, |k| shells; Sec. 2.2, Eq. dft) ----
 * Vt(eta, U) = sum_nu w(nu) m(U) V(U, nu) exp(-2 pi i eta nu / nc); F_j = inverse 3D FT of Vt on shell j;
 * for each candidate triangle (a,b,c): S_D = sum_x F_a F_b F_c over the nc*n*n voxels,
 * T3D = (nc n^2)^2 sum_x I_a I_b I_c (exact integer, I_j from the unit indicator of shell j),
 * rho3 = (1/nc) sum_nu w(nu)^3, N_eff = T3D rho3 and B = norm * nc * n^2 * S_D / N_eff (NaN if T3D == 0).
 * Outputs (device): B float64 [n_cand], N_tri int64 [n_cand] (= T3D), N_eff float64 [n_cand] (nullable).
 * Requires separable weights (BS_EUNSUPPORTED for per-cell N_g).  Counts depend only on the geometry and
 * are cached per (bins, uv_mask) in the context. */
int bs_estimate_3d(bs_ctx* ctx, const bs_bins* bins, const void* vis, const bs_weights* w,
                   int32_t precision, double norm, double* B, int64_t* N_tri, double* N_eff);

/* ---- seeded synthetic cubes (Sec. 4, Eq. mb1) ----
 * One realization of the validation field on the GPU: white noise from Philox4x64-10 (Salmon et al.
 * 2011) with key (seed, realization) and counter (i/4, 0, 0, 0) for voxel i = (z n + x) n + y, the
 * four outputs turned into 24-bit uniforms ((x >> 40) + 1/2) 2^-24 and two Box-Muller pairs;
 * g = irfftn(rfftn(white) sqrt(A P)), P = |k|^pk_index (P(0) = 0), A = sigma^2 N_vox / sum_k P;
 * delta = g + f_ng (g^2 - mean g^2); V[z] = rfft2(delta[z]) * chan_w[z] (chan_w NULL = ones).
 * Wave vectors: BS_K_CUBIC k = 2 pi (q_z/nc, q_x/n, q_y/n); BS_K_PHYSICAL k_par = 2 pi q_z /
 * (rprime nc dnu), k_perp = 2 pi du_lambda |q| / r_mpc (Mpc^-1).
 * vis: device complex64 [nc][n][n/2+1] (written).  Requires n % 4 == 0, n and nc of the form
 * 2^a 3^b, nc even, n <= 1024, nc <= 1536 (BS_EINVAL otherwise).  Work is FP32 with FP64 sums. */
#define BS_K_CUBIC 0
#define BS_K_PHYSICAL 1
typedef struct {
  int32_t n, nc, kind;
  double sigma, f_ng, pk_index;
  double du_lambda, r_mpc, rprime_mpc_per_mhz, dnu_mhz;
} bs_field_desc;
int bs_generate_cube(bs_ctx* ctx, const bs_field_desc* desc, uint64_t seed, uint64_t realization,
                     const float* chan_w, void* vis);

/* ---- Monte Carlo over seeded realizations of the 3D estimator (Sec. 4: ensemble means and
 * errors from independent realizations) ----
 * bs_mc_create: plan R realizations of desc's field through bs_estimate_3d with `bins` (BS_SHELL_K,
 *   same n and nc), weights `w` (separable; chan_w also zeroes the generated channels), precision
 *   BS_FP32 or BS_SPLIT_BF16 and `norm`.  The object owns its cube, field and accumulator buffers
 *   and its own HIP stream; bins and the weight arrays are borrowed and must outlive it.
 * bs_mc_run: realizations first .. first+count-1 of `seed`, each generated, estimated and added
 *   to FP64 per-triangle accumulators (count, mean, M2; Welford) on the device.  use_graph != 0
 *   captures one realization into a hipGraph on the first call and replays it (the realization
 *   index advances on the device); 0 launches the kernels directly.  Ordered after earlier work on
 *   the context's stream, and later work on that stream waits for it.
 * bs_mc_stats: per candidate triangle (host arrays [n_cand], each nullable): realizations
 *   accumulated (0 where N_tri = 0), mean B and unbiased variance (NaN with fewer than 2).
 * bs_mc_last: B and N_tri of the last realization (host arrays [n_cand], nullable).
 * bs_mc_reset: zero the accumulators.  bs_mc_destroy: free everything (NULL is a no-op). */
typedef struct bs_mc bs_mc;
int bs_mc_create(bs_ctx* ctx, const bs_bins* bins, const bs_field_desc* desc, const bs_weights* w,
                 int32_t precision, double norm, bs_mc** out);
int bs_mc_run(bs_mc* mc, uint64_t seed, uint64_t first_realization, int32_t count, int32_t use_graph);
int bs_mc_stats(bs_mc* mc, int64_t* n_host, double* mean_host, double* var_host);
int bs_mc_last(bs_mc* mc, double* B_host, int64_t* N_host);
int bs_mc_reset(bs_mc* mc);
void bs_mc_destroy(bs_mc* mc);

/* ---- batches of uneven cubes through the MABS (split-BF16 MFMA contraction) ----
 * Each cube i of `cubes` (n x n uv, n % 8 == 0, n >= 16; nc channels; the generator's size rules) is
 * generated from (seed, realization) with the field description `field` (its n and nc ignored),
 * binned in nrings log rings geomspace(1, umax + 1, nrings + 1) cells (umax = floor((n - 1) / 3)),
 * and estimated for every candidate triangle, the nu1 subset nu1_host (NULL = all channels) and all
 * (nu2, nu3), with unit weights and norm 1.  The output per cube is the ergodic collapse over the nu1
 * subset (Sec. 3.2 before Eq. dft, Sec. 5): Bbar[t][d1 + nc - 1][d2 + nc - 1] = mean over selected nu1
 * with nu1 - d1 and nu1 - d1 + d2 in the band of B(nu1, nu1 - d1 + d2, nu1 - d1) (NaN if none, or if
 * the triangle has no closed grid triangle), and N_nu[d1'][d2'] the number averaged.
 * bs_batch_create does every host-side step (bins, channel-independent counts, device tables) and
 * picks the tile shape and pixel-chunk count of each cube shape class (n, nc, n_nu1, nrings) by
 * timing candidates on the device (cached in the context; see bs_tune_set); cubes are packed in order
 * into waves whose workspaces fit budget_gib; every wave's contraction is one persistent launch per
 * tile shape in use (one block per CU pulls tiles of all the wave's cubes from per-XCD work queues,
 * largest tiles first); the whole batch is captured into one hipGraph.
 * bs_batch_run: one graph launch (ordered after earlier work on the context's stream; later work on
 *   that stream waits for it).
 * bs_batch_info: candidate count, wave, pixel chunks and products (valid triangles x n_nu1 x nc^2 x n^2)
 *   of cube i.  bs_batch_result: host copies of Bbar [n_cand][2nc-1][2nc-1], N_nu [2nc-1][2nc-1],
 *   T_perp [n_cand] and the candidate ring triples [n_cand][3] (each nullable; synchronises).
 * The batch owns its device memory (outputs of all cubes plus one arena of the largest wave). */
typedef struct {
  int32_t n, nc;
  uint64_t seed, realization;
  int32_t n_nu1;
  const int32_t* nu1_host;
} bs_batch_cube;
typedef struct bs_batch bs_batch;
int bs_batch_create(bs_ctx* ctx, const bs_batch_cube* cubes, int32_t ncubes, int32_t nrings,
                    const bs_field_desc* field, double budget_gib, bs_batch** out);
int bs_batch_run(bs_batch* batch);
int bs_batch_info(const bs_batch* batch, int32_t cube, int32_t* n_cand, int32_t* wave, int32_t* kchunks,
                  int64_t* products);
int bs_batch_result(bs_batch* batch, int32_t cube, double* Bbar_host, int32_t* N_nu_host, int64_t* T_perp_host,
                    int32_t* tri3_host);
void bs_batch_destroy(bs_batch* batch);
/* Tile choice of the batch contraction (the paper fixes none; Sec. 3.2 only parallelises over ring
 * and channel triples).  Shapes: tile_m x tile_n = 128 x 256 output rows (nu1, nu2) x columns nu3
 * (m1 = 0), or 256 x 192 whose rows are an m1 x (256 / m1) block of (nu1, nu2), m1 in {4, 8, 16, 32}
 * (needs n_nu1 >= 4 and m1 <= n_nu1 unless m1 = 4); kchunks in {1, 2, 4, 8} pixel chunks with n^2 /
 * kchunks a multiple of 32 and at least 1024.  A class is (n, nc, n_nu1, nrings).
 * bs_tune_set: store a choice for a class in the context's cache; bs_batch_create then uses it
 *   instead of timing (BS_EINVAL if the choice cannot run the class).
 * bs_tune_get: the cached choice of a class (all outputs 0 when it has none yet); outputs nullable.
 * bs_batch_tile: the choice used for cube i of a batch; outputs nullable. */
int bs_tune_set(bs_ctx* ctx, int32_t n, int32_t nc, int32_t n_nu1, int32_t nrings, int32_t tile_m, int32_t m1,
                int32_t kchunks);
int bs_tune_get(bs_ctx* ctx, int32_t n, int32_t nc, int32_t n_nu1, int32_t nrings, int32_t* tile_m, int32_t* tile_n,
                int32_t* m1, int32_t* kchunks);
int bs_batch_tile(const bs_batch* batch, int32_t cube, int32_t* tile_m, int32_t* tile_n, int32_t* m1, int32_t* kchunks);

/* ---- learned variance surrogate ----
 * Not part of the paper, which takes error bars from the scatter of independent realizations
 * (Sec. 4, Sec. 5): a 4 -> 256 -> 256 -> 256 -> 1 MLP with SiLU hidden units predicts log Var(B)
 * of a triangle from (log k1, log k2, log k3, rho), k_i the geometric centres of its shells
 * (Mpc^-1) and rho = sum_nu w(nu) / nc the flag summary, relative to the Gaussian-shaped baseline
 * log(N_vox / T3D) + n_s sum_i log k_i (P ~ k^n_s).  Training runs on the GPU in FP32 (hand-written
 * forward, backward and Adam kernels, one training step captured into a hipGraph and replayed);
 * prediction runs in FP32 or BF16 (MFMA).  Monte Carlo (bs_mc_*) makes the labels and evaluates it.
 * State: BS_MLP_NSTATE floats on the device: the 133,121 parameters (W1 [256][4], b1, W2 [256][256],
 *   b2, W3 [256][256], b3, w4 [256], b4, row-major) then mu_x[4], s_x[4], mu_t, s_t (normalisation
 *   x' = (x - mu_x) / s_x, t' = (t - mu_t) / s_t, fitted by bs_mlp_set_data).
 * bs_mlp_read_state / bs_mlp_write_state: copy the state to / from a host array (synchronising);
 *   a written state replaces parameters and normalisation (e.g. a saved, trained surrogate).
 * bs_mlp_create: parameters drawn from Philox4x64-10 with key (seed, 0x4D4C50), uniform in
 *   +-1/sqrt(fan_in); Adam moments zero.  max_batch bounds the training and prediction batch sizes.
 * bs_mlp_set_data: training inputs X (device float [n][4]) and targets t (device float [n]) are
 *   normalised into the object (the caller's arrays are not kept).
 * bs_mlp_loss_grad: loss = mean (y' - t')^2 and its gradient (device float [BS_MLP_NPARAM], nullable)
 *   at the current parameters.
 * bs_mlp_train: `steps` full-batch Adam steps (b1 0.9, b2 0.999, eps 1e-8; learning rate lr, or
 *   lr (1 + cos(pi k / steps)) / 2 at step k of this call when cosine != 0).  loss_host: the loss
 *   evaluated in the last step (before its update).
 * bs_mlp_predict: t = mu_t + s_t y'(x') for X (device float [n][4]) into y (device float [n]);
 *   bf16 != 0 evaluates layers 2-4 with bfloat16 weights and activations (FP32 accumulation).
 * bs_var_features (host only): X_host [n_cand][4] and, when T3D_host is given, base_host [n_cand]
 *   (the baseline above; -inf where T3D = 0) for the candidate triangles of 3D bins. */
#define BS_MLP_NPARAM 133121
#define BS_MLP_NSTATE 133131
typedef struct bs_mlp bs_mlp;
int bs_mlp_create(bs_ctx* ctx, uint64_t seed, int32_t max_batch, bs_mlp** out);
int bs_mlp_read_state(bs_mlp* mlp, float* state_host);
int bs_mlp_write_state(bs_mlp* mlp, const float* state_host);
int bs_mlp_set_data(bs_mlp* mlp, const float* X, const float* t, int32_t n);
int bs_mlp_loss_grad(bs_mlp* mlp, float* grad, double* loss_host);
int bs_mlp_train(bs_mlp* mlp, int32_t steps, double lr, int32_t cosine, double* loss_host);
int bs_mlp_predict(bs_mlp* mlp, const float* X, int32_t n, int32_t bf16, float* y);
void bs_mlp_destroy(bs_mlp* mlp);
int bs_var_features(const bs_bins* bins, const int64_t* T3D_host, double pk_index, double rho, float* X_host,
                    double* base_host);
/* Flag-aware surrogate inputs (the flag summary per triangle instead of the scalar rho).
 * Flags multiply the cube by w(nu) along frequency, which convolves every line of the delay
 * transform with the window's spectrum (Sec. 2.2 delay transform; Sec. 4 flagging): the Gaussian
 * power seen by the estimator is P_w(k_perp, eta) = sum_q |w~(q)|^2 / nc^2 P(k_perp, eta - q), with
 * P(k) = |k|^pk_index (P(0) = 0) on the bins' physical grid.  Power leaks from low |k| into shells of
 * high k_par, which for steep spectra raises the variance of some triangles by orders of magnitude.
 * bs_var_flag_proxy: G_host [n_cand] (host float64) = mean over the closed triangles of each
 *   candidate of P_w(k1) P_w(k2) P_w(k3) (the Gaussian variance of B up to N_vox / T3D and the
 *   N_eff normalisation), NaN where the triangle has no closed triangle.  chan_w_host: host float32
 *   [nc] weights (NULL = all ones).  Computed on the device: a cube whose delay transform is P_w
 *   (its channel form a(nu) xi(nu), a the window's autocorrelation, xi the inverse DFT of P along
 *   eta) goes through bs_estimate_3d in BS_FP64 with unit weights.  Needs 3D shell bins made with a
 *   context.  Synchronises the context's stream; about nc n (n/2+1) 16 bytes of context workspace.
 *   Errors: BS_EINVAL (not shell bins, a weight < 0 or not finite, all channels flagged), BS_ENOMEM,
 *   BS_EHIP and those of bs_estimate_3d.
 * bs_var_features_flag (host only): X_host [n_cand][4] = (log k1, log k2, log k3, log(G / G1) -
 *   2 log rho3), G from the flags and G1 from all ones (bs_var_flag_proxy), rho3 = (1/nc) sum w^3;
 *   base_host [n_cand] (nullable) = log(N_vox / T3D) + log G - 2 log rho3, the Gaussian log variance
 *   with flags up to a constant (-inf where T3D = 0 or G is not positive; X's last column NaN where
 *   G or G1 is not positive).  BS_EINVAL for NULL arrays or rho3 <= 0. */
int bs_var_flag_proxy(bs_ctx* ctx, const bs_bins* bins, double pk_index, const float* chan_w_host, double* G_host);
int bs_var_features_flag(const bs_bins* bins, const int64_t* T3D_host, const double* G_host, const double* G1_host,
                         double rho3, float* X_host, double* base_host);

/* ---- diagnostics ----
 * Time, in milliseconds, of the kernels of the last estimate call on this context, measured with HIP
 * events on the context's stream: out_ms_host[0] = whole call, [1] = the dominant contraction kernel,
 * [2] = fields/FFT kernels, [3] = the delay-axis grid length M the last 3D
 * contraction ran on (0 before any 3D call), [4] = algorithmic split-BF16 MFMA flops per
 * contracted voxel of the last 3D split-BF16 contraction when it ran the MFMA synthesis kernel
 * (12 sum_j (H_j + 1) for the eta synthesis of the Hermitian half spectra, H_j the largest |eta|
 * of field j, plus 6 (P min(F, 16) + P_hi max(F - 16, 0)) for the pair x field contraction, P product
 * rows, F fields and P_hi the rows that serve a triangle whose third field is 16 or later; 0 otherwise),
 * [5] = voxels contracted by that launch (M n^2).  n selects how many values are written (at most 6).
 * Returns BS_EINVAL if timing was not enabled with bs_set_timing(ctx, 1). */
int bs_set_timing(bs_ctx* ctx, int32_t enable);
int bs_last_timing(const bs_ctx* ctx, double* out_ms_host, int32_t n);
/* Certified triangle counts (Sec. 3.2, Eq. iFT_I: N_tri = N^2 sum I1 I2 I3 is an integer).
 * A count is computed in float64 as x = N^2 sum_x I_a I_b I_c from FFT'd bin indicators; before
 * rounding, the library bounds |x - N_tri| a priori from the bins' cell counts |S_j|, the FFT
 * lengths and the summation structure (first order in u = 2^-53: normwise FFT error per radix-2
 * stage mu + gamma_4 (sqrt 2 + mu), radix-3 stages counted twice, the whole doubled; Parseval
 * ||I_j||_2 = sqrt(|S_j| / N) and max |I_j| <= |S_j| / N; the longest chain of roundings in the
 * sum).  The call fails with BS_ECOUNT when that bound is not below 1/2 (rint(x) would not be
 * guaranteed to be N_tri) or when some |x - rint(x)| exceeds it (a computation outside the model).
 * bs_last_count_dev: the largest |x - rint(x)| over the counts of the last estimate (or of the
 * cached counts it used).  bs_last_count_bound: the bound that certified them (largest over the
 * call's triangles). */
int bs_last_count_dev(const bs_ctx* ctx, double* dev_host);
int bs_last_count_bound(const bs_ctx* ctx, double* bound_host);

#ifdef __cplusplus
}
#endif
#endif /* BS_H */
