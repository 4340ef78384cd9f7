// Kernel argument blocks and launch wrappers shared between the C ABI layer and the
// HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "fft_lds.h"

// Parts summed per group in the first stage of the fixed-order reduction of per-block partials
// (3D contractions).
constexpr int kReduceGroup = 32;

// ---------------------------------------------------------------- ring fields
struct MabsFieldArgs {
  const void* vis;          // complex64 (T=float) or complex128 (T=double), [nc][n][nh]
  const uint16_t* ng;       // per-cell counts or NULL
  const uint8_t* uvm;       // separable occupancy or NULL
  const float* chw;         // separable channel weights or NULL
  const int8_t* lut;        // ring of s = qu^2 + qv^2, s <= smax
  int smax;
  const int* bins;          // ring id per z block
  int n, nh, nc, vmax, G, CB, RB;
  int count_mode;           // 0: W V, 1: unit indicator [N_g > 0]
  int chan_offset;          // first channel of this launch (grid.y indexes channels from here)
  int ignore_chan;          // count mode, separable: channel-independent indicator
  void* out;                // T fields
  long long plane_stride;   // n*n
  long long bin_stride;     // between ring blocks
  const void* tw_n;         // Cx<T> exp(-2 pi i m / n), m < n
  FftPlan pcol;             // length n / G
  FftPlan prow;             // length n / 2
  double scale;             // 1 / n^2
};

// ------------------------------------------------------------- contractions
// Word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format, no swizzle); the
// kernels copy into LDS with buffer loads over one array or field plane, whose byte offsets must
// stay below 2^32.
constexpr int BUF_DWORD3 = 0x00020000;
inline bool buffer_fits(long long bytes) { return bytes >= 0 && bytes <= 0xFFFFFFFFll; }

struct MabsGemmArgs {
  const float* F;           // FP32 fields [nb][nc][P]
  const uint16_t* Fh;       // bf16 hi parts (bit patterns), same layout
  const uint16_t* Fl;       // bf16 lo parts
  const double* F64;        // FP64 fields
  const int* tri;           // [ntri][3] ring-block indices (b1, b2, b3)
  const int* nu1;           // selected nu1 channels [n_nu1]
  int nc, n_nu1, P, ntri;
  int kchunk, kchunks;      // pixels per chunk, number of chunks
  long long bin_stride;     // nc * P
  double* S;                // [kchunks][ntri][n_nu1*nc][nc]
  int tile_m1;              // 256 x 192 split tiles: nu1 rows per tile (4, 8, 16 or 32); 0 picks by n_nu1
};

struct MabsFinalArgs {
  const double* S;          // data sums [kchunks][ntri][rows][nc]
  int kchunks;
  const double* Sc;         // count sums (general N_g), same layout, or NULL
  int kchunks_c;
  const int64_t* Tperp;     // separable: n^4-scaled count per triangle [ntri]
  const float* chw;         // separable channel weights (NULL = all ones)
  const int* nu1;           // [n_nu1]
  int nc, n_nu1, ntri;
  double npix, norm;
  double* B;                // [ntri][n_nu1][nc][nc]
  int64_t* N;
  unsigned long long* bad;  // max |count - rint(count)| (double bits)
};

struct MabsCollapseArgs {
  const double* S; int kchunks;
  const double* Sc; int kchunks_c;
  const int64_t* Tperp; const float* chw;
  int nc, ntri, circular;
  double npix, norm;
  double* B;  int64_t* N;  int32_t* Nnu;   // [ntri][D][D]
  unsigned long long* bad;
};

struct MabsSubsetArgs {
  const double* S; int kchunks;        // partial sums [kchunks][ntri][n_nu1*nc][nc]
  const int64_t* Tperp;                // [ntri]
  const int* nu1; int n_nu1;
  int nc, ntri;
  double npix, norm;
  double* B;                           // [ntri][2nc-1][2nc-1]
  int32_t* Nnu;                        // [2nc-1][2nc-1]
};
void launch_mabs_collapse_subset(const MabsSubsetArgs& a, hipStream_t s);

void launch_mabs_fields_f32(const MabsFieldArgs& a, int nbins, int nchan, size_t lds, hipStream_t s);
void launch_mabs_fields_f64(const MabsFieldArgs& a, int nbins, int nchan, size_t lds, hipStream_t s);
void launch_split_bf16(const float* F, uint16_t* hi, uint16_t* lo, long long n, hipStream_t s);
void launch_mabs_gemm_split(const MabsGemmArgs& a, hipStream_t s);
void launch_mabs_gemm_f32(const MabsGemmArgs& a, hipStream_t s);
// Grouped split-BF16 contraction: groups_dev[g] owns blocks [offs_dev[g], offs_dev[g+1]) (offsets
// multiples of 8, each group's range >= mabs_split_blocks of it); all groups UNI or all not.
int mabs_split_blocks(const MabsGemmArgs& a);
void launch_mabs_gemm_split_grouped(const MabsGemmArgs* groups_dev, const int* offs_dev, int ngroups, int nblocks,
                                    hipStream_t s);
void launch_mabs_gemm_f64(const MabsGemmArgs& a, hipStream_t s);
// Persistent split-BF16 contraction over ngroups GEMMs of one tile kind (0: 128 x 256 tiles,
// 1: 256 x 192 tiles over nu1 x nu2 row blocks of tile_m1 x 256/tile_m1).  qoff[x][g] (x < 8, g <=
// ngroups) is the prefix over groups of the tiles that queue x holds: per = tiles/8 of group g,
// plus one when x < tiles mod 8.  counters: 8 ints of device memory, zeroed by the launch itself.
struct MabsPersistArgs {
  const MabsGemmArgs* groups;   // device [ngroups], largest tile cost first
  const int* qoff;              // device [8][ngroups + 1]
  int ngroups;
  int* counters;                // device [8]
};
int mabs_split3_tiles(const MabsGemmArgs& a);
void launch_mabs_gemm_persist(int kind, const MabsPersistArgs& p, int nblocks, hipStream_t s);
// Tsum[t] = npix^2 * sum_p I_b1 I_b2 I_b3 over channel-independent FP64 count fields [nb][P].
void launch_tperp(const double* I, const int* tri, int ntri, int P, double npix2, double* Tsum, hipStream_t s);
void launch_round_counts(const double* x, int n, int64_t* out, unsigned long long* maxdev, hipStream_t s);
void launch_mabs_finalize(const MabsFinalArgs& a, hipStream_t s);
void launch_mabs_collapse(const MabsCollapseArgs& a, hipStream_t s);

// ------------------------------------------------------------------ 3D path
// Shell geometry shared by the 3D kernels.  The uv support box is qu in [-vmax, vmax],
// qv in [0, vmax] (stored half plane) -> nub = 2 vmax + 1, nvb = vmax + 1.
struct Shell3Geom {
  int n, nh, nc, vmax, nub, nvb;
  int H;                    // delay planes stored: eta in [-H, H]
  int smax, S1;             // LUT row length S1 = smax + 1
  const int8_t* lut;        // shell of (|eta|, s)
  const uint8_t* uvm;       // uv occupancy [n][nh] or NULL
};

struct Delay3Args {
  Shell3Geom g;
  const void* vis;          // [nc][n][nh] complex (T)
  const float* chw;         // [nc] or NULL
  void* out;                // [2H+1][nub][nvb] complex (T)
  const void* tw;           // exp(-2 pi i m / nc)
  FftPlan plan;             // length nc
  int NL;                   // lines (consecutive qv) per block
  int ip;                   // 2 or 4: in-place FFT with that many butterflies per thread (one LDS buffer); 0: two buffers
};

// One work item = (shell block j, eta, start index) for the v and u passes, and
// (shell block j, start line) for the eta pass.
struct Work3 {
  int j, eta, start, pad;
};

struct Pass3Args {
  Shell3Geom g;
  const int* shell_of_block;   // shell id per block
  const Work3* work;
  const long long* off_in;     // per block element offset of the pass input
  const long long* off_out;    // per block element offset of the pass output
  const int* hj;               // per block: largest |eta| stored (H_j)
  const void* in;              // complex (T)
  void* out;                   // complex (T) or real (T) for the eta pass
  const void* tw;              // exp(-2 pi i m / L) for the pass length L
  FftPlan plan;
  int NL;
  int ip;                      // v / u pass: 2 or 4 = in-place FFT with that many butterflies per thread; 0 = two buffers
  int indicator;               // v pass: 1 = unit indicator of shell and support, 0 = data
  int shell_iv;                // v pass: 1 = shell membership from the item's s range (Work3::pad)
  int M;                       // eta pass: output length along eta
  double scale;                // eta pass: overall 1 / (M n^2); u pass with gs: the same, folded into gs
  long long fstride;           // eta pass: elements per output field (M n^2)
  void* gs;                    // u pass: when set, the spectra are written as bf16 MFMA fragments
                               // (layout of Dft3Args::Gs) instead of `out`
  const long long* off_gs;     // u pass: per block offset into gs (16-byte units)
};

struct Con3Args {
  const void* F;               // fields [nbu][vox] (T)
  long long vox;               // voxels per field
  int nbu;                     // fields (<= 32)
  const int* pairs;            // [npairs][2] field blocks (a, b)
  int npairs;                  // <= 112
  long long chunk;             // voxels per block (multiple of 128)
  double* partial;             // [gridDim.x][112][32]
};

struct Fin3Args {
  const double* partial; int nparts;  // reduce over parts: part p at partial + p * pstride * 112 * 32
  int pstride;                        // slots between parts (0 means 1)
  int nent;                           // entries of each [112][32] part that are summed (0 means all)
  const int* tri_pair; const int* tri_col;  // per triangle
  int ntri;
  const int64_t* T3D;          // counts (NULL when computing counts)
  double* Ssum;                // [ntri] output sums (count pass) or NULL
  double rho3, nvox, norm, sfac;
  double* B; int64_t* N; double* Neff;
};

void launch_delay3_f32(const Delay3Args& a, hipStream_t s, size_t lds);
void launch_delay3_f64(const Delay3Args& a, hipStream_t s, size_t lds);
void launch_vpass3(const Pass3Args& a, int nwork, bool fp64, hipStream_t s, size_t lds);
void launch_upass3(const Pass3Args& a, int nwork, bool fp64, hipStream_t s, size_t lds);
void launch_etapass3(const Pass3Args& a, int nwork, bool fp64, hipStream_t s, size_t lds);
void launch_contract3(const Con3Args& a, int mode, int nblocks, hipStream_t s);  // mode: 0 FP64, 1 FP32, 2 split
struct Fused3Args {
  const void* G;               // line-major delay spectra G_j[line][eta] (complex float)
  const long long* offG;       // per block
  const int* hj;               // per block
  int nbu;                     // fields (<= 32)
  long long nlines;            // n * n
  int M;                       // eta output length (even)
  FftPlan plan;                // length M / 2
  const void* tw;              // exp(-2 pi i m / M)
  double scale;                // 1 / (M n^2)
  const int* pairs; int npairs;
  long long lines_per_block;
  double* partial;             // [gridDim.x][112][32]
  int nlow;                    // leading blocks (H_j <= FUSED_DIRECT_H) summed directly instead of an FFT
};
constexpr int FUSED_DIRECT_H = 6;

// Split-BF16 synthesis along eta on MFMA + contraction.  The delay spectra arrive as bf16 hi/lo
// A-fragments of v_mfma_f32_16x16x32_bf16: for block j, line group g = x_v * (n / 16) + x_u / 16
// and K-step s (modes 16 s .. 16 s + 15), two 1 KB fragments (hi, lo) at
// Gs[offGs[j] + (g * S_j + s) * 128 + hl * 64 + lane]; lane l holds line x_u = 16 (x_u / 16) + l % 16
// and the reals (Re, Im) of modes 16 s + 4 (l / 16) + c, c = 0..3, scaled by a_q / (M n^2)
// (a_0 = 1 with Im dropped, a_q = 2).  W holds, for m = 0..M-1, the words (cos | -sin << 16) of the
// bf16 hi parts and of the lo parts of e^{2 pi i m / M}: the B-fragment word c of lane l for step s
// and t = 16 tt + l % 16 is entry (16 s + 4 (l / 16) + c) t mod M.
constexpr int DFT_MAX_FIELDS = 24, DFT_MAX_STEPS = 8, DFT_LDQ = 68;   // row stride: 16 rows hit distinct banks
// The per-field tables travel by value in the kernel arguments: the kernel reads them as uniform
// scalars, so a table read never waits for the fragment copies in flight.
struct Dft3Args {
  const void* Gs;                           // uint4 fragments
  const int* ctab;                          // [2 kb[nbu]][4] per stage fragment: offset of group 0
                                            // (16-byte units), per-group stride, H_j - 16 (s2 / 2), 0
  long long offGs[DFT_MAX_FIELDS];          // per field (16-byte units)
  int Sj[DFT_MAX_FIELDS];                   // per field: K-steps ceil((H_j + 1) / 16)
  int kb[DFT_MAX_FIELDS + 1];               // prefix of Sj
  int Hj[DFT_MAX_FIELDS];                   // per field: largest delay mode H_j
  int nbu;                                  // fields (<= DFT_MAX_FIELDS)
  int n, M, Smax;              // uv size (multiple of 16), delay grid, max Sj
  const void* W;               // [M] float2 (cos, sin) of 2 pi m / M
  const int* pairs; int npairs;
  int ct1_tiles;               // pair row tiles (the leading ones) contracted against fields 16..31 too
  int ngroups;                 // line groups n * n / 16
  int groups_per_block;
  int flush_vox;               // voxels per wave between FP64 flushes (8192: 256 FP32 MFMA accumulations)
  double* partial;             // [gridDim.x * DFT_WAVES][112][32]: one slot per wave
};
constexpr int DFT_SCHED = 28;  // schedule row: DFT_MAX_FIELDS fragment indices, chunk mask, padding to 16 bytes
constexpr int DFT_WAVES = 8;   // waves per block, two per SIMD (a power of two dividing M / 16)
void launch_dft3(const Dft3Args& a, int nblocks, size_t lds, hipStream_t s);

// Reduces the per-block partials into `reduced` ([112][32]) and finalises every triangle.
void launch_fin3(const Fin3Args& a, double* reduced, hipStream_t s);
void launch_fused3(const Fused3Args& a, int mode, int nblocks, size_t lds, hipStream_t s);

// ---- Eq. (dft): collapsed MABS -> cylindrical 3D BS ----
// Pass n: window of separations [-L/2, L/2)^2 laid out by residue (n mod L, m mod L), unsampled
// (NaN) entries as zero, two real columns packed into one complex FFT along n and split into their
// half spectra a < H.
// Pass m: FFT along m of NL half-spectrum rows, scaled, written with the Hermitian mirror rows.
struct MdftArgs {
  const double* B;   // [nt][S][S] collapsed MABS
  void* X;           // workspace, complex double [nt][H][L]
  void* out;         // complex double [nt][L][L]
  const void* tw;    // complex double exp(-2 pi i m / L), m < L
  FftPlan plan;
  int L, H, h, S, circ, nt;
  int nl, lgnl;      // pass n: column pairs per group (2^lgnl); pass m: rows per group
  int ld;            // LDS line stride of pass n
  int threads;       // block size, at most 512
  int bm;            // butterflies per thread of the in-place FFT (2 or 4)
  int grid;          // most blocks launched; each loops over (triangle, line block) groups
  double scale;
};
void launch_mdft_n(const MdftArgs& a, size_t lds, hipStream_t s);
void launch_mdft_m(const MdftArgs& a, size_t lds, hipStream_t s);

// ---- monopole B(k1, mu, t) of the cylindrical 3D BS (Eq. shape, Sec. 5 binning) ----
constexpr int MONO_MAX_K1 = 64;   // k1 bins
struct MonoArgs {
  const double* B;       // complex double [nt][nc][nc] (real parts read)
  const double* kperp;   // [nt][3]
  const double* k1e;     // [nk + 1] increasing k1 edges
  double* psum;          // per-block partial sums [nblocks][nk * 25]
  int* pcnt;             // per-block partial counts [nblocks][nk * 25]
  double* stage_s;       // group sums [part_groups(nblocks)][nk * 25] (multipoles: [..][n_lm][nk * 25])
  long long* stage_c;    // group counts [part_groups(nblocks)][nk * 25]
  double kpar_unit;
  int nc, nt, nk;
};
// The block partials are added in two fixed-order stages: groups of PART_KC consecutive blocks, then
// the groups; the result does not depend on scheduling.
constexpr int PART_KC = 32;
inline int part_groups(int nblocks) { return (nblocks + PART_KC - 1) / PART_KC; }
void launch_mono_bin(const MonoArgs& a, int nblocks, hipStream_t s);
// mean[b] = sum over blocks of psum / count (NaN where empty), count[b] as int64, fixed block order
void launch_mono_fin(const MonoArgs& a, int nblocks, double* mean, int64_t* count, hipStream_t s);

// Multipole moments (Eqs. orient, bs_lm): the monopole's cells and bins, n_lm = (lmax+1)(lmax+2)/2
// moments per bin in the order l = 0.., m = 0..l; per-block partials [nblocks][n_lm][nk * 25] and
// counts [nblocks][nk * 25]; lm_norm[i] = (2l+1) sqrt((l-m)! / (l+m)!).
constexpr int MULTI_MAX_LMAX = 4, MULTI_MAX_NLM = 15, MULTI_MAX_BINVALS = 6400;
struct MultiArgs {
  MonoArgs m;            // B, kperp, k1e, kpar_unit, nc, nt, nk (psum / pcnt: the partials below)
  int lmax, nlm;
  double lm_norm[MULTI_MAX_NLM];
};
void launch_multi_bin(const MultiArgs& a, int nblocks, hipStream_t s);
// moments[i][b] = sum over blocks (fixed order) / count (NaN where empty); count[b] int64
void launch_multi_fin(const MultiArgs& a, int nblocks, double* moments, int64_t* count, hipStream_t s);

// The cylindrical BS on a (k_par1, k_par2) grid (Sec. 5, Fig. 4): bin1[a] is the bin of index a on
// either axis (-1 outside the edges); a block adds the cells of one triangle's row slab into LDS
// bins and stores them as partials [nt][slabs][ne * ne]; the final kernel adds the slabs in order
// and divides by the counts.
constexpr int KPAR_MAX_BINS = 64;
struct KparArgs {
  const double* B;        // complex double [nt][nc][nc] (real parts read)
  const int* bin1;        // [nc]
  double* psum;           // [nt][slabs][ne * ne]
  const int64_t* count;   // [ne * ne]
  int nc, nt, ne, slabs;
  int jlo, jhi;           // the signed indices a' inside the edges: one interval (bins are monotone)
};
void launch_kpar_bin(const KparArgs& a, hipStream_t s);
void launch_kpar_fin(const KparArgs& a, double* mean, hipStream_t s);

// ---- Eq. (vg): nearest-grid-point gridding of visibilities ----
struct GridArgs {
  const double* uv;            // [nvis][2] baselines in wavelengths
  const float* vis;            // complex64 [nc][nvis], interleaved
  const unsigned char* flags;  // [nc][nvis], nonzero = flagged; may be null
  double* acc;                 // FP64 sums [nco][n][n/2+1][2]
  int* cnt;                    // [nco][n][n/2+1]
  long long nvis;
  int n, nc, chan_avg, nco;
  double du;
  // phase mode (vis and flags unused, chan_avg 1): the value of baseline i in output channel o is
  // exp(i k_o . delta_i), k_o = knode[2o], knode[2o+1] (radians per wavelength), delta_i = U_i - du q_i
  // its offset from its grid point
  const double* knode;
  // the LDS cells' block partials [nco][blocks][GRID_NHOT] (sums re, im and counts), stored whole
  // by every block and added over blocks in block order by launch_grid_hot
  double* hot_v;
  int* hot_c;
};
constexpr int GRID_HOT = 32;                                   // LDS cells: |q_u| < 32, q_v < 32
constexpr int GRID_NHOT = (2 * GRID_HOT - 1) * GRID_HOT;
constexpr int GRID_VPB = 16384;                                // visibilities a block
inline long long grid_blocks(long long nvis) { return (nvis + GRID_VPB - 1) / GRID_VPB; }
void launch_grid_hot(const GridArgs& a, hipStream_t s);
void launch_grid_zero(const GridArgs& a, hipStream_t s);
void launch_grid_scatter(const GridArgs& a, hipStream_t s);
// out: complex64 (fp64 == 0) or complex128 [nco][n][n/2+1]; ng: int32 of the same shape
void launch_grid_fin(const GridArgs& a, bool fp64, void* out, int32_t* ng, hipStream_t s);
