// Host-side plan of the 3D estimator, split into a prepare step (host work, allocations, uploads,
// synchronising reads) and an enqueue step (kernel launches only), so that a whole estimate can
// be replayed from a captured graph.
#pragma once
#include <string>
#include <vector>

#include "bs_ctx.h"
#include "bs_kernels.h"

const int kMaxFields = 32, kMaxPairs = 112;

// Host-side description of the shell blocks a 3D call works on.
struct Plan3 {
  std::vector<int> blocks;        // shell id per block
  std::vector<int> hj;            // largest |eta| per block
  std::vector<long long> offT, offG;
  long long totT = 0, totG = 0;
  int H = 0;
  std::vector<Work3> wv, wu, we;
  int NLv = 8, NLu = 8, NLe = 16, NLd = 8;
  // true when, for every v-pass item, the cells of its shell at its |eta| are one range of
  // s = qu^2 + qv^2, held in the item's pad as lo | hi << 16 (the v pass then needs no table reads)
  bool shell_iv = false;
};

// Device-side state of the field pipeline of one plan: workspaces and work lists.  Prepared once
// (allocations, uploads), then enqueued any number of times with launches only.
struct Fields3Dev {
  Shell3Geom g{};
  bool fp64 = false, indicator = false;
  const void* tw_nc = nullptr;
  const void* tw_n = nullptr;
  void* D = nullptr;
  void* Tm = nullptr;
  void* Gm = nullptr;
  int* d_shell = nullptr;
  int* d_hj = nullptr;
  long long* d_offT = nullptr;
  long long* d_offG = nullptr;
  Work3 *d_wv = nullptr, *d_wu = nullptr, *d_we = nullptr;
  void* Gs = nullptr;                // when set, the u pass writes bf16 A-fragments here
  long long* d_offGs = nullptr;
  int* d_ctab = nullptr;             // fragment copy table of the split-BF16 3D kernel
  double gscale = 1.0;               // folded into the fragments: 1 / (M n^2)
};

// Everything one 3D estimate needs besides the cube: resolved on the host once (plans, tables,
// counts, rho3, workspaces), then enqueued with launches only.
struct Est3 {
  std::string tag;
  int precision = BS_FP32;
  bool fp64 = false;
  int ntri = 0, npairs = 0;
  int ct1_tiles = 0;   // leading pair row tiles that serve a triangle with third shell >= 16
  int nhigh = 0;       // pairs that serve such a triangle
  std::vector<int> blocks;
  int *d_pairs = nullptr, *d_tp = nullptr, *d_tc = nullptr;
  long long nvox = 0, nblk = 0, chunk = 0;
  double *partial = nullptr, *reduced = nullptr;
  double rho3 = 1.0;
  const int64_t* d_counts = nullptr;
  double count_dev = 0.0, count_bound = 0.0;
  Plan3 pd;
  Fields3Dev fd;
  int M = 0;
  bool fused = false;
  double sfac = 1.0;
  void* F = nullptr;           // unfused: fields
  Fused3Args fa{};
  size_t lds = 0;
  int fblocks = 0;
  bool dft = false;            // split-BF16: eta synthesis on MFMA (k3_dft) instead of the FFT
  Dft3Args da{};
  size_t dlds = 0;
  int dblocks = 0;
};

void build_plan3(const bsplan::Plan& P, const std::vector<int>& blocks, bool fp64, Plan3& p);
int est3_prepare(bs_ctx* c, const bs_bins* b, const bs_weights* w, int32_t precision, const std::string& tag,
                 Est3& e);
int est3_enqueue(bs_ctx* c, const bs_bins* b, const void* vis, const bs_weights* w, Est3& e, double norm, double* B,
                 int64_t* N_tri, double* N_eff);
