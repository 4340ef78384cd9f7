// Internal context and plan objects behind the opaque handles of bs.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/bs.h"
#include "bs_plan.h"
#include "fft_lds.h"

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  std::vector<unsigned char> mirror;   // bytes last uploaded into p from the host (tables only)
};

struct CountCache {
  std::vector<int32_t> tri;       // triangle list the counts were made for
  int64_t* d_counts = nullptr;    // device int64 per triangle
  std::vector<int64_t> h_counts;  // host copy
  double dev = 0.0;               // max |count - rint(count)| when the counts were made
  double bound = 0.0;             // certified bound on that distance (bsplan::count_error_bound)
};

struct Est3;

struct bs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::map<std::string, DevBuf> ws;      // grow-only workspace slots
  std::map<int, void*> tw32, tw64;        // twiddle tables exp(-2 pi i m / L), by L
  std::map<long long, void*> dftw;       // eta-synthesis twiddle words, by M
  std::map<uint64_t, CountCache> counts;  // geometry-keyed count caches
  bool timing = false;
  hipEvent_t ev[8] = {};
  double last_ms[4] = {0, 0, 0, 0};
  bool have_timing = false;
  double last_count_dev = 0.0;
  double last_count_bound = 0.0;   // error bound that certified the rounding of the last counts
  int last_grid_M = 0;   // delay-axis grid of the last 3D contraction
  double last_flops_vox = 0.0, last_vox = 0.0;   // algorithmic MFMA flops per voxel, voxels (MFMA synthesis path)
  std::map<std::string, int> tuned;       // autotuned launch parameters, by shape key
  uint64_t ws_gen = 0;                    // bumped whenever a workspace is reallocated or re-uploaded
  // last prepared unweighted 3D estimate, reused while its key and ws_gen still match
  std::shared_ptr<Est3> est3;
  std::string est3_key;
  uint64_t est3_gen = 0;
};

struct bs_bins {
  bs_ctx* ctx = nullptr;
  bsplan::Plan P;
  int8_t* d_lut = nullptr;
};

// Device address of the allocation-free entry points' scratch array on `device` (current), looked
// up once per device (bs_noalloc.cpp).
int noalloc_scratch_init(int device);

// ---- helpers implemented in bs_api.cpp ----
// Certified bound on |x - T| of the FP64 ring counts of triangles `tri` ([n][3] bins) whose
// triple sum has a longest chain of `depth` roundings (bsplan::count_error_bound).
double ring_count_bound(const bsplan::Plan& P, const std::vector<int>& tri, double depth);
int ctx_fail(bs_ctx* c, int code, const std::string& msg);
void* ctx_ws(bs_ctx* c, const char* name, size_t bytes);       // grow-only; NULL on failure
const void* ctx_twiddle(bs_ctx* c, int L, bool fp64);          // NULL on failure
FftPlan make_fft_plan(int L);
// true when every pass of `p` over nl lines fits the in-place LDS FFT with `threads` threads and
// at most bmax butterflies per thread (bmax / 2 in radix-8 passes)
bool fft_ip_fits(const FftPlan& p, int nl, int threads, int bmax);
bool fft_len_ok(int L);
struct MabsFieldArgs;
int ring_fields_prepare(bs_ctx* c, const bs_bins* b, const bs_weights* w, bool fp64, bool count_mode,
                        bool ignore_chan, const int* d_bins, void* out, long long bin_stride, MabsFieldArgs& a,
                        size_t& lds);
void ring_fields_launch(MabsFieldArgs a, bool fp64, int nblocks, int nch, size_t lds, hipStream_t s);
