// Argument block and launchers of the seeded cube generator and the Monte Carlo accumulators.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/bs.h"
#include "fft_lds.h"

struct GenArgs {
  int n, nc, nh;                 // cube n x n x nc, half width nh = n/2 + 1
  double cz, cxy;                // k_z = cz q_z, k_x = cxy q_x, k_y = cxy q_y
  double index;                  // P = |k|^index
  int m2;                        // index == -2 exactly
  double sigma, fng;             // field rms, quadratic coefficient f
  const unsigned long long* state;   // device [seed, realization]
  double* stat;                  // device [sqrt(A), mean g^2]
  double* part;                  // device per-block partial sums (>= max(nc, row blocks))
  const float* chw;              // channel weights [nc] or NULL
  Cx<float>* W;                  // output / work cube [nc][n][nh]
  float* g;                      // real field [nc][n][n]
  const void* tw_n;              // exp(-2 pi i m / n)
  const void* tw_nc;             // exp(-2 pi i m / nc)
  FftPlan pn, pnc;               // lengths n and nc
  int NL;                        // row pairs per block (row passes)
  int NLx, NLz;                  // lines per block of the x and z passes
  int ipx, ipz;                  // their in-place FFT bound (butterflies per thread; 0: two buffers)
};

// sqrt(A) into stat[0] (sum of P over the full grid, reduced in a fixed order).
void launch_gen_amp(const GenArgs& a, hipStream_t s);
// One realization into a.W (reads the seed and realization from a.state).
void launch_gen_cube(const GenArgs& a, hipStream_t s);
int gen_row_blocks(const GenArgs& a);
void launch_gen_set_state(unsigned long long* state, unsigned long long seed, unsigned long long real, hipStream_t s);
// Welford update of per-triangle (count, mean, M2) with one realization's B; advances state[1].
void launch_mc_accumulate(const double* B, int ntri, long long* cnt, double* mean, double* m2,
                          unsigned long long* state, hipStream_t s);
void launch_mc_zero(long long* cnt, double* mean, double* m2, int ntri, hipStream_t s);
// Checks a field description and fills the shape-dependent part of a GenArgs (plans, twiddles,
// wave-vector scales); the device buffers are the caller's.
int gen_prepare(bs_ctx* c, const bs_field_desc* d, GenArgs& a);
