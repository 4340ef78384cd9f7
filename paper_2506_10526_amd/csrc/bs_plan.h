// Host-side bin planning shared by the C ABI layer (pure C++, no HIP).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace bsplan {

// Signed FFT index: i for i < n/2, i - n otherwise.
inline int signed_index(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

struct Plan {
  int kind = 0, n = 0, nc = 0, nh = 0, nbins = 0;
  double umax = 0.0;
  int smax = 0;          // largest q_u^2 + q_v^2 with 1 <= sqrt(.) <= umax
  int vmax = 0;          // largest |q| of any support cell along one axis
  double cperp = 0.0, cpar = 0.0;
  std::vector<double> edges;
  // LUT: RING_U -> lut[s] for s in [0, smax]; SHELL_K -> lut[|qeta| * (smax+1) + s], |qeta| <= nc/2.
  std::vector<int8_t> lut;
  std::vector<int64_t> modes;     // per bin, full Fourier grid
  std::vector<int32_t> tri;       // candidates [n][3]
  bool true_closure = false;
  int eta_max = 0;                // largest |q_eta| in any shell
  std::vector<int> eta_hi;        // per shell: largest |q_eta| with a mode in the shell (-1 if empty)
  std::vector<int> s_hi;          // per bin: largest s with a mode in the bin (-1 if empty)
  uint64_t hash = 0;              // geometry hash (edges, sizes, support, constants)
};

// Returns "" on success, else an error message.
std::string build_plan(int kind, int n, int nc, int nbins, const double* edges, double umax,
                       double du, double r_mpc, double rprime, double dnu, Plan& out);

}  // namespace bsplan
