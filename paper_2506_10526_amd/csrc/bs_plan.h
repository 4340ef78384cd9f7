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

// ---- certified rounding of float64 triangle counts (Sec. 3.2, Eq. iFT_I) ----
// A count is x = N^2 sum_x I_a I_b I_c in float64, I_j the inverse FFT (1/N) of the 0/1
// indicator of bin j, which has |S_j| cells on the N-cell grid; the exact count T is an integer.
// First-order error model in the unit roundoff u = 2^-53:
//  * each field has ||e_j||_2 <= eps_field u ||I_j||_2 (normwise FFT error: every radix-2 stage
//    contributes mu + gamma_4 (sqrt 2 + mu), mu <= u the twiddle error, as for the Cooley-Tukey
//    analysis in Higham, Accuracy and Stability of Numerical Algorithms, Thm 24.2; a radix-3 stage
//    is counted as two, and the whole is doubled for safety);
//  * ||I_j||_2 = sqrt(|S_j| / N) (Parseval) and max |I_j| <= |S_j| / N, so the field errors move
//    x by at most eps_field u sqrt(Sa Sb Sc) (sqrt min(Sb,Sc) + sqrt min(Sa,Sc) + sqrt min(Sa,Sb));
//  * products and the summation tree (longest chain of `depth` roundings) move it by at most
//    (depth + 3) u N^2 sum |I_a I_b I_c| <= (depth + 3) u min(sqrt(Sa Sb) Sc, ...), and the final
//    scaling by u T.
// If the bound is below 1/2, rint(x) is T.
// Stage-equivalents of an FFT of length L = 2^a 3^b: a + 2 b.
double fft_stage_units(int L);
// eps_field (units of u) of a field made by FFTs with `stages` stage-equivalents in total plus
// `scalings` rounded normalisations.
double field_error_units(double stages, int scalings);
// Bound on |x - T| for bins of Sa, Sb, Sc cells (see above).
double count_error_bound(double Sa, double Sb, double Sc, double eps_field, double depth);

// Returns "" on success, else an error message.
std::string build_plan(int kind, int n, int nc, int nbins, const double* edges, double umax,
                       double du, double r_mpc, double rprime, double dnu, Plan& out);

}  // namespace bsplan
