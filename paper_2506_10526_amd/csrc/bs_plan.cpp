// Bin planning (Sec. 3.2, Fig. 1: annular uv rings; |k| shells for the 3D estimator).
// Compiled without floating-point contraction so that every |U| and |k| is the
// correctly rounded float64 value of the documented expression.
#include "bs_plan.h"

#include <cmath>
#include <algorithm>
#include <cstring>

namespace bsplan {

static int bin_of(double x, const std::vector<double>& e) {
  // half-open e_j <= x < e_{j+1}
  int nb = (int)e.size() - 1;
  if (!(x >= e[0]) || !(x < e[nb])) return -1;
  int lo = 0, hi = nb;  // invariant e[lo] <= x < e[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (e[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

static uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ULL; }
  return h;
}

double fft_stage_units(int L) {
  double a = 0, b = 0;
  while (L > 1 && L % 2 == 0) { L /= 2; a += 1; }
  while (L > 1 && L % 3 == 0) { L /= 3; b += 1; }
  if (L > 1) a += std::ceil(std::log2((double)L)) * 2;   // not produced by the library's plans
  return a + 2 * b;
}

double field_error_units(double stages, int scalings) {
  const double u = std::ldexp(1.0, -53), mu = 1.0;       // twiddles rounded once from long double
  const double g4 = 4.0 / (1.0 - 4.0 * u);                // gamma_4 / u
  const double eta = mu + g4 * (std::sqrt(2.0) + mu * u); // per radix-2 stage, units of u
  return 2.0 * eta * stages + scalings;
}

double count_error_bound(double Sa, double Sb, double Sc, double eps_field, double depth) {
  const double u = std::ldexp(1.0, -53);
  const double r = std::sqrt(Sa * Sb * Sc);
  const double field = eps_field * r * (std::sqrt(std::min(Sb, Sc)) + std::sqrt(std::min(Sa, Sc)) + std::sqrt(std::min(Sa, Sb)));
  const double m = std::min(std::min(std::sqrt(Sa * Sb) * Sc, std::sqrt(Sa * Sc) * Sb), std::sqrt(Sb * Sc) * Sa);
  const double t = std::min(std::min(Sa * Sb, Sa * Sc), Sb * Sc);
  // second-order terms are below 1e-3 of the first-order ones for every bound below 1/2
  return 1.001 * u * (field + (depth + 3.0) * m + t);
}

std::string build_plan(int kind, int n, int nc, int nbins, const double* edges, double umax,
                       double du, double r_mpc, double rprime, double dnu, Plan& P) {
  if (kind != 0 && kind != 1) return "kind must be BS_RING_U or BS_SHELL_K";
  if (n < 8 || n > 1024 || (n & 1)) return "n must be even and in [8, 1024]";
  if (nc < 1 || nc > 1536) return "nc must be in [1, 1536]";
  if (nbins < 1 || nbins > 120) return "nbins must be in [1, 120]";
  if (!edges) return "edges_host is NULL";
  for (int j = 0; j <= nbins; ++j)
    if (!std::isfinite(edges[j])) return "edges must be finite";
  for (int j = 0; j < nbins; ++j)
    if (!(edges[j + 1] > edges[j])) return "edges must be strictly increasing";
  if (umax <= 0) umax = (double)((n - 1) / 3);
  if (!std::isfinite(umax)) return "umax must be finite";
  if (kind == 1) {
    if (!(du > 0) || !(r_mpc > 0) || !(rprime > 0) || !(dnu > 0) || !std::isfinite(du) || !std::isfinite(r_mpc) ||
        !std::isfinite(rprime) || !std::isfinite(dnu))
      return "SHELL_K needs positive finite du_lambda, r_mpc, rprime_mpc_per_mhz, dnu_mhz";
  }
  P = Plan();
  P.kind = kind; P.n = n; P.nc = nc; P.nh = n / 2 + 1; P.nbins = nbins; P.umax = umax;
  P.edges.assign(edges, edges + nbins + 1);
  // support radius in s = qu^2 + qv^2
  int smax = 0;
  int qlim = n / 2;
  for (int s = 0; s <= 2 * qlim * qlim; ++s) {
    double r = std::sqrt((double)s);
    if (r <= umax) smax = s; else break;
  }
  P.smax = smax;
  P.vmax = (int)std::floor(std::sqrt((double)smax));
  if (P.vmax > n / 2 - 1) P.vmax = n / 2 - 1;  // Nyquist never in support
  P.cperp = 2.0 * M_PI * du / r_mpc;
  P.cpar = 2.0 * M_PI / (rprime * (double)nc * dnu);
  const int S1 = smax + 1;
  P.modes.assign(nbins, 0);
  P.s_hi.assign(nbins, -1);
  if (kind == 0) {
    P.lut.assign(S1, (int8_t)-1);
    for (int s = 1; s <= smax; ++s) {
      double r = std::sqrt((double)s);
      if (r < 1.0 || r > umax) continue;
      P.lut[s] = (int8_t)bin_of(r, P.edges);
    }
  } else {
    const int E1 = nc / 2 + 1;
    P.lut.assign((size_t)E1 * S1, (int8_t)-1);
    P.eta_hi.assign(nbins, -1);
    const double cp2 = P.cperp * P.cperp, cl2 = P.cpar * P.cpar;
    for (int e = 0; e < E1; ++e) {
      if ((nc % 2 == 0) && e == nc / 2) continue;  // Nyquist delay plane excluded
      for (int s = 1; s <= smax; ++s) {
        double r = std::sqrt((double)s);
        if (r < 1.0 || r > umax) continue;
        double kp2 = cp2 * (double)s;
        double kl2 = cl2 * (double)((long long)e * e);
        double k = std::sqrt(kp2 + kl2);
        P.lut[(size_t)e * S1 + s] = (int8_t)bin_of(k, P.edges);
      }
    }
  }
  // Mode counts over the full grid by enumerating the half plane with multiplicities.
  const int nh = P.nh;
  for (int iu = 0; iu < n; ++iu) {
    int qu = signed_index(iu, n);
    if (qu == -n / 2) continue;
    for (int v = 0; v < nh; ++v) {
      if (v == n / 2) continue;
      long long s = (long long)qu * qu + (long long)v * v;
      if (s < 1 || s > smax) continue;
      int mult = (v == 0) ? 1 : 2;
      if (kind == 0) {
        int b = P.lut[s];
        if (b >= 0) { P.modes[b] += mult; if (s > P.s_hi[b]) P.s_hi[b] = (int)s; }
      } else {
        for (int ie = 0; ie < nc; ++ie) {
          int qe = signed_index(ie, nc);
          int ae = qe < 0 ? -qe : qe;
          if ((nc % 2 == 0) && ae == nc / 2) continue;
          int b = P.lut[(size_t)ae * S1 + s];
          if (b >= 0) {
            P.modes[b] += mult;
            if (ae > P.eta_hi[b]) P.eta_hi[b] = ae;
            if (s > P.s_hi[b]) P.s_hi[b] = (int)s;
          }
        }
      }
    }
  }
  if (kind == 1) {
    P.eta_max = 0;
    for (int b = 0; b < nbins; ++b) if (P.eta_hi[b] > P.eta_max) P.eta_max = P.eta_hi[b];
    P.true_closure = (3.0 * umax < (double)n) && (3 * P.eta_max < nc);
  } else {
    P.true_closure = 3.0 * umax < (double)n;
  }
  // Candidate triangles b1 >= b2 >= b3 over non-empty bins.
  for (int b1 = 0; b1 < nbins; ++b1) {
    if (!P.modes[b1]) continue;
    for (int b2 = 0; b2 <= b1; ++b2) {
      if (!P.modes[b2]) continue;
      for (int b3 = 0; b3 <= b2; ++b3) {
        if (!P.modes[b3]) continue;
        if (P.true_closure && !(P.edges[b2 + 1] + P.edges[b3 + 1] > P.edges[b1])) continue;
        P.tri.push_back(b1); P.tri.push_back(b2); P.tri.push_back(b3);
      }
    }
  }
  uint64_t h = 1469598103934665603ULL;
  int hdr[4] = {kind, n, nc, nbins};
  h = fnv(h, hdr, sizeof(hdr));
  h = fnv(h, P.edges.data(), P.edges.size() * sizeof(double));
  double c[3] = {umax, P.cperp, P.cpar};
  h = fnv(h, c, sizeof(c));
  P.hash = h;
  return "";
}

}  // namespace bsplan
