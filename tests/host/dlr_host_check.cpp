// Host-only driver of the DLR builder (csrc/dlr_host.cpp) for a sanitizer build on the CPU: builds node sets and
// maps for a range of cutoffs and accuracies, and prints per case the rank and how well the maps carry data the
// basis represents exactly (single poles on the DLR frequencies: G(tau) = -k(tau / beta, beta w_l) and
// G(i w_n) = 1 / (i w_n - w_l), fermionic; tanh(beta w_l / 2) / (i nu_n - w_l), bosonic), plus the quasiparticle row.
#include <cmath>
#include <complex>
#include <cstdio>
#include <string>
#include <vector>

#include "qgw_internal.h"

using cd = std::complex<double>;

static double kern(double t, double x) {
  return x >= 0.0 ? std::exp(-t * x) / (1.0 + std::exp(-x)) : std::exp((1.0 - t) * x) / (1.0 + std::exp(x));
}

// max |T a - b| / max |b| for an r x r map T
static double apply_defect(int r, const std::vector<cd>& t, const std::vector<cd>& a, const std::vector<cd>& b) {
  double worst = 0.0, scale = 0.0;
  for (int i = 0; i < r; ++i) {
    cd s = 0.0;
    for (int k = 0; k < r; ++k) s += t[size_t(i) * r + k] * a[k];
    worst = std::fmax(worst, std::abs(s - b[i]));
    scale = std::fmax(scale, std::abs(b[i]));
  }
  return worst / scale;
}

int main() {
  const double cases[][3] = {{10.0, 1e-6, 10.0}, {1250.0, 1e-10, 50.0}, {2500.0, 1e-10, 100.0},
                             {4000.0, 1e-12, 40.0}, {1.0, 1e-8, 1.0}};
  for (const auto& c : cases) {
    const double lambda = c[0], eps = c[1], beta = c[2];
    std::vector<double> x, tau_t;
    std::vector<int64_t> n_f, n_b;
    std::string err;
    const int r = qgw::dlr_build_host(lambda, eps, 96, x, tau_t, n_f, n_b, err);
    if (r <= 0) {
      std::printf("case %g %g error %s\n", lambda, eps, err.c_str());
      return 2;
    }
    std::vector<double> omega(x.size());
    for (size_t l = 0; l < x.size(); ++l) omega[l] = x[l] / beta;
    std::vector<cd> maps[qgw::kNumMaps];
    if (!qgw::dlr_maps_host(beta, omega, tau_t, n_f, n_b, maps, err)) {
      std::printf("case %g %g maps error %s\n", lambda, eps, err.c_str());
      return 3;
    }
    const double pi = 3.14159265358979323846;
    double df = 0.0, db = 0.0;
    for (int l0 : {0, r / 2, r - 1}) {
      std::vector<cd> gt(r), giw(r), wt(r), wiw(r);
      for (int k = 0; k < r; ++k) gt[k] = -kern(tau_t[k], x[l0]);
      for (int m = 0; m < r; ++m) {
        giw[m] = 1.0 / cd(-omega[l0], (2.0 * double(n_f[m]) + 1.0) * pi / beta);
        const double nu = 2.0 * double(n_b[m]) * pi / beta;
        wiw[m] = (nu == 0.0 && omega[l0] == 0.0) ? cd(-0.5 * beta) : std::tanh(0.5 * x[l0]) / cd(-omega[l0], nu);
      }
      for (int k = 0; k < r; ++k) wt[k] = gt[k];
      df = std::fmax(df, std::fmax(apply_defect(r, maps[2], gt, giw), apply_defect(r, maps[0], giw, gt)));
      db = std::fmax(db, std::fmax(apply_defect(r, maps[3], wt, wiw), apply_defect(r, maps[4], wiw, wt)));
    }
    std::vector<cd> row;
    if (!qgw::dlr_qp_row_host(beta, omega, n_f, row, err)) {
      std::printf("case %g %g row error %s\n", lambda, eps, err.c_str());
      return 4;
    }
    double rsum = 0.0;
    for (const cd& v : row) rsum += std::abs(v);
    std::printf("case lambda=%g eps=%g rank=%d fermion_defect=%.3e boson_defect=%.3e row_l1=%.6f\n", lambda, eps, r,
                df, db, rsum);
  }
  // too small a rank cap is an error, not a truncated basis
  std::vector<double> x, tau_t;
  std::vector<int64_t> n_f, n_b;
  std::string err;
  const int r = qgw::dlr_build_host(2500.0, 1e-12, 4, x, tau_t, n_f, n_b, err);
  std::printf("capped rank=%d error=%s\n", r, err.empty() ? "none" : "reported");
  return 0;
}
