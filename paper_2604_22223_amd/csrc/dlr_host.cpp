// Discrete Lehmann representation on the host, FP64.
//
// Construction of Kaye, Chen & Parcollet (PRB 105, 235115 (2022)), which the
// paper uses for every imaginary-time / Matsubara axis: the Lehmann kernel
// k(t, x) = exp(-t x) / (1 + exp(-x)) (t = tau / beta, x = beta * omega) is
// sampled on composite Chebyshev grids refined toward t = 0, 1 and x = 0;
// pivoted QR over the frequency columns picks the rank-r set x_l (pivots
// above eps times the first), pivoted QR over the time rows of k(t, x_l)
// picks t_k, and pivoted QR over the Matsubara rows of the fermionic and
// bosonic transforms of k picks the Matsubara nodes.  Maps between node
// values are k_out * k_in^{-1}, formed by LU solves with partial pivoting.
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <string>
#include <vector>

#include "qgw_internal.h"

namespace qgw {

using cd = std::complex<double>;

static const double kPi = 3.14159265358979323846264338327950288;

static inline double cconj(double v) { return v; }
static inline cd cconj(cd v) { return std::conj(v); }

// k(t, x) with tc = 1 - t supplied exactly by the caller
static double kernel_dimless(double t, double tc, double x) {
  if (x >= 0.0) return std::exp(-t * x) / (1.0 + std::exp(-x));
  return std::exp(tc * x) / (1.0 + std::exp(x));
}

static void chebyshev_panels(const std::vector<double>& edges, int order, std::vector<double>& out) {
  for (size_t p = 0; p + 1 < edges.size(); ++p) {
    const double a = edges[p], b = edges[p + 1];
    for (int j = order - 1; j >= 0; --j) {
      const double c = std::cos(kPi * (2.0 * j + 1.0) / (2.0 * order));
      out.push_back(0.5 * (a + b) + 0.5 * (b - a) * c);
    }
  }
}

// Column-pivoted Householder QR of the column-major m x n matrix a (in place).
// Stops after kmax steps, or (eps > 0) at the first pivot norm <= eps * the
// first one.  Returns the chosen column indices in order.
template <typename S>
static std::vector<int> pivoted_qr_columns(int m, int n, std::vector<S>& a, int kmax, double eps) {
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::vector<int> chosen;
  double first = -1.0;
  const int kcap = std::min(std::min(m, n), kmax);
  std::vector<double> norms(n);
  for (int j = 0; j < kcap; ++j) {
    // remaining column norms over rows j..m-1 (recomputed exactly)
    int best = j;
    double bestv = -1.0;
    for (int c = j; c < n; ++c) {
      double s = 0.0;
      const S* col = &a[size_t(c) * m];
      for (int i = j; i < m; ++i) s += std::norm(col[i]);
      norms[c] = s;
      if (s > bestv) {
        bestv = s;
        best = c;
      }
    }
    const double nrm = std::sqrt(bestv);
    if (first < 0.0) first = nrm;
    if (eps > 0.0 && !(nrm > eps * first)) break;
    if (best != j) {
      std::swap_ranges(a.begin() + size_t(j) * m, a.begin() + size_t(j + 1) * m, a.begin() + size_t(best) * m);
      std::swap(perm[j], perm[best]);
    }
    chosen.push_back(perm[j]);
    // Householder reflector for column j, rows j..m-1
    S* cj = &a[size_t(j) * m];
    const S x0 = cj[j];
    const double ax0 = std::abs(x0);
    const S phase = ax0 > 0.0 ? x0 / ax0 : S(1.0);
    const S alpha = -phase * nrm;
    std::vector<S> v(cj + j, cj + m);
    v[0] -= alpha;
    double vn = 0.0;
    for (auto& e : v) vn += std::norm(e);
    if (vn > 0.0) {
      const double inv_vn = 2.0 / vn;
      for (int c = j + 1; c < n; ++c) {
        S* cc = &a[size_t(c) * m];
        S dot = 0.0;
        for (int i = 0; i < m - j; ++i) dot += cconj(v[i]) * cc[j + i];
        dot *= inv_vn;
        for (int i = 0; i < m - j; ++i) cc[j + i] -= v[i] * dot;
      }
    }
    cj[j] = alpha;
    for (int i = j + 1; i < m; ++i) cj[i] = 0.0;
  }
  return chosen;
}

int dlr_build_host(double lambda, double eps, int max_rank, std::vector<double>& x,
                   std::vector<double>& tau_t, std::vector<int64_t>& n_f, std::vector<int64_t>& n_b,
                   std::string& err) {
  if (!(lambda > 0.0) || !(eps > 0.0) || !(eps < 1.0)) {
    err = "qgw_dlr_build: need lambda > 0 and 0 < eps < 1";
    return -1;
  }
  const int order = 24;
  const int npan = std::max(int(std::ceil(std::log2(lambda))), 1);
  // frequency grid: panels [0, lam 2^-(npan-1)], ..., [lam/2, lam], mirrored
  std::vector<double> xe{0.0};
  for (int j = npan - 1; j >= 0; --j) xe.push_back(lambda * std::ldexp(1.0, -j));
  std::vector<double> xpos;
  chebyshev_panels(xe, order, xpos);
  std::vector<double> xf;
  for (auto it = xpos.rbegin(); it != xpos.rend(); ++it) xf.push_back(-*it);
  xf.insert(xf.end(), xpos.begin(), xpos.end());
  // time grid: panels [0, 0.5 2^-npan], ..., [0.25, 0.5], mirrored with exact complements
  std::vector<double> te{0.0};
  for (int j = npan; j >= 0; --j) te.push_back(0.5 * std::ldexp(1.0, -j));
  std::vector<double> th;
  chebyshev_panels(te, order, th);
  std::vector<double> tf, tcf;
  for (double t : th) {
    tf.push_back(t);
    tcf.push_back(1.0 - t);
  }
  for (auto it = th.rbegin(); it != th.rend(); ++it) {
    tf.push_back(1.0 - *it);
    tcf.push_back(*it);
  }
  const int mt = int(tf.size()), nx = int(xf.size());
  // 1) frequencies
  std::vector<double> kf(size_t(mt) * nx);
  for (int c = 0; c < nx; ++c)
    for (int i = 0; i < mt; ++i) kf[size_t(c) * mt + i] = kernel_dimless(tf[i], tcf[i], xf[c]);
  std::vector<int> cols = pivoted_qr_columns<double>(mt, nx, kf, std::min(mt, nx), eps);
  const int r = int(cols.size());
  if (r > max_rank) {
    err = "qgw_dlr_build: rank " + std::to_string(r) + " exceeds max_rank";
    return -2;
  }
  x.clear();
  for (int c : cols) x.push_back(xf[c]);
  std::sort(x.begin(), x.end());
  // 2) times: columns of the r x mt matrix k(t, x_l)^T
  std::vector<double> kt(size_t(r) * mt);
  for (int c = 0; c < mt; ++c)
    for (int l = 0; l < r; ++l) kt[size_t(c) * r + l] = kernel_dimless(tf[c], tcf[c], x[l]);
  std::vector<int> trows = pivoted_qr_columns<double>(r, mt, kt, r, -1.0);
  tau_t.clear();
  for (int c : trows) tau_t.push_back(tf[c]);
  std::sort(tau_t.begin(), tau_t.end());
  // 3) Matsubara nodes
  const int nmax = std::max(int(std::ceil(2.0 * lambda)), 200);
  {
    const int nc = 2 * nmax;
    std::vector<cd> km(size_t(r) * nc);
    for (int c = 0; c < nc; ++c) {
      const double wn = kPi * (2.0 * (c - nmax) + 1.0);
      for (int l = 0; l < r; ++l) km[size_t(c) * r + l] = 1.0 / cd(-x[l], wn);
    }
    std::vector<int> sel = pivoted_qr_columns<cd>(r, nc, km, r, -1.0);
    n_f.clear();
    for (int c : sel) n_f.push_back(int64_t(c) - nmax);
    std::sort(n_f.begin(), n_f.end());
  }
  {
    const int nc = 2 * nmax + 1;
    std::vector<cd> km(size_t(r) * nc);
    for (int c = 0; c < nc; ++c) {
      const double nu = 2.0 * kPi * (c - nmax);
      for (int l = 0; l < r; ++l) {
        cd v;
        if (nu == 0.0 && x[l] == 0.0)
          v = -0.5;
        else
          v = std::tanh(0.5 * x[l]) / cd(-x[l], nu);
        km[size_t(c) * r + l] = v;
      }
    }
    std::vector<int> sel = pivoted_qr_columns<cd>(r, nc, km, r, -1.0);
    n_b.clear();
    for (int c : sel) n_b.push_back(int64_t(c) - nmax);
    std::sort(n_b.begin(), n_b.end());
  }
  return r;
}

// Solves A^T X = B^T for X (A: n x n, B: p x n, row-major); returns B A^{-1}.
static bool right_divide(int n, int p, std::vector<cd> a, const std::vector<cd>& b, std::vector<cd>& out) {
  // LU with partial pivoting of M = A^T (row-major)
  std::vector<cd> m(size_t(n) * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) m[size_t(i) * n + j] = a[size_t(j) * n + i];
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = std::abs(m[size_t(k) * n + k]);
    for (int i = k + 1; i < n; ++i) {
      const double v = std::abs(m[size_t(i) * n + k]);
      if (v > best) {
        best = v;
        pr = i;
      }
    }
    if (!(best > 0.0)) return false;
    piv[k] = pr;
    if (pr != k)
      for (int j = 0; j < n; ++j) std::swap(m[size_t(k) * n + j], m[size_t(pr) * n + j]);
    const cd d = m[size_t(k) * n + k];
    for (int i = k + 1; i < n; ++i) {
      const cd f = m[size_t(i) * n + k] / d;
      m[size_t(i) * n + k] = f;
      for (int j = k + 1; j < n; ++j) m[size_t(i) * n + j] -= f * m[size_t(k) * n + j];
    }
  }
  out.assign(size_t(p) * n, 0.0);
  std::vector<cd> y(n);
  for (int c = 0; c < p; ++c) {
    for (int i = 0; i < n; ++i) y[i] = b[size_t(c) * n + i];  // right-hand side B^T column c
    for (int k = 0; k < n; ++k)
      if (piv[k] != k) std::swap(y[k], y[piv[k]]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) y[i] -= m[size_t(i) * n + j] * y[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) y[i] -= m[size_t(i) * n + j] * y[j];
      y[i] /= m[size_t(i) * n + i];
    }
    for (int i = 0; i < n; ++i) out[size_t(c) * n + i] = y[i];
  }
  return true;
}

bool dlr_maps_host(double beta, const std::vector<double>& omega, const std::vector<double>& tau_t,
                   const std::vector<int64_t>& n_f, const std::vector<int64_t>& n_b,
                   std::vector<std::complex<double>> maps[kNumMaps], std::string& err) {
  const int r = int(omega.size());
  std::vector<cd> kt(size_t(r) * r), ktr(size_t(r) * r), kfm(size_t(r) * r), kbm(size_t(r) * r), kbeta(r);
  for (int l = 0; l < r; ++l) {
    const double x = beta * omega[l];
    for (int k = 0; k < r; ++k) {
      const double t = tau_t[k];
      kt[size_t(k) * r + l] = -kernel_dimless(t, 1.0 - t, x);
      ktr[size_t(k) * r + l] = -kernel_dimless(1.0 - t, t, x);
    }
    for (int m = 0; m < r; ++m) {
      const double wn = (2.0 * double(n_f[m]) + 1.0) * kPi / beta;
      kfm[size_t(m) * r + l] = 1.0 / cd(-omega[l], wn);
      const double nu = 2.0 * double(n_b[m]) * kPi / beta;
      if (nu == 0.0 && omega[l] == 0.0)
        kbm[size_t(m) * r + l] = -0.5 * beta;
      else
        kbm[size_t(m) * r + l] = std::tanh(0.5 * x) / cd(-omega[l], nu);
    }
    kbeta[l] = -kernel_dimless(1.0, 0.0, x);
  }
  bool ok = right_divide(r, r, kfm, kt, maps[0]) && right_divide(r, r, kfm, ktr, maps[1]) &&
            right_divide(r, r, kt, kfm, maps[2]) && right_divide(r, r, kt, kbm, maps[3]) &&
            right_divide(r, r, kbm, kt, maps[4]) && right_divide(r, 1, kfm, kbeta, maps[5]);
  // Matsubara sums: (1/beta) sum over all n of A(i w_n) B(i w_n) = sum_{l l'} a_l D_ll' b_l' for
  // fermionic DLR expansions, with D the divided differences of the Fermi function
  // f(x) = 1 / (1 + e^{beta x}) (partial fractions of 1 / ((i w - x)(i w - y)));
  // in node values Q = K_F^{-T} D K_F^{-1}, symmetric
  if (ok) {
    std::vector<double> f(r);
    for (int l = 0; l < r; ++l) f[l] = 0.5 * (1.0 - std::tanh(0.5 * beta * omega[l]));
    std::vector<cd> d(size_t(r) * r), b, bt(size_t(r) * r);
    for (int l = 0; l < r; ++l)
      for (int m = 0; m < r; ++m)
        d[size_t(l) * r + m] = (l == m) ? -beta * f[l] * (1.0 - f[l])
                                        : (f[l] - f[m]) / (omega[l] - omega[m]);
    ok = right_divide(r, r, kfm, d, b);  // D K^{-1}
    if (ok) {
      for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) bt[size_t(i) * r + j] = b[size_t(j) * r + i];
      ok = right_divide(r, r, kfm, bt, maps[6]);  // (D K^{-1})^T K^{-1} = K^{-T} D K^{-1}
    }
  }
  if (!ok) err = "DLR interpolation matrix is singular for the given nodes";
  return ok;
}

// The DLR interpolant of fermionic node values evaluated at the first
// Matsubara frequency i pi / beta: x(i pi / beta) = sum_m row[m] x(i w_m),
// row = K_F(i pi / beta, w_l) K_F^{-1} (the quasiparticle zero-frequency
// limit is taken at +-i pi / beta, where the expansion follows the function).
bool dlr_qp_row_host(double beta, const std::vector<double>& omega, const std::vector<int64_t>& n_f,
                     std::vector<std::complex<double>>& row, std::string& err) {
  const int r = int(omega.size());
  std::vector<cd> kfm(size_t(r) * r), k0(r);
  const double w0 = kPi / beta;
  for (int l = 0; l < r; ++l) {
    for (int m = 0; m < r; ++m) {
      const double wn = (2.0 * double(n_f[m]) + 1.0) * kPi / beta;
      kfm[size_t(m) * r + l] = 1.0 / cd(-omega[l], wn);
    }
    k0[l] = 1.0 / cd(-omega[l], w0);
  }
  if (!right_divide(r, 1, kfm, k0, row)) {
    err = "DLR interpolation matrix is singular for the given nodes";
    return false;
  }
  return true;
}

}  // namespace qgw
