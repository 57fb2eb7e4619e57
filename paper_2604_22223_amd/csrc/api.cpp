// C ABI of libqgw: argument validation, plans, the step calls and the
// self-consistent GW state.  Every compute step runs in the HIP kernels of
// this library; the host side only validates, sequences launches and builds
// the FP64 DLR maps once per plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qgw.h"
#include "qgw_internal.h"

namespace qgw {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

}  // namespace qgw

using namespace qgw;

struct qgw_state_s {
  qgw_plan plan = nullptr;
  double n_target = 0.0, mixing = 1.0, mu = 0.0;
  // static arrays
  void *H_k = nullptr, *V_R = nullptr, *V_q = nullptr, *V_qm = nullptr, *V_q0 = nullptr;
  // fermionic
  void *G_iw = nullptr, *Sig_iw = nullptr, *Sig_iw_old = nullptr, *SigHF_k = nullptr, *SigHF_old = nullptr;
  void *n_k = nullptr, *n_R = nullptr, *SigHF_R = nullptr, *Hs_k = nullptr;
  void *G_tau = nullptr, *G_reflt = nullptr, *Sig_tau_k = nullptr;
  // pair
  void *Pq = nullptr, *P_nu = nullptr, *Wc_nu = nullptr;
  void* hf_ws = nullptr;  // Hartree-Fock solve: eigenvectors and eigenvalues per k
  double* d_dsig = nullptr;
  double* d_blockmax = nullptr;
  // chemical-potential search of this state: scalars [16], partial sums, status
  double* d_scal = nullptr;
  double* d_part = nullptr;
  int* d_stat = nullptr;
  int mu_steps0 = 10;  // Newton steps queued in the first round of the next search
  int mu_steps_fixed = 0;  // > 0: that many instead (qgw_state_set_search_steps)
  double mu_g0 = NAN;  // mu of the state's last G0 at its target filling (the next G0's start if none is given)
  int last_evals = 0;  // evaluations the last search took
  // pinned host words of the search's per-iteration exchange (start point in, result out) and the
  // event the host polls for the result: no staging copy and no blocking wait per iteration
  double* h_io = nullptr;
  hipEvent_t ev_io = nullptr;
  // a12 runs on this side stream beside a1..a11 (fork and join events); default priority like every stream here
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // single-precision copies for the FP32 phase of the solve (allocated on first use)
  bool has32 = false;
  Plan p32;
  void *G32 = nullptr, *Gt32 = nullptr, *Gr32 = nullptr, *St32 = nullptr, *Siw32 = nullptr;
  void *Pq32 = nullptr, *Pnu32 = nullptr, *Wc32 = nullptr, *Vqm32 = nullptr;
  int prec_mode = 0;          // 0: FP64 only; 1: FP32 until |dSigma| <= switch_tol, then FP64
  double switch_tol = 1e-4;
  bool in_fp32 = false;
  int n_fp32 = 0, n_fp64 = 0, last_prec = 0;
  double last_dsig = INFINITY;
  // set when an iteration fails part-way (its arrays are then not one consistent state); cleared by a restart
  bool broken = false;
  // per-step timing with HIP events on the caller's stream
  bool prof = false;
  // two sets of step events, used by alternate iterations: one iteration's times are read after the next one
  // has been queued, so the reads do not hold up the GPU
  hipEvent_t ev[2][QGW_NUM_STEPS + 1] = {};
  hipEvent_t ev_a12[2] = {};  // end of a12 on the side stream (its start is ev[set][0], recorded there)
  int ev_set = 0;
  uint32_t prof_mask = (1u << QGW_NUM_STEPS) - 1;  // steps timed
  bool prof_in_line = false;                       // a12 on the caller's stream while timing
  double prof_ms[2][QGW_NUM_STEPS] = {};  // [FP64, FP32 iterations][step]
  int prof_iters[2] = {};
};

#define QGW_CHECK_HIP(expr, what)                                             \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_error(std::string(what) + ": " + hipGetErrorString(e_));            \
      return QGW_ERR_DEVICE;                                                  \
    }                                                                         \
  } while (0)

// Makes the device current and clears the runtime's last-error state, which any
// earlier HIP call of the process (the caller's included) may have left set, so
// that the launchers' hipGetLastError reports their own launches only.
static hipError_t enter_device(int dev) {
  const hipError_t e = hipSetDevice(dev);
  (void)hipGetLastError();
  return e;
}

#define QGW_REQUIRE(cond, code, msg) \
  do {                               \
    if (!(cond)) {                   \
      set_error(msg);                \
      return code;                   \
    }                                \
  } while (0)

static bool mesh_supported(int n, int dim) {
  if (dim == 3) {
    switch (n) {
#define QGW_CASE(NN) case NN:
      QGW_FOR_EACH_CUBE(QGW_CASE)
#undef QGW_CASE
      return true;
      default:
        return false;
    }
  }
  switch (n) {
#define QGW_CASE(NN) case NN:
    QGW_FOR_EACH_MESH(QGW_CASE)
#undef QGW_CASE
    return true;
    default:
      return false;
  }
}
static bool nb_supported(int nb) {
  switch (nb) {
#define QGW_CASE(NN) case NN:
    QGW_FOR_EACH_NB(QGW_CASE)
#undef QGW_CASE
    return true;
    default:
      return false;
  }
}

static size_t csize(const Plan& p) { return p.prec == 0 ? 16 : 8; }

static void free_plan_device(Plan& p) {
  for (int m = 0; m < kNumDevMaps; ++m) {
    if (p.dmaps64.m[m]) (void)hipFree(p.dmaps64.m[m]);
    if (p.dmaps32.m[m]) (void)hipFree(p.dmaps32.m[m]);
    p.dmaps64.m[m] = p.dmaps32.m[m] = nullptr;
  }
  void* ptrs[] = {p.d_tw64, p.d_tw32, p.d_pairs, p.terms.d_terms, p.terms.d_off, p.terms_lj.d_terms,
                  p.terms_lj.d_off, p.d_wn, p.d_qp_row, p.d_partials, p.d_status, p.d_scalars, p.d_mf};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  p.d_tw64 = nullptr;
  p.d_tw32 = nullptr;
  p.d_pairs = nullptr;
  p.terms.d_terms = p.terms.d_off = nullptr;
  p.terms_lj.d_terms = p.terms_lj.d_off = nullptr;
  p.d_wn = nullptr;
  p.d_qp_row = nullptr;
  p.d_partials = nullptr;
  p.d_status = nullptr;
  p.d_scalars = nullptr;
  p.d_mf = nullptr;
}

// e^{i pi q / den} with q reduced exactly modulo 2 den first
static zd cis_pi(int64_t q, int64_t den) {
  const int64_t per = 2 * den;
  q %= per;
  if (q < 0) q += per;
  const long double a = 3.141592653589793238462643383279502884L * (long double)q / (long double)den;
  return mk(double(cosl(a)), double(sinl(a)));
}

// Tables of the uniform-grid transforms (kernels_mf.hip), N = 2M nodes, fermionic w_m = (2m - N + 1) pi / beta,
// bosonic nu_m = (2m - N) pi / beta, tau_j = (j + 1/2) beta / N.  Each transform is
// out_k = post_k sum_j e^{s 2 pi i j k / N} pre_j in_j, from
//   w_m tau_j = 2 pi m j / N + pi m / N + pi (1 - N)(2j + 1) / (2N),   nu_m tau_j = 2 pi m j / N + pi m / N - pi (j + 1/2).
// Layout: e^{-2 pi i e / N} (N), the same for N1 and N2, then pre / post of iw -> tau (fermionic), tau -> iw
// (fermionic), tau -> i nu, i nu -> tau (N each), then the orbital-diagonal constant of iw -> tau,
// -(t_j + 1/2) with t_j = (1/beta) sum_m e^{-i w_m tau_j} / (i w_m) (the grid's sum of the 1/(iw) tail, whose
// exact transform is -1/2).
static std::vector<zd> mf_tables_host(int N, int n1, int n2, double beta) {
  std::vector<zd> t;
  t.reserve(size_t(10) * N + n1 + n2);
  for (int e = 0; e < N; ++e) t.push_back(cis_pi(-2 * e, N));
  for (int e = 0; e < n1; ++e) t.push_back(cis_pi(-2 * e, n1));
  for (int e = 0; e < n2; ++e) t.push_back(cis_pi(-2 * e, n2));
  const double ib = 1.0 / beta, bn = beta / double(N);
  auto push = [&](zd v, double s) { t.push_back(mk(v.re * s, v.im * s)); };
  // fermionic iw -> tau
  for (int m = 0; m < N; ++m) push(cis_pi(-m, N), ib);
  for (int j = 0; j < N; ++j) push(cis_pi(-int64_t(1 - N) * (2 * j + 1), 2 * int64_t(N)), 1.0);
  // fermionic tau -> iw
  for (int j = 0; j < N; ++j) push(cis_pi(int64_t(1 - N) * (2 * j + 1), 2 * int64_t(N)), bn);
  for (int m = 0; m < N; ++m) push(cis_pi(m, N), 1.0);
  // bosonic tau -> i nu
  for (int j = 0; j < N; ++j) push(cis_pi(-(2 * j + 1), 2), bn);
  for (int m = 0; m < N; ++m) push(cis_pi(m, N), 1.0);
  // bosonic i nu -> tau
  for (int m = 0; m < N; ++m) push(cis_pi(-m, N), ib);
  for (int j = 0; j < N; ++j) push(cis_pi(2 * j + 1, 2), 1.0);
  // orbital-diagonal constant of fermionic iw -> tau
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < N; ++j) {
    long double sr = 0.0L, si = 0.0L;
    for (int m = 0; m < N; ++m) {
      const int64_t k = 2 * int64_t(m) - N + 1;          // w_m = k pi / beta
      const zd e = cis_pi(-k * (2 * j + 1), 2 * int64_t(N));  // e^{-i w_m tau_j}
      // e / (i w_m) = -i e beta / (k pi); the 1/beta prefactor cancels beta
      const long double c = 1.0L / ((long double)k * pi);
      sr += (long double)e.im * c;
      si -= (long double)e.re * c;
    }
    t.push_back(mk(-double(sr + 0.5L), -double(si)));
  }
  return t;
}

template <typename V>
static hipError_t upload(void** dst, const V* src, size_t bytes) {
  hipError_t e = hipMalloc(dst, bytes);
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
}

extern "C" {

const char* qgw_last_error(void) { return g_err.c_str(); }

qgw_status qgw_dlr_build(double lambda, double eps, int32_t max_rank, double* x, double* tau_t,
                         int64_t* n_f, int64_t* n_b, int32_t* rank) {
  QGW_REQUIRE(x && tau_t && n_f && n_b && rank, QGW_ERR_INVALID_ARG, "qgw_dlr_build: null output");
  QGW_REQUIRE(max_rank > 0, QGW_ERR_INVALID_ARG, "qgw_dlr_build: max_rank must be positive");
  std::vector<double> xs, ts;
  std::vector<int64_t> nf, nb;
  std::string err;
  int r;
  try {
    r = dlr_build_host(lambda, eps, max_rank, xs, ts, nf, nb, err);
  } catch (const std::bad_alloc&) {
    set_error("qgw_dlr_build: out of host memory");
    return QGW_ERR_ALLOC;
  }
  if (r == -1) {
    set_error(err);
    return QGW_ERR_INVALID_ARG;
  }
  if (r < 0) {
    set_error(err);
    return QGW_ERR_SHAPE;
  }
  for (int i = 0; i < r; ++i) {
    x[i] = xs[i];
    tau_t[i] = ts[i];
    n_f[i] = nf[i];
    n_b[i] = nb[i];
  }
  *rank = r;
  return QGW_OK;
}

// mf_nodes == 0: DLR plan from the descriptor's node set; mf_nodes = N > 0: uniform Matsubara grid of N nodes
static qgw_status plan_create_impl(const qgw_plan_desc* d, int mf_nodes, qgw_plan* out) {
  QGW_REQUIRE(d && out, QGW_ERR_INVALID_ARG, "qgw_plan_create: null argument");
  *out = nullptr;
  QGW_REQUIRE(d->n >= 1, QGW_ERR_INVALID_ARG, "qgw_plan_create: mesh side must be >= 1");
  QGW_REQUIRE(d->dim == 0 || d->dim == 2 || d->dim == 3, QGW_ERR_INVALID_ARG,
              "qgw_plan_create: mesh dimension must be 2 or 3 (0 means 2)");
  const int dim = d->dim == 3 ? 3 : 2;
  QGW_REQUIRE(mesh_supported(d->n, dim), QGW_ERR_UNSUPPORTED,
              "qgw_plan_create: mesh side " + std::to_string(d->n) + " has no compiled " + std::to_string(dim) +
                  "-D transform");
  QGW_REQUIRE(d->n_sites >= 1 && d->site_norb, QGW_ERR_INVALID_ARG, "qgw_plan_create: need n_sites >= 1 and site_norb");
  QGW_REQUIRE(d->beta > 0.0 && std::isfinite(d->beta), QGW_ERR_INVALID_ARG, "qgw_plan_create: beta must be positive");
  int mf_n1 = 0, mf_n2 = 0;
  if (mf_nodes == 0) {
    QGW_REQUIRE(d->rank >= 1 && d->rank <= kMaxRank, QGW_ERR_UNSUPPORTED, "qgw_plan_create: DLR rank must be in [1, 96]");
    QGW_REQUIRE(d->omega && d->tau_t && d->n_f && d->n_b, QGW_ERR_INVALID_ARG, "qgw_plan_create: null DLR node array");
    QGW_REQUIRE(d->precision == QGW_F64 || d->precision == QGW_F32, QGW_ERR_INVALID_ARG, "qgw_plan_create: bad precision");
  } else {
    QGW_REQUIRE(mf_grid_split(mf_nodes, &mf_n1, &mf_n2), QGW_ERR_UNSUPPORTED,
                "qgw_plan_create_mf: " + std::to_string(mf_nodes) + " nodes have no compiled transform");
    QGW_REQUIRE(d->precision == QGW_F64, QGW_ERR_UNSUPPORTED, "qgw_plan_create_mf: the uniform grid runs in FP64");
  }
  int no = 0, nb = 0;
  for (int s = 0; s < d->n_sites; ++s) {
    QGW_REQUIRE(d->site_norb[s] >= 1, QGW_ERR_INVALID_ARG, "qgw_plan_create: site with no orbitals");
    no += d->site_norb[s];
    nb += d->site_norb[s] * d->site_norb[s];
  }
  QGW_REQUIRE(no <= 8, QGW_ERR_UNSUPPORTED, "qgw_plan_create: at most 8 orbitals per cell");
  QGW_REQUIRE(nb_supported(nb), QGW_ERR_UNSUPPORTED,
              "qgw_plan_create: pair basis size " + std::to_string(nb) + " has no compiled Dyson-W solver");
  for (int i = 0; mf_nodes == 0 && i < d->rank; ++i) {
    QGW_REQUIRE(d->tau_t[i] > 0.0 && d->tau_t[i] < 1.0, QGW_ERR_INVALID_ARG, "qgw_plan_create: tau_t must lie in (0, 1)");
    QGW_REQUIRE(std::isfinite(d->omega[i]), QGW_ERR_INVALID_ARG, "qgw_plan_create: non-finite omega");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    set_error("qgw_plan_create: no HIP device");
    return QGW_ERR_DEVICE;
  }
  QGW_REQUIRE(d->device >= 0 && d->device < ndev, QGW_ERR_INVALID_ARG, "qgw_plan_create: bad device ordinal");
  QGW_CHECK_HIP(enter_device(d->device), "hipSetDevice");

  qgw_plan h = new (std::nothrow) qgw_plan_s;
  QGW_REQUIRE(h, QGW_ERR_ALLOC, "qgw_plan_create: out of host memory");
  Plan& p = h->p;
  p.device = d->device;
  p.n = d->n;
  p.dim = dim;
  p.nk = dim == 3 ? d->n * d->n * d->n : d->n * d->n;
  p.no = no;
  p.nb = nb;
  p.prec = d->precision;
  p.beta = d->beta;
  p.site_norb.assign(d->site_norb, d->site_norb + d->n_sites);
  if (mf_nodes == 0) {
    p.r = d->rank;
    p.omega.assign(d->omega, d->omega + p.r);
    p.tau_t.assign(d->tau_t, d->tau_t + p.r);
    p.n_f.assign(d->n_f, d->n_f + p.r);
    p.n_b.assign(d->n_b, d->n_b + p.r);
  } else {
    // n = -M .. M-1 for both statistics, midpoint times; no real-frequency nodes
    p.grid = kGridMF;
    p.r = mf_nodes;
    p.mf_n1 = mf_n1;
    p.mf_n2 = mf_n2;
    p.ne_offset = double(no);
    p.omega.assign(p.r, 0.0);
    for (int j = 0; j < p.r; ++j) {
      p.tau_t.push_back((j + 0.5) / double(p.r));
      p.n_f.push_back(j - p.r / 2);
      p.n_b.push_back(j - p.r / 2);
    }
  }
  // orbital / pair bookkeeping
  p.pair_of.assign(size_t(no) * no, -1);
  int off = 0, al = 0;
  for (int s = 0; s < d->n_sites; ++s) {
    const int ns = d->site_norb[s];
    for (int i = 0; i < ns; ++i) p.orb_site.push_back(s);
    for (int i = 0; i < ns; ++i)
      for (int l = 0; l < ns; ++l) {
        p.pair_first.push_back(off + i);
        p.pair_second.push_back(off + l);
        p.pair_of[size_t(off + i) * no + off + l] = al++;
      }
    off += ns;
  }
  // term table: for output (i, k): alpha = (i, l), beta = (j, k)
  std::vector<int> terms, toff(size_t(no) * no + 1, 0);
  int max_terms = 0;
  for (int i = 0; i < no; ++i)
    for (int k = 0; k < no; ++k) {
      int cnt = 0;
      for (int a = 0; a < nb; ++a) {
        if (p.pair_first[a] != i) continue;
        for (int b = 0; b < nb; ++b) {
          if (p.pair_second[b] != k) continue;
          terms.push_back(a);
          terms.push_back(b);
          terms.push_back(p.pair_second[a]);
          terms.push_back(p.pair_first[b]);
          ++cnt;
        }
      }
      toff[size_t(i) * no + k + 1] = toff[size_t(i) * no + k] + cnt;
      if (cnt > max_terms) max_terms = cnt;
    }
  p.terms.max_terms = max_terms;
  // the same terms keyed by (l, j) = (second(alpha), first(beta)), entries (alpha, beta, i, k)
  std::vector<int> terms_lj, toff_lj(size_t(no) * no + 1, 0);
  int max_lj = 0;
  for (int l = 0; l < no; ++l)
    for (int j = 0; j < no; ++j) {
      int cnt = 0;
      for (int a = 0; a < nb; ++a) {
        if (p.pair_second[a] != l) continue;
        for (int b = 0; b < nb; ++b) {
          if (p.pair_first[b] != j) continue;
          terms_lj.push_back(a);
          terms_lj.push_back(b);
          terms_lj.push_back(p.pair_first[a]);
          terms_lj.push_back(p.pair_second[b]);
          ++cnt;
        }
      }
      toff_lj[size_t(l) * no + j + 1] = toff_lj[size_t(l) * no + j] + cnt;
      if (cnt > max_lj) max_lj = cnt;
    }
  p.terms_lj.max_terms = max_lj;
  // DLR maps (FP64, host)
  std::string err;
  if (p.grid == kGridMF) {
    // the density row only: G(beta^-) = -(1/beta) sum_m G(i w_m) - 1/2 on the orbital diagonal
    p.maps[QGW_F_IW2BETA].assign(p.r, std::complex<double>(-1.0 / p.beta, 0.0));
  } else if (!dlr_maps_host(p.beta, p.omega, p.tau_t, p.n_f, p.n_b, p.maps, err)) {
    delete h;
    set_error("qgw_plan_create: " + err);
    return QGW_ERR_INVALID_ARG;
  }
  // rows per chunk: minimise padded rows, then the number of chunks
  {
    const int cand[] = {8, 16, 20, 24, 28, 32};
    int best_mt = 32, best_cost = 1 << 30;
    for (int mt : cand) {
      const int chunks = (p.r + mt - 1) / mt;
      const int cost = chunks * mt * 4 + chunks;
      if (cost < best_cost) {
        best_cost = cost;
        best_mt = mt;
      }
    }
    p.dmaps64.mt = p.dmaps32.mt = best_mt;
    // zero rows past r so that every chunk size up to 32 reads inside the map
    p.dmaps64.rows_padded = p.dmaps32.rows_padded = ((p.r + 31) / 32) * 32 + 32;
  }
  hipError_t e = hipSuccess;
  {
    const int rp = p.dmaps64.rows_padded;
    for (int m = 0; m < kNumMaps && e == hipSuccess; ++m) {
      if (p.grid == kGridMF && m != QGW_F_IW2BETA) continue;
      const int rows = (m == 5) ? 1 : p.r;
      std::vector<zd> h64(size_t(rp) * p.r, mk(0.0, 0.0));
      std::vector<zf> h32(size_t(rp) * p.r, mk(0.0f, 0.0f));
      for (int i = 0; i < rows; ++i)
        for (int j = 0; j < p.r; ++j) {
          const std::complex<double> v = p.maps[m][size_t(i) * p.r + j];
          h64[size_t(i) * p.r + j] = mk(v.real(), v.imag());
          h32[size_t(i) * p.r + j] = mk(float(v.real()), float(v.imag()));
        }
      e = upload(&p.dmaps64.m[m], h64.data(), h64.size() * sizeof(zd));
      if (e == hipSuccess) e = upload(&p.dmaps32.m[m], h32.data(), h32.size() * sizeof(zf));
    }
    // adjoint maps T^H of the square maps (FP64 only: the adjoint calls run in FP64)
    for (int m = 0; m < kNumMaps && e == hipSuccess && p.grid == kGridDLR; ++m) {
      if (m == QGW_F_IW2BETA) continue;
      std::vector<zd> h64(size_t(rp) * p.r, mk(0.0, 0.0));
      for (int i = 0; i < p.r; ++i)
        for (int j = 0; j < p.r; ++j) {
          const std::complex<double> v = std::conj(p.maps[m][size_t(j) * p.r + i]);
          h64[size_t(i) * p.r + j] = mk(v.real(), v.imag());
        }
      e = upload(&p.dmaps64.m[kAdjMap0 + m], h64.data(), h64.size() * sizeof(zd));
    }
  }
  if (e == hipSuccess) {
    std::vector<zd> t64(p.n);
    std::vector<zf> t32(p.n);
    for (int j = 0; j < p.n; ++j) {
      const long double a = -2.0L * 3.141592653589793238462643383279502884L * j / p.n;
      t64[j] = mk(double(cosl(a)), double(sinl(a)));
      t32[j] = mk(float(cosl(a)), float(sinl(a)));
    }
    e = upload((void**)&p.d_tw64, t64.data(), t64.size() * sizeof(zd));
    if (e == hipSuccess) e = upload((void**)&p.d_tw32, t32.data(), t32.size() * sizeof(zf));
  }
  if (e == hipSuccess) {
    std::vector<int> pt(2 * nb + no * no);
    for (int a = 0; a < nb; ++a) {
      pt[a] = p.pair_first[a];
      pt[nb + a] = p.pair_second[a];
    }
    for (int i = 0; i < no * no; ++i) pt[2 * nb + i] = p.pair_of[i];
    e = upload((void**)&p.d_pairs, pt.data(), pt.size() * sizeof(int));
  }
  if (e == hipSuccess) e = upload((void**)&p.terms.d_terms, terms.data(), terms.size() * sizeof(int));
  if (e == hipSuccess) e = upload((void**)&p.terms.d_off, toff.data(), toff.size() * sizeof(int));
  if (e == hipSuccess) e = upload((void**)&p.terms_lj.d_terms, terms_lj.data(), terms_lj.size() * sizeof(int));
  if (e == hipSuccess) e = upload((void**)&p.terms_lj.d_off, toff_lj.data(), toff_lj.size() * sizeof(int));
  if (e == hipSuccess) {
    std::vector<double> wn(p.r);
    for (int m = 0; m < p.r; ++m) wn[m] = (2.0 * double(p.n_f[m]) + 1.0) * 3.14159265358979323846 / p.beta;
    e = upload((void**)&p.d_wn, wn.data(), wn.size() * sizeof(double));
  }
  if (e == hipSuccess && p.grid == kGridMF) {
    // i pi / beta is the grid's node n = 0 (index M)
    std::vector<zd> hr(p.r, mk(0.0, 0.0));
    hr[p.r / 2] = mk(1.0, 0.0);
    e = upload((void**)&p.d_qp_row, hr.data(), hr.size() * sizeof(zd));
    if (e == hipSuccess) {
      const std::vector<zd> tab = mf_tables_host(p.r, p.mf_n1, p.mf_n2, p.beta);
      e = upload((void**)&p.d_mf, tab.data(), tab.size() * sizeof(zd));
    }
  }
  if (e == hipSuccess && p.grid == kGridDLR) {
    std::vector<std::complex<double>> row;
    std::string rerr;
    if (!dlr_qp_row_host(p.beta, p.omega, p.n_f, row, rerr)) {
      free_plan_device(p);
      delete h;
      set_error("qgw_plan_create: " + rerr);
      return QGW_ERR_INVALID_ARG;
    }
    std::vector<zd> hr(p.r);
    for (int m = 0; m < p.r; ++m) hr[m] = mk(row[m].real(), row[m].imag());
    e = upload((void**)&p.d_qp_row, hr.data(), hr.size() * sizeof(zd));
  }
  if (e == hipSuccess) {
    p.max_blocks = 8192;
    e = hipMalloc((void**)&p.d_partials, size_t(2) * 4 * p.max_blocks * sizeof(double));
  }
  if (e == hipSuccess) e = hipMalloc((void**)&p.d_status, 16 * sizeof(int));
  if (e == hipSuccess) e = hipMemset(p.d_status, 0, 16 * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&p.d_scalars, 32 * sizeof(double));
  if (e != hipSuccess) {
    set_error(std::string("qgw_plan_create: ") + hipGetErrorString(e));
    free_plan_device(p);
    delete h;
    return QGW_ERR_ALLOC;
  }
  *out = h;
  return QGW_OK;
}

qgw_status qgw_plan_create(const qgw_plan_desc* d, qgw_plan* out) { return plan_create_impl(d, 0, out); }

qgw_status qgw_plan_create_mf(const qgw_plan_desc* d, int32_t n_nodes, qgw_plan* out) {
  QGW_REQUIRE(n_nodes > 0, QGW_ERR_INVALID_ARG, "qgw_plan_create_mf: the node count must be positive");
  return plan_create_impl(d, n_nodes, out);
}

int32_t qgw_mf_nodes_for(double beta, double omega_max) {
  if (!(beta > 0.0) || !(omega_max > 0.0) || !std::isfinite(beta * omega_max)) return 0;
  const double m = std::ceil(omega_max * beta / (2.0 * 3.14159265358979323846) + 0.5);  // (2M - 1) pi / beta >= omega_max
  const int need = 2 * int(m < 1.0 ? 1.0 : m);
  int best = 0;
#define QGW_CASE(NN, A, B) \
  if (NN >= need && (best == 0 || NN < best)) best = NN;
  QGW_FOR_EACH_MF_GRID(QGW_CASE)
#undef QGW_CASE
  return best;
}

qgw_status qgw_plan_destroy(qgw_plan h) {
  if (!h) return QGW_OK;
  (void)hipSetDevice(h->p.device);
  free_plan_device(h->p);
  delete h;
  return QGW_OK;
}

qgw_status qgw_plan_get_map(qgw_plan h, int32_t map, double* out) {
  QGW_REQUIRE(h && out, QGW_ERR_INVALID_ARG, "qgw_plan_get_map: null argument");
  QGW_REQUIRE(h->p.grid == kGridDLR, QGW_ERR_UNSUPPORTED, "qgw_plan_get_map: a uniform-grid plan holds no dense maps");
  QGW_REQUIRE(map >= 0 && map < kNumMaps, QGW_ERR_INVALID_ARG, "qgw_plan_get_map: bad map");
  const auto& v = h->p.maps[map];
  for (size_t i = 0; i < v.size(); ++i) {
    out[2 * i] = v[i].real();
    out[2 * i + 1] = v[i].imag();
  }
  return QGW_OK;
}

qgw_status qgw_plan_sizes(qgw_plan h, int32_t* rank, int32_t* n_o, int32_t* n_b, int32_t* n_k) {
  QGW_REQUIRE(h, QGW_ERR_INVALID_ARG, "qgw_plan_sizes: null plan");
  if (rank) *rank = h->p.r;
  if (n_o) *n_o = h->p.no;
  if (n_b) *n_b = h->p.nb;
  if (n_k) *n_k = h->p.nk;
  return QGW_OK;
}

// ------------------------------------------------------------------ steps

#define QGW_PLAN(h, name)                                                   \
  QGW_REQUIRE(h, QGW_ERR_INVALID_ARG, std::string(name) + ": null plan"); \
  const Plan& p = h->p;                                                     \
  QGW_CHECK_HIP(enter_device(p.device), "hipSetDevice")

qgw_status qgw_dlr_transform(qgw_plan h, int32_t map, int64_t ncols, double sre, double sim,
                             int32_t hermitian, const void* in, void* out, void* stream) {
  QGW_PLAN(h, "qgw_dlr_transform");
  QGW_REQUIRE(map >= 0 && map < kNumMaps, QGW_ERR_INVALID_ARG, "qgw_dlr_transform: bad map");
  QGW_REQUIRE(ncols >= 0, QGW_ERR_INVALID_ARG, "qgw_dlr_transform: negative ncols");
  if (ncols == 0) return QGW_OK;
  QGW_REQUIRE(in && out, QGW_ERR_INVALID_ARG, "qgw_dlr_transform: null array");
  QGW_REQUIRE(in != out, QGW_ERR_INVALID_ARG, "qgw_dlr_transform: in and out must differ");
  QGW_REQUIRE(hermitian >= 0 && hermitian <= 2, QGW_ERR_INVALID_ARG, "qgw_dlr_transform: bad hermitian mode");
  QGW_REQUIRE(hermitian == 0 || ncols == int64_t(p.no) * p.no * p.nk, QGW_ERR_SHAPE,
              "qgw_dlr_transform: the Hermitian modes need ncols = n_o^2 N_k");
  QGW_CHECK_HIP(launch_dlr(p, map, ncols, sre, sim, in, out, (hipStream_t)stream, hermitian), "qgw_dlr_transform");
  return QGW_OK;
}

qgw_status qgw_dlr_transform_pairs(qgw_plan h, int32_t map, int32_t in_layout, int32_t out_layout,
                                   const void* in, void* out, void* stream) {
  QGW_PLAN(h, "qgw_dlr_transform_pairs");
  QGW_REQUIRE(map >= 0 && map < 5, QGW_ERR_INVALID_ARG, "qgw_dlr_transform_pairs: bad map");
  QGW_REQUIRE((in_layout == 0 || in_layout == 1) && (out_layout == 0 || out_layout == 1), QGW_ERR_INVALID_ARG,
              "qgw_dlr_transform_pairs: bad layout");
  QGW_REQUIRE(in && out && in != out, QGW_ERR_INVALID_ARG, "qgw_dlr_transform_pairs: need distinct arrays");
  QGW_CHECK_HIP(launch_dlr_pairs(p, map, in_layout, out_layout, in, out, (hipStream_t)stream),
                "qgw_dlr_transform_pairs");
  return QGW_OK;
}

qgw_status qgw_lattice_fft(qgw_plan h, int32_t dir, int64_t batch, const void* in, void* out, void* stream) {
  QGW_PLAN(h, "qgw_lattice_fft");
  QGW_REQUIRE(dir == QGW_R_TO_K || dir == QGW_K_TO_R, QGW_ERR_INVALID_ARG, "qgw_lattice_fft: bad direction");
  QGW_REQUIRE(batch >= 0, QGW_ERR_INVALID_ARG, "qgw_lattice_fft: negative batch");
  if (batch == 0) return QGW_OK;
  QGW_REQUIRE(in && out, QGW_ERR_INVALID_ARG, "qgw_lattice_fft: null array");
  QGW_CHECK_HIP(launch_lattice_fft(p, dir, batch, in, out, (hipStream_t)stream), "qgw_lattice_fft");
  return QGW_OK;
}

qgw_status qgw_bubble(qgw_plan h, const void* gt, const void* gr, int32_t out_q, void* P, void* stream) {
  QGW_PLAN(h, "qgw_bubble");
  QGW_REQUIRE(gt && gr && P, QGW_ERR_INVALID_ARG, "qgw_bubble: null array");
  QGW_REQUIRE(P != gt && P != gr, QGW_ERR_INVALID_ARG, "qgw_bubble: output aliases an input");
  QGW_CHECK_HIP(launch_bubble(p, gt, gr, out_q ? 1 : 0, P, (hipStream_t)stream), "qgw_bubble");
  return QGW_OK;
}

qgw_status qgw_dyson_W(qgw_plan h, const void* V_q, const void* P_nu, void* Wc_nu, void* stream) {
  QGW_PLAN(h, "qgw_dyson_W");
  QGW_REQUIRE(V_q && P_nu && Wc_nu, QGW_ERR_INVALID_ARG, "qgw_dyson_W: null array");
  QGW_CHECK_HIP(launch_dyson_w(p, V_q, P_nu, Wc_nu, (hipStream_t)stream), "qgw_dyson_W");
  return QGW_OK;
}

qgw_status qgw_sigma(qgw_plan h, const void* gt, const void* wc, int32_t in_q, int32_t out_k, void* sig,
                     void* stream) {
  QGW_PLAN(h, "qgw_sigma");
  QGW_REQUIRE(gt && wc && sig, QGW_ERR_INVALID_ARG, "qgw_sigma: null array");
  QGW_REQUIRE(sig != gt && sig != wc, QGW_ERR_INVALID_ARG, "qgw_sigma: output aliases an input");
  QGW_CHECK_HIP(launch_sigma(p, gt, wc, in_q ? 1 : 0, out_k ? 1 : 0, sig, (hipStream_t)stream), "qgw_sigma");
  return QGW_OK;
}

qgw_status qgw_hartree_fock(qgw_plan h, const void* V_R, const void* n_R, void* SigHF_R, void* stream) {
  QGW_PLAN(h, "qgw_hartree_fock");
  QGW_REQUIRE(V_R && n_R && SigHF_R, QGW_ERR_INVALID_ARG, "qgw_hartree_fock: null array");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_hartree_fock: FP64 plans only");
  // V(q = 0) in the plan's status scratch is too small: use the partials buffer
  const size_t need = size_t(p.nb) * p.nb * sizeof(zd);
  QGW_REQUIRE(need <= size_t(2) * 4 * p.max_blocks * sizeof(double), QGW_ERR_UNSUPPORTED, "qgw_hartree_fock: pair basis too large");
  hipStream_t s = (hipStream_t)stream;
  QGW_CHECK_HIP(launch_pair_sum_r(p, V_R, p.d_partials, s), "qgw_hartree_fock");
  QGW_CHECK_HIP(launch_hartree_fock(p, V_R, p.d_partials, n_R, SigHF_R, s), "qgw_hartree_fock");
  return QGW_OK;
}

// extra_src / extra_dst: one more device scalar read back with the search's
// result (the iteration's |dSigma|), end_ev: recorded after the last kernel
static qgw_status run_dyson_g(const Plan& p, const void* H_k, const void* Sig_iw, double n_target,
                              double* mu, void* G_iw, hipStream_t s, double* evals, double* scal = nullptr,
                              double* part = nullptr, int* stat = nullptr, const double* extra_src = nullptr,
                              double* extra_dst = nullptr, hipEvent_t end_ev = nullptr, int steps0 = 6,
                              double* h_io = nullptr, hipEvent_t io_ev = nullptr, int track = 0,
                              const double* dpart = nullptr, int dnblk = 0, int* rounds_out = nullptr,
                              void (*on_queued)(void*) = nullptr, void* on_ctx = nullptr,
                              const double* bmax = nullptr, int nbmax = 0, double* dsig_out = nullptr) {
  const int mode = std::isnan(n_target) ? 0 : 1;
  if (!scal) {
    scal = p.d_scalars;
    part = p.d_partials;
    stat = p.d_status;
  }
  // with pinned words (h_io[0..9] result, h_io[16..17] start point) the copies need no staging
  // buffer and the host polls an event for the result instead of blocking on the stream
  double sc_pageable[2] = {*mu, n_target};
  double* sc = sc_pageable;
  if (h_io) {
    sc = h_io + 16;
    sc[0] = *mu;
    sc[1] = n_target;
  }
  // the search's first launch takes the start point as arguments and resets the status word; a fixed-mu call
  // has no search and gets mu by a copy
  if (mode == 1) {
    // with the diagonal sums of H from a14 at hand and a finite start, no Gershgorin pass is needed
    const bool use_d = dpart && std::isfinite(sc[0]);
    QGW_CHECK_HIP(launch_dyson_g_begin(p, H_k, scal, part, stat, track, s, 1, sc[0], sc[1], use_d ? dpart : nullptr,
                                       dnblk, bmax, nbmax, dsig_out),
                  "qgw_dyson_G");
  } else {
    QGW_CHECK_HIP(hipMemcpyAsync(scal, sc, 2 * sizeof(double), hipMemcpyHostToDevice, s), "qgw_dyson_G");
    QGW_CHECK_HIP(hipMemsetAsync(stat, 0, sizeof(int), s), "qgw_dyson_G");
  }
  // scal[0..9]: mu, n_target, evaluations, N_e, search state, status, extra
  double res[10] = {};
  int st = 0;
  int rounds = 0;
  for (int round = 0;; ++round) {
    rounds = round + 1;
    // a few Newton evaluations, G at the current mu, one read-back; more rounds only if needed
    const int steps = mode == 1 ? (round == 0 ? steps0 : 16) : 0;
    if (mode == 1)
      QGW_CHECK_HIP(launch_dyson_g_steps(p, H_k, Sig_iw, scal, part, stat, steps, s), "qgw_dyson_G");
    QGW_CHECK_HIP(launch_dyson_g_final(p, H_k, Sig_iw, mode, G_iw, scal, part, stat, s, extra_src, steps),
                  "qgw_dyson_G");
    if (end_ev) QGW_CHECK_HIP(hipEventRecord(end_ev, s), "qgw_dyson_G");
    if (h_io) {
      QGW_CHECK_HIP(hipMemcpyAsync(h_io, scal, sizeof(res), hipMemcpyDeviceToHost, s), "qgw_dyson_G");
      QGW_CHECK_HIP(hipEventRecord(io_ev, s), "qgw_dyson_G");
      // work the caller queues behind the read-back (on_queued), so the GPU has it while the host waits
      if (round == 0 && on_queued) on_queued(on_ctx);
      hipError_t q;
      while ((q = hipEventQuery(io_ev)) == hipErrorNotReady) {
      }
      QGW_CHECK_HIP(q, "qgw_dyson_G");
      std::memcpy(res, h_io, sizeof(res));
    } else {
      QGW_CHECK_HIP(hipMemcpyAsync(res, scal, sizeof(res), hipMemcpyDeviceToHost, s), "qgw_dyson_G");
      QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_dyson_G");
    }
    st = int(res[8]);
    if (extra_src && round == 0) *extra_dst = res[9];
    if (mode == 0 || st != 2 || res[2] >= 200.0) break;
    QGW_CHECK_HIP(hipMemsetAsync(stat, 0, sizeof(int), s), "qgw_dyson_G");
  }
  if (rounds_out) *rounds_out = rounds;
  if (mode == 1) {
    *mu = res[0];
    if (evals) *evals = res[2];
    if (st == 1) {
      set_error("qgw_dyson_G: no finite starting point for the chemical potential");
      return QGW_ERR_NOT_CONVERGED;
    }
    if (st == 2) {
      set_error("qgw_dyson_G: chemical potential search did not converge");
      return QGW_ERR_NOT_CONVERGED;
    }
    if (!std::isfinite(res[0])) {
      set_error("qgw_dyson_G: non-finite chemical potential");
      return QGW_ERR_NONFINITE;
    }
  }
  return QGW_OK;
}

qgw_status qgw_dyson_G(qgw_plan h, const void* H_k, const void* Sig_iw, double n_target, double* mu,
                       void* G_iw, void* stream) {
  QGW_PLAN(h, "qgw_dyson_G");
  QGW_REQUIRE(H_k && G_iw && mu, QGW_ERR_INVALID_ARG, "qgw_dyson_G: null argument");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_dyson_G: the Dyson G solve is FP64");
  if (!std::isnan(n_target))
    QGW_REQUIRE(n_target > 0.0 && n_target < 2.0 * p.no, QGW_ERR_INVALID_ARG,
                "qgw_dyson_G: target filling must lie in (0, 2 n_o)");
  else
    QGW_REQUIRE(std::isfinite(*mu), QGW_ERR_INVALID_ARG, "qgw_dyson_G: fixed mu must be finite");
  return run_dyson_g(p, H_k, Sig_iw, n_target, mu, G_iw, (hipStream_t)stream, nullptr);
}

// ------------------------------------------------------ Dyson G without allocation
// The search scratch of qgw_dyson_G_noalloc: 32 scalars, the per-block partial sums of the start and of the
// evaluations, and 16 status words, in a file-scope device array.  Each GPU the library runs on holds its own
// copy until the process ends.  Host code uses it only through the address hipGetSymbolAddress returns for the
// current device (the array's name on the host is not a device address).
constexpr int kNaScalars = 32;
constexpr int kNaPartials = 4096;
constexpr int kNaStatus = 16;
constexpr size_t kNaBytes = (kNaScalars + kNaPartials) * sizeof(double) + kNaStatus * sizeof(int);
constexpr int kNaMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNaBytes];

static std::mutex g_na_mutex;
static void* g_na_ptr[kNaMaxDevices] = {};

// the device address of this device's copy of ``scratch``, looked up once per device (that device current)
static hipError_t noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_na_mutex);
  if (!g_na_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_na_ptr[dev] = ptr;
  }
  *out = g_na_ptr[dev];
  return hipSuccess;
}

qgw_status qgw_dyson_G_noalloc(qgw_plan h, const void* H_k, const void* Sig_iw, double n_target, double* mu,
                               void* G_iw, void* stream) {
  QGW_PLAN(h, "qgw_dyson_G_noalloc");
  QGW_REQUIRE(H_k && G_iw && mu, QGW_ERR_INVALID_ARG, "qgw_dyson_G_noalloc: null argument");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_dyson_G_noalloc: the Dyson G solve is FP64");
  QGW_REQUIRE(p.device >= 0 && p.device < kNaMaxDevices, QGW_ERR_UNSUPPORTED,
              "qgw_dyson_G_noalloc: device ordinal beyond the static scratch table");
  if (!std::isnan(n_target))
    QGW_REQUIRE(n_target > 0.0 && n_target < 2.0 * p.no, QGW_ERR_INVALID_ARG,
                "qgw_dyson_G_noalloc: target filling must lie in (0, 2 n_o)");
  else
    QGW_REQUIRE(std::isfinite(*mu), QGW_ERR_INVALID_ARG, "qgw_dyson_G_noalloc: fixed mu must be finite");
  const int need = dyson_g_partials_needed(p);
  QGW_REQUIRE(need <= kNaPartials, QGW_ERR_UNSUPPORTED,
              "qgw_dyson_G_noalloc: the search needs " + std::to_string(need) +
                  " partial sums; the static scratch holds " + std::to_string(kNaPartials));
  void* base = nullptr;
  QGW_CHECK_HIP(noalloc_scratch(p.device, &base), "qgw_dyson_G_noalloc: scratch address");
  double* scal = (double*)base;
  double* part = scal + kNaScalars;
  int* stat = (int*)(part + kNaPartials);
  // every word the search reads is written first (scalars from the host, status by the start or a clear), so
  // the previous call's contents need no clearing; calls that overlap on one GPU race on the array
  return run_dyson_g(p, H_k, Sig_iw, n_target, mu, G_iw, (hipStream_t)stream, nullptr, scal, part, stat);
}

// ------------------------------------------------------------------ adjoints

// bytes of caller-provided scratch each call needs on plan p (0: none)
static int64_t workspace_need(const Plan& p, int op) {
  const int64_t so = int64_t(p.no) * p.no * p.nk * int64_t(sizeof(zd));  // static orbital array
  const int64_t se = int64_t(p.no) * p.nk * int64_t(sizeof(double));     // one energy per band and k
  const int64_t fo = so * p.r;                                           // orbital array with nodes
  switch (op) {
    case QGW_OP_SIGMA_BWD:
      return fo;  // Sigma-bar(k) -> R
    case QGW_OP_DYSON_W_BWD:  // W^C and X = (I - V P)^{-H} Wbar per matrix, V-bar partials per chunk
      return (2 * int64_t(p.r) + (p.r < 8 ? p.r : 8)) * p.nb * p.nb * p.nk * int64_t(sizeof(zd));
    case QGW_OP_HARTREE_FOCK_BWD:
      return int64_t(p.nb) * p.nb * int64_t(sizeof(zd));  // V(q = 0)
    case QGW_OP_ENERGY:
      return 2 * so + fo + int64_t(2) * 4096 * int64_t(sizeof(double)) + 64;  // n, y, block partials, sums
    case QGW_OP_ENERGY_BWD:
      return 2 * so + 2 * fo;  // n, n-bar, y, y-bar
    case QGW_OP_HF_DENSITY:
      return so + se + 64 * int64_t(sizeof(double));  // eigenvectors, eigenvalues, search scalars, status
    case QGW_OP_QUASIPARTICLE:
      return 64;  // status flag
    default:
      return -1;
  }
}

// the caller's scratch for op: non-null and at least the size qgw_workspace_size reports
#define QGW_WORKSPACE(op, ws, ws_bytes, name)                                                          \
  do {                                                                                                 \
    const int64_t need_ = workspace_need(p, op);                                                      \
    QGW_REQUIRE(need_ == 0 || (ws && ws_bytes >= need_), QGW_ERR_INVALID_ARG,                          \
                std::string(name) + ": workspace of " + std::to_string(need_) + " bytes required (" +  \
                    std::to_string(ws ? ws_bytes : 0) + " given)");                                   \
  } while (0)

#define QGW_BWD_PLAN(h, name)                                                                        \
  QGW_PLAN(h, name);                                                                                 \
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, std::string(name) + ": adjoints need an FP64 plan"); \
  QGW_REQUIRE(p.grid == kGridDLR, QGW_ERR_UNSUPPORTED, std::string(name) + ": adjoints need a DLR plan")

qgw_status qgw_dlr_transform_bwd(qgw_plan h, int32_t map, int64_t ncols, double sre, double sim,
                                 int32_t hermitian, const void* ybar, void* xbar, void* stream) {
  QGW_BWD_PLAN(h, "qgw_dlr_transform_bwd");
  QGW_REQUIRE(map >= 0 && map < kNumMaps, QGW_ERR_INVALID_ARG, "qgw_dlr_transform_bwd: bad map");
  QGW_REQUIRE(ncols >= 0, QGW_ERR_INVALID_ARG, "qgw_dlr_transform_bwd: negative ncols");
  if (ncols == 0) return QGW_OK;
  QGW_REQUIRE(ybar && xbar && ybar != xbar, QGW_ERR_INVALID_ARG, "qgw_dlr_transform_bwd: need distinct arrays");
  QGW_REQUIRE(hermitian >= 0 && hermitian <= 2, QGW_ERR_INVALID_ARG, "qgw_dlr_transform_bwd: bad hermitian mode");
  QGW_REQUIRE(hermitian == 0 || ncols == int64_t(p.no) * p.no * p.nk, QGW_ERR_SHAPE,
              "qgw_dlr_transform_bwd: the Hermitian modes need ncols = n_o^2 N_k");
  hipStream_t s = (hipStream_t)stream;
  if (map == QGW_F_IW2BETA) {
    QGW_CHECK_HIP(launch_row_map_bwd(p, ncols, sre, sim, hermitian, ybar, xbar, s), "qgw_dlr_transform_bwd");
    return QGW_OK;
  }
  // y = herm_out(s T herm_in(x)): xbar = herm_in(conj(s) T^H herm_out(ybar))
  const int hb = hermitian == 1 ? 2 : (hermitian == 2 ? 1 : 0);
  QGW_CHECK_HIP(launch_dlr(p, kAdjMap0 + map, ncols, sre, -sim, ybar, xbar, s, hb), "qgw_dlr_transform_bwd");
  return QGW_OK;
}

qgw_status qgw_dlr_transform_pairs_bwd(qgw_plan h, int32_t map, int32_t in_layout, int32_t out_layout,
                                       const void* ybar, void* xbar, void* stream) {
  QGW_BWD_PLAN(h, "qgw_dlr_transform_pairs_bwd");
  QGW_REQUIRE(map >= 0 && map < 5, QGW_ERR_INVALID_ARG, "qgw_dlr_transform_pairs_bwd: bad map");
  QGW_REQUIRE((in_layout == 0 || in_layout == 1) && (out_layout == 0 || out_layout == 1), QGW_ERR_INVALID_ARG,
              "qgw_dlr_transform_pairs_bwd: bad layout");
  QGW_REQUIRE(ybar && xbar && ybar != xbar, QGW_ERR_INVALID_ARG, "qgw_dlr_transform_pairs_bwd: need distinct arrays");
  QGW_CHECK_HIP(launch_dlr_pairs(p, kAdjMap0 + map, out_layout, in_layout, ybar, xbar, (hipStream_t)stream),
                "qgw_dlr_transform_pairs_bwd");
  return QGW_OK;
}

qgw_status qgw_lattice_fft_bwd(qgw_plan h, int32_t dir, int64_t batch, const void* ybar, void* xbar,
                               void* stream) {
  QGW_BWD_PLAN(h, "qgw_lattice_fft_bwd");
  QGW_REQUIRE(dir == QGW_R_TO_K || dir == QGW_K_TO_R, QGW_ERR_INVALID_ARG, "qgw_lattice_fft_bwd: bad direction");
  QGW_REQUIRE(batch >= 0, QGW_ERR_INVALID_ARG, "qgw_lattice_fft_bwd: negative batch");
  if (batch == 0) return QGW_OK;
  QGW_REQUIRE(ybar && xbar, QGW_ERR_INVALID_ARG, "qgw_lattice_fft_bwd: null array");
  // adjoint of k -> R (1/N_k, e^{+ik.R}) is e^{-ik.R} with 1/N_k; of R -> k it is e^{+ik.R} unscaled
  const int sign = dir == QGW_K_TO_R ? -1 : +1;
  const double sc = dir == QGW_K_TO_R ? 1.0 / double(p.nk) : 1.0;
  QGW_CHECK_HIP(launch_lattice_fft_scaled(p, sign, sc, batch, ybar, xbar, (hipStream_t)stream),
                "qgw_lattice_fft_bwd");
  return QGW_OK;
}

qgw_status qgw_bubble_bwd(qgw_plan h, const void* gt, const void* gr, const void* Pbar_q, void* Gbar_tau,
                          void* Gbar_reflt, void* stream) {
  QGW_BWD_PLAN(h, "qgw_bubble_bwd");
  QGW_REQUIRE(gt && gr && Pbar_q && Gbar_tau && Gbar_reflt, QGW_ERR_INVALID_ARG, "qgw_bubble_bwd: null array");
  QGW_REQUIRE(Gbar_tau != Gbar_reflt && Gbar_tau != gt && Gbar_tau != gr && Gbar_reflt != gt && Gbar_reflt != gr,
              QGW_ERR_INVALID_ARG, "qgw_bubble_bwd: outputs alias inputs");
  hipStream_t s = (hipStream_t)stream;
  QGW_CHECK_HIP(launch_contract_bwd(p, 1, Pbar_q, gr, Gbar_tau, s), "qgw_bubble_bwd");
  QGW_CHECK_HIP(launch_contract_bwd(p, 2, Pbar_q, gt, Gbar_reflt, s), "qgw_bubble_bwd");
  return QGW_OK;
}

qgw_status qgw_sigma_bwd(qgw_plan h, const void* gt, const void* wc_q, int32_t out_k, const void* Sigbar,
                         void* Gbar_tau, void* Wcbar_q, void* workspace, int64_t workspace_bytes, void* stream) {
  QGW_BWD_PLAN(h, "qgw_sigma_bwd");
  QGW_REQUIRE(gt && wc_q && Sigbar && Gbar_tau && Wcbar_q, QGW_ERR_INVALID_ARG, "qgw_sigma_bwd: null array");
  QGW_REQUIRE(Gbar_tau != gt && Wcbar_q != wc_q && Gbar_tau != Wcbar_q, QGW_ERR_INVALID_ARG,
              "qgw_sigma_bwd: outputs alias inputs");
  hipStream_t s = (hipStream_t)stream;
  const void* sbar_r = Sigbar;
  if (out_k) {
    QGW_WORKSPACE(QGW_OP_SIGMA_BWD, workspace, workspace_bytes, "qgw_sigma_bwd");
    QGW_REQUIRE(workspace != gt && workspace != wc_q && workspace != Sigbar && workspace != Gbar_tau &&
                    workspace != Wcbar_q, QGW_ERR_INVALID_ARG, "qgw_sigma_bwd: workspace aliases an array");
    QGW_CHECK_HIP(launch_lattice_fft_scaled(p, +1, 1.0, int64_t(p.r) * p.no * p.no, Sigbar, workspace, s),
                  "qgw_sigma_bwd");
    sbar_r = workspace;
  }
  QGW_CHECK_HIP(launch_contract_bwd(p, 0, wc_q, sbar_r, Gbar_tau, s), "qgw_sigma_bwd");
  QGW_CHECK_HIP(launch_sigma_bwd_wc(p, gt, sbar_r, Wcbar_q, s), "qgw_sigma_bwd");
  return QGW_OK;
}

qgw_status qgw_dyson_W_bwd(qgw_plan h, const void* V_q, const void* P_nu, const void* Wcbar_nu, void* Pbar_nu,
                           void* Vbar_q, void* workspace, int64_t workspace_bytes, void* stream) {
  QGW_BWD_PLAN(h, "qgw_dyson_W_bwd");
  QGW_REQUIRE(V_q && P_nu && Wcbar_nu && Pbar_nu && Vbar_q, QGW_ERR_INVALID_ARG, "qgw_dyson_W_bwd: null array");
  QGW_REQUIRE(Pbar_nu != P_nu && Pbar_nu != Wcbar_nu && Vbar_q != V_q, QGW_ERR_INVALID_ARG,
              "qgw_dyson_W_bwd: outputs alias inputs");
  const int chunks = p.r < 8 ? p.r : 8;
  const int64_t nv = int64_t(p.nb) * p.nb * p.nk;
  QGW_WORKSPACE(QGW_OP_DYSON_W_BWD, workspace, workspace_bytes, "qgw_dyson_W_bwd");
  hipStream_t s = (hipStream_t)stream;
  QGW_CHECK_HIP(launch_dyson_w_bwd(p, V_q, P_nu, Wcbar_nu, Pbar_nu, workspace, chunks, s), "qgw_dyson_W_bwd");
  const zd* vpart = (const zd*)workspace + 2 * int64_t(p.r) * nv;
  QGW_CHECK_HIP(launch_sum_chunks(nv, chunks, vpart, Vbar_q, s), "qgw_dyson_W_bwd");
  return QGW_OK;
}

qgw_status qgw_hartree_fock_bwd(qgw_plan h, const void* V_R, const void* n_R, const void* Sbar_R, void* nbar_R,
                                void* Vbar_R, void* workspace, int64_t workspace_bytes, void* stream) {
  QGW_BWD_PLAN(h, "qgw_hartree_fock_bwd");
  QGW_REQUIRE(V_R && n_R && Sbar_R && (nbar_R || Vbar_R), QGW_ERR_INVALID_ARG, "qgw_hartree_fock_bwd: null array");
  QGW_WORKSPACE(QGW_OP_HARTREE_FOCK_BWD, workspace, workspace_bytes, "qgw_hartree_fock_bwd");
  hipStream_t s = (hipStream_t)stream;
  QGW_CHECK_HIP(launch_pair_sum_r(p, V_R, workspace, s), "qgw_hartree_fock_bwd");
  QGW_CHECK_HIP(launch_hartree_fock_bwd(p, V_R, workspace, n_R, Sbar_R, nbar_R, Vbar_R, s), "qgw_hartree_fock_bwd");
  return QGW_OK;
}

qgw_status qgw_dyson_G_bwd(qgw_plan h, const void* H_k, const void* Sig_iw, double mu, double n_target,
                           double mubar, const void* Gbar, void* Sigbar, void* Hbar, void* stream) {
  QGW_BWD_PLAN(h, "qgw_dyson_G_bwd");
  QGW_REQUIRE(H_k && Gbar && Sigbar, QGW_ERR_INVALID_ARG, "qgw_dyson_G_bwd: null array");
  QGW_REQUIRE(std::isfinite(mu), QGW_ERR_INVALID_ARG, "qgw_dyson_G_bwd: mu must be finite");
  QGW_REQUIRE(Sigbar != Gbar && Sigbar != H_k && Sigbar != Sig_iw, QGW_ERR_INVALID_ARG,
              "qgw_dyson_G_bwd: Sigbar aliases an input");
  hipStream_t s = (hipStream_t)stream;
  QGW_CHECK_HIP(launch_dyson_g_bwd(p, H_k, Sig_iw, mu, n_target, mubar, Gbar, Sigbar, s), "qgw_dyson_G_bwd");
  if (Hbar) QGW_CHECK_HIP(launch_sum_nodes(p, Sigbar, Hbar, s), "qgw_dyson_G_bwd");
  return QGW_OK;
}

// ---------------------------------------------------------------- energy

qgw_status qgw_energy(qgw_plan h, const void* H_k, const void* SigHF_k, const void* Sig_iw, const void* G_iw,
                      double* e_out, void* workspace, int64_t workspace_bytes, void* stream) {
  QGW_BWD_PLAN(h, "qgw_energy");
  QGW_REQUIRE(H_k && SigHF_k && Sig_iw && G_iw && e_out, QGW_ERR_INVALID_ARG, "qgw_energy: null argument");
  const size_t so = size_t(p.no) * p.no * p.nk * sizeof(zd);
  const size_t fo = so * p.r;
  QGW_WORKSPACE(QGW_OP_ENERGY, workspace, workspace_bytes, "qgw_energy");
  char* ws = (char*)workspace;
  void* n_k = ws;
  void* y = ws + 2 * so;
  double* part = (double*)(ws + 2 * so + fo);
  double* sums = part + 2 * 4096;
  hipStream_t s = (hipStream_t)stream;
  const int64_t ncol = int64_t(p.no) * p.no * p.nk;
  QGW_CHECK_HIP(launch_dlr(p, QGW_F_IW2BETA, ncol, -1.0, 0.0, G_iw, n_k, s, 2), "qgw_energy");
  QGW_CHECK_HIP(launch_dlr(p, QGW_F_IW2GM, ncol, 1.0, 0.0, Sig_iw, y, s), "qgw_energy");
  QGW_CHECK_HIP(launch_energy_sums(p, H_k, SigHF_k, n_k, y, G_iw, part, sums, s), "qgw_energy");
  double host[2];
  QGW_CHECK_HIP(hipMemcpyAsync(host, sums, sizeof(host), hipMemcpyDeviceToHost, s), "qgw_energy");
  QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_energy");
  const double e_hf = 2.0 / double(p.nk) * host[0];
  const double e_c = host[1] / double(p.nk);
  e_out[0] = e_hf + e_c;
  e_out[1] = e_hf;
  e_out[2] = e_c;
  return QGW_OK;
}

qgw_status qgw_energy_bwd(qgw_plan h, const void* H_k, const void* SigHF_k, const void* Sig_iw, const void* G_iw,
                          double ebar, void* Hbar, void* SigHFbar, void* Sigbar, void* Gbar, void* workspace,
                          int64_t workspace_bytes, void* stream) {
  QGW_BWD_PLAN(h, "qgw_energy_bwd");
  QGW_REQUIRE(H_k && SigHF_k && Sig_iw && G_iw && Hbar && SigHFbar && Sigbar && Gbar, QGW_ERR_INVALID_ARG,
              "qgw_energy_bwd: null argument");
  QGW_REQUIRE(Gbar != G_iw && Sigbar != Sig_iw && Sigbar != Gbar, QGW_ERR_INVALID_ARG,
              "qgw_energy_bwd: outputs alias inputs");
  const size_t so = size_t(p.no) * p.no * p.nk * sizeof(zd);
  const size_t fo = so * p.r;
  QGW_WORKSPACE(QGW_OP_ENERGY_BWD, workspace, workspace_bytes, "qgw_energy_bwd");
  char* ws = (char*)workspace;
  void* n_k = ws;
  void* nbar = ws + so;
  void* y = ws + 2 * so;
  void* ybar = ws + 2 * so + fo;
  hipStream_t s = (hipStream_t)stream;
  const int64_t ncol = int64_t(p.no) * p.no * p.nk;
  QGW_CHECK_HIP(launch_dlr(p, QGW_F_IW2BETA, ncol, -1.0, 0.0, G_iw, n_k, s, 2), "qgw_energy_bwd");
  QGW_CHECK_HIP(launch_dlr(p, QGW_F_IW2GM, ncol, 1.0, 0.0, Sig_iw, y, s), "qgw_energy_bwd");
  QGW_CHECK_HIP(launch_energy_bwd_static(p, H_k, SigHF_k, n_k, 2.0 * ebar / double(p.nk), Hbar, SigHFbar, nbar, s),
                "qgw_energy_bwd");
  QGW_CHECK_HIP(launch_row_map_bwd(p, ncol, -1.0, 0.0, 2, nbar, Gbar, s), "qgw_energy_bwd");
  QGW_CHECK_HIP(launch_energy_bwd_nodes(p, y, G_iw, ebar / double(p.nk), Gbar, ybar, s), "qgw_energy_bwd");
  QGW_CHECK_HIP(launch_dlr(p, kAdjMap0 + QGW_F_IW2GM, ncol, 1.0, 0.0, ybar, Sigbar, s), "qgw_energy_bwd");
  return QGW_OK;
}

// ----------------------------------------------------------- Hartree-Fock

qgw_status qgw_hf_density(qgw_plan h, const void* H_k, double n_target, double* mu, void* n_k, void* workspace,
                          int64_t workspace_bytes, void* stream) {
  QGW_PLAN(h, "qgw_hf_density");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_hf_density: FP64 plans only");
  QGW_REQUIRE(H_k && mu && n_k, QGW_ERR_INVALID_ARG, "qgw_hf_density: null argument");
  if (!std::isnan(n_target))
    QGW_REQUIRE(n_target > 0.0 && n_target < 2.0 * p.no, QGW_ERR_INVALID_ARG,
                "qgw_hf_density: target filling must lie in (0, 2 n_o)");
  else
    QGW_REQUIRE(std::isfinite(*mu), QGW_ERR_INVALID_ARG, "qgw_hf_density: fixed mu must be finite");
  const size_t so = size_t(p.no) * p.no * p.nk * sizeof(zd);
  const size_t se = size_t(p.no) * p.nk * sizeof(double);
  QGW_WORKSPACE(QGW_OP_HF_DENSITY, workspace, workspace_bytes, "qgw_hf_density");
  char* ws = (char*)workspace;
  double* scal = (double*)(ws + so + se);
  int* stat = (int*)(scal + 16);
  hipStream_t s = (hipStream_t)stream;
  double sc[2] = {*mu, n_target};
  QGW_CHECK_HIP(hipMemcpyAsync(scal, sc, sizeof(sc), hipMemcpyHostToDevice, s), "qgw_hf_density");
  QGW_CHECK_HIP(launch_hf_density(p, H_k, scal, stat, ws, (double*)(ws + so), n_k, s), "qgw_hf_density");
  double res[4];
  int bad = 0;
  QGW_CHECK_HIP(hipMemcpyAsync(res, scal, sizeof(res), hipMemcpyDeviceToHost, s), "qgw_hf_density");
  QGW_CHECK_HIP(hipMemcpyAsync(&bad, stat, sizeof(int), hipMemcpyDeviceToHost, s), "qgw_hf_density");
  QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_hf_density");
  QGW_REQUIRE(bad == 0, QGW_ERR_NONFINITE, "qgw_hf_density: non-finite chemical potential or filling");
  *mu = res[0];
  return QGW_OK;
}

qgw_status qgw_state_hf_solve(qgw_state st, double tol, int32_t max_iter, int32_t* iters_done, double* d_sigma,
                              double* mu_out, void* stream) {
  QGW_REQUIRE(st, QGW_ERR_INVALID_ARG, "qgw_state_hf_solve: null state");
  QGW_REQUIRE(max_iter >= 0, QGW_ERR_INVALID_ARG, "qgw_state_hf_solve: negative max_iter");
  qgw_plan h = st->plan;
  const Plan& p = h->p;
  QGW_CHECK_HIP(enter_device(p.device), "hipSetDevice");
  if (std::isnan(st->n_target))
    QGW_REQUIRE(std::isfinite(st->mu), QGW_ERR_INVALID_ARG, "qgw_state_hf_solve: fixed mu must be finite");
  const int64_t so_n = int64_t(p.no) * p.no * p.nk;
  const size_t so = size_t(so_n) * sizeof(zd);
  const size_t se = size_t(p.no) * p.nk * sizeof(double);
  st->broken = true;  // until the solve has left a consistent state
  void* u = st->hf_ws;
  double* eps = (double*)((char*)st->hf_ws + so);
  hipStream_t s = (hipStream_t)stream;
  // start: Sigma_HF = 0 and the density of H0 at the target filling (or at the state's mu)
  QGW_CHECK_HIP(hipMemsetAsync(st->SigHF_k, 0, so, s), "qgw_state_hf_solve");
  QGW_CHECK_HIP(hipMemsetAsync(st->SigHF_old, 0, so, s), "qgw_state_hf_solve");
  double sc[2] = {st->mu, st->n_target};
  QGW_CHECK_HIP(hipMemcpyAsync(st->d_scal, sc, sizeof(sc), hipMemcpyHostToDevice, s), "qgw_state_hf_solve");
  QGW_CHECK_HIP(launch_hf_density(p, st->H_k, st->d_scal, st->d_stat, u, eps, st->n_k, s), "qgw_state_hf_solve");
  double res[4] = {};
  double dsig = NAN;
  int bad = 0, done = 0;
  for (int it = 0; it < max_iter; ++it) {
    // SigH + SigF from n, the change and mixing, H = H0 + Sigma_HF, then mu and n (H class)
    QGW_CHECK_HIP(launch_lattice_fft(p, QGW_K_TO_R, int64_t(p.no) * p.no, st->n_k, st->n_R, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(launch_hartree_fock(p, st->V_R, st->V_q0, st->n_R, st->SigHF_R, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(launch_lattice_fft(p, QGW_R_TO_K, int64_t(p.no) * p.no, st->SigHF_R, st->SigHF_k, s),
                  "qgw_state_hf_solve");
    QGW_CHECK_HIP(launch_hf_delta_mix(p, st->SigHF_k, st->SigHF_old, st->mixing, st->d_dsig, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(launch_add(p, so_n, st->H_k, st->SigHF_k, st->Hs_k, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(launch_hf_density(p, st->Hs_k, st->d_scal, st->d_stat, u, eps, st->n_k, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(hipMemcpyAsync(&dsig, st->d_dsig, sizeof(double), hipMemcpyDeviceToHost, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(hipMemcpyAsync(res, st->d_scal, sizeof(res), hipMemcpyDeviceToHost, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(hipMemcpyAsync(&bad, st->d_stat, sizeof(int), hipMemcpyDeviceToHost, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_state_hf_solve");
    ++done;
    QGW_REQUIRE(bad == 0, QGW_ERR_NONFINITE, "qgw_state_hf_solve: non-finite chemical potential or filling");
    QGW_REQUIRE(std::isfinite(dsig), QGW_ERR_NONFINITE, "qgw_state_hf_solve: non-finite Hartree-Fock self-energy");
    if (dsig <= tol) break;
  }
  if (done == 0) {
    QGW_CHECK_HIP(hipMemcpyAsync(res, st->d_scal, sizeof(res), hipMemcpyDeviceToHost, s), "qgw_state_hf_solve");
    QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_state_hf_solve");
  }
  st->mu = res[0];
  // G = [(i w + mu) - H0 - Sigma_HF]^{-1} with Sigma^C = 0, so that a GW solve can continue from HF
  QGW_CHECK_HIP(hipMemsetAsync(st->Sig_iw, 0, so * p.r, s), "qgw_state_hf_solve");
  QGW_CHECK_HIP(hipMemsetAsync(st->Sig_iw_old, 0, so * p.r, s), "qgw_state_hf_solve");
  QGW_CHECK_HIP(launch_add(p, so_n, st->H_k, st->SigHF_k, st->Hs_k, s), "qgw_state_hf_solve");
  QGW_CHECK_HIP(launch_dyson_g_final(p, st->Hs_k, nullptr, 0, st->G_iw, st->d_scal, st->d_part, st->d_stat, s),
                "qgw_state_hf_solve");
  // the next GW search starts from the HF mu: no shift from a mean level of before the HF solve
  const double nan_word = NAN;
  QGW_CHECK_HIP(hipMemcpyAsync(st->d_scal + 10, &nan_word, sizeof(double), hipMemcpyHostToDevice, s),
                "qgw_state_hf_solve");
  QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_state_hf_solve");
  st->last_dsig = INFINITY;
  st->broken = false;
  if (iters_done) *iters_done = done;
  if (d_sigma) *d_sigma = dsig;
  if (mu_out) *mu_out = st->mu;
  return QGW_OK;
}

// ---------------------------------------------------------- quasiparticle

qgw_status qgw_quasiparticle(qgw_plan h, const void* H_k, const void* SigHF_k, const void* Sig_iw, double mu,
                             void* Sig0, void* Z, void* Hqp, double* bands, void* workspace, int64_t workspace_bytes,
                             void* stream) {
  QGW_PLAN(h, "qgw_quasiparticle");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_quasiparticle: FP64 plans only");
  QGW_REQUIRE(H_k && SigHF_k && Sig_iw && Sig0 && Z && Hqp && bands, QGW_ERR_INVALID_ARG,
              "qgw_quasiparticle: null argument");
  QGW_REQUIRE(std::isfinite(mu), QGW_ERR_INVALID_ARG, "qgw_quasiparticle: mu must be finite");
  QGW_WORKSPACE(QGW_OP_QUASIPARTICLE, workspace, workspace_bytes, "qgw_quasiparticle");
  int* flag = (int*)workspace;
  hipStream_t s = (hipStream_t)stream;
  QGW_CHECK_HIP(hipMemsetAsync(flag, 0, sizeof(int), s), "qgw_quasiparticle");
  QGW_CHECK_HIP(launch_quasiparticle(p, H_k, SigHF_k, Sig_iw, mu, Sig0, Z, Hqp, bands, flag, s),
                "qgw_quasiparticle");
  int bad = 0;
  QGW_CHECK_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s), "qgw_quasiparticle");
  QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_quasiparticle");
  QGW_REQUIRE(bad == 0, QGW_ERR_NONFINITE, "qgw_quasiparticle: Z(k)^{-1} is not positive definite at some k");
  return QGW_OK;
}

static int64_t qp_path_bytes(const Plan& p, int64_t npt) {
  const int64_t nab = int64_t(p.no) * p.no;
  return 256 + 16 * nab * (4 * int64_t(p.nk) + 3 * npt) + 8 * int64_t(p.dim) * npt;
}

qgw_status qgw_quasiparticle_path_workspace(qgw_plan h, int32_t n_path, int64_t* bytes) {
  QGW_REQUIRE(h && bytes, QGW_ERR_INVALID_ARG, "qgw_quasiparticle_path_workspace: null argument");
  QGW_REQUIRE(n_path >= 1 && n_path <= 65536, QGW_ERR_INVALID_ARG,
              "qgw_quasiparticle_path_workspace: n_path must be in [1, 65536]");
  *bytes = qp_path_bytes(h->p, n_path);
  return QGW_OK;
}

qgw_status qgw_quasiparticle_path(qgw_plan h, const void* H_k, const void* SigHF_k, const void* Sig_iw, double mu,
                                  const double* kfrac, int32_t n_path, void* Sig0, void* Z, void* Hqp, double* bands,
                                  void* workspace, int64_t workspace_bytes, void* stream) {
  QGW_PLAN(h, "qgw_quasiparticle_path");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_quasiparticle_path: FP64 plans only");
  QGW_REQUIRE(H_k && SigHF_k && Sig_iw && kfrac && Sig0 && Z && Hqp && bands && workspace, QGW_ERR_INVALID_ARG,
              "qgw_quasiparticle_path: null argument");
  QGW_REQUIRE(std::isfinite(mu), QGW_ERR_INVALID_ARG, "qgw_quasiparticle_path: mu must be finite");
  QGW_REQUIRE(n_path >= 1 && n_path <= 65536, QGW_ERR_INVALID_ARG,
              "qgw_quasiparticle_path: n_path must be in [1, 65536]");
  QGW_REQUIRE(workspace_bytes >= qp_path_bytes(p, n_path), QGW_ERR_INVALID_ARG,
              "qgw_quasiparticle_path: workspace needs " + std::to_string(qp_path_bytes(p, n_path)) + " bytes");
  const int64_t nf = int64_t(n_path) * p.dim;
  for (int64_t i = 0; i < nf; ++i)
    QGW_REQUIRE(std::isfinite(kfrac[i]), QGW_ERR_NONFINITE, "qgw_quasiparticle_path: non-finite kfrac");
  // [flag | pad to 256][S_k, X_R (3), X_path (3)][kfrac]
  int* flag = (int*)workspace;
  char* base = (char*)workspace + 256;
  const int64_t nab = int64_t(p.no) * p.no;
  double* d_kf = (double*)(base + 16 * nab * (4 * int64_t(p.nk) + 3 * int64_t(n_path)));
  hipStream_t s = (hipStream_t)stream;
  QGW_CHECK_HIP(hipMemsetAsync(flag, 0, sizeof(int), s), "qgw_quasiparticle_path");
  QGW_CHECK_HIP(hipMemcpyAsync(d_kf, kfrac, size_t(nf) * sizeof(double), hipMemcpyHostToDevice, s),
                "qgw_quasiparticle_path");
  QGW_CHECK_HIP(launch_quasiparticle_path(p, H_k, SigHF_k, Sig_iw, d_kf, n_path, mu, base, Sig0, Z, Hqp, bands,
                                          flag, s),
                "qgw_quasiparticle_path");
  int bad = 0;
  QGW_CHECK_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s), "qgw_quasiparticle_path");
  QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_quasiparticle_path");
  QGW_REQUIRE(bad == 0, QGW_ERR_NONFINITE,
              "qgw_quasiparticle_path: Z(k')^{-1} is not positive definite at some path point");
  return QGW_OK;
}

qgw_status qgw_add(qgw_plan h, int64_t count, const void* a, const void* b, void* out, void* stream) {
  QGW_PLAN(h, "qgw_add");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_add: FP64 plans only");
  QGW_REQUIRE(count >= 0, QGW_ERR_INVALID_ARG, "qgw_add: negative count");
  if (count == 0) return QGW_OK;
  QGW_REQUIRE(a && b && out, QGW_ERR_INVALID_ARG, "qgw_add: null array");
  QGW_CHECK_HIP(launch_add(p, count, a, b, out, (hipStream_t)stream), "qgw_add");
  return QGW_OK;
}

qgw_status qgw_pair_layout(qgw_plan h, int32_t in_layout, int32_t out_layout, int64_t nn, const void* in, void* out,
                           void* stream) {
  QGW_PLAN(h, "qgw_pair_layout");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_pair_layout: FP64 plans only");
  QGW_REQUIRE((in_layout == 0 && out_layout == 1) || (in_layout == 1 && out_layout == 0), QGW_ERR_INVALID_ARG,
              "qgw_pair_layout: layouts must differ");
  QGW_REQUIRE(nn >= 0, QGW_ERR_INVALID_ARG, "qgw_pair_layout: negative count");
  if (nn == 0) return QGW_OK;
  QGW_REQUIRE(in && out && in != out, QGW_ERR_INVALID_ARG, "qgw_pair_layout: need distinct arrays");
  QGW_CHECK_HIP(launch_pair_layout(p, out_layout == 1 ? 1 : 0, nn, in, out, (hipStream_t)stream), "qgw_pair_layout");
  return QGW_OK;
}

qgw_status qgw_check_finite(qgw_plan h, const void* x, int64_t count, void* stream) {
  QGW_PLAN(h, "qgw_check_finite");
  QGW_REQUIRE(x || count == 0, QGW_ERR_INVALID_ARG, "qgw_check_finite: null array");
  QGW_REQUIRE(count >= 0, QGW_ERR_INVALID_ARG, "qgw_check_finite: negative count");
  hipStream_t s = (hipStream_t)stream;
  int zero = 0, cnt = 0;
  QGW_CHECK_HIP(hipMemcpyAsync(p.d_status + 8, &zero, sizeof(int), hipMemcpyHostToDevice, s), "qgw_check_finite");
  QGW_CHECK_HIP(launch_count_nonfinite(p, x, count, p.d_status + 8, s), "qgw_check_finite");
  QGW_CHECK_HIP(hipMemcpyAsync(&cnt, p.d_status + 8, sizeof(int), hipMemcpyDeviceToHost, s), "qgw_check_finite");
  QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_check_finite");
  if (cnt) {
    set_error("qgw_check_finite: " + std::to_string(cnt) + " non-finite values");
    return QGW_ERR_NONFINITE;
  }
  return QGW_OK;
}

qgw_status qgw_workspace_size(qgw_plan h, int32_t op, int64_t* bytes) {
  QGW_REQUIRE(h && bytes, QGW_ERR_INVALID_ARG, "qgw_workspace_size: null argument");
  const int64_t b = workspace_need(h->p, op);
  QGW_REQUIRE(b >= 0, QGW_ERR_INVALID_ARG, "qgw_workspace_size: unknown operation " + std::to_string(op));
  *bytes = b;
  return QGW_OK;
}

// reads and clears the plan's device condition word once the stream has drained
static qgw_status take_conditions(const Plan& p, hipStream_t s, int* flags) {
  int host = 0;
  const int zero = 0;
  QGW_CHECK_HIP(hipMemcpyAsync(&host, p.d_status + kCondWord, sizeof(int), hipMemcpyDeviceToHost, s), "qgw_sync_status");
  QGW_CHECK_HIP(hipMemcpyAsync(p.d_status + kCondWord, &zero, sizeof(int), hipMemcpyHostToDevice, s), "qgw_sync_status");
  QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_sync_status");
  *flags = host;
  return QGW_OK;
}

qgw_status qgw_sync_status(qgw_plan h, void* stream) {
  QGW_PLAN(h, "qgw_sync_status");
  int flags = 0;
  const qgw_status rc = take_conditions(p, (hipStream_t)stream, &flags);
  if (rc != QGW_OK) return rc;
  QGW_REQUIRE(!(flags & kCondSingular), QGW_ERR_SINGULAR,
              "qgw_sync_status: a Dyson-W system I - V P had a zero or non-finite pivot");
  return QGW_OK;
}

// ------------------------------------------------------------------ state

static void free_state(qgw_state st) {
  for (auto& set : st->ev)
    for (auto& e : set)
      if (e) (void)hipEventDestroy(e);
  if (st->ev_io) (void)hipEventDestroy(st->ev_io);
  for (auto& e : st->ev_a12)
    if (e) (void)hipEventDestroy(e);
  if (st->ev_fork) (void)hipEventDestroy(st->ev_fork);
  if (st->ev_join) (void)hipEventDestroy(st->ev_join);
  if (st->side) (void)hipStreamDestroy(st->side);
  if (st->h_io) (void)hipHostFree(st->h_io);
  void* ptrs[] = {st->H_k, st->V_R, st->V_q, st->V_qm, st->V_q0, st->G_iw, st->Sig_iw, st->Sig_iw_old,
                  st->SigHF_k, st->SigHF_old, st->n_k, st->n_R, st->SigHF_R, st->Hs_k, st->G_tau,
                  st->G_reflt, st->Sig_tau_k, st->Pq, st->P_nu, st->Wc_nu, st->d_dsig, st->d_blockmax,
                  st->G32, st->Gt32, st->Gr32, st->St32, st->Siw32, st->Pq32, st->Pnu32, st->Wc32,
                  st->Vqm32, st->d_scal, st->d_part, st->d_stat, st->hf_ws};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
}

// buffers of the single-precision phase, allocated when first needed
static hipError_t ensure_fp32(qgw_state st) {
  if (st->has32) return hipSuccess;
  const Plan& p = st->plan->p;
  const size_t so = size_t(p.no) * p.no * p.nk * 8;
  const size_t sp = size_t(p.nb) * p.nb * p.nk * 8;
  const size_t fo = so * p.r, fp = sp * p.r;
  struct {
    void** ptr;
    size_t bytes;
  } allocs[] = {{&st->G32, fo},  {&st->Gt32, fo},  {&st->Gr32, fo},  {&st->St32, fo}, {&st->Siw32, fo},
                {&st->Pq32, fp}, {&st->Pnu32, fp}, {&st->Wc32, size_t(state_w_ld(p)) * p.nk * 8 * p.r},
                {&st->Vqm32, sp}};
  hipError_t e = hipSuccess;
  for (auto& a : allocs) {
    if (e != hipSuccess) break;
    if (!*a.ptr) e = hipMalloc(a.ptr, a.bytes);
  }
  if (e == hipSuccess) e = launch_convert(int64_t(p.nb) * p.nb * p.nk, st->V_qm, st->Vqm32, 1, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e == hipSuccess) st->has32 = true;
  return e;
}

qgw_status qgw_state_create(qgw_plan h, const void* H0_R, const void* V_R, double n_target, double mixing,
                            qgw_state* out) {
  QGW_PLAN(h, "qgw_state_create");
  QGW_REQUIRE(out && H0_R && V_R, QGW_ERR_INVALID_ARG, "qgw_state_create: null argument");
  QGW_REQUIRE(p.prec == 0, QGW_ERR_UNSUPPORTED, "qgw_state_create: FP64 plans only");
  QGW_REQUIRE(mixing > 0.0 && mixing <= 1.0, QGW_ERR_INVALID_ARG, "qgw_state_create: mixing must be in (0, 1]");
  if (!std::isnan(n_target))
    QGW_REQUIRE(n_target > 0.0 && n_target < 2.0 * p.no, QGW_ERR_INVALID_ARG,
                "qgw_state_create: target filling must lie in (0, 2 n_o)");
  *out = nullptr;
  qgw_state st = new (std::nothrow) qgw_state_s;
  QGW_REQUIRE(st, QGW_ERR_ALLOC, "qgw_state_create: out of host memory");
  st->plan = h;
  st->n_target = n_target;
  st->mixing = mixing;
  const size_t so = size_t(p.no) * p.no * p.nk * 16;         // static orbital
  const size_t sp = size_t(p.nb) * p.nb * p.nk * 16;         // static pair
  const size_t fo = so * p.r;                                // fermionic orbital
  const size_t fp = sp * p.r;                                // pair with nodes
  const size_t fw = size_t(state_w_ld(p)) * p.nk * 16 * p.r;  // W^C: matrix rows padded to whole lines
  hipError_t e = hipSuccess;
  struct {
    void** ptr;
    size_t bytes;
  } allocs[] = {{&st->H_k, so},       {&st->V_R, sp},     {&st->V_q, sp},        {&st->V_qm, sp},
                {&st->V_q0, size_t(p.nb) * p.nb * 16},    {&st->G_iw, fo},       {&st->Sig_iw, fo},
                {&st->Sig_iw_old, fo}, {&st->SigHF_k, so}, {&st->SigHF_old, so},  {&st->n_k, so},
                {&st->n_R, so},       {&st->SigHF_R, so}, {&st->Hs_k, so},       {&st->G_tau, fo},
                {&st->G_reflt, fo},   {&st->Sig_tau_k, fo}, {&st->Pq, fp},       {&st->P_nu, fp},
                {&st->Wc_nu, fw},     {(void**)&st->d_dsig, 64}, {(void**)&st->d_blockmax, 8192 * sizeof(double)},
                {(void**)&st->d_scal, 32 * sizeof(double)},
                {(void**)&st->d_part, size_t(8) * p.max_blocks * sizeof(double)},
                {(void**)&st->d_stat, 16 * sizeof(int)},
                {&st->hf_ws, so + size_t(p.no) * p.nk * sizeof(double)}};
  for (auto& a : allocs) {
    if (e != hipSuccess) break;
    e = hipMalloc(a.ptr, a.bytes);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&st->h_io, 32 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&st->ev_io, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&st->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&st->ev_join, hipEventDisableTiming);
  st->p32 = p;
  st->p32.prec = QGW_F32;
  hipStream_t s = nullptr;
  if (e == hipSuccess) e = hipMemcpyAsync(st->V_R, V_R, sp, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_lattice_fft(p, QGW_R_TO_K, int64_t(p.no) * p.no, H0_R, st->H_k, s);
  if (e == hipSuccess) e = launch_lattice_fft(p, QGW_R_TO_K, int64_t(p.nb) * p.nb, V_R, st->V_q, s);
  if (e == hipSuccess) e = launch_slab_to_matrix_static(p, st->V_q, st->V_qm, s);
  if (e == hipSuccess) e = launch_pair_sum_r(p, V_R, st->V_q0, s);
  if (e == hipSuccess) {
    double sc[16];
    for (double& v : sc) v = NAN;
    sc[1] = n_target;
    e = hipMemcpy(st->d_scal, sc, sizeof(sc), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(st->d_stat, 0, 16 * sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(st->Sig_iw, 0, fo, s);
  if (e == hipSuccess) e = hipMemsetAsync(st->Sig_iw_old, 0, fo, s);
  if (e == hipSuccess) e = hipMemsetAsync(st->SigHF_k, 0, so, s);
  if (e == hipSuccess) e = hipMemsetAsync(st->SigHF_old, 0, so, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error(std::string("qgw_state_create: ") + hipGetErrorString(e));
    free_state(st);
    delete st;
    return QGW_ERR_DEVICE;
  }
  *out = st;
  return QGW_OK;
}

qgw_status qgw_state_destroy(qgw_state st) {
  if (!st) return QGW_OK;
  (void)hipSetDevice(st->plan->p.device);
  free_state(st);
  delete st;
  return QGW_OK;
}

qgw_status qgw_state_init_g0(qgw_state st, double* mu, void* stream) {
  QGW_REQUIRE(st && mu, QGW_ERR_INVALID_ARG, "qgw_state_init_g0: null argument");
  const Plan& p = st->plan->p;
  st->mu_steps0 = 10;
  QGW_CHECK_HIP(enter_device(p.device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const size_t so = size_t(p.no) * p.no * p.nk * 16;
  const size_t fo = so * p.r;
  QGW_CHECK_HIP(hipMemsetAsync(st->Sig_iw_old, 0, fo, s), "qgw_state_init_g0");
  QGW_CHECK_HIP(hipMemsetAsync(st->SigHF_old, 0, so, s), "qgw_state_init_g0");
  double m = *mu;
  // with a target filling and no finite start given, the search starts from the state's previous G0 (the same
  // H0, so the same mu up to the search's tolerance): a couple of Newton steps instead of a search from the
  // Gershgorin centre
  const bool warm = !std::isnan(st->n_target) && !std::isfinite(m) && std::isfinite(st->mu_g0);
  if (warm) m = st->mu_g0;
  qgw_status rc = run_dyson_g(p, st->H_k, nullptr, st->n_target, &m, st->G_iw, s, nullptr, st->d_scal,
                              st->d_part, st->d_stat, nullptr, nullptr, nullptr, warm ? 3 : 6, st->h_io, st->ev_io);
  if (rc != QGW_OK) return rc;
  if (!std::isnan(st->n_target)) st->mu_g0 = m;
  st->mu = m;
  *mu = m;
  st->broken = false;
  st->in_fp32 = st->prec_mode != 0;
  st->n_fp32 = st->n_fp64 = 0;
  st->last_dsig = INFINITY;
  return QGW_OK;
}

qgw_status qgw_state_set_search_steps(qgw_state st, int32_t first_round) {
  QGW_REQUIRE(st, QGW_ERR_INVALID_ARG, "qgw_state_set_search_steps: null state");
  QGW_REQUIRE(first_round >= 0 && first_round <= 64, QGW_ERR_INVALID_ARG,
              "qgw_state_set_search_steps: first_round must be in [0, 64]");
  st->mu_steps_fixed = first_round;
  return QGW_OK;
}

qgw_status qgw_state_set_precision(qgw_state st, int32_t mode, double switch_tol) {
  QGW_REQUIRE(st, QGW_ERR_INVALID_ARG, "qgw_state_set_precision: null state");
  QGW_REQUIRE(mode >= 0 && mode <= 2, QGW_ERR_INVALID_ARG, "qgw_state_set_precision: mode must be 0, 1 or 2");
  QGW_REQUIRE(switch_tol > 0.0, QGW_ERR_INVALID_ARG, "qgw_state_set_precision: switch_tol must be positive");
  QGW_REQUIRE(mode == 0 || st->plan->p.grid == kGridDLR, QGW_ERR_UNSUPPORTED,
              "qgw_state_set_precision: a uniform-grid plan runs in FP64 only");
  if (mode != 0) {
    QGW_CHECK_HIP(enter_device(st->plan->p.device), "hipSetDevice");
    QGW_CHECK_HIP(ensure_fp32(st), "qgw_state_set_precision: single-precision buffers");
  }
  st->prec_mode = mode;
  st->switch_tol = switch_tol;
  st->in_fp32 = mode != 0;
  st->last_dsig = INFINITY;
  return QGW_OK;
}

qgw_status qgw_state_info(qgw_state st, int32_t* last_prec, int32_t* n_fp32, int32_t* n_fp64, int32_t* mu_evals) {
  QGW_REQUIRE(st, QGW_ERR_INVALID_ARG, "qgw_state_info: null state");
  if (mu_evals) *mu_evals = st->last_evals;
  if (last_prec) *last_prec = st->last_prec;
  if (n_fp32) *n_fp32 = st->n_fp32;
  if (n_fp64) *n_fp64 = st->n_fp64;
  return QGW_OK;
}

// a1 of an iteration, G(tau) and G(beta - tau), on s; with `fork` first the event that a12 waits on for G.  Queued
// by enqueue_steps, or ahead of time into event set `set` while the previous iteration's host waits for its search.
static hipError_t enqueue_a1(qgw_state st, bool f32, bool prof, hipStream_t s, bool fork, int set) {
  const Plan& p = st->plan->p;
  const int64_t ncol_g = int64_t(p.no) * p.no * p.nk;
  hipError_t e = hipSuccess;
  auto run = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  if (fork) run(hipEventRecord(st->ev_fork, s));
  if (prof && (st->prof_mask & 2u)) run(hipEventRecord(st->ev[set][1], s));
  if (!f32) {
    if (p.grid == kGridMF) {
      run(launch_mf_g_tau(p, st->G_iw, st->G_tau, st->G_reflt, s));  // one transform, both time orders
    } else {
      run(launch_dlr2(p, QGW_F_IW2TAU, QGW_F_IW2TAUR, ncol_g, st->G_iw, st->G_tau, st->G_reflt, s));
    }
  } else {
    st->p32.tune = p.has_tune32 ? p.tune32 : p.tune;
    run(launch_dlr2_from_f64(st->p32, QGW_F_IW2TAU, QGW_F_IW2TAUR, ncol_g, st->G_iw, st->Gt32, st->Gr32, st->G32, s));
  }
  return e;
}

// a12, a1-a11 (FP64 or single precision), a14 and the static H + Sigma_HF of a13,
// enqueued on s; with `prof` HIP events mark the step boundaries 0 .. 10.  fork: a12 on the state's side stream
// (eager iterations); without it (batch capture) everything goes on s.
static hipError_t enqueue_steps(qgw_state st, bool f32, bool prof, hipStream_t s, bool fork, bool a1_queued = false) {
  const Plan& p = st->plan->p;
  const int64_t no2 = int64_t(p.no) * p.no;
  const int64_t ncol_g = no2 * p.nk;
  st->p32.tune = p.has_tune32 ? p.tune32 : p.tune;
  hipError_t e = hipSuccess;
  hipEvent_t* ev = st->ev[st->ev_set];
  const uint32_t m = prof ? st->prof_mask : 0u;
  if (prof && st->prof_in_line) fork = false;
  // boundary i opens step i and closes step i - 1 (steps 1 .. 10; step 0 has events of its own)
  auto mark = [&](int i) {
    if (e == hipSuccess && (((m >> i) & 1u) || (i >= 2 && ((m >> (i - 1)) & 1u)))) e = hipEventRecord(ev[i], s);
  };
  auto run = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  // a12: density of the incoming G (Hermitian part), Hartree-Fock.  It reads only G and writes only n and
  // Sigma_HF, which a14 and a13 use.  In an eager iteration it runs on the state's side stream beside a1..a11 and
  // joins before a14, so its small, latency-bound launches overlap the pair-array steps instead of adding to them;
  // the pair-array steps are queued first, so the caller's stream has work as soon as the iteration starts, and
  // a12 waits for G through an event recorded ahead of them.  A batch capture keeps a12 on the worker stream, in
  // front (a fork from an already forked stream is not recorded).
  auto a12 = [&](hipStream_t a) {
    if (e == hipSuccess && (m & 1u)) e = hipEventRecord(ev[0], a);
    run(launch_dlr(p, QGW_F_IW2BETA, ncol_g, -1.0, 0.0, st->G_iw, st->n_k, a, 2));
    run(launch_lattice_fft(p, QGW_K_TO_R, no2, st->n_k, st->n_R, a));
    run(launch_hartree_fock(p, st->V_R, st->V_q0, st->n_R, st->SigHF_R, a));
    run(launch_lattice_fft(p, QGW_R_TO_K, no2, st->SigHF_R, st->SigHF_k, a));
    if (e == hipSuccess && (m & 1u)) e = hipEventRecord(st->ev_a12[st->ev_set], a);
  };
  // a1_queued: a1 and the fork event are already on s (queued during the previous iteration's wait)
  if (!fork) a12(s);
  if (!a1_queued) run(enqueue_a1(st, f32, prof, s, fork, st->ev_set));
  if (!f32) {
    mark(2);  // a2
    run(launch_lattice_fft2(p, QGW_K_TO_R, no2 * p.r, st->G_tau, st->G_tau, st->G_reflt, st->G_reflt, s));
    mark(3);  // a3 + a4
    run(launch_bubble(p, st->G_tau, st->G_reflt, 1, st->Pq, s));
    mark(4);  // a5
    run(launch_dlr_pairs(p, QGW_B_TAU2IW, QGW_LAYOUT_SLAB, QGW_LAYOUT_MATRIX, st->Pq, st->P_nu, s));
    mark(5);  // a6
    run(launch_dyson_w(p, st->V_qm, st->P_nu, st->Wc_nu, s, state_w_ld(p)));
    mark(6);  // a7
    run(launch_dlr_pairs(p, QGW_B_IW2TAU, QGW_LAYOUT_MATRIX, QGW_LAYOUT_SLAB, st->Wc_nu, st->Pq, s, state_w_ld(p)));
    mark(7);  // a8 + a9 + a10
    run(launch_sigma(p, st->G_tau, st->Pq, 1, 1, st->Sig_tau_k, s));
    mark(8);  // a11 (Hermitian part of Sigma^C(k, tau))
    run(launch_dlr(p, QGW_F_TAU2IW, ncol_g, 1.0, 0.0, st->Sig_tau_k, st->Sig_iw, s, 1));
  } else {
    // the same steps in single precision (defect-correction phase of the solve)
    const Plan& q = st->p32;
    mark(2);
    run(launch_lattice_fft2(q, QGW_K_TO_R, no2 * p.r, st->Gt32, st->Gt32, st->Gr32, st->Gr32, s));
    mark(3);
    run(launch_bubble(q, st->Gt32, st->Gr32, 1, st->Pq32, s));
    mark(4);
    run(launch_dlr_pairs(q, QGW_B_TAU2IW, QGW_LAYOUT_SLAB, QGW_LAYOUT_MATRIX, st->Pq32, st->Pnu32, s));
    mark(5);
    run(launch_dyson_w(q, st->Vqm32, st->Pnu32, st->Wc32, s, state_w_ld(p)));
    mark(6);
    run(launch_dlr_pairs(q, QGW_B_IW2TAU, QGW_LAYOUT_MATRIX, QGW_LAYOUT_SLAB, st->Wc32, st->Pq32, s, state_w_ld(p)));
    mark(7);
    run(launch_sigma(q, st->Gt32, st->Pq32, 1, 1, st->St32, s));
    mark(8);
    run(launch_dlr_to_f64(q, QGW_F_TAU2IW, ncol_g, 1.0, 0.0, st->St32, st->Sig_iw, st->Siw32, s, 1));
  }
  if (fork) {
    run(hipStreamWaitEvent(st->side, st->ev_fork, 0));
    a12(st->side);
    run(hipEventRecord(st->ev_join, st->side));
  }
  // a14 and the static part of a13 (H0 + Sigma_HF) in one pass, once a12 has joined
  if (fork) run(hipStreamWaitEvent(s, st->ev_join, 0));
  mark(9);
  // with a target filling the search's first launch reduces the block maxima into |dSigma| (one launch less)
  run(launch_delta_and_mix(p, st->SigHF_k, st->Sig_iw, st->SigHF_old, st->Sig_iw_old, st->mixing, st->d_dsig,
                           st->d_blockmax, s, st->H_k, st->Hs_k, std::isnan(st->n_target)));
  mark(10);
  return e;
}

// The next iteration's a1, queued behind an iteration's search read-back while the host waits for it.  Its
// precision is the current one; it is kept if the search ended in its first round (G is final) and the next
// iteration runs in that precision, and queued again otherwise.  A solve that stops there leaves it as the
// G(tau) of the final G.
struct NextA1 {
  qgw_state st;
  hipStream_t s;
  bool f32;
  int set;
  bool queued;
  hipError_t err;
};

static void queue_next_a1(void* c) {
  NextA1* x = static_cast<NextA1*>(c);
  x->err = enqueue_a1(x->st, x->f32, x->st->prof, x->s, true, x->set);
  x->queued = true;
}

qgw_status qgw_gw_iteration(qgw_state st, int32_t n_iter, double tol, int32_t* iters_done, double* d_sigma,
                            double* mu_out, void* stream) {
  QGW_REQUIRE(st, QGW_ERR_INVALID_ARG, "qgw_gw_iteration: null state");
  QGW_REQUIRE(n_iter >= 0, QGW_ERR_INVALID_ARG, "qgw_gw_iteration: negative n_iter");
  QGW_REQUIRE(!st->broken, QGW_ERR_INVALID_ARG,
              "qgw_gw_iteration: an earlier iteration of this state failed; restart it with qgw_state_init_g0");
  const Plan& p = st->plan->p;
  QGW_CHECK_HIP(enter_device(p.device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  double dsig = NAN;
  int done = 0;
  // step times of the last finished iteration (event set `pend`, -1: none), read once the next iteration is queued
  int pend = -1;
  bool pend_f32 = false;
  auto read_times = [&]() -> hipError_t {
    if (pend < 0) return hipSuccess;
    const hipEvent_t* ev = st->ev[pend];
    float ms[QGW_NUM_STEPS] = {};
    for (int i = 0; i < QGW_NUM_STEPS; ++i) {
      if (!((st->prof_mask >> i) & 1u)) continue;
      // step 0 (a12) runs from ev[0] to ev_a12
      const hipError_t e = hipEventElapsedTime(&ms[i], ev[i], i == 0 ? st->ev_a12[pend] : ev[i + 1]);
      if (e != hipSuccess) return e;
    }
    for (int i = 0; i < QGW_NUM_STEPS; ++i) st->prof_ms[pend_f32 ? 1 : 0][i] += ms[i];
    ++st->prof_iters[pend_f32 ? 1 : 0];
    pend = -1;
    return hipSuccess;
  };
  bool a1_next = false, a1_next_f32 = false;  // the next iteration's a1 is on s, in that precision
  for (int it = 0; it < n_iter; ++it) {
    const bool f32 = st->prec_mode == 2 || (st->prec_mode == 1 && st->in_fp32);
    st->ev_set = pend == 0 ? 1 : 0;
    const hipError_t qe = enqueue_steps(st, f32, st->prof, s, true, a1_next && a1_next_f32 == f32);
    a1_next = false;
    if (qe != hipSuccess) {
      st->broken = true;
      set_error(std::string("qgw_gw_iteration: ") + hipGetErrorString(qe));
      return QGW_ERR_DEVICE;
    }
    QGW_CHECK_HIP(read_times(), "profile");
    // a13: Dyson G with the chemical potential
    // |dSigma| (a14, already enqueued) comes back with the search's result: one wait per iteration
    // the first round queues the previous search's evaluation count + 2 Newton steps (3 .. 12; 10 after G0)
    double m = st->mu, evals = 0.0;
    // not with a12 timed in line (it must stay ahead of a1), nor past this call's last iteration
    NextA1 nx{st, s, f32, st->prof ? (st->ev_set ^ 1) : 0, false, hipSuccess};
    const bool ahead = it + 1 < n_iter && !(st->prof && st->prof_in_line);
    int rounds = 0;
    qgw_status rc = run_dyson_g(p, st->Hs_k, st->Sig_iw, st->n_target, &m, st->G_iw, s, &evals, st->d_scal,
                                st->d_part, st->d_stat, st->d_dsig, &dsig,
                                st->prof && ((st->prof_mask >> 10) & 1u) ? st->ev[st->ev_set][QGW_NUM_STEPS] : nullptr,
                                st->mu_steps_fixed > 0 ? st->mu_steps_fixed : st->mu_steps0, st->h_io,
                                st->ev_io, 1,
                                st->d_blockmax + 4096, dyson_g_diag_blocks(p), &rounds,
                                ahead ? queue_next_a1 : nullptr, &nx, st->d_blockmax, dyson_g_diag_blocks(p),
                                st->d_dsig);
    if (nx.queued && nx.err != hipSuccess) {
      st->broken = true;
      set_error(std::string("qgw_gw_iteration: ") + hipGetErrorString(nx.err));
      return QGW_ERR_DEVICE;
    }
    a1_next = nx.queued && rounds == 1;
    a1_next_f32 = nx.f32;
    st->last_evals = int(evals);
    // a singular Dyson-W system or a non-finite self-energy is named as the cause, also of a failed search
    if (rc != QGW_ERR_DEVICE && (rc != QGW_OK || !std::isfinite(dsig))) {
      int flags = 0;
      const qgw_status rc2 = take_conditions(p, s, &flags);
      if (rc2 != QGW_OK) {
        rc = rc2;
      } else if (flags & kCondSingular) {
        set_error("qgw_gw_iteration: a Dyson-W system I - V P had a zero or non-finite pivot");
        rc = QGW_ERR_SINGULAR;
      } else if (!std::isfinite(dsig)) {
        set_error("qgw_gw_iteration: non-finite self-energy (max |Delta Sigma| is not finite)");
        rc = QGW_ERR_NONFINITE;
      }
    }
    if (rc != QGW_OK) {
      st->broken = true;
      if (iters_done) *iters_done = done;
      return rc;
    }
    st->mu = m;
    st->mu_steps0 = std::min(12, std::max(3, int(evals) + 2));
    if (st->prof) {
      pend = st->ev_set;
      pend_f32 = f32;
    }
    ++done;
    st->last_prec = f32 ? 1 : 0;
    if (f32) {
      ++st->n_fp32;
      // leave the single-precision phase at its tolerance, or once it stalls
      if (st->prec_mode == 1 && (dsig <= st->switch_tol || dsig > 0.5 * st->last_dsig)) st->in_fp32 = false;
    } else {
      ++st->n_fp64;
    }
    st->last_dsig = dsig;
    if (dsig <= tol && !(st->prec_mode != 0 && f32)) break;
  }
  QGW_CHECK_HIP(read_times(), "profile");
  if (iters_done) *iters_done = done;
  if (d_sigma) *d_sigma = dsig;
  if (mu_out) *mu_out = st->mu;
  return QGW_OK;
}

// ------------------------------------------------------------------ batches

struct qgw_batch_s {
  std::vector<qgw_state> states;
  int device = 0;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> workers;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void free_batch(qgw_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  for (hipStream_t w : b->workers) (void)hipStreamDestroy(w);
  if (b->cap) (void)hipStreamDestroy(b->cap);
}

// Estimated time of one iteration of a plan (ns), from the sizes that set each step's work: Dyson W grows with
// N_k r N_b^3 (plus a per-matrix cost of the serial pivot steps), the pair maps with N_k N_b^2 r^2, bubble and
// self-energy with N_k N_b^2 r, and about 0.1 ms goes to latency-bound steps.  The coefficients are the FP64 rates
// measured at the five-orbital 24 x 24 workload and on the 64-instance sweep; only the ratios matter.
static double iteration_cost_ns(const Plan& p) {
  const double nk = p.nk, r = p.r, nb = p.nb;
  return nk * r * (0.8e-3 * nb * nb * nb + 1.5 + 4.5e-4 * nb * nb * r + 0.0105 * nb * nb) + 1e5;
}

qgw_status qgw_batch_create(int32_t n, const qgw_state* states, int32_t precision, int32_t n_iter,
                            int32_t mu_steps, qgw_batch* out) {
  QGW_REQUIRE(out && states && n > 0, QGW_ERR_INVALID_ARG, "qgw_batch_create: need states");
  QGW_REQUIRE(precision == 0 || precision == 1, QGW_ERR_INVALID_ARG, "qgw_batch_create: bad precision");
  QGW_REQUIRE(n_iter >= 1 && n_iter <= 64, QGW_ERR_INVALID_ARG, "qgw_batch_create: n_iter must be in [1, 64]");
  QGW_REQUIRE(mu_steps >= 1 && mu_steps <= 64, QGW_ERR_INVALID_ARG, "qgw_batch_create: mu_steps must be in [1, 64]");
  *out = nullptr;
  const int dev = states[0] ? states[0]->plan->p.device : 0;
  for (int i = 0; i < n; ++i) {
    QGW_REQUIRE(states[i], QGW_ERR_INVALID_ARG, "qgw_batch_create: null state");
    QGW_REQUIRE(states[i]->plan->p.device == dev, QGW_ERR_INVALID_ARG, "qgw_batch_create: states on different devices");
    QGW_REQUIRE(!states[i]->prof, QGW_ERR_INVALID_ARG, "qgw_batch_create: disable profiling first");
    QGW_REQUIRE(states[i]->plan->p.grid == kGridDLR, QGW_ERR_UNSUPPORTED, "qgw_batch_create: DLR plans only");
    QGW_REQUIRE(!states[i]->broken, QGW_ERR_INVALID_ARG, "qgw_batch_create: a state needs a restart (failed iteration)");
    for (int j = 0; j < i; ++j)
      QGW_REQUIRE(states[j] != states[i], QGW_ERR_INVALID_ARG, "qgw_batch_create: a state appears twice");
  }
  QGW_CHECK_HIP(enter_device(dev), "hipSetDevice");
  if (precision == 1)
    for (int i = 0; i < n; ++i) QGW_CHECK_HIP(ensure_fp32(states[i]), "qgw_batch_create: single-precision buffers");
  // the sticky failure words start clear (earlier eager searches may have raised them between their rounds)
  for (int i = 0; i < n; ++i)
    QGW_CHECK_HIP(hipMemset(states[i]->d_stat + 1, 0, sizeof(int)), "qgw_batch_create");
  qgw_batch b = new (std::nothrow) qgw_batch_s;
  QGW_REQUIRE(b, QGW_ERR_ALLOC, "qgw_batch_create: out of host memory");
  b->states.assign(states, states + n);
  b->device = dev;
  const int nw = n < 4 ? n : 4;
  hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  for (int w = 0; w < nw && e == hipSuccess; ++w) {
    hipStream_t ws = nullptr;
    e = hipStreamCreateWithFlags(&ws, hipStreamNonBlocking);
    if (e == hipSuccess) b->workers.push_back(ws);
  }
  for (int w = 0; w <= nw && e == hipSuccess; ++w) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->events.push_back(ev);
  }
  // instances to workers, longest estimated time first, each to the worker with the least estimated work so far (a
  // round-robin deal left one worker with twice the work of another on the uneven sweep)
  std::vector<int> worker(n, 0);
  {
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::vector<double> cost(n);
    for (int i = 0; i < n; ++i) cost[i] = iteration_cost_ns(states[i]->plan->p);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    std::vector<double> load(nw, 0.0);
    for (int i : order) {
      const int w = int(std::min_element(load.begin(), load.end()) - load.begin());
      worker[i] = w;
      load[w] += cost[i];
    }
  }
  // capture: fork the workers from the capture stream, each instance on its worker, join
  if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t ce = hipEventRecord(b->events[nw], b->cap);
    for (int w = 0; w < nw && ce == hipSuccess; ++w) ce = hipStreamWaitEvent(b->workers[w], b->events[nw], 0);
    for (int it = 0; it < n_iter && ce == hipSuccess; ++it)
      for (int i = 0; i < n && ce == hipSuccess; ++i) {
        qgw_state st = states[i];
        const Plan& p = st->plan->p;
        hipStream_t ws = b->workers[worker[i]];
        ce = enqueue_steps(st, precision == 1, false, ws, false);
        if (ce == hipSuccess)
          ce = launch_dyson_g_chain(p, st->Hs_k, st->Sig_iw, std::isnan(st->n_target) ? 0 : 1, st->G_iw, st->d_scal,
                                    st->d_part, st->d_stat, mu_steps, st->d_stat + 1, ws, st->d_blockmax + 4096,
                                    dyson_g_diag_blocks(p), st->d_blockmax, dyson_g_diag_blocks(p), st->d_dsig);
      }
    for (int w = 0; w < nw && ce == hipSuccess; ++w) {
      ce = hipEventRecord(b->events[w], b->workers[w]);
      if (ce == hipSuccess) ce = hipStreamWaitEvent(b->cap, b->events[w], 0);
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(b->cap, &g);
    b->graph = g;
    e = ce != hipSuccess ? ce : ee;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    set_error(std::string("qgw_batch_create: ") + hipGetErrorString(e));
    free_batch(b);
    delete b;
    return QGW_ERR_DEVICE;
  }
  *out = b;
  return QGW_OK;
}

qgw_status qgw_batch_launch(qgw_batch b, void* stream) {
  QGW_REQUIRE(b, QGW_ERR_INVALID_ARG, "qgw_batch_launch: null batch");
  QGW_CHECK_HIP(enter_device(b->device), "hipSetDevice");
  QGW_CHECK_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream), "qgw_batch_launch");
  return QGW_OK;
}

qgw_status qgw_batch_read(qgw_batch b, double* d_sigma, double* mu, int32_t* status, int32_t* evals, void* stream) {
  QGW_REQUIRE(b, QGW_ERR_INVALID_ARG, "qgw_batch_read: null batch");
  QGW_CHECK_HIP(enter_device(b->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const size_t n = b->states.size();
  std::vector<double> ds(n), m(n), ev(n);
  std::vector<int> stt(n);
  const int zero = 0;
  for (size_t i = 0; i < n; ++i) {
    qgw_state st = b->states[i];
    QGW_CHECK_HIP(hipMemcpyAsync(&ds[i], st->d_dsig, sizeof(double), hipMemcpyDeviceToHost, s), "qgw_batch_read");
    QGW_CHECK_HIP(hipMemcpyAsync(&m[i], st->d_scal, sizeof(double), hipMemcpyDeviceToHost, s), "qgw_batch_read");
    QGW_CHECK_HIP(hipMemcpyAsync(&ev[i], st->d_scal + 2, sizeof(double), hipMemcpyDeviceToHost, s), "qgw_batch_read");
    // the sticky word: the worst search status of every replay since the last read
    QGW_CHECK_HIP(hipMemcpyAsync(&stt[i], st->d_stat + 1, sizeof(int), hipMemcpyDeviceToHost, s), "qgw_batch_read");
    QGW_CHECK_HIP(hipMemcpyAsync(st->d_stat + 1, &zero, sizeof(int), hipMemcpyHostToDevice, s), "qgw_batch_read");
  }
  QGW_CHECK_HIP(hipStreamSynchronize(s), "qgw_batch_read");
  for (size_t i = 0; i < n; ++i) {
    b->states[i]->mu = m[i];
    if (stt[i] != 0) b->states[i]->broken = true;
    if (d_sigma) d_sigma[i] = ds[i];
    if (mu) mu[i] = m[i];
    if (status) status[i] = stt[i];
    if (evals) evals[i] = int32_t(ev[i]);
  }
  return QGW_OK;
}

qgw_status qgw_batch_destroy(qgw_batch b) {
  if (!b) return QGW_OK;
  (void)hipSetDevice(b->device);
  free_batch(b);
  delete b;
  return QGW_OK;
}

qgw_status qgw_state_copy(qgw_state st, int32_t which, void* dst, int64_t* bytes, void* stream) {
  QGW_REQUIRE(st, QGW_ERR_INVALID_ARG, "qgw_state_copy: null state");
  const Plan& p = st->plan->p;
  const size_t so = size_t(p.no) * p.no * p.nk * 16;
  const size_t fp = size_t(p.nb) * p.nb * p.nk * 16 * p.r;
  const void* src = nullptr;
  size_t n = 0;
  switch (which) {
    case 0: src = st->G_iw; n = so * p.r; break;
    case 1: src = st->Sig_iw; n = so * p.r; break;
    case 2: src = st->SigHF_k; n = so; break;
    case 3: src = st->P_nu; n = fp; break;
    case 4: src = st->Wc_nu; n = fp; break;  // rows padded to state_w_ld: copied row by row below
    case 5: src = st->n_k; n = so; break;
    default:
      set_error("qgw_state_copy: bad selector");
      return QGW_ERR_INVALID_ARG;
  }
  if (bytes) *bytes = int64_t(n);
  if (!dst) return QGW_OK;
  QGW_CHECK_HIP(enter_device(p.device), "hipSetDevice");
  const int64_t nb2 = int64_t(p.nb) * p.nb, ld = state_w_ld(p);
  if (which == 4 && ld != nb2)
    QGW_CHECK_HIP(hipMemcpy2DAsync(dst, size_t(nb2) * 16, src, size_t(ld) * 16, size_t(nb2) * 16,
                                   size_t(p.r) * p.nk, hipMemcpyDeviceToDevice, (hipStream_t)stream),
                  "qgw_state_copy");
  else
    QGW_CHECK_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, (hipStream_t)stream), "qgw_state_copy");
  return QGW_OK;
}

qgw_status qgw_state_profile_select(qgw_state st, uint32_t step_mask, int32_t in_line) {
  QGW_REQUIRE(st, QGW_ERR_INVALID_ARG, "qgw_state_profile_select: null state");
  QGW_REQUIRE((step_mask >> QGW_NUM_STEPS) == 0u, QGW_ERR_INVALID_ARG,
              "qgw_state_profile_select: step_mask has bits past the last step");
  QGW_REQUIRE(!st->prof, QGW_ERR_INVALID_ARG, "qgw_state_profile_select: disable timing first (mode 0)");
  st->prof_mask = step_mask;
  st->prof_in_line = in_line != 0;
  return QGW_OK;
}

qgw_status qgw_state_profile(qgw_state st, int32_t mode, double* ms, int32_t* iters) {
  QGW_REQUIRE(st, QGW_ERR_INVALID_ARG, "qgw_state_profile: null state");
  QGW_REQUIRE(mode >= 0 && mode <= 2, QGW_ERR_INVALID_ARG, "qgw_state_profile: bad mode");
  QGW_CHECK_HIP(enter_device(st->plan->p.device), "hipSetDevice");
  if (mode == 1) {
    for (auto& set : st->ev)
      for (auto& e : set)
        if (!e) QGW_CHECK_HIP(hipEventCreate(&e), "qgw_state_profile");
    for (auto& e : st->ev_a12)
      if (!e) QGW_CHECK_HIP(hipEventCreate(&e), "qgw_state_profile");
    for (auto& row : st->prof_ms)
      for (double& v : row) v = 0.0;
    st->prof_iters[0] = st->prof_iters[1] = 0;
    st->prof = true;
  } else if (mode == 0) {
    st->prof = false;
  }
  if (ms)
    for (int k = 0; k < 2; ++k)
      for (int i = 0; i < QGW_NUM_STEPS; ++i) ms[k * QGW_NUM_STEPS + i] = st->prof_ms[k][i];
  if (iters) iters[0] = st->prof_iters[0], iters[1] = st->prof_iters[1];
  return QGW_OK;
}

}  // extern "C"
