// Internal declarations shared by the libqgw translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "qgw_complex.h"

namespace qgw {

// Mesh sides with a compiled transform (radix 2, 3, 5; at most 48).
#define QGW_FOR_EACH_MESH(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(9) X(10) X(12) X(15) X(16) X(18) X(20) X(24) X(25) X(27) X(30) X(32) X(36) X(40) X(45) X(48)

// Sides of a cubic N x N x N mesh with a compiled 3-D transform.
#define QGW_FOR_EACH_CUBE(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12)

// Node counts N = N1 N2 of the uniform Matsubara grid with a compiled transform, X(N, N1, N2).
#define QGW_FOR_EACH_MF_GRID(X)                                                                              \
  X(16, 4, 4) X(32, 4, 8) X(48, 6, 8) X(64, 8, 8) X(80, 8, 10) X(96, 8, 12) X(128, 8, 16) X(160, 10, 16)      \
  X(192, 12, 16) X(200, 10, 20) X(256, 16, 16) X(320, 16, 20) X(400, 16, 25) X(512, 16, 32) X(640, 20, 32) \
  X(800, 25, 32) X(1024, 32, 32)

// Pair-basis sizes with a compiled Dyson-W solver.
#define QGW_FOR_EACH_NB(X) X(1) X(2) X(4) X(5) X(8) X(9) X(16) X(25)

// Orbital counts with a compiled Dyson-G solver.
#define QGW_FOR_EACH_NO(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

constexpr int kMaxRank = 96;
constexpr int kGridDLR = 0, kGridMF = 1;
constexpr int kNumMaps = 7;
// device map slots: 0-6 the forward maps, 7 + m the adjoint T^H of the square map m (m != 5)
constexpr int kAdjMap0 = 7;
constexpr int kNumDevMaps = 14;
// d_status[kCondWord] of a plan: device-detected conditions, bits set by kernels and cleared by the host
// (qgw_sync_status); kCondSingular: a zero or non-finite pivot in the Dyson-W solve
constexpr int kCondWord = 12;
constexpr int kCondSingular = 1;

struct DeviceMaps {
  void* m[kNumDevMaps] = {nullptr};  // rows padded to a multiple of mt, zero-filled
  int mt = 32;                    // output rows per thread block chunk
  int rows_padded = 0;
};

// Term lists of the Fock / self-energy contraction: for output (i, k),
// every (alpha, beta) with first(alpha) = i, second(beta) = k, stored as
// (alpha, beta, l = second(alpha), j = first(beta)).
struct TermTable {
  int* d_terms = nullptr;  // int4 per term
  int* d_off = nullptr;    // [n_o * n_o + 1] offsets into terms
  int max_terms = 0;
};

// Launch shapes picked by the autotuner (0 or -1: the built-in heuristic).
struct Tune {
  int fft_spb = 0;      // slabs per block of the lattice transform
  int bubble_spb = 0;   // slabs per block of the bubble
  int sigma_spb = 0;    // term lanes per block of the self-energy
  int mfma_bpc = 0;     // resident blocks per CU of the MFMA DLR maps
  int orb_valu = -1;    // orbital-array maps: 1 VALU kernel, 0 matrix cores
  int orb_mt = 0;       // rows per block chunk of the VALU map kernel
  int w25_mfma = -1;    // Dyson W with N_b = 25: 1 V P on the matrix cores, 0 on the VALU, -1 the default (0)
};

struct Plan {
  int device = 0;
  int n = 0, dim = 2, nk = 0, no = 0, nb = 0, r = 0, prec = 0;  // mesh side n, N_k = n^dim
  // node axis: kGridDLR (r DLR nodes) or kGridMF (r = N uniform Matsubara frequencies / midpoint times)
  int grid = 0;
  int mf_n1 = 0, mf_n2 = 0;   // N = N1 N2 (kGridMF)
  zd* d_mf = nullptr;         // kGridMF transform tables (kernels_mf.hip)
  double ne_offset = 0.0;     // N_e = -(2/N_k) sum Re rho_m Tr G_m + ne_offset (n_o on the uniform grid)
  double beta = 0.0;
  std::vector<int> site_norb, pair_first, pair_second, orb_site, pair_of;  // pair_of[a*no+b] or -1
  std::vector<double> omega, tau_t;
  std::vector<int64_t> n_f, n_b;
  std::vector<std::complex<double>> maps[kNumMaps];  // host FP64, r x r (IW2BETA: 1 x r)
  DeviceMaps dmaps64, dmaps32;
  zd* d_tw64 = nullptr;
  zf* d_tw32 = nullptr;
  int* d_pairs = nullptr;  // [2 * nb]: first, second
  TermTable terms;     // keyed by (i, k): entries (alpha, beta, l, j)
  TermTable terms_lj;  // keyed by (l, j): entries (alpha, beta, i, k)
  double* d_wn = nullptr;  // fermionic Matsubara frequencies (r)
  zd* d_qp_row = nullptr;  // node values -> value at i pi / beta (r)
  // Dyson-G scratch: partial sums (2 x max blocks x 4), status words ([0] search status, [8] count of
  // non-finite values, [kCondWord] device conditions)
  double* d_partials = nullptr;
  int* d_status = nullptr;
  double* d_scalars = nullptr;  // [8]: mu, n_target, d_sigma, ...
  int max_blocks = 0;
  Tune tune;
  Tune tune32;              // shapes of the FP32 kernels of an FP64 plan (a state's single-precision iterations)
  bool has_tune32 = false;
};

void set_error(const std::string& msg);

// Hartree-Fock density of the static Hamiltonian hs (FP64): eigen-decomposition per k into u, eps
// (workspace: n_o^2 N_k complex, n_o N_k double), mu at the filling scal[1] (or scal[0] if scal[1] is
// NaN) into scal[0], n = U f U^H into n
hipError_t launch_hf_density(const Plan& p, const void* hs, double* scal, int* status, void* u, double* eps, void* n,
                             hipStream_t s);
// d_out = max |x_new - x_old| over a static orbital array, then x_new <- x_old + alpha (x_new - x_old), x_old <- x_new
hipError_t launch_hf_delta_mix(const Plan& p, void* x_new, void* x_old, double alpha, double* d_out, hipStream_t s);

// quasiparticle outputs per k (FP64); status[0] is set to 1 where Z^{-1} is not positive definite
hipError_t launch_quasiparticle(const Plan& p, const void* h_k, const void* shf_k, const void* sig_iw, double mu,
                                void* sig0, void* z, void* hqp, double* bands, int* status, hipStream_t s);
// the same at npt path points (device kfrac [npt][dim]) by Fourier interpolation from the mesh; workspace:
// (4 N_k + 3 npt) n_o^2 complex
hipError_t launch_quasiparticle_path(const Plan& p, const void* h_k, const void* shf_k, const void* sig_iw,
                                     const double* kfrac, int npt, double mu, void* ws, void* sig0, void* z,
                                     void* hqp, double* bands, int* status, hipStream_t s);

// ---- kernels (each returns hipSuccess or the launch error) ----------------
hipError_t launch_lattice_fft(const Plan& p, int dir, int64_t batch, const void* in, void* out,
                              hipStream_t s);
// the same transform of two arrays of ``batch`` slabs each, in one launch on a square mesh
hipError_t launch_lattice_fft2(const Plan& p, int dir, int64_t batch, const void* in1, void* out1, const void* in2,
                               void* out2, hipStream_t s);
hipError_t launch_bubble(const Plan& p, const void* g_tau_r, const void* g_reflt_r, int out_q,
                         void* out, hipStream_t s);
hipError_t launch_sigma(const Plan& p, const void* g_tau_r, const void* wc, int in_q, int out_k,
                        void* sig, hipStream_t s);
// herm: 0 plain, 1 Hermitian part of the input, 2 of the output (orbital arrays)
hipError_t launch_dlr(const Plan& p, int map, int64_t ncols, double sre, double sim, const void* in,
                      void* out, hipStream_t s, int herm = 0);
// two maps of the same input (scale 1), in one launch where the matrix-core path splits the map's row tiles
hipError_t launch_dlr2(const Plan& p, int map1, int map2, int64_t ncols, const void* in, void* out1, void* out2,
                       hipStream_t s);
// in_ld: row stride (elements) of a matrix-layout input, 0 for N_b^2 (only the matrix-core path takes another)
hipError_t launch_dlr_pairs(const Plan& p, int map, int in_layout, int out_layout, const void* in,
                            void* out, hipStream_t s, int64_t in_ld = 0);
// out_ld: row stride (elements) of the W^C matrices written, 0 for N_b^2
hipError_t launch_dyson_w(const Plan& p, const void* v_q, const void* p_nu, void* wc_nu,
                          hipStream_t s, int64_t out_ld = 0);
// row stride of the W^C matrices a state keeps: rounded up to 128-byte lines (16 complex FP32 values) when the
// matrix-core pair maps read them, so that the matrix -> slab map reads whole lines
inline int64_t state_w_ld(const Plan& p) {
  const int64_t na = int64_t(p.nb) * p.nb;
  return (p.grid == kGridDLR && p.r <= 64) ? (na + 15) / 16 * 16 : na;
}
hipError_t launch_hartree_fock(const Plan& p, const void* v_r, const void* v_q0, const void* n_r,
                               void* sig_hf_r, hipStream_t s);
hipError_t launch_pair_sum_r(const Plan& p, const void* v_r, void* v_q0, hipStream_t s);
// Dyson G with the chemical-potential search as a chain of launches.  Scalar
// block scal[16] ([0] mu, [1] n_target, [2] evaluations, [3] last N_e,
// [4-6] bracket and step cap, [7] done flag), partial sums [8 max_blocks],
// status word.  begin: Gershgorin start if mu is not finite, resets the
// search; steps: `steps` Newton evaluations (no-ops once done); final: G at
// mu (mode 0: mu as given; mode 1: also status 2 if the search has not
// converged).  chain = begin + steps + final (graph-capturable).
// track = 1: a state's search, whose start moves with the mean diagonal of H since its previous search (scal[10]);
// set = 1: scal[0..1] = (mu0, nt) first (the host's start point as kernel arguments, no copy)
// dpart (optional): dnblk block sums of the diagonal of h_k already at hand (from a14); the Gershgorin pass is then
// skipped, and a start that is not finite is reported as status 1 instead of replaced by the Gershgorin centre
// bmax (optional): a14's nbmax block maxima of |Delta Sigma|, reduced into *dsig by the same launch (a14 then runs
// without its own reduction)
hipError_t launch_dyson_g_begin(const Plan& p, const void* h_k, double* scal, double* partials, int* status,
                                int track, hipStream_t s, int set = 0, double mu0 = 0.0, double nt = 0.0,
                                const double* dpart = nullptr, int dnblk = 0, const double* bmax = nullptr,
                                int nbmax = 0, double* dsig = nullptr);
// number of the diagonal block sums a14 leaves for the search (one per 64 static entries)
inline int dyson_g_diag_blocks(const Plan& p) { return int((int64_t(p.no) * p.no * p.nk + 63) / 64); }
// doubles of partial sums one chemical-potential search on plan p uses (start and evaluations)
int dyson_g_partials_needed(const Plan& p);
hipError_t launch_dyson_g_steps(const Plan& p, const void* h_k, const void* sig_iw, double* scal, double* partials,
                                int* status, int steps, hipStream_t s);
// also copies the status to scal[8] and, if extra is given, *extra to scal[9]; ``steps`` is the number of
// evaluations launch_dyson_g_steps queued in this round (the final pass takes the step of the last one).
// scal holds 32 doubles: the host-visible words 0..9 and the two state slots of a round at 16..31.
// fail_word (optional): raised to a failing status of the search and never lowered by the kernels (the sticky
// report of a batch graph, whose every replay restarts status[0])
hipError_t launch_dyson_g_final(const Plan& p, const void* h_k, const void* sig_iw, int mode, void* g_iw,
                                double* scal, double* partials, int* status, hipStream_t s,
                                const double* extra = nullptr, int steps = 0, int* fail_word = nullptr);
hipError_t launch_dyson_g_chain(const Plan& p, const void* h_k, const void* sig_iw, int mode, void* g_iw,
                                double* scal, double* partials, int* status, int steps, int* fail_word,
                                hipStream_t s, const double* dpart = nullptr, int dnblk = 0,
                                const double* bmax = nullptr, int nbmax = 0, double* dsig = nullptr);
hipError_t launch_slab_to_matrix_static(const Plan& p, const void* in, void* out, hipStream_t s);
hipError_t launch_add(const Plan& p, int64_t count, const void* a, const void* b, void* out,
                      hipStream_t s);
// d_sigma = max |(hf_new + c_new) - (hf_old + c_old)| (non-finite entries count as +inf); then optional mixing
// new <- old + alpha (new - old), and old <- new; with h0 also hs = h0 + (mixed) hf_new.  block_scratch holds up to
// 4096 block maxima of 64 static entries (n_o^2 N_k <= 262144), and with h0, at block_scratch + 4096, the blocks'
// sums of the diagonal of hs (dyson_g_diag_blocks of them): the mean level a state's next search starts from.
// reduce = false leaves the block maxima unreduced (d_out untouched) for the chemical-potential search's first
// launch to reduce (launch_dyson_g_begin with bmax).
hipError_t launch_delta_and_mix(const Plan& p, void* hf_new, void* c_new, void* hf_old,
                                void* c_old, double alpha, double* d_out, double* block_scratch,
                                hipStream_t s, const void* h0 = nullptr, void* hs = nullptr, bool reduce = true);
// complex128 <-> complex64 copies (to_f32 = 1: double -> float)
hipError_t launch_convert(int64_t count, const void* in, void* out, int to_f32, hipStream_t s);
// FP32 plans: the two maps of an FP64 input (rounded as read), and a map whose result is widened to FP64 as stored;
// `stage` (r ncols FP32 values) serves the conversion pass where the matrix-core path does not apply
hipError_t launch_dlr2_from_f64(const Plan& p, int map1, int map2, int64_t ncols, const void* in64, void* out1,
                                void* out2, void* stage, hipStream_t s);
hipError_t launch_dlr_to_f64(const Plan& p, int map, int64_t ncols, double sre, double sim, const void* in,
                             void* out64, void* stage, hipStream_t s, int herm);
hipError_t launch_count_nonfinite(const Plan& p, const void* x, int64_t count, int* d_count,
                                  hipStream_t s);

// ---- adjoints (FP64 plans) ----------------------------------------------
// batched 2-D DFT with sign and output scale given explicitly
hipError_t launch_lattice_fft_scaled(const Plan& p, int sign, double out_scale, int64_t batch,
                                     const void* in, void* out, hipStream_t s);
// xbar[t][c] = conj(s rho_t) ybar[c] for the density row (herm as in launch_dlr)
hipError_t launch_row_map_bwd(const Plan& p, int64_t ncols, double sre, double sim, int herm,
                              const void* ybar, void* xbar, hipStream_t s);
// Wc^bar(q) from Sigma^bar(R): -conj(G_lj(R)) Sbar_ik(R), then R -> q with 1/N_k
hipError_t launch_sigma_bwd_wc(const Plan& p, const void* g_tau_r, const void* sbar_r, void* wcbar_q,
                               hipStream_t s);
// contraction adjoints (see kernels_bwd.hip): mode 0 Sigma -> G, 1 bubble -> G(tau),
// 2 bubble -> G(beta - tau)
hipError_t launch_contract_bwd(const Plan& p, int mode, const void* x_pair, const void* y_orb,
                               void* out, hipStream_t s);
// the same five steps on a cubic mesh (p.dim == 3); the 2-D launchers route to them
hipError_t launch_lattice_fft3(const Plan& p, int sign, double out_scale, int64_t batch, const void* in, void* out,
                               hipStream_t s);
hipError_t launch_bubble3(const Plan& p, const void* gt, const void* gr, int out_q, void* out, hipStream_t s);
hipError_t launch_sigma3(const Plan& p, const void* gt, const void* wc, int in_q, int out_k, void* sig, hipStream_t s);
hipError_t launch_sigma_bwd_wc3(const Plan& p, const void* gt, const void* sbar, void* out, hipStream_t s);
hipError_t launch_contract_bwd3(const Plan& p, int mode, const void* xq, const void* y, void* out, hipStream_t s);
// uniform-grid (MF) plans: the transforms behind launch_dlr / launch_dlr_pairs, G(tau) and G(beta - tau) in one
// pass, the split N = N1 N2 of a supported node count
hipError_t launch_mf(const Plan& p, int map, int64_t ncols, double sre, double sim, const void* in, void* out,
                     hipStream_t s, int herm);
hipError_t launch_mf_pairs(const Plan& p, int map, int in_layout, int out_layout, const void* in, void* out,
                           hipStream_t s);
hipError_t launch_mf_g_tau(const Plan& p, const void* g_iw, void* g_tau, void* g_reflt, hipStream_t s);
bool mf_grid_split(int n, int* n1, int* n2);
// the density row y = s sum_m row_m x_m (map 5), with the Hermitian part of the input (herm 1) or output (herm 2)
hipError_t launch_row_map(const Plan& p, int64_t ncols, double sre, double sim, int herm, const void* in, void* out,
                          hipStream_t s);

// threads per slab line set: n for a square mesh, n^2 for a cube
inline int lines_per_slab(const Plan& p) { return p.dim == 3 ? p.n * p.n : p.n; }
// workspace: W^C and X = (I - V P)^{-H} Wbar (r N_k N_b^2 complex each), then the Vbar partials (chunks N_k N_b^2)
hipError_t launch_dyson_w_bwd(const Plan& p, const void* v_q, const void* p_nu, const void* wcbar,
                              void* pbar, void* workspace, int chunks, hipStream_t s);
hipError_t launch_sum_chunks(int64_t n, int chunks, const void* partial, void* out, hipStream_t s);
// Dyson G adjoint: sbar = G^H Gbar G^H (+ the chemical-potential term when n_target is finite)
hipError_t launch_dyson_g_bwd(const Plan& p, const void* h_k, const void* sig_iw, double mu,
                              double n_target, double mubar, const void* gbar, void* sigbar,
                              hipStream_t s);
// hbar[ab][k] = sum_m x[m][ab][k]
hipError_t launch_sum_nodes(const Plan& p, const void* x, void* out, hipStream_t s);
hipError_t launch_hartree_fock_bwd(const Plan& p, const void* v_r, const void* v_q0, const void* n_r,
                                   const void* sbar_r, void* nbar_r, void* vbar_r, hipStream_t s);
// total energy: parts[2] = (sum Re (H + Sigma_HF/2)_ab n_ba, sum Re Y_m,ab G_m,ba) over all entries
hipError_t launch_energy_sums(const Plan& p, const void* h_k, const void* shf_k, const void* n_k, const void* y,
                              const void* g, double* partials, double* out2, hipStream_t s);
// energy adjoint pieces: abar -> hbar, shfbar (= abar / 2), nbar (static); then gbar += c conj(Y^T), ybar = c conj(G^T)
hipError_t launch_energy_bwd_static(const Plan& p, const void* h_k, const void* shf_k, const void* n_k, double c,
                                    void* hbar, void* shfbar, void* nbar, hipStream_t s);
hipError_t launch_energy_bwd_nodes(const Plan& p, const void* y, const void* g, double c, void* gbar, void* ybar,
                                   hipStream_t s);
// pair arrays with nn leading blocks: slab [nn][A][B][k] <-> matrix [nn][k][A][B]
hipError_t launch_pair_layout(const Plan& p, int to_matrix, int64_t nn, const void* in, void* out,
                              hipStream_t s);

// ---- host DLR -------------------------------------------------------------
int dlr_build_host(double lambda, double eps, int max_rank, std::vector<double>& x,
                   std::vector<double>& tau_t, std::vector<int64_t>& n_f,
                   std::vector<int64_t>& n_b, std::string& err);
bool dlr_qp_row_host(double beta, const std::vector<double>& omega, const std::vector<int64_t>& n_f,
                     std::vector<std::complex<double>>& row, std::string& err);
bool dlr_maps_host(double beta, const std::vector<double>& omega, const std::vector<double>& tau_t,
                   const std::vector<int64_t>& n_f, const std::vector<int64_t>& n_b,
                   std::vector<std::complex<double>> maps[kNumMaps], std::string& err);

}  // namespace qgw

// opaque handle of the C ABI
struct qgw_plan_s {
  qgw::Plan p;
};
