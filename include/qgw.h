/*
 * libqgw -- one GW iteration on a tight-binding lattice, HIP kernels for gfx950.
 *
 * C ABI.  Every function returns a qgw_status; qgw_last_error() gives a
 * thread-local message for the last failing call on that thread.  No C++
 * exception crosses this boundary.
 *
 * Physics (arXiv:2604.22223, method section):
 *   H0(k)         Eq. eq:fourier-transform-kr applied to H0(R) (cell-periodic gauge)
 *   G(k, i w)     Eq. full-green-freq with G0^{-1} = (i w + mu) - H0(k)
 *   P(q, i nu)    Eq. eq-polarizability (spin sum 2, fermionic antiperiodicity)
 *   W(q, i nu)    Eq. eq-screened-coulomb, W^C = W - V
 *   Sigma^C       Eq. eq-gw-self-energy
 *   Sigma^H, ^F   Eqs. eq-hartree-self-energy, eq-fock-self-energy
 *   density       n = -G(beta^-), mu adjusted to the target filling
 *                 (G class paragraph of Fig. fig-self (b))
 *   time/frequency axes in the discrete Lehmann representation (DLR; the
 *   sentence after Eq. eq:bare-green-freq)
 *
 * Index conventions.  Orbitals a = 0 .. n_o-1 are numbered site by site.
 * Pair ("product") indices alpha = (p; i, l), i and l orbitals of site p,
 * numbered site-major then i then l; N_b = sum_p n_p^2.  A pair array
 * X[alpha][beta] holds the paper's X_{ijkl} with alpha = (i, l) and
 * beta = (j, k); with that labelling W = V + V P W is a matrix product.
 *
 * Data.  All device arrays are complex, interleaved (re, im), C-contiguous,
 * 16-byte aligned for double precision and 8-byte aligned for single, and
 * owned by the caller.  The mesh is square, n x n, N_k = n * n, with the
 * flat index k = k1 * n + k2 (fastest); k.R = 2 pi (k1 R1 + k2 R2) / n.
 * Layouts (r = DLR rank):
 *   orbital array  [r][n_o][n_o][N_k]      ("G layout")
 *   pair slab      [r][N_b][N_b][N_k]      (mesh fastest; transforms over R/q)
 *   pair matrix    [r][N_k][N_b][N_b]      (one N_b x N_b matrix per (node, q))
 *   static orbital [n_o][n_o][N_k], static pair [N_b][N_b][N_k]
 *
 * Streams.  ``stream`` is a hipStream_t passed as void* (NULL = the default
 * stream).  Compute calls only enqueue work, allocate nothing and return
 * once the work is queued.  Calls that return a value computed on the device
 * to the host (the chemical potential, the energy, a status) wait for their
 * stream; each such call says so.
 *
 * Scratch.  Calls marked "workspace" take caller-owned device scratch
 * (``workspace``, ``workspace_bytes``) of at least the size
 * qgw_workspace_size reports for the plan and the call, so the caller's
 * allocator owns it.  It must stay valid until the queued work has run, and
 * two calls in flight at once must not share it.  Too small or NULL (where
 * bytes are needed): QGW_ERR_INVALID_ARG before anything is queued.
 *
 * Device conditions.  Kernels that meet a condition the host cannot check
 * beforehand (a zero or non-finite pivot in the Dyson-W solve) set a bit in a
 * plan-owned device status word; qgw_sync_status reads and clears it.
 */
#ifndef QGW_H
#define QGW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qgw_status;

enum {
  QGW_OK = 0,
  QGW_ERR_INVALID_ARG = 1,   /* null pointer, negative size, bad enum            */
  QGW_ERR_SHAPE = 2,         /* sizes inconsistent with the plan                 */
  QGW_ERR_UNSUPPORTED = 3,   /* mesh side, N_b or rank outside the built set    */
  QGW_ERR_DEVICE = 4,        /* HIP error, or no GPU                             */
  QGW_ERR_NOT_CONVERGED = 5, /* chemical potential search did not converge      */
  QGW_ERR_NONFINITE = 6,     /* NaN / Inf met (inputs or a singular solve)       */
  QGW_ERR_ALLOC = 7,         /* device or host allocation failed (plan set-up)  */
  QGW_ERR_SINGULAR = 8       /* a Dyson-W system I - V P had a zero pivot        */
};

/* Calls that take caller-provided scratch (qgw_workspace_size). */
enum {
  QGW_OP_SIGMA_BWD = 0,         /* qgw_sigma_bwd with out_k = 1 (out_k = 0 needs none) */
  QGW_OP_DYSON_W_BWD = 1,       /* qgw_dyson_W_bwd                                     */
  QGW_OP_HARTREE_FOCK_BWD = 2,  /* qgw_hartree_fock_bwd                                */
  QGW_OP_ENERGY = 3,            /* qgw_energy                                          */
  QGW_OP_ENERGY_BWD = 4,        /* qgw_energy_bwd                                      */
  QGW_OP_HF_DENSITY = 5,        /* qgw_hf_density                                      */
  QGW_OP_QUASIPARTICLE = 6      /* qgw_quasiparticle                                   */
};

/* Arithmetic of the bulk arrays. */
enum { QGW_F64 = 0, QGW_F32 = 1 };

/* DLR maps (qgw_dlr_transform).  Each maps the r node values of a function
 * to r node values of the same function elsewhere (construction of Kaye,
 * Chen & Parcollet, PRB 105, 235115 (2022), cited by the paper for the DLR):
 *   QGW_F_IW2TAU   fermionic Matsubara nodes -> tau_k
 *   QGW_F_IW2TAUR  fermionic Matsubara nodes -> beta - tau_k
 *   QGW_F_TAU2IW   tau_k -> fermionic Matsubara nodes
 *   QGW_B_TAU2IW   tau_k -> bosonic Matsubara nodes
 *   QGW_B_IW2TAU   bosonic Matsubara nodes -> tau_k
 *   QGW_F_IW2BETA  fermionic Matsubara nodes -> beta^- (one output row)
 *   QGW_F_IW2GM    fermionic Matsubara nodes -> Matsubara-sum weights: with
 *                  Y = T x, sum_m Y_m B_m = (1/beta) sum over all n of
 *                  x(i w_n) B(i w_n) for fermionic DLR functions x and B
 *                  (T = K_F^{-T} D K_F^{-1}, D the divided differences of the
 *                  Fermi function; the Galitskii-Migdal correlation energy) */
enum {
  QGW_F_IW2TAU = 0,
  QGW_F_IW2TAUR = 1,
  QGW_F_TAU2IW = 2,
  QGW_B_TAU2IW = 3,
  QGW_B_IW2TAU = 4,
  QGW_F_IW2BETA = 5,
  QGW_F_IW2GM = 6
};

/* Pair-array layouts. */
enum { QGW_LAYOUT_SLAB = 0, QGW_LAYOUT_MATRIX = 1 };

/* Transform directions for qgw_lattice_fft (Eq. eq:fourier-transform-kr). */
enum {
  QGW_R_TO_K = -1,  /* X(k) = sum_R X(R) e^{-i k.R}                 */
  QGW_K_TO_R = +1   /* X(R) = (1/N_k) sum_k X(k) e^{+i k.R}         */
};

typedef struct qgw_plan_s *qgw_plan;

/* Plan description.  The DLR nodes are data: pass the node set produced by
 * qgw_dlr_build (or any other node set of the same rank).  All host arrays
 * are read during qgw_plan_create only. */
typedef struct {
  int32_t n;                 /* mesh side: N_k = n * n (n^3 when dim is 3)        */
  int32_t n_sites;           /* basis sites per cell                               */
  const int32_t *site_norb;  /* [n_sites] orbitals per site                        */
  double beta;               /* inverse temperature (1/eV)                         */
  int32_t rank;              /* DLR rank r                                         */
  const double *omega;       /* [r] DLR real frequencies (eV)                      */
  const double *tau_t;       /* [r] DLR times as tau / beta in (0, 1)              */
  const int64_t *n_f;        /* [r] fermionic nodes: w = (2 n + 1) pi / beta       */
  const int64_t *n_b;        /* [r] bosonic nodes:   nu = 2 n pi / beta            */
  int32_t precision;         /* QGW_F64 or QGW_F32                                 */
  int32_t device;            /* HIP device ordinal                                 */
  int32_t dim;               /* mesh dimension: 2 (n x n; 0 also means 2) or 3     */
                             /* (simple cubic n x n x n, N_k = n^3, index          */
                             /* (R1 n + R2) n + R3)                                */
} qgw_plan_desc;

/* ------------------------------------------------------------------ set-up */

/* DLR node selection on the host in FP64 (DLR paragraph of the method
 * section; Kaye, Chen & Parcollet 2022): pivoted QR of the Lehmann kernel
 * K(t, x) = exp(-t x) / (1 + exp(-x)) on composite Chebyshev grids, with
 * dimensionless cutoff lambda = beta * omega_max and tolerance eps.
 * Outputs (caller-owned, capacity max_rank each): x = beta * omega_l,
 * tau_t, n_f, n_b, all sorted ascending; *rank receives r.  Returns
 * QGW_ERR_SHAPE if r would exceed max_rank. */
qgw_status qgw_dlr_build(double lambda, double eps, int32_t max_rank,
                         double *x, double *tau_t, int64_t *n_f, int64_t *n_b,
                         int32_t *rank);

/* Creates a plan: validates the description, forms the r x r DLR maps in
 * FP64 on the host by LU solves (never an explicit inverse), uploads them,
 * builds FFT twiddles and allocates the plan's private device scratch.
 * Supported: n in {1,2,3,4,5,6,8,9,10,12,15,16,18,20,24,25,27,30,32,36,40,
 * 45,48} for a square mesh, n in {1,2,3,4,5,6,8,10,12} for a cubic one (the
 * 8 x 8 x 8 mesh of the performance section); N_b in {1,2,4,5,8,9,16,25};
 * 1 <= r <= 96.  Any other dim is QGW_ERR_INVALID_ARG. */
qgw_status qgw_plan_create(const qgw_plan_desc *desc, qgw_plan *plan);
qgw_status qgw_plan_destroy(qgw_plan plan);

/* Uniform-grid plan: the same iteration on the conventional Matsubara grid
 * that the performance section compares the DLR with (its "MF" rows).  The
 * node axis holds n_nodes = N = 2M points: fermionic w_n = (2n + 1) pi / beta
 * and bosonic nu_n = 2 n pi / beta for n = -M .. M-1 (index n + M), and
 * midpoint times tau_j = (j + 1/2) beta / N (so beta - tau_j = tau_{N-1-j}).
 * desc's mesh, sites, beta and device are used; rank and the node arrays are
 * ignored and may be NULL; precision must be QGW_F64.  N must be one of
 * {16, 32, 48, 64, 80, 96, 128, 160, 192, 200, 256, 320, 400, 512, 640, 800,
 * 1024} (QGW_ERR_UNSUPPORTED otherwise); qgw_mf_nodes_for picks one.
 *
 * On such a plan the map calls apply the grid's transforms along the node
 * axis (FFTs), in the same argument conventions:
 *   QGW_F_IW2TAU   G(tau_j) = (1/beta) sum_n e^{-i w_n tau_j} G(i w_n)
 *                  - delta_ab (t_j + 1/2), t_j the grid's own sum of the
 *                  1/(i w_n) tail, whose exact transform is -1/2 (so the tail
 *                  of the orbital diagonal is transformed exactly);
 *   QGW_F_IW2TAUR  the same at beta - tau_j;
 *   QGW_F_TAU2IW   (beta/N) sum_j e^{i w_n tau_j} X(tau_j) (midpoint rule);
 *   QGW_B_TAU2IW   (beta/N) sum_j e^{i nu_n tau_j} X(tau_j);
 *   QGW_B_IW2TAU   (1/beta) sum_n e^{-i nu_n tau_j} X(i nu_n);
 *   QGW_F_IW2BETA  G(beta^-) = -(1/beta) sum_n G(i w_n) - delta_ab / 2.
 * F_IW2TAU, F_IW2TAUR and F_IW2BETA take orbital arrays (ncols = n_o^2 N_k,
 * QGW_ERR_DEVICE otherwise); the scale multiplies the whole affine result.
 * qgw_dlr_transform_pairs with a layout change transposes into out and then
 * transforms out in place (in is not modified).  Dyson G, the chemical
 * potential (N_e = 2/N_k sum_k Re Tr n(k) with n as above), Hartree-Fock,
 * bubble, Dyson W, Sigma, the composite iteration, the Hartree-Fock solve and
 * qgw_quasiparticle (i pi / beta is node n = 0) work unchanged.  Not
 * available on a uniform-grid plan (QGW_ERR_UNSUPPORTED): qgw_plan_get_map,
 * the adjoint calls, qgw_energy / qgw_energy_bwd, the FP32 schedules of
 * qgw_state_set_precision, batches and the autotuner. */
qgw_status qgw_plan_create_mf(const qgw_plan_desc *desc, int32_t n_nodes, qgw_plan *plan);

/* The smallest supported uniform-grid node count N with w_{M-1} >= omega_max
 * (M = N / 2), or 0 if none is large enough or the arguments are not positive. */
int32_t qgw_mf_nodes_for(double beta, double omega_max);

/* Copies the FP64 r x r map (row-major, interleaved complex, r*r*2 doubles;
 * r*2 for QGW_F_IW2BETA) of ``map`` to host memory ``out``. */
qgw_status qgw_plan_get_map(qgw_plan plan, int32_t map, double *out);

/* Launch-shape autotuner: times the candidate shapes of the kernels whose
 * best shape depends on the instance, on scratch arrays of the plan's sizes
 * (allocated and freed inside the call; waits for ``stream``), and keeps the
 * fastest in the plan for every later call (and for states built on it):
 * slabs per block of the lattice transform and of the bubble, term lanes of
 * the self-energy, resident blocks per CU of the matrix-core DLR maps, and
 * the kernel of the orbital-array maps (matrix cores, or the VALU kernel with
 * 8, 16 or 32 rows per chunk), and for N_b = 25 where the Dyson-W product
 * V P runs (1 = matrix cores, 0 = VALU).  choices[7] (may be NULL) receives
 * them in that order (orbital maps as two entries: 1 = VALU, and its chunk).
 * The candidates compute the same values; the self-energy lane count, the
 * orbital-map kernel and the Dyson-W product change only the order of
 * floating-point sums.  An FP64 plan is tuned a second time for its FP32
 * kernels, which a state's single-precision iterations use (choices reports
 * the FP64 shapes). */
qgw_status qgw_plan_autotune(qgw_plan plan, int32_t *choices, void *stream);

/* Sets the launch shapes directly, in qgw_plan_autotune's order (choices[7];
 * 0, or -1 for the two kernel selectors, leaves a knob at its default): to
 * restore shapes tuned earlier or to pin one kernel variant.  precision
 * QGW_F64 sets the plan's own shapes, QGW_F32 (FP64 plans only) those of its
 * FP32 kernels.  Applies to calls enqueued after it; batches keep the shapes
 * they were captured with.  QGW_ERR_INVALID_ARG for a choice outside its
 * range (slabs and lanes 0 .. 256 / (mesh lines per slab), blocks per CU
 * 0 .. 8, orbital-map chunk 0, 8, 16 or 32). */
qgw_status qgw_plan_set_tuning(qgw_plan plan, int32_t precision, const int32_t *choices);

/* Sizes of the plan: any output pointer may be NULL. */
qgw_status qgw_plan_sizes(qgw_plan plan, int32_t *rank, int32_t *n_o,
                          int32_t *n_b, int32_t *n_k);

/* Bytes of caller-provided scratch that call ``op`` (QGW_OP_*) needs on this
 * plan (0: none).  QGW_ERR_INVALID_ARG for an unknown op. */
qgw_status qgw_workspace_size(qgw_plan plan, int32_t op, int64_t *bytes);

/* Waits for ``stream``, then reads and clears the plan's device status word:
 * QGW_ERR_SINGULAR if a Dyson-W solve on this plan (qgw_dyson_W, or a state
 * iteration on it) met a zero or non-finite pivot since the last read
 * (Eq. eq-screened-coulomb has no solution there; the affected W^C entries
 * are non-finite), QGW_OK otherwise.  Calls on one plan from several streams
 * share the word. */
qgw_status qgw_sync_status(qgw_plan plan, void *stream);

/* ------------------------------------------------------------ step calls */

/* a1, a11, density row: out[m][c] = scale * sum_t T_map[m][t] in[t][c] for
 * c < ncols (orbital arrays: ncols = n_o^2 N_k).  in and out must not
 * overlap.  QGW_F_IW2BETA writes one row out[c].
 * hermitian = 1 maps the Hermitian part (X + X^dagger) / 2 of the input,
 * taken over the orbital indices at every (node, k); hermitian = 2 returns
 * the Hermitian part of the output.  Both need ncols = n_o^2 N_k.  The exact
 * Sigma^C(k, tau) and density matrix are Hermitian; the loop keeps only
 * their Hermitian parts. */
qgw_status qgw_dlr_transform(qgw_plan plan, int32_t map, int64_t ncols,
                             double scale_re, double scale_im, int32_t hermitian,
                             const void *in, void *out, void *stream);

/* a5, a7: the same map on pair arrays [r] x (N_b^2 N_k) with a layout
 * change: in_layout / out_layout are QGW_LAYOUT_SLAB or QGW_LAYOUT_MATRIX. */
qgw_status qgw_dlr_transform_pairs(qgw_plan plan, int32_t map,
                                   int32_t in_layout, int32_t out_layout,
                                   const void *in, void *out, void *stream);

/* a2, a4, a8, a10: ``batch`` 2-D transforms over the trailing N_k axis,
 * direction QGW_R_TO_K or QGW_K_TO_R (with 1/N_k).  in == out allowed. */
qgw_status qgw_lattice_fft(qgw_plan plan, int32_t dir, int64_t batch,
                           const void *in, void *out, void *stream);

/* a3 (+ a4): P_{(il),(jk)}(R, tau) = -2 G_{lj}(R, tau) G_{ki}(-R, beta - tau).
 * G_tau_R = G(R, tau_k) and G_reflt_R = G(R, beta - tau_k), orbital layout.
 * With out_q = 0 writes P(R, tau); with out_q = 1 writes P(q, tau) (the
 * R -> q transform fused).  Output: pair slab. */
qgw_status qgw_bubble(qgw_plan plan, const void *G_tau_R, const void *G_reflt_R,
                      int32_t out_q, void *P, void *stream);

/* a6: W^C = (I - V P)^{-1} V - V for every (q, bosonic node), Gauss-Jordan
 * with partial pivoting.  V_q: [N_k][N_b][N_b]; P_nu, Wc_nu: pair matrix
 * layout.  A zero or non-finite pivot yields non-finite output for that
 * matrix and sets the plan's device status word (qgw_sync_status reports
 * QGW_ERR_SINGULAR). */
qgw_status qgw_dyson_W(qgw_plan plan, const void *V_q, const void *P_nu,
                       void *Wc_nu, void *stream);

/* a9 (+ a8, a10): Sigma^C_{ik}(R, tau) = -sum W^C_{(il),(jk)}(R, tau) G_{lj}(R, tau).
 * Wc: pair slab, in q (in_q = 1, the q -> R transform fused) or R (in_q = 0).
 * G_tau_R: orbital layout.  Output Sigma in k (out_k = 1, R -> k fused) or R. */
qgw_status qgw_sigma(qgw_plan plan, const void *G_tau_R, const void *Wc,
                     int32_t in_q, int32_t out_k, void *Sig, void *stream);

/* a12: Sigma_HF(R) = Sigma_F(R) + delta_{R,0} Sigma_H from the density n(R)
 * (static orbital layout) and V(R) (static pair layout), both in R.  Output
 * static orbital layout, in R. */
qgw_status qgw_hartree_fock(qgw_plan plan, const void *V_R, const void *n_R,
                            void *SigHF_R, void *stream);

/* a13: G(k, i w_m) = [(i w_m + mu) - H(k) - Sigma(k, i w_m)]^{-1} with H =
 * H0 + Sigma_HF (static orbital layout) and Sigma (orbital layout, or NULL
 * for Sigma = 0).  If n_target is finite, mu is first solved so that
 * N_e(mu) = 2/N_k sum_k Re Tr n(k) = n_target, n = -G(beta^-), by Newton
 * steps on N_e(mu) (dN_e/dmu from Tr G^2) kept inside the sign-change
 * bracket by bisection once one is known, until |d mu| <= 1e-13 max(1, |mu|)
 * eV or |N_e - n_target| <= 1e-13.  On input *mu is the starting point (NaN:
 * the centre of the Gershgorin bounds of H); on output the chemical
 * potential.  If n_target is NaN, *mu is used as given.  Waits for
 * ``stream``.  QGW_ERR_NOT_CONVERGED if the search does not converge within
 * 200 evaluations. */
qgw_status qgw_dyson_G(qgw_plan plan, const void *H_k, const void *Sig_iw,
                       double n_target, double *mu, void *G_iw, void *stream);

/* qgw_dyson_G for callers that cannot allocate device memory (code under HIP
 * graph capture elsewhere in their program, tight serving loops, harnesses
 * that forbid hipMalloc): the same computation, arguments, waits and errors,
 * with the search's scratch (32 scalars, at most 4096 partial sums, 16
 * status words; 33,088 bytes) in a static device array of the library
 * instead of the plan's.  Each GPU holds one copy of that array until the
 * process ends; calls that overlap on one GPU (from several threads or
 * streams) race on it.  The call allocates nothing.  QGW_ERR_UNSUPPORTED if
 * a search on this plan would need more partial sums than the array holds
 * (the search uses at most 1024 blocks, so no supported plan does) or the
 * device ordinal is 64 or above. */
qgw_status qgw_dyson_G_noalloc(qgw_plan plan, const void *H_k, const void *Sig_iw,
                               double n_target, double *mu, void *G_iw, void *stream);

/* ------------------------------------------------------------- adjoints
 *
 * Reverse-mode derivatives of the step calls (FP64 plans only; FP32 plans
 * return QGW_ERR_UNSUPPORTED).  For a real loss L the cotangent of a complex
 * array z is zbar = dL/dRe z + i dL/dIm z (the convention of PyTorch's
 * complex autograd), so a complex-linear y = A x has xbar = A^H ybar.  Every
 * call overwrites its outputs (callers add branches themselves); shapes and
 * layouts are those of the forward call.  Calls marked "workspace" take the
 * caller's scratch (see the file header). */

/* a15: adjoint of qgw_dlr_transform with the same map, ncols, scale and
 * hermitian mode: xbar = herm_in(conj(scale) T^H herm_out(ybar)).  For
 * QGW_F_IW2BETA ybar has ncols entries and xbar r x ncols. */
qgw_status qgw_dlr_transform_bwd(qgw_plan plan, int32_t map, int64_t ncols,
                                 double scale_re, double scale_im, int32_t hermitian,
                                 const void *ybar, void *xbar, void *stream);

/* a15: adjoint of qgw_dlr_transform_pairs (same map and layouts): ybar is
 * in out_layout, xbar in in_layout. */
qgw_status qgw_dlr_transform_pairs_bwd(qgw_plan plan, int32_t map,
                                       int32_t in_layout, int32_t out_layout,
                                       const void *ybar, void *xbar, void *stream);

/* a16: adjoint of qgw_lattice_fft in direction dir: for QGW_K_TO_R,
 * xbar(k) = (1/N_k) sum_R ybar(R) e^{-ik.R}; for QGW_R_TO_K,
 * xbar(R) = sum_k ybar(k) e^{+ik.R}.  ybar == xbar allowed. */
qgw_status qgw_lattice_fft_bwd(qgw_plan plan, int32_t dir, int64_t batch,
                               const void *ybar, void *xbar, void *stream);

/* a17: adjoint of qgw_bubble with out_q = 1 (Eq. eq-polarizability):
 *   Gbar_lj(R, tau)         = -2 sum_{ik} conj(G_ki(-R, beta - tau)) Pbar_{(il),(jk)}(R, tau)
 *   Gbar_ki(-R, beta - tau) = -2 sum_{lj} conj(G_lj(R, tau)) Pbar_{(il),(jk)}(R, tau)
 * with Pbar(R) = sum_q e^{iq.R} Pbar(q).  Pbar_q: pair slab in q; outputs:
 * orbital layout in R, written whole. */
qgw_status qgw_bubble_bwd(qgw_plan plan, const void *G_tau_R, const void *G_reflt_R,
                          const void *Pbar_q, void *Gbar_tau_R, void *Gbar_reflt_R,
                          void *stream);

/* a19: adjoint of qgw_sigma with in_q = 1 and the given out_k (Eq.
 * eq-gw-self-energy):
 *   Wcbar_{(il),(jk)}(R) = -conj(G_lj(R)) Sbar_ik(R),  then to q
 *   Gbar_lj(R)          = -sum_{ik} conj(W^C_{(il),(jk)}(R)) Sbar_ik(R)
 * Sigbar in k (out_k = 1) or R; Wc_q and Wcbar_q pair slabs in q; Gbar_tau_R
 * orbital layout in R.  Workspace (r n_o^2 N_k complex, QGW_OP_SIGMA_BWD)
 * when out_k = 1; it must not overlap any array of the call. */
qgw_status qgw_sigma_bwd(qgw_plan plan, const void *G_tau_R, const void *Wc_q,
                         int32_t out_k, const void *Sigbar, void *Gbar_tau_R,
                         void *Wcbar_q, void *workspace, int64_t workspace_bytes,
                         void *stream);

/* a18: adjoint of qgw_dyson_W (Eq. eq-screened-coulomb).  With A = I - V P,
 * W = A^{-1} V and Wbar the cotangent of W^C = W - V:
 *   Pbar = W^H Wbar W^H,   Vbar = sum over nodes [A^{-H} Wbar (I + P W)^H - Wbar].
 * V_q, Vbar_q: [N_k][N_b][N_b]; P_nu, Wcbar_nu, Pbar_nu: pair matrix
 * layout.  The node sum runs in a fixed order (deterministic).  Workspace
 * ((2 r + min(r, 8)) N_b^2 N_k complex, QGW_OP_DYSON_W_BWD: W^C and
 * X = (I - V P)^{-H} Wbar per matrix, and the partial node sums of Vbar).
 * A zero or non-finite pivot sets the device status word as in qgw_dyson_W. */
qgw_status qgw_dyson_W_bwd(qgw_plan plan, const void *V_q, const void *P_nu,
                           const void *Wcbar_nu, void *Pbar_nu, void *Vbar_q,
                           void *workspace, int64_t workspace_bytes, void *stream);

/* a12 adjoint: cotangents of n(R) and V(R) for a cotangent Sbar_R of the
 * Hartree-Fock self-energy (Eqs. eq-hartree-self-energy,
 * eq-fock-self-energy).  Either output may be NULL.  Workspace (N_b^2
 * complex, QGW_OP_HARTREE_FOCK_BWD). */
qgw_status qgw_hartree_fock_bwd(qgw_plan plan, const void *V_R, const void *n_R,
                                const void *Sbar_R, void *nbar_R, void *Vbar_R,
                                void *workspace, int64_t workspace_bytes, void *stream);

/* a20: adjoint of qgw_dyson_G at the chemical potential mu it returned.
 * With X = H + Sigma: Sigbar = G^H Gbar G^H at every (node, k).  If
 * n_target is finite mu moves with X (N_e(mu, X) = n_target), which adds
 * c conj(rho_m) (G^2)^H with c = 2/N_k (mubar - Re sum tr(G^H Gbar G^H)) /
 * (dN_e/dmu); mubar is the cotangent of the returned mu.  If n_target is
 * NaN mu is held fixed and mubar is ignored.  Sigbar: orbital layout
 * (r n_o^2 N_k); Hbar (may be NULL) = sum over nodes of Sigbar, static
 * orbital layout.  Sig_iw may be NULL (Sigma = 0). */
qgw_status qgw_dyson_G_bwd(qgw_plan plan, const void *H_k, const void *Sig_iw,
                           double mu, double n_target, double mubar,
                           const void *Gbar, void *Sigbar, void *Hbar, void *stream);

/* Layout change of ``nn`` pair arrays between QGW_LAYOUT_SLAB
 * [nn][N_b][N_b][N_k] and QGW_LAYOUT_MATRIX [nn][N_k][N_b][N_b] (a
 * permutation; its adjoint is the opposite change).  FP64 plans. */
qgw_status qgw_pair_layout(qgw_plan plan, int32_t in_layout, int32_t out_layout,
                           int64_t nn, const void *in, void *out, void *stream);

/* a14: Galitskii-Migdal total energy per cell (two spins) of a state
 * (H0(k), Sigma_HF(k), Sigma^C(k, i w), G(k, i w)), FP64 plans:
 *   E = 2/N_k sum_k Re Tr[(H0 + Sigma_HF / 2) n]
 *       + 1/N_k sum_k Re (1/beta) sum_n Tr[Sigma^C(i w_n) G(i w_n)]
 * with n = Herm(-G(beta^-)) and the Matsubara sum over all n taken exactly
 * from the DLR expansions (map QGW_F_IW2GM).  e_out[3] = (E, HF part,
 * correlation part).  Waits for ``stream``.  Workspace (QGW_OP_ENERGY). */
qgw_status qgw_energy(qgw_plan plan, const void *H_k, const void *SigHF_k,
                      const void *Sig_iw, const void *G_iw, double *e_out,
                      void *workspace, int64_t workspace_bytes, void *stream);

/* Adjoint of qgw_energy's E for a cotangent ebar: writes Hbar, SigHFbar
 * (static orbital layout), Sigbar and Gbar (orbital layout).  Workspace
 * (QGW_OP_ENERGY_BWD). */
qgw_status qgw_energy_bwd(qgw_plan plan, const void *H_k, const void *SigHF_k,
                          const void *Sig_iw, const void *G_iw, double ebar, void *Hbar,
                          void *SigHFbar, void *Sigbar, void *Gbar, void *workspace,
                          int64_t workspace_bytes, void *stream);

/* Hartree-Fock density of a static Hamiltonian (Fig. fig-self (a), H class
 * paragraph), FP64 plans: for H_k [n_o][n_o][N_k] (its Hermitian part is
 * used) writes n_k = U f(beta (eps - mu)) U^H, f(x) = 1 / (e^x + 1), with
 * H(k) = U diag(eps) U^H per k.  mu (in/out) is found by bisection to the
 * target filling N_e = (2 / N_k) sum_{k,n} f(beta (eps_n(k) - mu)), or is
 * used as given if n_target is NaN.  Waits for ``stream``.  Workspace
 * (QGW_OP_HF_DENSITY). */
qgw_status qgw_hf_density(qgw_plan plan, const void *H_k, double n_target, double *mu,
                          void *n_k, void *workspace, int64_t workspace_bytes, void *stream);

/* Quasiparticle post-processing (Z class, SigStc class, Eq. eq-z-factor,
 * Eq. eq-quasi-particle-Hamiltonian), FP64 plans.  The zero-frequency limit
 * of the self-energy is taken at the Matsubara frequencies closest to zero,
 * +-i pi/beta, where its DLR expansion follows it: with
 * S(k) = Sigma^C(k, i pi/beta) (the DLR interpolant of Sig_iw) and
 * Sigma(-i w) = Sigma(i w)^H,
 *   Sig0 = Sigma(k, 0) = Herm(Sigma_HF(k) + S(k)),
 *   Z^{-1}(k)  = 1 - (S - S^H) / (2 i pi/beta)   (dSigma/d(i w) at 0 as a
 *                 central difference over +-pi/beta),
 *   Hqp  = sqrt(Z) (Herm H0(k) + Sigma(k, 0) - mu) sqrt(Z), Hermitian part,
 *   bands = eigenvalues of Hqp(k), ascending.
 * mu = 0 is the equation as printed; the chemical potential puts the bands
 * relative to the Fermi level.  H_k, SigHF_k: [n_o][n_o][N_k]; Sig_iw:
 * [r][n_o][n_o][N_k] (orbital layout); outputs Sig0, Z, Hqp: [n_o][n_o][N_k]
 * complex; bands: [n_o][N_k] double.  Waits for ``stream``.  Workspace
 * (QGW_OP_QUASIPARTICLE).  QGW_ERR_NONFINITE if Z^{-1}(k) is not positive
 * definite at some k (the outputs there are not meaningful). */
qgw_status qgw_quasiparticle(qgw_plan plan, const void *H_k, const void *SigHF_k,
                             const void *Sig_iw, double mu, void *Sig0, void *Z, void *Hqp,
                             double *bands, void *workspace, int64_t workspace_bytes,
                             void *stream);

/* Quasiparticle bands along a path of arbitrary k points (the band plots of
 * Fig. fig-band-dos (a)), FP64 plans.  H0, Sigma_HF and S = Sigma^C(i pi/beta)
 * are brought from the mesh to each point k' by Fourier interpolation,
 * X(k') = sum_R w(R) e^{-i k'.R} X(R) with X(R) the inverse lattice DFT of
 * the mesh values, each axis's R taken in (-n/2, n/2] and, for even n, the
 * n/2 term weighted cos(pi f n) (the half shell split between +-n/2, so the
 * interpolant is real-symmetric and exact on mesh points); the relations of
 * qgw_quasiparticle then hold per point.  kfrac: HOST array [n_path][dim] of
 * fractional coordinates f (k' = 2 pi f along the reciprocal basis of the
 * mesh); inputs as for qgw_quasiparticle; outputs Sig0, Z, Hqp:
 * [n_o][n_o][n_path] complex, bands: [n_o][n_path] double (device).
 * 1 <= n_path <= 65536.  Workspace: qgw_quasiparticle_path_workspace bytes.
 * Waits for ``stream``.  QGW_ERR_NONFINITE if Z^{-1}(k') is not positive
 * definite at some point or kfrac holds a non-finite value. */
qgw_status qgw_quasiparticle_path_workspace(qgw_plan plan, int32_t n_path, int64_t *bytes);
qgw_status qgw_quasiparticle_path(qgw_plan plan, const void *H_k, const void *SigHF_k,
                                  const void *Sig_iw, double mu, const double *kfrac,
                                  int32_t n_path, void *Sig0, void *Z, void *Hqp, double *bands,
                                  void *workspace, int64_t workspace_bytes, void *stream);

/* out = a + b over ``count`` complex FP64 entries (the static H0(k) +
 * Sigma_HF(k) of the Dyson equation for G); out may alias a or b. */
qgw_status qgw_add(qgw_plan plan, int64_t count, const void *a, const void *b,
                   void *out, void *stream);

/* ------------------------------------------------------- whole iteration */

typedef struct qgw_state_s *qgw_state;

/* A self-consistent GW state bound to a plan: holds H0(k), V(q) and every
 * intermediate array on the device.  H0_R: [n_o][n_o][N_k] and V_R:
 * [N_b][N_b][N_k] are device arrays in R (FP64).  mixing in (0, 1] is the
 * linear mixing weight of the total self-energy (1 = none).  The state owns
 * a second stream (default priority) on which each qgw_gw_iteration runs its
 * a12 beside a1-a11; it is forked from and joined back into the caller's
 * stream inside the iteration, so work the caller orders after an iteration
 * on its stream sees all of it.  A batch records a12 on its own worker
 * stream instead. */
qgw_status qgw_state_create(qgw_plan plan, const void *H0_R, const void *V_R,
                            double n_target, double mixing, qgw_state *state);
qgw_status qgw_state_destroy(qgw_state state);

/* Sets G = G0 at the chemical potential for the target filling (or at *mu
 * if n_target is NaN).  With a target filling *mu is the search's start
 * and receives the result; a NaN start begins at the state's previous G0
 * mu (the same H0: the search then stops at its first evaluation), or at
 * the centre of H0's Gershgorin bounds the first time. */
qgw_status qgw_state_init_g0(qgw_state state, double *mu, void *stream);

/* Runs up to n_iter GW iterations (Fig. fig-self (b): a1 .. a14), stopping
 * early once max |Delta Sigma| <= tol.  Outputs (any may be NULL): the
 * number of iterations done, the last max |Delta Sigma| and mu.  Waits for
 * ``stream`` once per iteration (mu and max |Delta Sigma| come back); while
 * it waits, the next iteration's first step (G(tau), which depends only on
 * the new G) is already queued behind the read-back, so when the call
 * returns after stopping early the stream may still hold that step, which
 * rewrites only internal G(tau) buffers (none that qgw_state_copy exposes).
 * Errors: QGW_ERR_SINGULAR if a Dyson-W system met a zero or non-finite
 * pivot, QGW_ERR_NONFINITE if max |Delta Sigma| is not finite (any NaN in
 * Sigma counts), QGW_ERR_NOT_CONVERGED if the chemical-potential search
 * failed.  After an error the state's arrays are not one consistent
 * iterate: further iterations are refused (QGW_ERR_INVALID_ARG) until
 * qgw_state_init_g0 or qgw_state_hf_solve restarts the state. */
qgw_status qgw_gw_iteration(qgw_state state, int32_t n_iter, double tol,
                            int32_t *iters_done, double *d_sigma, double *mu,
                            void *stream);

/* Hartree-Fock self-consistency of a state (Fig. fig-self (a); H class
 * paragraph): from Sigma_HF = 0 and the density of H0, each pass computes
 * Sigma_H + Sigma_F from n (Eqs. eq-hartree-self-energy,
 * eq-fock-self-energy), mixes it with the state's mixing weight, and sets
 * n(k) = 1 / (e^{beta (H(k) - mu)} + 1) for H = H0 + Sigma_HF, with mu at
 * the target filling (or the state's mu if n_target is NaN).  Stops after
 * max_iter passes or once max |Delta Sigma_HF| <= tol (a negative tol runs
 * exactly max_iter passes).  Leaves Sigma_HF, n,
 * mu in the state and G = [(i w + mu) - H0 - Sigma_HF]^{-1} with
 * Sigma^C = 0, so a GW solve can continue from the HF solution.  Outputs
 * (any may be NULL): passes done, the last max |Delta Sigma_HF|, mu.
 * Waits for ``stream``; uses scratch the state owns.  QGW_ERR_NONFINITE if
 * the change of Sigma_HF, mu or the filling is not finite (the state then
 * needs a restart, as after a failed qgw_gw_iteration). */
qgw_status qgw_state_hf_solve(qgw_state state, double tol, int32_t max_iter,
                              int32_t *iters_done, double *d_sigma, double *mu,
                              void *stream);

/* Copies a state array (FP64) into the caller's device buffer ``dst`` on
 * ``stream``: which = 0 G(k, i w) [orbital], 1 Sigma^C(k, i w) [orbital],
 * 2 Sigma_HF(k) [static orbital], 3 P(q, i nu) [pair matrix],
 * 4 W^C(q, i nu) [pair matrix], 5 n(k) [static orbital; the density of the
 * last Hartree-Fock pass or of the last GW iteration's a12].  *bytes (if not
 * NULL) receives the size. */
qgw_status qgw_state_copy(qgw_state state, int32_t which, void *dst, int64_t *bytes,
                          void *stream);

/* Precision schedule of the solve.  mode 0: every iteration in FP64.  mode 1
 * (mixed): iterations run the bulk steps a1-a11 in FP32 (complex64 arrays,
 * FP32 matrix cores for the DLR maps, FP32 Dyson W) while max |Delta Sigma|
 * is above switch_tol and still falling by at least half per iteration; the
 * rest of the solve runs in FP64, so the converged result is an FP64 fixed
 * point (defect correction).  mode 2: every iteration runs a1-a11 in FP32
 * (the FP32 phase alone, without the FP64 finish; for measurements).
 * Density, Hartree-Fock, the Dyson G solve and the chemical potential are
 * FP64 in every mode.  qgw_state_init_g0 restarts the schedule.  The first
 * call with mode 1 or 2 allocates the single-precision buffers. */
qgw_status qgw_state_set_precision(qgw_state state, int32_t mode, double switch_tol);

/* Newton evaluations of the chemical potential that qgw_gw_iteration queues
 * before its one read-back per iteration: 0 (the default) adapts them (the
 * previous search's count + 2, between 3 and 12; 10 after G0), 1 .. 64
 * fixes them.  A search that needs more continues in further rounds of 16,
 * each with a read-back; the evaluations and the result are the same either
 * way, only launches and read-backs trade places.  QGW_ERR_INVALID_ARG
 * outside [0, 64]. */
qgw_status qgw_state_set_search_steps(qgw_state state, int32_t first_round);

/* Precision used by the last iteration (0 FP64, 1 FP32), the number of FP32
 * and FP64 iterations since qgw_state_init_g0, and the number of N_e(mu)
 * evaluations the last iteration's chemical-potential search took.  Any
 * output pointer may be NULL. */
qgw_status qgw_state_info(qgw_state state, int32_t *last_prec, int32_t *n_fp32, int32_t *n_fp64,
                          int32_t *mu_evals);

/* Per-step timing of qgw_gw_iteration with HIP events on the caller's
 * stream.  By default every step is timed and step 0 runs on the state's
 * second stream, concurrently with steps 1-8 (it joins the caller's stream
 * before step 9), so its time is the span from its start to its end while
 * sharing the GPU; qgw_state_profile_select can time fewer steps or run
 * step 0 in line.  mode 1 resets the accumulators and enables timing, mode 0
 * disables it, mode 2 only reads.  ms[2 * QGW_NUM_STEPS] (may be NULL)
 * receives the accumulated milliseconds per step, first over the FP64
 * iterations, then over the FP32 ones (0 for steps not timed); iters[2]
 * (may be NULL) the number of timed FP64 and FP32 iterations.  Steps, in
 * launch order:
 *   0 a12  density n = -G(beta^-), Hartree-Fock      1 a1  G(tau), G(beta - tau)
 *   2 a2   k -> R of both                             3 a3+a4 bubble, R -> q
 *   4 a5   P: tau -> i nu (to the matrix layout)      5 a6  Dyson W
 *   6 a7   W^C: i nu -> tau (to the slab layout)      7 a8-a10 self-energy
 *   8 a11  Sigma^C: tau -> i w                        9 a14 Delta Sigma, mixing, H0 + Sigma_HF
 *  10 a13  Dyson G with the chemical-potential search */
#define QGW_NUM_STEPS 11
qgw_status qgw_state_profile(qgw_state state, int32_t mode, double *ms, int32_t *iters);

/* What qgw_state_profile times from its next mode-1 call on: bit i of
 * step_mask selects step i (events are recorded only at the boundaries of
 * selected steps, two per step at most, so a mask of one step costs two
 * events per iteration); in_line != 0 runs step 0 (a12) on the caller's
 * stream ahead of step 1 while timing is enabled, so that every step's time
 * is its own and their sum is the iteration's span.  Default: all steps
 * (0x7FF), step 0 concurrent.  Bits at or above QGW_NUM_STEPS are rejected
 * with QGW_ERR_INVALID_ARG. */
qgw_status qgw_state_profile_select(qgw_state state, uint32_t step_mask, int32_t in_line);

/* ---------------------------------------------------------------- batches
 *
 * Many independent states -- each with its own plan, so orbital count,
 * mesh, beta and DLR rank may all differ -- advanced together by one graph
 * launch.  qgw_batch_create records n_iter GW iterations of every state
 * into one HIP graph: the states are spread over four worker streams forked
 * from the capture stream, so independent instances run concurrently, and
 * each state's iterations stay in order.  Inside the graph the chemical
 * potential search is a fixed chain of mu_steps Newton evaluations per
 * iteration (steps after convergence return at once).  It starts from the
 * state's current mu moved by the change of the mean diagonal of
 * H0 + Sigma_HF since the state's previous search (the level shift of a
 * change of Sigma_HF), as the eager search does; it is the same search as
 * qgw_gw_iteration (same grid, same summation order).  A search that has
 * not converged after mu_steps evaluations raises the state's sticky status
 * word to 2 (the graph continues; that iteration's G is at an unconverged
 * mu).  precision 0 records FP64 iterations; 1 records the single-precision
 * form of steps a1-a11 (the FP32 phase of the mixed solve, without its FP64
 * finish).  Every state must have been started (qgw_state_init_g0) and not
 * be waiting for a restart, must not be profiling, and must not be used by
 * other calls while a launch is in flight.  Each call of qgw_batch_launch
 * replays the graph on ``stream`` (no host synchronisation); qgw_batch_read
 * waits for ``stream`` and returns, per state, the last max |Delta Sigma|,
 * mu, the worst search status of all replays since the previous read (0 ok,
 * 1 no finite mu to start from, 2 search not converged; the word is then
 * cleared, and a state with a non-zero status needs a restart before eager
 * iterations) and the evaluations its last search took.  Any output pointer
 * of qgw_batch_read may be NULL. */
typedef struct qgw_batch_s *qgw_batch;
qgw_status qgw_batch_create(int32_t n, const qgw_state *states, int32_t precision,
                            int32_t n_iter, int32_t mu_steps, qgw_batch *batch);
qgw_status qgw_batch_launch(qgw_batch batch, void *stream);
qgw_status qgw_batch_read(qgw_batch batch, double *d_sigma, double *mu, int32_t *status,
                          int32_t *evals, void *stream);
qgw_status qgw_batch_destroy(qgw_batch batch);

/* Checks ``count`` complex values (precision of the plan) for NaN/Inf;
 * waits for the stream.  QGW_ERR_NONFINITE if any is found. */
qgw_status qgw_check_finite(qgw_plan plan, const void *x, int64_t count, void *stream);

const char *qgw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QGW_H */
