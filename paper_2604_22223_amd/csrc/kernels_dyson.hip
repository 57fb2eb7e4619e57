// Dyson equations.
//
// Screened interaction (Eq. eq-screened-coulomb): for every (bosonic node,
// q) solve (I - V P) W = V and return W^C = W - V.  One lane owns one row of
// the augmented system [I - V P | V] in registers; the lanes of one matrix
// form a power-of-two segment of the wavefront.  Gauss-Jordan elimination
// with partial pivoting: the pivot row is found by a segmented arg-max over
// the unused rows (ties go to the lower row), broadcast through LDS, and
// eliminated from every other row, so each lane ends with the solution row
// of the column it pivoted.
//
// Green's function (Eq. full-green-freq): one thread per (fermionic node, k)
// inverts the n_o x n_o matrix (i w + mu) - H(k) - Sigma(k, i w) in registers
// (in-place Gauss-Jordan with partial pivoting).  The chemical potential for
// the target filling is found inside one cooperative launch: every
// evaluation of N_e(mu) = -2/N_k sum_{k,m} Re rho_m Tr G(k, i w_m) ends in a
// grid-wide barrier after which every block sums the same per-block partials
// in the same order, so all blocks take identical root-finding steps.
#include <hip/hip_cooperative_groups.h>

#include "qgw_internal.h"

namespace cg = cooperative_groups;

namespace qgw {

constexpr int pow2_ceil(int n) {
  int p = 1;
  while (p < n) p *= 2;
  return p;
}

// ---------------------------------------------------------------------------
// W^C = (I - V P)^{-1} V - V
// ---------------------------------------------------------------------------
template <int NB, typename T>
__global__ __launch_bounds__(64) void k_dyson_w(const cpx<T>* __restrict__ vq,
                                                const cpx<T>* __restrict__ pnu,
                                                cpx<T>* __restrict__ wc, int64_t nmat, int nk) {
  constexpr int SEG = pow2_ceil(NB);
  constexpr int MPW = 64 / SEG;
  constexpr int NN = NB * NB;
  __shared__ cpx<T> sp[MPW * NN];
  __shared__ cpx<T> piv[2][MPW][2 * NB];
  const int lane = threadIdx.x;
  const int mw = lane / SEG, row = lane % SEG;
  const int64_t mat0 = int64_t(blockIdx.x) * MPW;
  const int64_t mat = mat0 + mw;
  const bool valid = (mat < nmat) && (row < NB);
  const int q = int(valid ? mat % nk : 0);
  // stage the block's P matrices (contiguous in the matrix layout)
  const int64_t nload = (nmat - mat0 < MPW ? nmat - mat0 : MPW) * NN;
  for (int e = lane; e < MPW * NN; e += 64) sp[e] = e < nload ? pnu[mat0 * NN + e] : mk(T(0), T(0));
  cpx<T> a[NB], b[NB];
  if (valid) {
#pragma unroll
    for (int c = 0; c < NB; ++c) b[c] = vq[(int64_t(q) * NB + row) * NB + c];
  }
  __syncthreads();
  if (valid) {
    const cpx<T>* pm = sp + mw * NN;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      cpx<T> s = mk(T(c == row ? 1 : 0), T(0));
#pragma unroll
      for (int j = 0; j < NB; ++j) s = fms(s, b[j], pm[j * NB + c]);
      a[c] = s;
    }
  }
  bool used = false;
  int my_step = 0;
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    T val = (valid && !used) ? norm2(a[s]) : T(-1);
    int idx = row;
#pragma unroll
    for (int off = SEG / 2; off >= 1; off >>= 1) {
      const T ov = __shfl_xor(val, off, SEG);
      const int oi = __shfl_xor(idx, off, SEG);
      if (ov > val || (ov == val && oi < idx)) {
        val = ov;
        idx = oi;
      }
    }
    const bool me = valid && (row == idx);
    if (me) {
      used = true;
      my_step = s;
#pragma unroll
      for (int c = s; c < NB; ++c) piv[s & 1][mw][c] = a[c];
#pragma unroll
      for (int c = 0; c < NB; ++c) piv[s & 1][mw][NB + c] = b[c];
    }
    __syncthreads();
    if (valid) {
      const cpx<T>* pr = piv[s & 1][mw];
      const cpx<T> pinv = inv(pr[s]);
      if (me) {
#pragma unroll
        for (int c = s + 1; c < NB; ++c) a[c] = a[c] * pinv;
        a[s] = mk(T(1), T(0));
#pragma unroll
        for (int c = 0; c < NB; ++c) b[c] = b[c] * pinv;
      } else {
        const cpx<T> f = a[s] * pinv;
#pragma unroll
        for (int c = s + 1; c < NB; ++c) a[c] = fms(a[c], f, pr[c]);
        a[s] = mk(T(0), T(0));
#pragma unroll
        for (int c = 0; c < NB; ++c) b[c] = fms(b[c], f, pr[NB + c]);
      }
    }
  }
  // W^C row my_step = b - V row my_step; stage in LDS, store contiguously
  if (valid) {
    const cpx<T>* vr = vq + (int64_t(q) * NB + my_step) * NB;
#pragma unroll
    for (int c = 0; c < NB; ++c) sp[mw * NN + my_step * NB + c] = b[c] - vr[c];
  }
  __syncthreads();
  for (int e = lane; e < nload; e += 64) wc[mat0 * NN + e] = sp[e];
}

// ---------------------------------------------------------------------------
// n_o x n_o inverse in registers, Gauss-Jordan with partial pivoting
// ---------------------------------------------------------------------------
template <int NO>
__device__ __forceinline__ void invert_inplace(cpx<double> (&a)[NO][NO]) {
  int perm[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    int p = k;
    double best = norm2(a[k][k]);
#pragma unroll
    for (int i = k + 1; i < NO; ++i) {
      const double v = norm2(a[i][k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    perm[k] = p;
#pragma unroll
    for (int i = k + 1; i < NO; ++i) {
      const bool sw = (p == i);
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        const cpx<double> t = a[k][j];
        a[k][j] = sw ? a[i][j] : t;
        a[i][j] = sw ? t : a[i][j];
      }
    }
    const cpx<double> pinv = inv(a[k][k]);
    a[k][k] = mk(1.0, 0.0);
#pragma unroll
    for (int j = 0; j < NO; ++j) a[k][j] = a[k][j] * pinv;
#pragma unroll
    for (int i = 0; i < NO; ++i) {
      if (i == k) continue;
      const cpx<double> f = a[i][k];
      a[i][k] = mk(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < NO; ++j) a[i][j] = fms(a[i][j], f, a[k][j]);
    }
  }
#pragma unroll
  for (int k = NO - 1; k >= 0; --k) {
#pragma unroll
    for (int c = k + 1; c < NO; ++c) {
      const bool sw = (perm[k] == c);
#pragma unroll
      for (int i = 0; i < NO; ++i) {
        const cpx<double> t = a[i][k];
        a[i][k] = sw ? a[i][c] : t;
        a[i][c] = sw ? t : a[i][c];
      }
    }
  }
}

struct DysonGArgs {
  const zd* hk;       // [no][no][nk]
  const zd* sig;      // [r][no][no][nk] or null
  const double* wn;   // [r]
  const zd* rho;      // [r]: G(beta^-) = sum_m rho_m G(i w_m)
  zd* g;              // [r][no][no][nk]
  double* scal;       // [0] mu (in/out), [1] n_target, [2] evaluations, [3] final N_e
  double* partials;   // [2][4][max_blocks]
  int* status;        // 0 ok, 1 no bracket, 2 not converged
  int r, nk, mode, max_evals;
  double beta, tol_mu, tol_n;
};

template <int NO>
__device__ __forceinline__ void load_base(const DysonGArgs& A, int64_t gi, cpx<double> (&bm)[NO][NO]) {
  const int m = int(gi / A.nk), k = int(gi - int64_t(m) * A.nk);
  const double w = A.wn[m];
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const zd h = A.hk[(int64_t(i) * NO + j) * A.nk + k];
      cpx<double> v = mk(-h.re, -h.im);
      if (A.sig) {
        const zd sg = A.sig[((int64_t(m) * NO + i) * NO + j) * A.nk + k];
        v = v - sg;
      }
      if (i == j) v.im += w;
      bm[i][j] = v;
    }
}

// block-level deterministic sum (one wavefront per block)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

template <int NO>
__device__ double count_electrons(const DysonGArgs& A, double mu, cg::grid_group& grid, int buf) {
  const int64_t total = int64_t(A.r) * A.nk;
  const int64_t stride = int64_t(gridDim.x) * 64;
  double acc = 0.0;
  for (int64_t gi = int64_t(blockIdx.x) * 64 + threadIdx.x; gi < total; gi += stride) {
    cpx<double> a[NO][NO];
    load_base<NO>(A, gi, a);
#pragma unroll
    for (int i = 0; i < NO; ++i) a[i][i].re += mu;
    invert_inplace<NO>(a);
    cpx<double> tr = mk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < NO; ++i) tr = tr + a[i][i];
    const int m = int(gi / A.nk);
    const zd rh = A.rho[m];
    acc += rh.re * tr.re - rh.im * tr.im;
  }
  acc = wave_sum(acc);
  double* part = A.partials + int64_t(buf) * 4 * gridDim.x;
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
  grid.sync();
  double s = 0.0;
  for (int b = threadIdx.x; b < int(gridDim.x); b += 64) s += part[b];
  s = wave_sum(s);
  return -2.0 * s / double(A.nk);
}

template <int NO>
__global__ __launch_bounds__(64) void k_dyson_g(DysonGArgs A) {
  cg::grid_group grid = cg::this_grid();
  const int64_t total = int64_t(A.r) * A.nk;
  const int64_t stride = int64_t(gridDim.x) * 64;
  double mu = A.scal[0];
  int status = 0, evals = 0;
  double n_final = 0.0;
  if (A.mode == 1) {
    const double nt = A.scal[1];
    // Gershgorin bounds of H plus a bound on |Sigma|
    double glo = 1e300, ghi = -1e300, smax = 0.0;
    for (int64_t gi = int64_t(blockIdx.x) * 64 + threadIdx.x; gi < total; gi += stride) {
      const int m = int(gi / A.nk), k = int(gi - int64_t(m) * A.nk);
      for (int i = 0; i < NO; ++i) {
        double rad = 0.0;
        for (int j = 0; j < NO; ++j) {
          const zd h = A.hk[(int64_t(i) * NO + j) * A.nk + k];
          if (j != i) rad += sqrt(norm2(h));
          if (A.sig) smax = fmax(smax, sqrt(norm2(A.sig[((int64_t(m) * NO + i) * NO + j) * A.nk + k])));
        }
        const double d = A.hk[(int64_t(i) * NO + i) * A.nk + k].re;
        glo = fmin(glo, d - rad);
        ghi = fmax(ghi, d + rad);
      }
    }
    glo = wave_min(glo);
    ghi = wave_max(ghi);
    smax = wave_max(smax);
    double* part = A.partials + int64_t(1) * 4 * gridDim.x;
    if (threadIdx.x == 0) {
      part[blockIdx.x] = glo;
      part[gridDim.x + blockIdx.x] = ghi;
      part[2 * gridDim.x + blockIdx.x] = smax;
    }
    grid.sync();
    glo = 1e300;
    ghi = -1e300;
    smax = 0.0;
    for (int b = threadIdx.x; b < int(gridDim.x); b += 64) {
      glo = fmin(glo, part[b]);
      ghi = fmax(ghi, part[gridDim.x + b]);
      smax = fmax(smax, part[2 * gridDim.x + b]);
    }
    glo = wave_min(glo);
    ghi = wave_max(ghi);
    smax = wave_max(smax);
    const double pad = 10.0 / A.beta + NO * smax + 1.0;
    double lo = glo - pad, hi = ghi + pad;
    int buf = 0;
    double flo = count_electrons<NO>(A, lo, grid, buf) - nt;
    buf ^= 1;
    double fhi = count_electrons<NO>(A, hi, grid, buf) - nt;
    buf ^= 1;
    evals = 2;
    int widen = 0;
    while (!(flo < 0.0 && fhi > 0.0) && widen < 60) {
      const double w = hi - lo;
      lo -= w;
      hi += w;
      flo = count_electrons<NO>(A, lo, grid, buf) - nt;
      buf ^= 1;
      fhi = count_electrons<NO>(A, hi, grid, buf) - nt;
      buf ^= 1;
      evals += 2;
      ++widen;
    }
    if (!(flo < 0.0 && fhi > 0.0)) {
      status = 1;
      mu = 0.5 * (lo + hi);
    } else {
      // Illinois false position, every third step a bisection
      int side = 0;
      double c = 0.5 * (lo + hi), fc = 0.0;
      bool done = false;
      for (int it = 0; it < A.max_evals && !done; ++it) {
        if (it % 3 == 2) {
          c = 0.5 * (lo + hi);
        } else {
          c = hi - fhi * (hi - lo) / (fhi - flo);
          if (!(c > lo && c < hi)) c = 0.5 * (lo + hi);
        }
        fc = count_electrons<NO>(A, c, grid, buf) - nt;
        buf ^= 1;
        ++evals;
        if (fc < 0.0) {
          lo = c;
          flo = fc;
          if (side == -1) fhi *= 0.5;
          side = -1;
        } else if (fc > 0.0) {
          hi = c;
          fhi = fc;
          if (side == +1) flo *= 0.5;
          side = +1;
        } else {
          done = true;
        }
        if (hi - lo <= A.tol_mu || fabs(fc) <= A.tol_n) done = true;
      }
      mu = (fabs(fc) <= A.tol_n || hi - lo > A.tol_mu) ? c : 0.5 * (lo + hi);
      if (!done) status = 2;
      n_final = fc + nt;
    }
  }
  // G at the final mu
  for (int64_t gi = int64_t(blockIdx.x) * 64 + threadIdx.x; gi < total; gi += stride) {
    cpx<double> a[NO][NO];
    load_base<NO>(A, gi, a);
#pragma unroll
    for (int i = 0; i < NO; ++i) a[i][i].re += mu;
    invert_inplace<NO>(a);
    const int m = int(gi / A.nk), k = int(gi - int64_t(m) * A.nk);
#pragma unroll
    for (int i = 0; i < NO; ++i)
#pragma unroll
      for (int j = 0; j < NO; ++j) A.g[((int64_t(m) * NO + i) * NO + j) * A.nk + k] = a[i][j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.scal[0] = mu;
    A.scal[2] = double(evals);
    A.scal[3] = n_final;
    A.status[0] = status;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

template <int NB, typename T>
hipError_t dyson_w_nb(const Plan& p, const void* v_q, const void* p_nu, void* wc_nu, hipStream_t s) {
  constexpr int MPW = 64 / pow2_ceil(NB);
  const int64_t nmat = int64_t(p.r) * p.nk;
  const unsigned blocks = unsigned((nmat + MPW - 1) / MPW);
  hipLaunchKernelGGL((k_dyson_w<NB, T>), dim3(blocks), dim3(64), 0, s, (const cpx<T>*)v_q,
                     (const cpx<T>*)p_nu, (cpx<T>*)wc_nu, nmat, p.nk);
  return hipGetLastError();
}

template <int NO>
hipError_t dyson_g_no(const Plan& p, const void* h_k, const void* sig_iw, int mode, void* g_iw,
                      hipStream_t s) {
  DysonGArgs A;
  A.hk = (const zd*)h_k;
  A.sig = (const zd*)sig_iw;
  A.wn = p.d_wn;
  A.rho = (const zd*)p.dmaps64.m[5];
  A.g = (zd*)g_iw;
  A.scal = p.d_scalars;
  A.partials = p.d_partials;
  A.status = p.d_status;
  A.r = p.r;
  A.nk = p.nk;
  A.mode = mode;
  A.max_evals = 200;
  A.beta = p.beta;
  A.tol_mu = 1e-13;
  A.tol_n = 1e-13;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_dyson_g<NO>, 64, 0);
  if (e != hipSuccess) return e;
  int dev = 0, ncu = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  int64_t need = (int64_t(p.r) * p.nk + 63) / 64;
  int64_t cap = int64_t(per_cu) * ncu;
  if (cap > p.max_blocks) cap = p.max_blocks;
  const int blocks = int(need < cap ? need : cap);
  if (blocks < 1) return hipErrorInvalidConfiguration;
  void* args[] = {&A};
  return hipLaunchCooperativeKernel((const void*)k_dyson_g<NO>, dim3(blocks), dim3(64), args, 0, s);
}

}  // namespace

hipError_t launch_dyson_w(const Plan& p, const void* v_q, const void* p_nu, void* wc_nu,
                          hipStream_t s) {
  switch (p.nb) {
#define QGW_CASE(NBV) \
  case NBV:           \
    return p.prec == 0 ? dyson_w_nb<NBV, double>(p, v_q, p_nu, wc_nu, s) : dyson_w_nb<NBV, float>(p, v_q, p_nu, wc_nu, s);
    QGW_FOR_EACH_NB(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_dyson_g(const Plan& p, const void* h_k, const void* sig_iw, int mode, void* g_iw,
                          hipStream_t s) {
  switch (p.no) {
#define QGW_CASE(NOV) \
  case NOV:           \
    return dyson_g_no<NOV>(p, h_k, sig_iw, mode, g_iw, s);
    QGW_FOR_EACH_NO(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace qgw
