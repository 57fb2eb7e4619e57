// Hartree-Fock density (Fig. fig-self (a), H class paragraph), FP64.  For the
// static Hamiltonian H(k) = U diag(eps) U^H the density matrix is
//   n(k) = 1 / (e^{beta (H(k) - mu)} + 1) = U f(beta (eps - mu)) U^H,
// f(x) = 1 / (e^x + 1), with mu at the target filling
//   N_e(mu) = (2 / N_k) sum_{k, n} f(beta (eps_n(k) - mu)).
//   k_hf_eig      one thread per k: Jacobi eigen-decomposition (qgw_herm.h)
//   k_hf_mu       one block: safeguarded Newton for mu over all N_k n_o
//                 eigenvalues, each evaluation a fixed-order block reduction
//   k_hf_density  one thread per k: n = U f U^H
//   k_hf_delta_mix  one block: max |Sigma_new - Sigma_old|, then linear mixing
#include "qgw_herm.h"

namespace qgw {

namespace {

__device__ __forceinline__ double fermi_fn(double x) { return 0.5 * (1.0 - tanh(0.5 * x)); }

template <int NO>
__global__ __launch_bounds__(64) void k_hf_eig(const zd* __restrict__ hs, double* __restrict__ eps,
                                               zd* __restrict__ u, int nk) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= nk) return;
  HermEig<NO> h;
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const cpx<double> a = hs[int64_t(i * NO + j) * nk + k], b = hs[int64_t(j * NO + i) * nk + k];
      h.a[i][j] = scale(a + conj(b), 0.5);
    }
  herm_eig<NO>(h);
#pragma unroll
  for (int n = 0; n < NO; ++n) eps[int64_t(n) * nk + k] = h.a[n][n].re;
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int n = 0; n < NO; ++n) u[int64_t(i * NO + n) * nk + k] = h.v[i][n];
}

// block sums of f(beta (eps - mu)) and beta f (1 - f) over all eigenvalues (1024 threads), the same
// order on every call: per-thread sums, a xor butterfly in each wave, the 16 wave sums in a fixed order
__device__ void counts_at(const double* __restrict__ eps, int64_t count, double beta, double mu, double* red,
                          double& s0, double& s1) {
  double v0 = 0.0, v1 = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 1024) {
    const double f = fermi_fn(beta * (eps[i] - mu));
    v0 += f;
    v1 += beta * f * (1.0 - f);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    v0 += __shfl_xor(v0, off, 64);
    v1 += __shfl_xor(v1, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w] = v0;
    red[16 + w] = v1;
  }
  __syncthreads();
  s0 = s1 = 0.0;
  for (int i = 0; i < 16; ++i) {
    s0 += red[i];
    s1 += red[16 + i];
  }
  __syncthreads();
}

// scal: [0] mu (in: fixed mu when [1] is NaN, else the starting point if it lies inside the spectrum's
// bracket; out), [1] n_target, [2] evaluations, [3] N_e(mu).  Safeguarded Newton on
// N_e(mu) - n_target (dN_e/dmu = (2 / N_k) sum beta f (1 - f) > 0), kept inside the bracket that the
// evaluations shrink, with bisection where a step would leave it; stops at |d mu| <= 1e-13 max(1, |mu|)
// or |N_e - n_target| <= 1e-14 max(1, n_target).
__global__ __launch_bounds__(1024) void k_hf_mu(const double* __restrict__ eps, int64_t count, int nk, double beta,
                                                double* __restrict__ scal, int* __restrict__ status) {
  __shared__ double red[32];
  const double nt = scal[1];
  const double norm = 2.0 / double(nk);
  double mu = scal[0];
  int evals = 0;
  double s0 = 0.0, s1 = 0.0;
  if (isfinite(nt)) {
    double lo = 1e300, hi = -1e300;
    for (int64_t i = threadIdx.x; i < count; i += 1024) {
      lo = fmin(lo, eps[i]);
      hi = fmax(hi, eps[i]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, off, 64));
      hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6] = lo;
      red[16 + (threadIdx.x >> 6)] = hi;
    }
    __syncthreads();
    for (int i = 0; i < 16; ++i) {
      lo = fmin(lo, red[i]);
      hi = fmax(hi, red[16 + i]);
    }
    __syncthreads();
    lo -= 50.0 / beta + 1.0;
    hi += 50.0 / beta + 1.0;
    if (!(mu > lo && mu < hi)) mu = 0.5 * (lo + hi);
    for (int step = 0; step < 400; ++step) {
      counts_at(eps, count, beta, mu, red, s0, s1);
      ++evals;
      const double f = norm * s0 - nt, df = norm * s1;
      if (fabs(f) <= 1e-14 * fmax(1.0, nt)) break;
      if (f < 0.0)
        lo = mu;
      else
        hi = mu;
      double nxt = df > 0.0 ? mu - f / df : 0.5 * (lo + hi);
      if (!(nxt > lo && nxt < hi)) nxt = 0.5 * (lo + hi);
      const bool small = fabs(nxt - mu) <= 1e-13 * fmax(1.0, fabs(mu)) || hi - lo <= 1e-13 * fmax(1.0, fabs(mu));
      mu = nxt;
      if (small) break;
    }
  }
  counts_at(eps, count, beta, mu, red, s0, s1);
  if (threadIdx.x == 0) {
    scal[0] = mu;
    scal[2] = double(evals);
    scal[3] = norm * s0;
    status[0] = isfinite(mu) && isfinite(s0) ? 0 : 1;
  }
}

template <int NO>
__global__ __launch_bounds__(64) void k_hf_density(const double* __restrict__ eps, const zd* __restrict__ u,
                                                   const double* __restrict__ scal, double beta, zd* __restrict__ n,
                                                   int nk) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= nk) return;
  const double mu = scal[0];
  double occ[NO];
#pragma unroll
  for (int m = 0; m < NO; ++m) occ[m] = fermi_fn(beta * (eps[int64_t(m) * nk + k] - mu));
  cpx<double> v[NO][NO];
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int m = 0; m < NO; ++m) v[i][m] = u[int64_t(i * NO + m) * nk + k];
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      cpx<double> acc = mk(0.0, 0.0);
#pragma unroll
      for (int m = 0; m < NO; ++m) acc = acc + scale(v[i][m] * conj(v[j][m]), occ[m]);
      n[int64_t(i * NO + j) * nk + k] = acc;
    }
}

__global__ __launch_bounds__(256) void k_hf_delta_mix(zd* __restrict__ x_new, zd* __restrict__ x_old, int64_t count,
                                                      double alpha, double* __restrict__ d_out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) {
    cpx<double> a = x_new[i];
    const cpx<double> o = x_old[i];
    v = fmax(v, finite_or_inf(sqrt(norm2(a - o))));
    if (alpha != 1.0) {
      a = o + scale(a - o, alpha);
      x_new[i] = a;
    }
    x_old[i] = a;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) d_out[0] = red[0];
}

template <int NO>
hipError_t hf_density_no(const Plan& p, const void* hs, double* scal, int* status, void* u, double* eps, void* n,
                         hipStream_t s) {
  const unsigned blocks = unsigned((p.nk + 63) / 64);
  hipLaunchKernelGGL((k_hf_eig<NO>), dim3(blocks), dim3(64), 0, s, (const zd*)hs, eps, (zd*)u, p.nk);
  hipLaunchKernelGGL(k_hf_mu, dim3(1), dim3(1024), 0, s, (const double*)eps, int64_t(NO) * p.nk, p.nk, p.beta, scal,
                     status);
  hipLaunchKernelGGL((k_hf_density<NO>), dim3(blocks), dim3(64), 0, s, (const double*)eps, (const zd*)u,
                     (const double*)scal, p.beta, (zd*)n, p.nk);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_hf_density(const Plan& p, const void* hs, double* scal, int* status, void* u, double* eps, void* n,
                             hipStream_t s) {
  switch (p.no) {
#define QGW_CASE(NOV) \
  case NOV:           \
    return hf_density_no<NOV>(p, hs, scal, status, u, eps, n, s);
    QGW_FOR_EACH_NO(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_hf_delta_mix(const Plan& p, void* x_new, void* x_old, double alpha, double* d_out, hipStream_t s) {
  hipLaunchKernelGGL(k_hf_delta_mix, dim3(1), dim3(256), 0, s, (zd*)x_new, (zd*)x_old,
                     int64_t(p.no) * p.no * p.nk, alpha, d_out);
  return hipGetLastError();
}

}  // namespace qgw
