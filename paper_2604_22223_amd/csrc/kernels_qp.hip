// Quasiparticle post-processing of a GW self-energy (Z class, SigStc class,
// Eq. eq-z-factor, Eq. eq-quasi-particle-Hamiltonian), FP64.
//
// The zero-frequency limit is taken at the Matsubara frequencies closest to
// zero, +-i pi/beta, where the DLR expansion of Sigma(k, i w) follows the
// function; with S = Sigma^C(k, i pi/beta) (one row of the DLR interpolant
// applied to the node values) and Sigma(-i w) = Sigma(i w)^H:
//   Sigma(k, 0)  = Sigma_HF(k) + (S + S^H) / 2
//   Z(k)^{-1}    = 1 - (S - S^H) / (2 i pi/beta)     (central difference)
//   H_QP(k)      = sqrt(Z) (H0 + Sigma(k, 0) - mu) sqrt(Z)
// and the bands are the eigenvalues of H_QP(k), ascending.
//
// One thread per k: the n_o x n_o Hermitian matrices stay in registers and
// are diagonalised by the Jacobi routine of qgw_herm.h.
//
// Off the mesh (bands along a path, Fig. fig-band-dos (a)), H0, Sigma_HF and
// S come from the mesh by Fourier interpolation: X(k') = sum_R w(R)
// e^{-2 pi i f.R} X(R), X(R) the inverse DFT of the mesh values, each axis's R
// taken in (-n/2, n/2] and, for even n, the n/2 term split equally between
// +n/2 and -n/2 (weight cos(pi f n)); on mesh points that is the mesh value.
// The same per-point kernel then runs on the path points.
#include "qgw_herm.h"

namespace qgw {

namespace {

template <int NO>
__global__ __launch_bounds__(64) void k_quasiparticle(const zd* __restrict__ hk, const zd* __restrict__ shf,
                                                      const zd* __restrict__ sig, const zd* __restrict__ row, int r,
                                                      int nk, double w0, double mu, zd* __restrict__ sig0,
                                                      zd* __restrict__ zout, zd* __restrict__ hqp,
                                                      double* __restrict__ bands, int* __restrict__ status) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= nk) return;
  auto at = [&](int i, int j) { return int64_t(i * NO + j) * nk + k; };
  // S = sum_m row[m] Sigma^C(i w_m)
  cpx<double> s[NO][NO];
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) s[i][j] = mk(0.0, 0.0);
  for (int m = 0; m < r; ++m) {
    const cpx<double> w = row ? row[m] : mk(1.0, 0.0);  // no row: sig already holds S (r = 1)
    const zd* sm = sig + int64_t(m) * NO * NO * nk;
#pragma unroll
    for (int i = 0; i < NO; ++i)
#pragma unroll
      for (int j = 0; j < NO; ++j) s[i][j] = fma(s[i][j], w, sm[at(i, j)]);
  }
  // Z^{-1} = 1 - (S - S^H) / (2 i w0); Sigma(k, 0) = Herm(Sigma_HF + S) goes to t
  HermEig<NO> h;
  cpx<double> t[NO][NO], sq[NO][NO];
  const double inv2w = 0.5 / w0;
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const cpx<double> d = s[i][j] - conj(s[j][i]);  // (S - S^H)_ij; d / (2 i w0) = -i d / (2 w0)
      h.a[i][j] = mk((i == j ? 1.0 : 0.0) - d.im * inv2w, d.re * inv2w);
      const cpx<double> hs = shf[at(i, j)], hst = shf[at(j, i)];
      t[i][j] = scale((hs + conj(hst)) + (s[i][j] + conj(s[j][i])), 0.5);
    }
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) sig0[at(i, j)] = t[i][j];
  herm_eig<NO>(h);
  double fz[NO], fs[NO];
  bool pos = true;
#pragma unroll
  for (int n = 0; n < NO; ++n) {
    const double lam = h.a[n][n].re;
    pos = pos && lam > 0.0;
    fz[n] = 1.0 / lam;
    fs[n] = 1.0 / sqrt(lam);
  }
  if (!pos) status[0] = 1;
  spectral<NO>(h.v, fz, s);  // Z
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) zout[at(i, j)] = s[i][j];
  spectral<NO>(h.v, fs, sq);  // sqrt(Z)
  // A = Herm(H0) + Sigma(k, 0) - mu, in s
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const cpx<double> a0 = hk[at(i, j)], a1 = hk[at(j, i)];
      s[i][j] = scale(a0 + conj(a1), 0.5) + t[i][j];
      if (i == j) s[i][j].re -= mu;
    }
  // H_QP = sqrt(Z) A sqrt(Z): t = A sqrt(Z), s = sqrt(Z) t
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      cpx<double> acc = mk(0.0, 0.0);
#pragma unroll
      for (int n = 0; n < NO; ++n) acc = fma(acc, s[i][n], sq[n][j]);
      t[i][j] = acc;
    }
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      cpx<double> acc = mk(0.0, 0.0);
#pragma unroll
      for (int n = 0; n < NO; ++n) acc = fma(acc, sq[i][n], t[n][j]);
      s[i][j] = acc;
    }
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      h.a[i][j] = scale(s[i][j] + conj(s[j][i]), 0.5);
      hqp[at(i, j)] = h.a[i][j];
    }
  herm_eig<NO>(h);
  double ev[NO];
#pragma unroll
  for (int n = 0; n < NO; ++n) ev[n] = h.a[n][n].re;
  // ascending order (exchange sort on registers)
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = i + 1; j < NO; ++j) {
      const double lo = fmin(ev[i], ev[j]), hi = fmax(ev[i], ev[j]);
      ev[i] = lo;
      ev[j] = hi;
    }
#pragma unroll
  for (int n = 0; n < NO; ++n) bands[int64_t(n) * nk + k] = ev[n];
}

// out[c] = sum_m row[m] in[m][c]: the DLR interpolant at i pi / beta of node values
__global__ __launch_bounds__(256) void k_row_apply(const zd* __restrict__ in, const zd* __restrict__ row, int r,
                                                   int64_t ncols, zd* __restrict__ out) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= ncols) return;
  cpx<double> s = mk(0.0, 0.0);
  for (int m = 0; m < r; ++m) s = fma(s, row[m], in[int64_t(m) * ncols + c]);
  out[c] = s;
}

// per-axis factor w(R) e^{-2 pi i f R} of the interpolation (R a mesh index 0 .. n-1)
__device__ __forceinline__ cpx<double> interp_phase(double f, int R, int n) {
  if (2 * R == n) return mk(cospi(f * double(n)), 0.0);
  const int rep = 2 * R < n ? R : R - n;
  double sn, cs;
  sincospi(-2.0 * f * double(rep), &sn, &cs);
  return mk(cs, sn);
}

// x_R: `narr` arrays of `nab` slabs [nab][N_k] in R, one after the other; out: [narr][nab][npt]
__global__ __launch_bounds__(256) void k_interp(const zd* __restrict__ x_r, int narr, int nab, int n, int dim,
                                                const double* __restrict__ kfrac, int npt, zd* __restrict__ out) {
  const int64_t gi = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t total = int64_t(narr) * nab * npt;
  if (gi >= total) return;
  const int pt = int(gi % npt);
  const int64_t slab = gi / npt;  // array * nab + ab
  const int64_t nk = dim == 3 ? int64_t(n) * n * n : int64_t(n) * n;
  const zd* x = x_r + slab * nk;
  const double f1 = kfrac[pt * dim], f2 = kfrac[pt * dim + 1], f3 = dim == 3 ? kfrac[pt * dim + 2] : 0.0;
  cpx<double> acc = mk(0.0, 0.0);
  for (int r1 = 0; r1 < n; ++r1) {
    const cpx<double> p1 = interp_phase(f1, r1, n);
    for (int r2 = 0; r2 < n; ++r2) {
      const cpx<double> p12 = p1 * interp_phase(f2, r2, n);
      if (dim == 3) {
        for (int r3 = 0; r3 < n; ++r3)
          acc = fma(acc, p12 * interp_phase(f3, r3, n), x[(int64_t(r1) * n + r2) * n + r3]);
      } else {
        acc = fma(acc, p12, x[int64_t(r1) * n + r2]);
      }
    }
  }
  out[slab * npt + pt] = acc;
}

template <int NO>
hipError_t quasiparticle_no(const Plan& p, const void* h_k, const void* shf_k, const void* sig_iw, double mu,
                            void* sig0, void* z, void* hqp, double* bands, int* status, hipStream_t s) {
  const double w0 = 3.14159265358979323846 / p.beta;
  hipLaunchKernelGGL((k_quasiparticle<NO>), dim3(unsigned((p.nk + 63) / 64)), dim3(64), 0, s, (const zd*)h_k,
                     (const zd*)shf_k, (const zd*)sig_iw, p.d_qp_row, p.r, p.nk, w0, mu, (zd*)sig0, (zd*)z,
                     (zd*)hqp, bands, status);
  return hipGetLastError();
}

template <int NO>
hipError_t quasiparticle_points_no(const Plan& p, int npt, const void* h, const void* shf, const void* sp, double mu,
                                   void* sig0, void* z, void* hqp, double* bands, int* status, hipStream_t s) {
  const double w0 = 3.14159265358979323846 / p.beta;
  hipLaunchKernelGGL((k_quasiparticle<NO>), dim3(unsigned((npt + 63) / 64)), dim3(64), 0, s, (const zd*)h,
                     (const zd*)shf, (const zd*)sp, (const zd*)nullptr, 1, npt, w0, mu, (zd*)sig0, (zd*)z, (zd*)hqp,
                     bands, status);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_quasiparticle_path(const Plan& p, const void* h_k, const void* shf_k, const void* sig_iw,
                                     const double* kfrac, int npt, double mu, void* ws, void* sig0, void* z,
                                     void* hqp, double* bands, int* status, hipStream_t s) {
  const int64_t nab = int64_t(p.no) * p.no, so = nab * p.nk;
  zd* s_k = (zd*)ws;       // S(k) on the mesh
  zd* x_r = s_k + so;      // H0, Sigma_HF, S in R
  zd* x_p = x_r + 3 * so;  // the same at the path points
  hipLaunchKernelGGL(k_row_apply, dim3(unsigned((so + 255) / 256)), dim3(256), 0, s, (const zd*)sig_iw,
                     (const zd*)p.d_qp_row, p.r, so, s_k);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_lattice_fft(p, +1, nab, h_k, x_r, s);  // k -> R with 1/N_k
  if (e == hipSuccess) e = launch_lattice_fft(p, +1, nab, shf_k, x_r + so, s);
  if (e == hipSuccess) e = launch_lattice_fft(p, +1, nab, s_k, x_r + 2 * so, s);
  if (e != hipSuccess) return e;
  const int64_t total = 3 * nab * npt;
  hipLaunchKernelGGL(k_interp, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, (const zd*)x_r, 3, int(nab),
                     p.n, p.dim, kfrac, npt, x_p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const zd* hp = x_p;
  const zd* shp = x_p + nab * npt;
  const zd* sp = x_p + 2 * nab * npt;
  switch (p.no) {
#define QGW_CASE(NOV) \
  case NOV:           \
    return quasiparticle_points_no<NOV>(p, npt, hp, shp, sp, mu, sig0, z, hqp, bands, status, s);
    QGW_FOR_EACH_NO(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_quasiparticle(const Plan& p, const void* h_k, const void* shf_k, const void* sig_iw, double mu,
                                void* sig0, void* z, void* hqp, double* bands, int* status, hipStream_t s) {
  switch (p.no) {
#define QGW_CASE(NOV) \
  case NOV:           \
    return quasiparticle_no<NOV>(p, h_k, shf_k, sig_iw, mu, sig0, z, hqp, bands, status, s);
    QGW_FOR_EACH_NO(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace qgw
