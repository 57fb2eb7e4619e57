// Per-thread eigen-decomposition of small Hermitian matrices held in
// registers (n_o <= 8), for the static problems per k: the quasiparticle
// Hamiltonian and the Hartree-Fock density.  Cyclic complex Jacobi: each
// rotation first turns a_pq real with a phase on column q, then zeroes it
// with a real plane rotation; sweeps stop at an off-diagonal norm below
// 1e-30 of the total (at most 30 sweeps).
#pragma once

#include "qgw_internal.h"

namespace qgw {

template <int NO>
struct HermEig {
  cpx<double> a[NO][NO];  // in: Hermitian matrix; out: diagonal holds the eigenvalues
  cpx<double> v[NO][NO];  // eigenvectors (columns)
};

template <int NO>
__device__ __forceinline__ double offdiag2(const cpx<double> (&a)[NO][NO], double& total) {
  double off = 0.0, all = 0.0;
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const double v = norm2(a[i][j]);
      all += v;
      if (i != j) off += v;
    }
  total = all;
  return off;
}

template <int NO, int P, int Q>
__device__ __forceinline__ void jacobi_rotate(HermEig<NO>& h) {
  const cpx<double> apq = h.a[P][Q];
  const double g = sqrt(norm2(apq));
  if (g == 0.0) return;
  const cpx<double> e = mk(apq.re / g, apq.im / g);  // a_pq = g e
  const double app = h.a[P][P].re, aqq = h.a[Q][Q].re;
  const double tau = (aqq - app) / (2.0 * g);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
  // W on the (P, Q) plane: W_PP = c, W_PQ = s, W_QP = -s conj(e), W_QQ = c conj(e)
  const cpx<double> ce = conj(e);
  // columns: A <- A W, V <- V W
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const cpx<double> ap = h.a[i][P], aq = h.a[i][Q];
    h.a[i][P] = scale(ap, c) - scale(aq * ce, s);
    h.a[i][Q] = scale(ap, s) + scale(aq * ce, c);
    const cpx<double> vp = h.v[i][P], vq = h.v[i][Q];
    h.v[i][P] = scale(vp, c) - scale(vq * ce, s);
    h.v[i][Q] = scale(vp, s) + scale(vq * ce, c);
  }
  // rows: A <- W^H A (W^H_PP = c, W^H_PQ = -s e, W^H_QP = s, W^H_QQ = c e)
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    const cpx<double> ap = h.a[P][j], aq = h.a[Q][j];
    h.a[P][j] = scale(ap, c) - scale(e * aq, s);
    h.a[Q][j] = scale(ap, s) + scale(e * aq, c);
  }
  h.a[P][Q] = mk(0.0, 0.0);
  h.a[Q][P] = mk(0.0, 0.0);
  h.a[P][P].im = 0.0;
  h.a[Q][Q].im = 0.0;
}

template <int NO, int P, int Q>
__device__ __forceinline__ void jacobi_row(HermEig<NO>& h) {
  if constexpr (Q < NO) {
    jacobi_rotate<NO, P, Q>(h);
    jacobi_row<NO, P, Q + 1>(h);
  }
}

template <int NO, int P>
__device__ __forceinline__ void jacobi_sweep(HermEig<NO>& h) {
  if constexpr (P < NO - 1) {
    jacobi_row<NO, P, P + 1>(h);
    jacobi_sweep<NO, P + 1>(h);
  }
}

template <int NO>
__device__ __forceinline__ void herm_eig(HermEig<NO>& h) {
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) h.v[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
  for (int sweep = 0; sweep < 30; ++sweep) {
    double total = 0.0;
    const double off = offdiag2<NO>(h.a, total);
    if (!(off > 1e-30 * total)) break;
    jacobi_sweep<NO, 0>(h);
  }
}

// out = V diag(f) V^H, Hermitian by construction
template <int NO>
__device__ __forceinline__ void spectral(const cpx<double> (&v)[NO][NO], const double (&f)[NO],
                                         cpx<double> (&out)[NO][NO]) {
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      cpx<double> acc = mk(0.0, 0.0);
#pragma unroll
      for (int n = 0; n < NO; ++n) acc = acc + scale(v[i][n] * conj(v[j][n]), f[n]);
      out[i][j] = acc;
    }
}

}  // namespace qgw
