// Small kernels: Hartree-Fock self-energy (Eqs. eq-hartree-self-energy,
// eq-fock-self-energy), V(q = 0), layout changes of static arrays, the
// self-energy change / mixing of the self-consistency loop, finiteness check.
#include <algorithm>

#include "qgw_internal.h"

namespace qgw {

// Sigma_HF_{ik}(R) = - sum_terms V_{(il),(jk)}(R) n_{lj}(R)
//                    + delta_{R,0} 2 sum_beta V_{(ik),beta}(q=0) n_{k_beta j_beta}(0)
// Four adjacent lanes share one output (i, k, R): each sums every fourth term, and two xor shuffles add the four
// partial sums in a fixed order.
__global__ __launch_bounds__(256) void k_hartree_fock(const zd* __restrict__ v_r, const zd* __restrict__ v_q0,
                                                      const zd* __restrict__ n_r, zd* __restrict__ out,
                                                      int no, int nb, int nk, const int* __restrict__ pairs,
                                                      const int4* __restrict__ terms,
                                                      const int* __restrict__ term_off) {
  const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int part = int(g & 3);
  const int64_t gi = g >> 2;
  const bool valid = gi < int64_t(no) * no * nk;
  const int rr = valid ? int(gi % nk) : 0;
  const int ik = valid ? int(gi / nk) : 0;
  const int i = ik / no, k = ik % no;
  cpx<double> s = mk(0.0, 0.0);
  if (valid) {
    for (int t = term_off[ik] + part; t < term_off[ik + 1]; t += 4) {
      const int4 tm = terms[t];
      s = fms(s, v_r[(int64_t(tm.x) * nb + tm.y) * nk + rr], n_r[(int64_t(tm.z) * no + tm.w) * nk + rr]);
    }
  }
  // every lane of the wave takes part in the shuffles
  s.re += __shfl_xor(s.re, 1, 64);
  s.im += __shfl_xor(s.im, 1, 64);
  s.re += __shfl_xor(s.re, 2, 64);
  s.im += __shfl_xor(s.im, 2, 64);
  if (!valid || part != 0) return;
  if (rr == 0) {
    const int al = pairs[2 * nb + i * no + k];  // pair (i, k) if on one site
    if (al >= 0) {
      cpx<double> h = mk(0.0, 0.0);
      for (int be = 0; be < nb; ++be) {
        const int j = pairs[be], kk = pairs[nb + be];
        h = fma(h, v_q0[int64_t(al) * nb + be], n_r[(int64_t(kk) * no + j) * nk]);
      }
      s = s + scale(h, 2.0);
    }
  }
  out[gi] = s;
}

// V(q = 0) = sum_R V(R), fixed summation order
// V(q = 0) = sum_R V(R): one wavefront per pair entry, lanes striding over R (coalesced), then a xor butterfly
// in a fixed order (the same bits in every lane)
__global__ __launch_bounds__(64) void k_pair_sum_r(const zd* __restrict__ v_r, zd* __restrict__ v_q0, int nbb,
                                                   int nk) {
  const int ab = blockIdx.x;
  const zd* row = v_r + int64_t(ab) * nk;
  double re = 0.0, im = 0.0;
  for (int rr = threadIdx.x; rr < nk; rr += 64) {
    const zd v = row[rr];
    re += v.re;
    im += v.im;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (threadIdx.x == 0 && ab < nbb) v_q0[ab] = mk(re, im);
}

// [A][q] -> [q][A] for a static pair array
__global__ void k_static_transpose(const zd* __restrict__ in, zd* __restrict__ out, int na, int nq) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= int64_t(na) * nq) return;
  const int a = int(gi % na);
  const int64_t q = gi / na;
  out[gi] = in[int64_t(a) * nq + q];
}

__global__ void k_add(const zd* __restrict__ a, const zd* __restrict__ b, zd* __restrict__ out, int64_t n) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi < n) out[gi] = a[gi] + b[gi];
}

// a14 in one pass.  A block owns 64 static entries st; its four waves split the r node entries of the
// self-energy at those st (wave g takes nodes g, g + 4, ..).  Per-block max of |(hf_new + c_new) - (hf_old + c_old)|
// (a non-finite entry counts as +inf), new <- old + alpha (new - old) and old <- new for the node entries; after a
// barrier (every wave has read the static Sigma_HF(st)) wave 0 mixes and copies Sigma_HF(st) and, with h0 given,
// writes the static H = H0 + Sigma_HF of the Dyson equation for G into hs.
__global__ __launch_bounds__(256) void k_delta_mix(zd* __restrict__ hf_new, zd* __restrict__ c_new,
                                                   zd* __restrict__ hf_old, zd* __restrict__ c_old, int64_t ns,
                                                   int r, double alpha, double* __restrict__ block_max,
                                                   const zd* __restrict__ h0, zd* __restrict__ hs, int no, int nk,
                                                   double* __restrict__ diag_sum) {
  __shared__ double red[256];
  const int g = threadIdx.x >> 6;
  const int64_t st = int64_t(blockIdx.x) * 64 + (threadIdx.x & 63);
  const bool ok = st < ns;
  double v = 0.0;
  cpx<double> h = mk(0.0, 0.0), ho = mk(0.0, 0.0);
  if (ok) {
    h = hf_new[st];
    ho = hf_old[st];
    for (int m = g; m < r; m += 4) {
      const int64_t gi = int64_t(m) * ns + st;
      cpx<double> c = c_new[gi];
      const cpx<double> co = c_old[gi];
      const cpx<double> d = (h + c) - (ho + co);
      v = fmax(v, finite_or_inf(sqrt(norm2(d))));
      if (alpha != 1.0) {
        c = co + scale(c - co, alpha);
        c_new[gi] = c;
      }
      c_old[gi] = c;
    }
  }
  red[threadIdx.x] = v;
  __syncthreads();  // every wave has read hf_new[st] and hf_old[st]
  if (g == 0) {
    double dv = 0.0;
    if (ok) {
      if (alpha != 1.0) {
        h = ho + scale(h - ho, alpha);
        hf_new[st] = h;
      }
      hf_old[st] = h;
      if (h0) {
        const cpx<double> t = h0[st] + h;
        hs[st] = t;
        if (int(st / nk) % (no + 1) == 0) dv = t.re;  // a diagonal entry (i, i)
      }
    }
    if (diag_sum) {
      // this block's part of the diagonal sum of H0 + Sigma_HF, for the start of the next search (fixed order)
      for (int off = 32; off >= 1; off >>= 1) dv += __shfl_xor(dv, off, 64);
      if (threadIdx.x == 0) diag_sum[blockIdx.x] = dv;
    }
  }
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) block_max[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_max_reduce(const double* __restrict__ in, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v = fmax(v, in[i]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

template <typename T>
__global__ void k_count_nonfinite(const cpx<T>* __restrict__ x, int64_t n, int* __restrict__ count) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  const cpx<T> v = x[gi];
  if (!isfinite(v.re) || !isfinite(v.im)) atomicAdd(count, 1);
}

// precision changes of complex arrays (round to nearest)
__global__ void k_to_f32(const zd* __restrict__ in, zf* __restrict__ out, int64_t n) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi < n) out[gi] = cast<float>(in[gi]);
}
__global__ void k_to_f64(const zf* __restrict__ in, zd* __restrict__ out, int64_t n) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi < n) out[gi] = cast<double>(in[gi]);
}


// ---- adjoints -------------------------------------------------------------

// out[e] = sum_c partial[c][e], chunks in a fixed order
__global__ void k_sum_chunks(const zd* __restrict__ part, zd* __restrict__ out, int64_t n, int chunks) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  cpx<double> s = part[gi];
  for (int c = 1; c < chunks; ++c) s = s + part[int64_t(c) * n + gi];
  out[gi] = s;
}

// out[ab][k] = sum_m x[m][ab][k]
__global__ void k_sum_nodes(const zd* __restrict__ x, zd* __restrict__ out, int64_t n, int r) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  cpx<double> s = mk(0.0, 0.0);
  for (int m = 0; m < r; ++m) s = s + x[int64_t(m) * n + gi];
  out[gi] = s;
}

// Adjoint of the Hartree-Fock self-energy in the density:
//   nbar_lj(R) = -sum_{(il),(jk)} conj(V_{(il),(jk)}(R)) Sbar_ik(R)
//                + delta_{R,0} 2 sum_alpha conj(V_{alpha,beta}(q = 0)) Sbar_alpha(0), beta = (j', k') with (k', j') = (l, j)
__global__ __launch_bounds__(256) void k_hf_bwd_n(const zd* __restrict__ v_r, const zd* __restrict__ v_q0,
                                                  const zd* __restrict__ sbar, zd* __restrict__ nbar, int no,
                                                  int nb, int nk, const int* __restrict__ pairs,
                                                  const int4* __restrict__ terms_lj,
                                                  const int* __restrict__ off_lj) {
  const int64_t gi = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (gi >= int64_t(no) * no * nk) return;
  const int rr = int(gi % nk);
  const int lj = int(gi / nk);
  cpx<double> s = mk(0.0, 0.0);
  for (int t = off_lj[lj]; t < off_lj[lj + 1]; ++t) {
    const int4 tm = terms_lj[t];
    s = fms(s, conj(v_r[(int64_t(tm.x) * nb + tm.y) * nk + rr]), sbar[(int64_t(tm.z) * no + tm.w) * nk + rr]);
  }
  if (rr == 0) {
    const int a = lj / no, b = lj % no;
    const int be = pairs[2 * nb + b * no + a];  // pair (b, a): first b, second a
    if (be >= 0) {
      cpx<double> h = mk(0.0, 0.0);
      for (int al = 0; al < nb; ++al) {
        const int i = pairs[al], l = pairs[nb + al];
        h = fma(h, conj(v_q0[int64_t(al) * nb + be]), sbar[(int64_t(i) * no + l) * nk]);
      }
      s = s + scale(h, 2.0);
    }
  }
  nbar[gi] = s;
}

// Adjoint in V(R): Vbar_{(il),(jk)}(R) = -conj(n_lj(R)) Sbar_ik(R) + 2 conj(n_kj(0)) Sbar_il(0)
// (the Hartree term sees V(q = 0) = sum_R V(R))
__global__ __launch_bounds__(256) void k_hf_bwd_v(const zd* __restrict__ n_r, const zd* __restrict__ sbar,
                                                  zd* __restrict__ vbar, int no, int nb, int nk,
                                                  const int* __restrict__ pairs) {
  const int64_t gi = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (gi >= int64_t(nb) * nb * nk) return;
  const int rr = int(gi % nk);
  const int ab = int(gi / nk);
  const int al = ab / nb, be = ab % nb;
  const int i = pairs[al], l = pairs[nb + al], j = pairs[be], k = pairs[nb + be];
  cpx<double> v = -(conj(n_r[(int64_t(l) * no + j) * nk + rr]) * sbar[(int64_t(i) * no + k) * nk + rr]);
  v = v + scale(conj(n_r[(int64_t(k) * no + j) * nk]) * sbar[(int64_t(i) * no + l) * nk], 2.0);
  vbar[gi] = v;
}

// pair arrays: slab [nn][A][k] <-> matrix [nn][k][A], A = (alpha, beta)
__global__ void k_pair_layout(const zd* __restrict__ in, zd* __restrict__ out, int64_t total, int na, int nq,
                              int to_matrix) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= total) return;
  const int64_t plane = int64_t(na) * nq;
  const int64_t n = gi / plane, rem = gi - n * plane;
  if (to_matrix) {
    const int64_t q = rem / na, a = rem - q * na;
    out[gi] = in[n * plane + a * nq + q];
  } else {
    const int64_t a = rem / nq, q = rem - a * nq;
    out[gi] = in[n * plane + q * na + a];
  }
}

// ---- total energy ----------------------------------------------------------

// per-block partial sums of Re (H + Sigma_HF / 2)_ab n_ba (static entries) and of
// Re Y_m,ab G_m,ba (node entries), orbital transposes read directly
__global__ __launch_bounds__(256) void k_energy_sums(const zd* __restrict__ h, const zd* __restrict__ shf,
                                                     const zd* __restrict__ n, const zd* __restrict__ y,
                                                     const zd* __restrict__ g, int no, int nk, int r,
                                                     double* __restrict__ part) {
  __shared__ double red[2][256];
  const int64_t ns = int64_t(no) * no * nk, nt = ns * r;
  const int64_t stride = int64_t(gridDim.x) * 256;
  double a = 0.0, b = 0.0;
  for (int64_t gi = int64_t(blockIdx.x) * 256 + threadIdx.x; gi < nt; gi += stride) {
    const int64_t k = gi % nk, mab = gi / nk;
    const int ab = int(mab % (int64_t(no) * no));
    const int64_t m = mab / (int64_t(no) * no);
    const int i = ab / no, j = ab % no;
    const int64_t tr = (m * no * no + int64_t(j) * no + i) * nk + k;
    const cpx<double> p = y[gi] * g[tr];
    b += p.re;
    if (gi < ns) {
      const cpx<double> av = h[gi] + scale(shf[gi], 0.5);
      const cpx<double> q = av * n[(int64_t(j) * no + i) * nk + k];
      a += q.re;
    }
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = red[0][0];
    part[gridDim.x + blockIdx.x] = red[1][0];
  }
}

__global__ __launch_bounds__(256) void k_energy_final(const double* __restrict__ part, int nblk,
                                                      double* __restrict__ out) {
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) {
    a += part[i];
    b += part[nblk + i];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

// Abar = c conj(n^T): hbar = Abar, shfbar = Abar / 2; nbar = c conj(A^T), A = H + Sigma_HF / 2
__global__ void k_energy_bwd_static(const zd* __restrict__ h, const zd* __restrict__ shf, const zd* __restrict__ n,
                                    double c, zd* __restrict__ hbar, zd* __restrict__ shfbar, zd* __restrict__ nbar,
                                    int no, int nk) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= int64_t(no) * no * nk) return;
  const int64_t k = gi % nk;
  const int ab = int(gi / nk), i = ab / no, j = ab % no;
  const int64_t tr = (int64_t(j) * no + i) * nk + k;
  const cpx<double> abar = scale(conj(n[tr]), c);
  hbar[gi] = abar;
  shfbar[gi] = scale(abar, 0.5);
  nbar[gi] = scale(conj(h[tr] + scale(shf[tr], 0.5)), c);
}

// gbar += c conj(Y^T); ybar = c conj(G^T) (transpose over the orbital pair at each node and k)
__global__ void k_energy_bwd_nodes(const zd* __restrict__ y, const zd* __restrict__ g, double c,
                                   zd* __restrict__ gbar, zd* __restrict__ ybar, int no, int nk, int r) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nt = int64_t(no) * no * nk * r;
  if (gi >= nt) return;
  const int64_t k = gi % nk, mab = gi / nk;
  const int ab = int(mab % (int64_t(no) * no));
  const int64_t m = mab / (int64_t(no) * no);
  const int i = ab / no, j = ab % no;
  const int64_t tr = (m * no * no + int64_t(j) * no + i) * nk + k;
  gbar[gi] = gbar[gi] + scale(conj(y[tr]), c);
  ybar[gi] = scale(conj(g[tr]), c);
}

static unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

hipError_t launch_convert(int64_t count, const void* in, void* out, int to_f32, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (to_f32)
    hipLaunchKernelGGL(k_to_f32, dim3(nblk(count, 256)), dim3(256), 0, s, (const zd*)in, (zf*)out, count);
  else
    hipLaunchKernelGGL(k_to_f64, dim3(nblk(count, 256)), dim3(256), 0, s, (const zf*)in, (zd*)out, count);
  return hipGetLastError();
}

hipError_t launch_hartree_fock(const Plan& p, const void* v_r, const void* v_q0, const void* n_r,
                               void* sig_hf_r, hipStream_t s) {
  const int64_t n = int64_t(p.no) * p.no * p.nk;
  hipLaunchKernelGGL(k_hartree_fock, dim3(nblk(4 * n, 256)), dim3(256), 0, s, (const zd*)v_r,
                     (const zd*)v_q0, (const zd*)n_r, (zd*)sig_hf_r, p.no, p.nb, p.nk, p.d_pairs,
                     (const int4*)p.terms.d_terms, p.terms.d_off);
  return hipGetLastError();
}

hipError_t launch_pair_sum_r(const Plan& p, const void* v_r, void* v_q0, hipStream_t s) {
  const int nbb = p.nb * p.nb;
  hipLaunchKernelGGL(k_pair_sum_r, dim3(unsigned(nbb)), dim3(64), 0, s, (const zd*)v_r, (zd*)v_q0, nbb, p.nk);
  return hipGetLastError();
}

hipError_t launch_slab_to_matrix_static(const Plan& p, const void* in, void* out, hipStream_t s) {
  const int na = p.nb * p.nb;
  const int64_t n = int64_t(na) * p.nk;
  hipLaunchKernelGGL(k_static_transpose, dim3(nblk(n, 256)), dim3(256), 0, s, (const zd*)in, (zd*)out, na, p.nk);
  return hipGetLastError();
}

hipError_t launch_add(const Plan& p, int64_t count, const void* a, const void* b, void* out, hipStream_t s) {
  (void)p;
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add, dim3(nblk(count, 256)), dim3(256), 0, s, (const zd*)a, (const zd*)b, (zd*)out, count);
  return hipGetLastError();
}

hipError_t launch_delta_and_mix(const Plan& p, void* hf_new, void* c_new, void* hf_old, void* c_old,
                                double alpha, double* d_out, double* block_scratch, hipStream_t s, const void* h0,
                                void* hs, bool reduce) {
  const int64_t ns = int64_t(p.no) * p.no * p.nk;
  const int64_t blocks = nblk(ns, 64);
  if (blocks > 4096) return hipErrorInvalidValue;  // the state's block scratch holds 4096 maxima
  hipLaunchKernelGGL(k_delta_mix, dim3(unsigned(blocks)), dim3(256), 0, s, (zd*)hf_new, (zd*)c_new, (zd*)hf_old,
                     (zd*)c_old, ns, p.r, alpha, block_scratch, (const zd*)h0, (zd*)hs, p.no, p.nk,
                     h0 ? block_scratch + 4096 : nullptr);
  if (reduce)
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, (const double*)block_scratch, int(blocks), d_out);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const Plan& p, const void* x, int64_t count, int* d_count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (p.prec == 0)
    hipLaunchKernelGGL(k_count_nonfinite<double>, dim3(nblk(count, 256)), dim3(256), 0, s, (const zd*)x, count, d_count);
  else
    hipLaunchKernelGGL(k_count_nonfinite<float>, dim3(nblk(count, 256)), dim3(256), 0, s, (const zf*)x, count, d_count);
  return hipGetLastError();
}

hipError_t launch_sum_chunks(int64_t n, int chunks, const void* partial, void* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_chunks, dim3(nblk(n, 256)), dim3(256), 0, s, (const zd*)partial, (zd*)out, n, chunks);
  return hipGetLastError();
}

hipError_t launch_sum_nodes(const Plan& p, const void* x, void* out, hipStream_t s) {
  const int64_t n = int64_t(p.no) * p.no * p.nk;
  hipLaunchKernelGGL(k_sum_nodes, dim3(nblk(n, 256)), dim3(256), 0, s, (const zd*)x, (zd*)out, n, p.r);
  return hipGetLastError();
}

hipError_t launch_hartree_fock_bwd(const Plan& p, const void* v_r, const void* v_q0, const void* n_r,
                                   const void* sbar_r, void* nbar_r, void* vbar_r, hipStream_t s) {
  const int64_t nn = int64_t(p.no) * p.no * p.nk;
  const int64_t nv = int64_t(p.nb) * p.nb * p.nk;
  if (nbar_r)
    hipLaunchKernelGGL(k_hf_bwd_n, dim3(nblk(nn, 256)), dim3(256), 0, s, (const zd*)v_r, (const zd*)v_q0,
                       (const zd*)sbar_r, (zd*)nbar_r, p.no, p.nb, p.nk, p.d_pairs, (const int4*)p.terms_lj.d_terms,
                       p.terms_lj.d_off);
  if (vbar_r)
    hipLaunchKernelGGL(k_hf_bwd_v, dim3(nblk(nv, 256)), dim3(256), 0, s, (const zd*)n_r, (const zd*)sbar_r,
                       (zd*)vbar_r, p.no, p.nb, p.nk, p.d_pairs);
  return hipGetLastError();
}

hipError_t launch_energy_sums(const Plan& p, const void* h_k, const void* shf_k, const void* n_k, const void* y,
                              const void* g, double* partials, double* out2, hipStream_t s) {
  const int64_t nt = int64_t(p.no) * p.no * p.nk * p.r;
  const int blocks = int(std::min<int64_t>((nt + 255) / 256, 4096));
  hipLaunchKernelGGL(k_energy_sums, dim3(blocks), dim3(256), 0, s, (const zd*)h_k, (const zd*)shf_k, (const zd*)n_k,
                     (const zd*)y, (const zd*)g, p.no, p.nk, p.r, partials);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, s, (const double*)partials, blocks, out2);
  return hipGetLastError();
}

hipError_t launch_energy_bwd_static(const Plan& p, const void* h_k, const void* shf_k, const void* n_k, double c,
                                    void* hbar, void* shfbar, void* nbar, hipStream_t s) {
  const int64_t n = int64_t(p.no) * p.no * p.nk;
  hipLaunchKernelGGL(k_energy_bwd_static, dim3(nblk(n, 256)), dim3(256), 0, s, (const zd*)h_k, (const zd*)shf_k,
                     (const zd*)n_k, c, (zd*)hbar, (zd*)shfbar, (zd*)nbar, p.no, p.nk);
  return hipGetLastError();
}

hipError_t launch_energy_bwd_nodes(const Plan& p, const void* y, const void* g, double c, void* gbar, void* ybar,
                                   hipStream_t s) {
  const int64_t n = int64_t(p.no) * p.no * p.nk * p.r;
  hipLaunchKernelGGL(k_energy_bwd_nodes, dim3(nblk(n, 256)), dim3(256), 0, s, (const zd*)y, (const zd*)g, c,
                     (zd*)gbar, (zd*)ybar, p.no, p.nk, p.r);
  return hipGetLastError();
}

hipError_t launch_pair_layout(const Plan& p, int to_matrix, int64_t nn, const void* in, void* out, hipStream_t s) {
  const int na = p.nb * p.nb;
  const int64_t total = nn * na * p.nk;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_layout, dim3(nblk(total, 256)), dim3(256), 0, s, (const zd*)in, (zd*)out, total, na,
                     p.nk, to_matrix);
  return hipGetLastError();
}

}  // namespace qgw
