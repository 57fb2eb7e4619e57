// Small kernels: Hartree-Fock self-energy (Eqs. eq-hartree-self-energy,
// eq-fock-self-energy), V(q = 0), layout changes of static arrays, the
// self-energy change / mixing of the self-consistency loop, finiteness check.
#include "qgw_internal.h"

namespace qgw {

// Sigma_HF_{ik}(R) = - sum_terms V_{(il),(jk)}(R) n_{lj}(R)
//                    + delta_{R,0} 2 sum_beta V_{(ik),beta}(q=0) n_{k_beta j_beta}(0)
__global__ __launch_bounds__(256) void k_hartree_fock(const zd* __restrict__ v_r, const zd* __restrict__ v_q0,
                                                      const zd* __restrict__ n_r, zd* __restrict__ out,
                                                      int no, int nb, int nk, const int* __restrict__ pairs,
                                                      const int4* __restrict__ terms,
                                                      const int* __restrict__ term_off) {
  const int64_t gi = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (gi >= int64_t(no) * no * nk) return;
  const int rr = int(gi % nk);
  const int ik = int(gi / nk);
  const int i = ik / no, k = ik % no;
  cpx<double> s = mk(0.0, 0.0);
  for (int t = term_off[ik]; t < term_off[ik + 1]; ++t) {
    const int4 tm = terms[t];
    s = fms(s, v_r[(int64_t(tm.x) * nb + tm.y) * nk + rr], n_r[(int64_t(tm.z) * no + tm.w) * nk + rr]);
  }
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
__global__ void k_pair_sum_r(const zd* __restrict__ v_r, zd* __restrict__ v_q0, int nbb, int nk) {
  const int ab = blockIdx.x * blockDim.x + threadIdx.x;
  if (ab >= nbb) return;
  cpx<double> s = mk(0.0, 0.0);
  for (int rr = 0; rr < nk; ++rr) s = s + v_r[int64_t(ab) * nk + rr];
  v_q0[ab] = s;
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

// per-block max of |(hf_new + c_new) - (hf_old + c_old)| over (m, ab, k)
__global__ __launch_bounds__(256) void k_delta(const zd* __restrict__ hf_new, const zd* __restrict__ c_new,
                                               const zd* __restrict__ hf_old, const zd* __restrict__ c_old,
                                               int64_t n_static, int64_t n_total, double* __restrict__ block_max) {
  __shared__ double red[256];
  double v = 0.0;
  for (int64_t gi = int64_t(blockIdx.x) * 256 + threadIdx.x; gi < n_total; gi += int64_t(gridDim.x) * 256) {
    const int64_t st = gi % n_static;
    const cpx<double> d = (hf_new[st] + c_new[gi]) - (hf_old[st] + c_old[gi]);
    v = fmax(v, sqrt(norm2(d)));
  }
  red[threadIdx.x] = v;
  __syncthreads();
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

// x_new <- x_old + alpha (x_new - x_old); x_old <- x_new
__global__ void k_mix_copy(zd* __restrict__ x_new, zd* __restrict__ x_old, int64_t n, double alpha) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  cpx<double> v = x_new[gi];
  if (alpha != 1.0) {
    const cpx<double> o = x_old[gi];
    v = o + scale(v - o, alpha);
    x_new[gi] = v;
  }
  x_old[gi] = v;
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
  hipLaunchKernelGGL(k_hartree_fock, dim3(nblk(n, 256)), dim3(256), 0, s, (const zd*)v_r,
                     (const zd*)v_q0, (const zd*)n_r, (zd*)sig_hf_r, p.no, p.nb, p.nk, p.d_pairs,
                     (const int4*)p.terms.d_terms, p.terms.d_off);
  return hipGetLastError();
}

hipError_t launch_pair_sum_r(const Plan& p, const void* v_r, void* v_q0, hipStream_t s) {
  const int nbb = p.nb * p.nb;
  hipLaunchKernelGGL(k_pair_sum_r, dim3(nblk(nbb, 64)), dim3(64), 0, s, (const zd*)v_r, (zd*)v_q0, nbb, p.nk);
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
                                double alpha, double* d_out, double* block_scratch, hipStream_t s) {
  const int64_t ns = int64_t(p.no) * p.no * p.nk;
  const int64_t nt = ns * p.r;
  const int blocks = 256;
  hipLaunchKernelGGL(k_delta, dim3(blocks), dim3(256), 0, s, (const zd*)hf_new, (const zd*)c_new,
                     (const zd*)hf_old, (const zd*)c_old, ns, nt, block_scratch);
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, (const double*)block_scratch, blocks, d_out);
  hipLaunchKernelGGL(k_mix_copy, dim3(nblk(ns, 256)), dim3(256), 0, s, (zd*)hf_new, (zd*)hf_old, ns, alpha);
  hipLaunchKernelGGL(k_mix_copy, dim3(nblk(nt, 256)), dim3(256), 0, s, (zd*)c_new, (zd*)c_old, nt, alpha);
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

}  // namespace qgw
