// Lattice transforms (Eq. eq:fourier-transform-kr, cell-periodic gauge), the
// polarizability bubble (Eq. eq-polarizability) with the R -> q transform
// fused, and the GW self-energy (Eq. eq-gw-self-energy) with the q -> R and
// R -> k transforms fused.
//
// A slab is one N x N mesh of complex values (R or k fastest, row-major:
// index = x1 * N + x2).  In LDS a slab is stored with a row stride of N + 1
// elements so that the strided column reads of the second pass spread over
// the banks.  One thread owns one mesh line per pass and transforms it in
// registers (qgw_fft_reg.h).
#include "qgw_fft_reg.h"
#include "qgw_internal.h"

namespace qgw {

// ---------------------------------------------------------------------------
// plain batched 2-D transform
// ---------------------------------------------------------------------------
template <int N, int SIGN, typename T>
__global__ __launch_bounds__(256) void k_lattice_fft(const cpx<T>* __restrict__ in1,
                                                     cpx<T>* __restrict__ out1, int64_t nslabs1,
                                                     int spb, const cpx<T>* __restrict__ tw,
                                                     T out_scale, const cpx<T>* __restrict__ in2,
                                                     cpx<T>* __restrict__ out2, int64_t nslabs2) {
  using M = MeshShape<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  // two arrays in one launch (both time orders of G): the first nb1 blocks take array 1, the rest array 2
  const int64_t nb1 = (nslabs1 + spb - 1) / spb;
  const bool second = int64_t(blockIdx.x) >= nb1;
  const cpx<T>* in = second ? in2 : in1;
  cpx<T>* out = second ? out2 : out1;
  const int64_t nslabs = second ? nslabs2 : nslabs1;
  const int64_t s0 = (int64_t(blockIdx.x) - (second ? nb1 : 0)) * spb;
  const int nloc = int(nslabs - s0 < spb ? nslabs - s0 : spb);
  // coalesced load
  for (int e = threadIdx.x; e < nloc * M::NN; e += blockDim.x) {
    const int sl = e / M::NN, rem = e - sl * M::NN;
    const int r1 = rem / N, r2 = rem - r1 * N;
    lds[sl * M::SLAB + r1 * M::LD + r2] = in[(s0 + sl) * M::NN + rem];
  }
  __syncthreads();
  const int sl = threadIdx.x / N, line = threadIdx.x - sl * N;
  const bool act = sl < nloc;
  cpx<T> x[N];
  if (act) {
    cpx<T>* slab = lds + sl * M::SLAB;
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = slab[line * M::LD + j];
    fft_reg<N, SIGN>(x, tw);
#pragma unroll
    for (int j = 0; j < N; ++j) slab[line * M::LD + j] = x[j];
  }
  __syncthreads();
  if (act) {
    const cpx<T>* slab = lds + sl * M::SLAB;
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = slab[j * M::LD + line];
    fft_reg<N, SIGN>(x, tw);
    cpx<T>* o = out + (s0 + sl) * M::NN;
#pragma unroll
    for (int j = 0; j < N; ++j) o[j * N + line] = scale(x[j], out_scale);
  }
}

// ---------------------------------------------------------------------------
// bubble: P_{(il),(jk)}(R, tau) = -2 G_{lj}(R, tau) G_{ki}(-R, beta - tau)
// slab index = (t * nb + alpha) * nb + beta
// ---------------------------------------------------------------------------
template <int N, bool OUTQ, typename T>
__global__ __launch_bounds__(256) void k_bubble(const cpx<T>* __restrict__ gt,
                                                const cpx<T>* __restrict__ gr,
                                                cpx<T>* __restrict__ out, int64_t nslabs, int spb,
                                                int no, int nb, const int* __restrict__ pairs,
                                                const cpx<T>* __restrict__ tw) {
  using M = MeshShape<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int64_t s0 = xcd_block(blockIdx.x, gridDim.x) * spb;
  const int nloc = int(nslabs - s0 < spb ? nslabs - s0 : spb);
  const int sl = threadIdx.x / N, line = threadIdx.x - sl * N;
  const bool act = sl < nloc;
  const T two = T(2);
  if (!OUTQ) {
    // no transform: stream the product straight out
    for (int e = threadIdx.x; e < nloc * M::NN; e += blockDim.x) {
      const int sl2 = e / M::NN, rem = e - sl2 * M::NN;
      const int64_t s = s0 + sl2;
      const int be = int(s % nb), al = int((s / nb) % nb);
      const int64_t t = s / (int64_t(nb) * nb);
      const int i = pairs[al], l = pairs[nb + al], j = pairs[be], k = pairs[nb + be];
      const int r1 = rem / N, r2 = rem - r1 * N;
      const int mr = ((N - r1) % N) * N + (N - r2) % N;
      const cpx<T> a = gt[((t * no + l) * no + j) * M::NN + rem];
      const cpx<T> b = gr[((t * no + k) * no + i) * M::NN + mr];
      out[s * M::NN + rem] = scale(a * b, -two);
    }
    return;
  }
  cpx<T> x[N];
  if (act) {
    // column pass straight from global memory: thread owns column r2 = line
    const int64_t s = s0 + sl;
    const int be = int(s % nb), al = int((s / nb) % nb);
    const int64_t t = s / (int64_t(nb) * nb);
    const int i = pairs[al], l = pairs[nb + al], j = pairs[be], k = pairs[nb + be];
    const cpx<T>* a = gt + ((t * no + l) * no + j) * M::NN;
    const cpx<T>* b = gr + ((t * no + k) * no + i) * M::NN;
    const int mr2 = (N - line) % N;
#pragma unroll
    for (int r1 = 0; r1 < N; ++r1) {
      const int mr1 = (N - r1) % N;
      x[r1] = scale(a[r1 * N + line] * b[mr1 * N + mr2], -two);
    }
    fft_reg<N, -1>(x, tw);  // along R1 -> q1
    cpx<T>* slab = lds + sl * M::SLAB;
#pragma unroll
    for (int q1 = 0; q1 < N; ++q1) slab[q1 * M::LD + line] = x[q1];
  }
  __syncthreads();
  if (act) {
    cpx<T>* slab = lds + sl * M::SLAB;
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = slab[line * M::LD + j];
    fft_reg<N, -1>(x, tw);  // along R2 -> q2
#pragma unroll
    for (int j = 0; j < N; ++j) slab[line * M::LD + j] = x[j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nloc * M::NN; e += blockDim.x) {
    const int sl2 = e / M::NN, rem = e - sl2 * M::NN;
    const int q1 = rem / N, q2 = rem - q1 * N;
    out[(s0 + sl2) * M::NN + rem] = lds[sl2 * M::SLAB + q1 * M::LD + q2];
  }
}

// ---------------------------------------------------------------------------
// self-energy: Sigma_{ik}(R, tau) = - sum_{(il),(jk)} W^C_{(il),(jk)}(R, tau) G_{lj}(R, tau)
// One block per output slab (t, i, k); ``spb`` term lanes work on different
// (alpha, beta) terms at once and are summed at the end.  Per term a thread
// loads one column of the W^C(q) slab straight into registers (24
// independent, coalesced loads), transforms it along q1, passes it through
// LDS once to hold a row R1 of the slab, transforms along q2, and
// accumulates -W G for that row.  The summed slab goes R -> k through LDS.
// ---------------------------------------------------------------------------
template <int N, bool INQ, bool OUTK, typename T>
__global__ __launch_bounds__(256) void k_sigma(const cpx<T>* __restrict__ gt,
                                               const cpx<T>* __restrict__ wc,
                                               cpx<T>* __restrict__ sig, int spb, int no, int nb,
                                               const int4* __restrict__ terms,
                                               const int* __restrict__ term_off,
                                               const cpx<T>* __restrict__ tw) {
  using M = MeshShape<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int out_slab = int(xcd_block(blockIdx.x, gridDim.x));  // (t * no + i) * no + k
  const int ik = out_slab % (no * no);
  const int64_t t = out_slab / (no * no);
  const int tb = term_off[ik], te = term_off[ik + 1];
  const int lane = threadIdx.x / N, line = threadIdx.x - lane * N;
  const bool act = lane < spb;
  const T inv_nk = INQ ? T(1) / T(M::NN) : T(1);
  cpx<T> acc[N];  // row R1 = line of this lane's partial sum
#pragma unroll
  for (int j = 0; j < N; ++j) acc[j] = mk(T(0), T(0));
  cpx<T> x[N];
  cpx<T>* slab = lds + lane * M::SLAB;
  for (int c0 = tb; c0 < te; c0 += spb) {
    const bool mine = act && c0 + lane < te;
    int4 tm = make_int4(0, 0, 0, 0);
    if (mine) {
      tm = terms[c0 + lane];
      const cpx<T>* w = wc + ((t * nb + tm.x) * nb + tm.y) * M::NN;
      if (INQ) {
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = w[j * N + line];  // column q2 = line
        fft_reg<N, +1>(x, tw);                                 // q1 -> R1
#pragma unroll
        for (int j = 0; j < N; ++j) slab[j * M::LD + line] = x[j];
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = w[line * N + j];  // row R1 = line
      }
    }
    if (INQ) {
      __syncthreads();
      if (mine) {
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = slab[line * M::LD + j];  // row R1 = line
        fft_reg<N, +1>(x, tw);                                       // q2 -> R2
      }
      __syncthreads();  // the slab is free for the next term
    }
    if (mine) {
      const cpx<T>* g = gt + ((t * no + tm.z) * no + tm.w) * M::NN + line * N;
#pragma unroll
      for (int j = 0; j < N; ++j) acc[j] = fms(acc[j], x[j], g[j]);
    }
  }
  // reduce the term lanes: lane partial rows -> LDS, lane 0 threads add up
  if (act) {
#pragma unroll
    for (int j = 0; j < N; ++j) slab[line * M::LD + j] = acc[j];
  }
  __syncthreads();
  const bool lead = threadIdx.x < N;
  if (lead) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cpx<T> s = lds[line * M::LD + j];
      for (int l2 = 1; l2 < spb; ++l2) s = s + lds[l2 * M::SLAB + line * M::LD + j];
      x[j] = scale(s, inv_nk);
    }
  }
  if (!OUTK) {
    if (lead) {
      cpx<T>* o = sig + int64_t(out_slab) * M::NN + line * N;
#pragma unroll
      for (int j = 0; j < N; ++j) o[j] = x[j];
    }
    return;
  }
  // forward transform of the summed slab: R2 -> k2 along the row, then R1 -> k1
  __syncthreads();  // every lane has read its partial sums
  if (lead) {
    fft_reg<N, -1>(x, tw);
#pragma unroll
    for (int j = 0; j < N; ++j) lds[line * M::LD + j] = x[j];
  }
  __syncthreads();
  if (lead) {
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = lds[j * M::LD + line];
    fft_reg<N, -1>(x, tw);
#pragma unroll
    for (int j = 0; j < N; ++j) lds[j * M::LD + line] = x[j];
  }
  __syncthreads();
  cpx<T>* o = sig + int64_t(out_slab) * M::NN;
  for (int e = threadIdx.x; e < M::NN; e += blockDim.x) {
    const int k1 = e / N, k2 = e - k1 * N;
    o[e] = lds[k1 * M::LD + k2];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace {

constexpr int kLdsBudget = 64 * 1024;

// slabs per block: the tuned value if set (within the LDS and 256-thread limits), else the default
template <typename T>
int tuned_spb(int n, int want) {
  const int cap = slabs_per_block<T>(n, kLdsBudget);
  if (want <= 0) return cap;
  return want < cap ? want : cap;
}

template <typename T>
const cpx<T>* twiddles(const Plan& p);
template <>
const cpx<double>* twiddles<double>(const Plan& p) {
  return p.d_tw64;
}
template <>
const cpx<float>* twiddles<float>(const Plan& p) {
  return p.d_tw32;
}

template <int N, typename T>
hipError_t fft_signed(const Plan& p, int sign, T sc, int64_t batch, const void* in, void* out, hipStream_t s,
                      const void* in2 = nullptr, void* out2 = nullptr) {
  if (batch <= 0) return hipSuccess;
  const int spb = tuned_spb<T>(N, p.tune.fft_spb);
  const size_t lds = size_t(spb) * MeshShape<N>::SLAB * sizeof(cpx<T>);
  const int64_t blocks = (batch + spb - 1) / spb + (in2 ? (batch + spb - 1) / spb : 0);
  if (sign > 0)
    hipLaunchKernelGGL((k_lattice_fft<N, +1, T>), dim3(unsigned(blocks)), dim3(spb * N), lds, s,
                       (const cpx<T>*)in, (cpx<T>*)out, batch, spb, twiddles<T>(p), sc, (const cpx<T>*)in2,
                       (cpx<T>*)out2, batch);
  else
    hipLaunchKernelGGL((k_lattice_fft<N, -1, T>), dim3(unsigned(blocks)), dim3(spb * N), lds, s,
                       (const cpx<T>*)in, (cpx<T>*)out, batch, spb, twiddles<T>(p), sc, (const cpx<T>*)in2,
                       (cpx<T>*)out2, batch);
  return hipGetLastError();
}

// X(R) = (1/N_k) sum_k X(k) e^{+ik.R} for dir > 0, X(k) = sum_R X(R) e^{-ik.R} for dir < 0
template <int N, typename T>
hipError_t fft_n(const Plan& p, int dir, int64_t batch, const void* in, void* out, hipStream_t s,
                 const void* in2 = nullptr, void* out2 = nullptr) {
  return fft_signed<N, T>(p, dir > 0 ? +1 : -1, dir > 0 ? T(1) / T(N * N) : T(1), batch, in, out, s, in2, out2);
}

template <int N, typename T>
hipError_t bubble_n(const Plan& p, const void* gt, const void* gr, int out_q, void* out,
                    hipStream_t s) {
  const int64_t nslabs = int64_t(p.r) * p.nb * p.nb;
  // untuned: the FP64 transform holds 150 VGPRs per thread on meshes from 16 up, and two slabs per block (more,
  // smaller blocks) measured fastest at 24 x 24 (0.097 -> 0.083 ms); otherwise as many slabs as fit
  const int want = p.tune.bubble_spb > 0 ? p.tune.bubble_spb : (sizeof(T) == 8 && N >= 16 ? 2 : 0);
  const int spb = tuned_spb<T>(N, want);
  const int64_t blocks = (nslabs + spb - 1) / spb;
  if (out_q) {
    const size_t lds = size_t(spb) * MeshShape<N>::SLAB * sizeof(cpx<T>);
    hipLaunchKernelGGL((k_bubble<N, true, T>), dim3(unsigned(blocks)), dim3(spb * N), lds, s,
                       (const cpx<T>*)gt, (const cpx<T>*)gr, (cpx<T>*)out, nslabs, spb, p.no, p.nb,
                       p.d_pairs, twiddles<T>(p));
  } else {
    hipLaunchKernelGGL((k_bubble<N, false, T>), dim3(unsigned(blocks)), dim3(spb * N), 0, s,
                       (const cpx<T>*)gt, (const cpx<T>*)gr, (cpx<T>*)out, nslabs, spb, p.no, p.nb,
                       p.d_pairs, twiddles<T>(p));
  }
  return hipGetLastError();
}

template <int N, typename T>
hipError_t sigma_n(const Plan& p, const void* gt, const void* wc, int in_q, int out_k, void* sig,
                   hipStream_t s) {
  // term lanes: the largest divisor of the per-output term count that fits
  const int terms = p.terms.max_terms;
  int cap = slabs_per_block<T>(N, kLdsBudget);
  int spb = 1;
  for (int d = 1; d <= terms && d <= cap; ++d)
    if (terms % d == 0) spb = d;
  if (p.tune.sigma_spb > 0) spb = p.tune.sigma_spb < cap ? p.tune.sigma_spb : cap;
  const size_t lds = size_t(spb) * MeshShape<N>::SLAB * sizeof(cpx<T>);
  const unsigned blocks = unsigned(int64_t(p.r) * p.no * p.no);
  const dim3 blk(spb * N);
  auto args = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), blk, lds, s, (const cpx<T>*)gt, (const cpx<T>*)wc,
                       (cpx<T>*)sig, spb, p.no, p.nb, (const int4*)p.terms.d_terms,
                       p.terms.d_off, twiddles<T>(p));
  };
  if (in_q && out_k) args(k_sigma<N, true, true, T>);
  else if (in_q) args(k_sigma<N, true, false, T>);
  else if (out_k) args(k_sigma<N, false, true, T>);
  else args(k_sigma<N, false, false, T>);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lattice_fft(const Plan& p, int dir, int64_t batch, const void* in, void* out,
                              hipStream_t s) {
  if (p.dim == 3) return launch_lattice_fft3(p, dir > 0 ? +1 : -1, dir > 0 ? 1.0 / double(p.nk) : 1.0, batch, in, out, s);
  switch (p.n) {
#define QGW_CASE(NN) \
  case NN:           \
    return p.prec == 0 ? fft_n<NN, double>(p, dir, batch, in, out, s) : fft_n<NN, float>(p, dir, batch, in, out, s);
    QGW_FOR_EACH_MESH(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_lattice_fft2(const Plan& p, int dir, int64_t batch, const void* in1, void* out1, const void* in2,
                               void* out2, hipStream_t s) {
  if (p.dim == 3) {
    hipError_t e = launch_lattice_fft(p, dir, batch, in1, out1, s);
    return e == hipSuccess ? launch_lattice_fft(p, dir, batch, in2, out2, s) : e;
  }
  switch (p.n) {
#define QGW_CASE(NN)                                                                       \
  case NN:                                                                                 \
    return p.prec == 0 ? fft_n<NN, double>(p, dir, batch, in1, out1, s, in2, out2)         \
                       : fft_n<NN, float>(p, dir, batch, in1, out1, s, in2, out2);
    QGW_FOR_EACH_MESH(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_lattice_fft_scaled(const Plan& p, int sign, double out_scale, int64_t batch,
                                     const void* in, void* out, hipStream_t s) {
  if (p.dim == 3) return launch_lattice_fft3(p, sign, out_scale, batch, in, out, s);
  switch (p.n) {
#define QGW_CASE(NN)                                                                                   \
  case NN:                                                                                             \
    return p.prec == 0 ? fft_signed<NN, double>(p, sign, out_scale, batch, in, out, s)                \
                       : fft_signed<NN, float>(p, sign, float(out_scale), batch, in, out, s);
    QGW_FOR_EACH_MESH(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_bubble(const Plan& p, const void* gt, const void* gr, int out_q, void* out,
                         hipStream_t s) {
  if (p.dim == 3) return launch_bubble3(p, gt, gr, out_q, out, s);
  switch (p.n) {
#define QGW_CASE(NN) \
  case NN:           \
    return p.prec == 0 ? bubble_n<NN, double>(p, gt, gr, out_q, out, s) : bubble_n<NN, float>(p, gt, gr, out_q, out, s);
    QGW_FOR_EACH_MESH(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_sigma(const Plan& p, const void* gt, const void* wc, int in_q, int out_k,
                        void* sig, hipStream_t s) {
  if (p.dim == 3) return launch_sigma3(p, gt, wc, in_q, out_k, sig, s);
  switch (p.n) {
#define QGW_CASE(NN) \
  case NN:           \
    return p.prec == 0 ? sigma_n<NN, double>(p, gt, wc, in_q, out_k, sig, s) : sigma_n<NN, float>(p, gt, wc, in_q, out_k, sig, s);
    QGW_FOR_EACH_MESH(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace qgw
