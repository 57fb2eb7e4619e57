// Lattice transforms (Eq. eq:fourier-transform-kr), the polarizability bubble
// (Eq. eq-polarizability) with R -> q fused, the GW self-energy
// (Eq. eq-gw-self-energy) with q -> R and R -> k fused, and the adjoints of the
// last two, on a cubic N x N x N mesh (the 8 x 8 x 8 mesh of the performance
// section).
//
// A slab is one mesh of N^3 complex values, row-major: index = (i1 N + i2) N + i3.
// A transform is three passes of length-N DFTs, one along each axis; in each
// pass a thread owns one mesh line (N^2 lines per slab) and transforms it in
// registers (qgw_fft_reg.h).  The pass along axis 1 reads or writes global
// memory directly: its N^2 lines are the N^2 consecutive elements of each
// plane, so a wavefront's accesses are contiguous.  The other passes go
// through LDS, where the slab is stored with strides S2 = N + 1 (axis 2) and
// S1 = N (N + 1) (axis 1) so that the lines of the axis-3 pass, N + 1
// elements apart, spread over the banks.
#include "qgw_fft_reg.h"
#include "qgw_internal.h"

namespace qgw {

template <int N>
struct Cube {
  static constexpr int NK = N * N * N;
  static constexpr int LINES = N * N;  // lines per slab in every pass
  static constexpr int S2 = N + 1;
  static constexpr int S1 = N * (N + 1);
  static constexpr int SLAB = N * S1;  // LDS elements per slab
  // LDS offset of line l of the pass along axis A (0, 1, 2) and the element stride along A
  template <int A>
  __device__ static int base(int l) {
    const int u = l / N, v = l - u * N;
    if constexpr (A == 0) return u * S2 + v;  // l = (i2, i3)
    else if constexpr (A == 1) return u * S1 + v;  // l = (i1, i3)
    else return u * S1 + v * S2;  // l = (i1, i2)
  }
  template <int A>
  static constexpr int stride() {
    return A == 0 ? S1 : A == 1 ? S2 : 1;
  }
  // global index of -R for the element (i1, i2, i3) = (j, l / N, l % N) of an axis-1 line
  __device__ static int neg_axis1(int j, int l) {
    const int i2 = l / N, i3 = l - i2 * N;
    return (((N - j) % N) * N + (N - i2) % N) * N + (N - i3) % N;
  }
  // global index of -R for the element (i1, i2, i3) = (l / N, l % N, j) of an axis-3 line
  __device__ static int neg_axis3(int l, int j) {
    const int i1 = l / N, i2 = l - i1 * N;
    return (((N - i1) % N) * N + (N - i2) % N) * N + (N - j) % N;
  }
};

// DFT of line l along axis A of an LDS slab, in place
template <int N, int A, int SIGN, typename T>
__device__ __forceinline__ void lds_line_pass(cpx<T>* slab, int l, const cpx<T>* __restrict__ tw) {
  using C = Cube<N>;
  const int b = C::template base<A>(l);
  constexpr int st = C::template stride<A>();
  cpx<T> x[N];
#pragma unroll
  for (int j = 0; j < N; ++j) x[j] = slab[b + j * st];
  fft_reg<N, SIGN>(x, tw);
#pragma unroll
  for (int j = 0; j < N; ++j) slab[b + j * st] = x[j];
}

template <int N, typename T>
__device__ __forceinline__ void store_axis1(cpx<T>* slab, int l, const cpx<T> (&x)[N]) {
  using C = Cube<N>;
  const int b = C::template base<0>(l);
#pragma unroll
  for (int j = 0; j < N; ++j) slab[b + j * C::S1] = x[j];
}

// Block-uniform q -> R transform of one slab per term lane: the axis-1 line l of
// w (global, skipped where !on) is transformed, then axes 2 and 3 through LDS.
// On return x[j] holds X(R = (l / N, l % N, j)) and the LDS slab is free again.
template <int N, typename T>
__device__ __forceinline__ void q_to_R_axis3(const cpx<T>* __restrict__ w, bool on, cpx<T>* slab, int l,
                                             cpx<T> (&x)[N], const cpx<T>* __restrict__ tw) {
  using C = Cube<N>;
  if (on) {
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = w[j * C::LINES + l];
    fft_reg<N, +1>(x, tw);
    store_axis1<N>(slab, l, x);
  }
  __syncthreads();
  if (on) lds_line_pass<N, 1, +1>(slab, l, tw);
  __syncthreads();
  if (on) {
    const int b = C::template base<2>(l);
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = slab[b + j];
    fft_reg<N, +1>(x, tw);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// plain batched 3-D transform
// ---------------------------------------------------------------------------
template <int N, int SIGN, typename T>
__global__ __launch_bounds__(256) void k_lattice_fft3(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                                      int64_t nslabs, int spb, const cpx<T>* __restrict__ tw,
                                                      T out_scale) {
  using C = Cube<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int64_t s0 = int64_t(blockIdx.x) * spb;
  const int nloc = int(nslabs - s0 < spb ? nslabs - s0 : spb);
  const int sl = threadIdx.x / C::LINES, l = threadIdx.x - sl * C::LINES;
  const bool act = sl < nloc;
  cpx<T>* slab = lds + sl * C::SLAB;
  if (act) {
    const cpx<T>* src = in + (s0 + sl) * C::NK;
    cpx<T> x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = src[j * C::LINES + l];
    fft_reg<N, SIGN>(x, tw);
    store_axis1<N>(slab, l, x);
  }
  __syncthreads();
  if (act) lds_line_pass<N, 1, SIGN>(slab, l, tw);
  __syncthreads();
  if (act) lds_line_pass<N, 2, SIGN>(slab, l, tw);
  __syncthreads();
  for (int e = threadIdx.x; e < nloc * C::NK; e += blockDim.x) {
    const int s2 = e / C::NK, rem = e - s2 * C::NK;
    const int i1 = rem / C::LINES, i23 = rem - i1 * C::LINES, i2 = i23 / N, i3 = i23 - i2 * N;
    out[(s0 + s2) * C::NK + rem] = scale(lds[s2 * C::SLAB + i1 * C::S1 + i2 * C::S2 + i3], out_scale);
  }
}

// ---------------------------------------------------------------------------
// bubble: P_{(il),(jk)}(R, tau) = -2 G_{lj}(R, tau) G_{ki}(-R, beta - tau), slab (t, alpha, beta)
// ---------------------------------------------------------------------------
template <int N, bool OUTQ, typename T>
__global__ __launch_bounds__(256) void k_bubble3(const cpx<T>* __restrict__ gt, const cpx<T>* __restrict__ gr,
                                                 cpx<T>* __restrict__ out, int64_t nslabs, int spb, int no, int nb,
                                                 const int* __restrict__ pairs, const cpx<T>* __restrict__ tw) {
  using C = Cube<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int64_t s0 = xcd_block(blockIdx.x, gridDim.x) * spb;
  const int nloc = int(nslabs - s0 < spb ? nslabs - s0 : spb);
  const int sl = threadIdx.x / C::LINES, l = threadIdx.x - sl * C::LINES;
  const bool act = sl < nloc;
  const T two = T(2);
  if (!OUTQ) {
    for (int e = threadIdx.x; e < nloc * C::NK; e += blockDim.x) {
      const int s2 = e / C::NK, rem = e - s2 * C::NK;
      const int64_t s = s0 + s2;
      const int be = int(s % nb), al = int((s / nb) % nb);
      const int64_t t = s / (int64_t(nb) * nb);
      const int i = pairs[al], li = pairs[nb + al], j = pairs[be], k = pairs[nb + be];
      const int i1 = rem / C::LINES, i23 = rem - i1 * C::LINES;
      const cpx<T> a = gt[((t * no + li) * no + j) * C::NK + rem];
      const cpx<T> b = gr[((t * no + k) * no + i) * C::NK + C::neg_axis1(i1, i23)];
      out[s * C::NK + rem] = scale(a * b, -two);
    }
    return;
  }
  cpx<T>* slab = lds + sl * C::SLAB;
  if (act) {
    const int64_t s = s0 + sl;
    const int be = int(s % nb), al = int((s / nb) % nb);
    const int64_t t = s / (int64_t(nb) * nb);
    const int i = pairs[al], li = pairs[nb + al], j = pairs[be], k = pairs[nb + be];
    const cpx<T>* a = gt + ((t * no + li) * no + j) * C::NK;
    const cpx<T>* b = gr + ((t * no + k) * no + i) * C::NK;
    cpx<T> x[N];
#pragma unroll
    for (int r1 = 0; r1 < N; ++r1) x[r1] = scale(a[r1 * C::LINES + l] * b[C::neg_axis1(r1, l)], -two);
    fft_reg<N, -1>(x, tw);  // R1 -> q1
    store_axis1<N>(slab, l, x);
  }
  __syncthreads();
  if (act) lds_line_pass<N, 1, -1>(slab, l, tw);  // R2 -> q2
  __syncthreads();
  if (act) lds_line_pass<N, 2, -1>(slab, l, tw);  // R3 -> q3
  __syncthreads();
  for (int e = threadIdx.x; e < nloc * C::NK; e += blockDim.x) {
    const int s2 = e / C::NK, rem = e - s2 * C::NK;
    const int i1 = rem / C::LINES, i23 = rem - i1 * C::LINES, i2 = i23 / N, i3 = i23 - i2 * N;
    out[(s0 + s2) * C::NK + rem] = lds[s2 * C::SLAB + i1 * C::S1 + i2 * C::S2 + i3];
  }
}

// ---------------------------------------------------------------------------
// self-energy: Sigma_{ik}(R, tau) = - sum_{(il),(jk)} W^C_{(il),(jk)}(R, tau) G_{lj}(R, tau)
// One block per output slab (t, i, k); ``spb`` term lanes work on different
// (alpha, beta) terms at once.  Per term a lane takes its W^C(q) slab to R
// (three passes) and accumulates -W G along its axis-3 lines; the lanes'
// partial slabs are summed at the end and the sum goes R -> k.
// ---------------------------------------------------------------------------
template <int N, bool INQ, bool OUTK, typename T>
__global__ __launch_bounds__(256) void k_sigma3(const cpx<T>* __restrict__ gt, const cpx<T>* __restrict__ wc,
                                                cpx<T>* __restrict__ sig, int spb, int no, int nb,
                                                const int4* __restrict__ terms, const int* __restrict__ term_off,
                                                const cpx<T>* __restrict__ tw) {
  using C = Cube<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int out_slab = int(xcd_block(blockIdx.x, gridDim.x));  // (t * no + i) * no + k
  const int ik = out_slab % (no * no);
  const int64_t t = out_slab / (no * no);
  const int tb = term_off[ik], te = term_off[ik + 1];
  const int lane = threadIdx.x / C::LINES, l = threadIdx.x - lane * C::LINES;
  const bool act = lane < spb;
  const T inv_nk = INQ ? T(1) / T(C::NK) : T(1);
  cpx<T> acc[N];  // R = (l / N, l % N, j)
#pragma unroll
  for (int j = 0; j < N; ++j) acc[j] = mk(T(0), T(0));
  cpx<T> x[N];
  cpx<T>* slab = lds + lane * C::SLAB;
  for (int c0 = tb; c0 < te; c0 += spb) {
    const bool mine = act && c0 + lane < te;
    int4 tm = make_int4(0, 0, 0, 0);
    if (mine) tm = terms[c0 + lane];
    const cpx<T>* w = wc + ((t * nb + tm.x) * nb + tm.y) * C::NK;
    if (INQ) {
      q_to_R_axis3<N>(w, mine, slab, l, x, tw);
    } else if (mine) {
#pragma unroll
      for (int j = 0; j < N; ++j) x[j] = w[l * N + j];
    }
    if (mine) {
      const cpx<T>* g = gt + ((t * no + tm.z) * no + tm.w) * C::NK + l * N;
#pragma unroll
      for (int j = 0; j < N; ++j) acc[j] = fms(acc[j], x[j], g[j]);
    }
  }
  if (act) {
    const int b = C::template base<2>(l);
#pragma unroll
    for (int j = 0; j < N; ++j) slab[b + j] = acc[j];
  }
  __syncthreads();
  const bool lead = threadIdx.x < C::LINES;
  if (lead) {
    const int b = C::template base<2>(l);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cpx<T> s = lds[b + j];
      for (int l2 = 1; l2 < spb; ++l2) s = s + lds[l2 * C::SLAB + b + j];
      x[j] = scale(s, inv_nk);
    }
  }
  if (!OUTK) {
    if (lead) {
      cpx<T>* o = sig + int64_t(out_slab) * C::NK + l * N;
#pragma unroll
      for (int j = 0; j < N; ++j) o[j] = x[j];
    }
    return;
  }
  // R -> k: axis 3 on the summed lines, axis 2 in LDS, axis 1 straight to global memory
  __syncthreads();  // every lane has read its partial sums
  if (lead) {
    fft_reg<N, -1>(x, tw);
    const int b = C::template base<2>(l);
#pragma unroll
    for (int j = 0; j < N; ++j) lds[b + j] = x[j];
  }
  __syncthreads();
  if (lead) lds_line_pass<N, 1, -1>(lds, l, tw);
  __syncthreads();
  if (lead) {
    const int b = C::template base<0>(l);
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = lds[b + j * C::S1];
    fft_reg<N, -1>(x, tw);
    cpx<T>* o = sig + int64_t(out_slab) * C::NK;
#pragma unroll
    for (int j = 0; j < N; ++j) o[j * C::LINES + l] = x[j];
  }
}

// ---------------------------------------------------------------------------
// adjoints (FP64), the 3-D forms of the self-energy and bubble adjoints:
//   Wbar(q) = (1/N_k) sum_R e^{-iq.R} [-conj(G_lj(R)) Sbar_ik(R)], slab (t, alpha, beta)
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_sigma_bwd_wc3(const zd* __restrict__ gt, const zd* __restrict__ sbar,
                                                       zd* __restrict__ out, int64_t nslabs, int spb, int no, int nb,
                                                       const int* __restrict__ pairs, const zd* __restrict__ tw) {
  using C = Cube<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<double>* lds = reinterpret_cast<cpx<double>*>(smem_raw);
  const int64_t s0 = int64_t(blockIdx.x) * spb;
  const int nloc = int(nslabs - s0 < spb ? nslabs - s0 : spb);
  const int sl = threadIdx.x / C::LINES, l = threadIdx.x - sl * C::LINES;
  const bool act = sl < nloc;
  const double c = -1.0 / double(C::NK);
  cpx<double>* slab = lds + sl * C::SLAB;
  if (act) {
    const int64_t s = s0 + sl;
    const int be = int(s % nb), al = int((s / nb) % nb);
    const int64_t t = s / (int64_t(nb) * nb);
    const int i = pairs[al], li = pairs[nb + al], j = pairs[be], k = pairs[nb + be];
    const zd* a = gt + ((t * no + li) * no + j) * C::NK;
    const zd* b = sbar + ((t * no + i) * no + k) * C::NK;
    cpx<double> x[N];
#pragma unroll
    for (int r1 = 0; r1 < N; ++r1) x[r1] = scale(conj(a[r1 * C::LINES + l]) * b[r1 * C::LINES + l], c);
    fft_reg<N, -1>(x, tw);
    store_axis1<N>(slab, l, x);
  }
  __syncthreads();
  if (act) lds_line_pass<N, 1, -1>(slab, l, tw);
  __syncthreads();
  if (act) lds_line_pass<N, 2, -1>(slab, l, tw);
  __syncthreads();
  for (int e = threadIdx.x; e < nloc * C::NK; e += blockDim.x) {
    const int s2 = e / C::NK, rem = e - s2 * C::NK;
    const int i1 = rem / C::LINES, i23 = rem - i1 * C::LINES, i2 = i23 / N, i3 = i23 - i2 * N;
    out[(s0 + s2) * C::NK + rem] = lds[s2 * C::SLAB + i1 * C::S1 + i2 * C::S2 + i3];
  }
}

// contraction adjoints; one block per output slab (t, key), modes as in the 2-D form:
//   MODE 0: X = conj(W^C(R)), W^C(R) = (1/N_k) sum_q e^{iq.R} W^C(q); Y = Sbar_ik(R); c = -1
//   MODE 1: X = Pbar(R) = sum_q e^{iq.R} Pbar(q); Y = conj(G_ki(-R, beta - t)); c = -2
//   MODE 2: key (i, k); X = Pbar(R); Y = conj(G_lj(R, t)); c = -2; stored in slab (t, k, i) at -R
template <int N, int MODE>
__global__ __launch_bounds__(256) void k_contract_bwd3(const zd* __restrict__ xq, const zd* __restrict__ y,
                                                       zd* __restrict__ out, int spb, int no, int nb,
                                                       const int4* __restrict__ terms,
                                                       const int* __restrict__ term_off, const zd* __restrict__ tw) {
  using C = Cube<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<double>* lds = reinterpret_cast<cpx<double>*>(smem_raw);
  const int out_slab = blockIdx.x;
  const int key = out_slab % (no * no);
  const int64_t t = out_slab / (no * no);
  const int tb = term_off[key], te = term_off[key + 1];
  const int lane = threadIdx.x / C::LINES, l = threadIdx.x - lane * C::LINES;
  const bool act = lane < spb;
  cpx<double> acc[N];  // R = (l / N, l % N, j)
#pragma unroll
  for (int j = 0; j < N; ++j) acc[j] = mk(0.0, 0.0);
  cpx<double> x[N];
  cpx<double>* slab = lds + lane * C::SLAB;
  for (int c0 = tb; c0 < te; c0 += spb) {
    const bool mine = act && c0 + lane < te;
    int4 tm = make_int4(0, 0, 0, 0);
    if (mine) tm = terms[c0 + lane];
    q_to_R_axis3<N>(xq + ((t * nb + tm.x) * nb + tm.y) * C::NK, mine, slab, l, x, tw);
    if (mine) {
      if (MODE == 0) {
        const zd* g = y + ((t * no + tm.z) * no + tm.w) * C::NK + l * N;
#pragma unroll
        for (int j = 0; j < N; ++j) acc[j] = fma(acc[j], conj(x[j]), g[j]);
      } else if (MODE == 1) {
        const zd* g = y + ((t * no + tm.w) * no + tm.z) * C::NK;
#pragma unroll
        for (int j = 0; j < N; ++j) acc[j] = fma(acc[j], x[j], conj(g[C::neg_axis3(l, j)]));
      } else {
        const zd* g = y + ((t * no + tm.z) * no + tm.w) * C::NK + l * N;
#pragma unroll
        for (int j = 0; j < N; ++j) acc[j] = fma(acc[j], x[j], conj(g[j]));
      }
    }
  }
  if (act) {
    const int b = C::template base<2>(l);
#pragma unroll
    for (int j = 0; j < N; ++j) slab[b + j] = acc[j];
  }
  __syncthreads();
  if (threadIdx.x < C::LINES) {
    const double c = MODE == 0 ? -1.0 / double(C::NK) : -2.0;
    int oslab = out_slab;
    if (MODE == 2) {
      const int i = key / no, k = key - i * no;
      oslab = int(t) * no * no + k * no + i;
    }
    zd* o = out + int64_t(oslab) * C::NK;
    const int b = C::template base<2>(l);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cpx<double> s = lds[b + j];
      for (int l2 = 1; l2 < spb; ++l2) s = s + lds[l2 * C::SLAB + b + j];
      s = scale(s, c);
      if (MODE == 2)
        o[C::neg_axis3(l, j)] = s;
      else
        o[l * N + j] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace {

constexpr int kLdsBudget3 = 64 * 1024;

// slabs (or term lanes) per block: at most 256 threads and the LDS budget, or the tuned value below that
template <int N, typename T>
int cube_cap() {
  int s = 256 / Cube<N>::LINES;
  if (s < 1) s = 1;
  while (s > 1 && s * Cube<N>::SLAB * int(sizeof(cpx<T>)) > kLdsBudget3) --s;
  return s;
}
template <int N, typename T>
int cube_spb(int want) {
  const int cap = cube_cap<N, T>();
  return want > 0 && want < cap ? want : cap;
}

template <typename T>
const cpx<T>* tw3(const Plan& p);
template <>
const cpx<double>* tw3<double>(const Plan& p) {
  return p.d_tw64;
}
template <>
const cpx<float>* tw3<float>(const Plan& p) {
  return p.d_tw32;
}

template <int N, typename T>
hipError_t fft3_n(const Plan& p, int sign, T sc, int64_t batch, const void* in, void* out, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int spb = cube_spb<N, T>(p.tune.fft_spb);
  const size_t lds = size_t(spb) * Cube<N>::SLAB * sizeof(cpx<T>);
  const int64_t blocks = (batch + spb - 1) / spb;
  const dim3 blk(spb * Cube<N>::LINES);
  if (sign > 0)
    hipLaunchKernelGGL((k_lattice_fft3<N, +1, T>), dim3(unsigned(blocks)), blk, lds, s, (const cpx<T>*)in,
                       (cpx<T>*)out, batch, spb, tw3<T>(p), sc);
  else
    hipLaunchKernelGGL((k_lattice_fft3<N, -1, T>), dim3(unsigned(blocks)), blk, lds, s, (const cpx<T>*)in,
                       (cpx<T>*)out, batch, spb, tw3<T>(p), sc);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t bubble3_n(const Plan& p, const void* gt, const void* gr, int out_q, void* out, hipStream_t s) {
  const int64_t nslabs = int64_t(p.r) * p.nb * p.nb;
  const int spb = cube_spb<N, T>(p.tune.bubble_spb);
  const int64_t blocks = (nslabs + spb - 1) / spb;
  const dim3 blk(spb * Cube<N>::LINES);
  if (out_q)
    hipLaunchKernelGGL((k_bubble3<N, true, T>), dim3(unsigned(blocks)), blk,
                       size_t(spb) * Cube<N>::SLAB * sizeof(cpx<T>), s, (const cpx<T>*)gt, (const cpx<T>*)gr,
                       (cpx<T>*)out, nslabs, spb, p.no, p.nb, p.d_pairs, tw3<T>(p));
  else
    hipLaunchKernelGGL((k_bubble3<N, false, T>), dim3(unsigned(blocks)), blk, 0, s, (const cpx<T>*)gt,
                       (const cpx<T>*)gr, (cpx<T>*)out, nslabs, spb, p.no, p.nb, p.d_pairs, tw3<T>(p));
  return hipGetLastError();
}

template <int N, typename T>
hipError_t sigma3_n(const Plan& p, const void* gt, const void* wc, int in_q, int out_k, void* sig, hipStream_t s) {
  const int cap = cube_cap<N, T>();
  int spb = p.terms.max_terms < cap ? (p.terms.max_terms > 0 ? p.terms.max_terms : 1) : cap;
  if (p.tune.sigma_spb > 0 && p.tune.sigma_spb < spb) spb = p.tune.sigma_spb;
  const size_t lds = size_t(spb) * Cube<N>::SLAB * sizeof(cpx<T>);
  const unsigned blocks = unsigned(int64_t(p.r) * p.no * p.no);
  const dim3 blk(spb * Cube<N>::LINES);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), blk, lds, s, (const cpx<T>*)gt, (const cpx<T>*)wc, (cpx<T>*)sig, spb,
                       p.no, p.nb, (const int4*)p.terms.d_terms, p.terms.d_off, tw3<T>(p));
  };
  if (in_q && out_k) go(k_sigma3<N, true, true, T>);
  else if (in_q) go(k_sigma3<N, true, false, T>);
  else if (out_k) go(k_sigma3<N, false, true, T>);
  else go(k_sigma3<N, false, false, T>);
  return hipGetLastError();
}

template <int N>
hipError_t sigma_bwd_wc3_n(const Plan& p, const void* gt, const void* sbar, void* out, hipStream_t s) {
  const int64_t nslabs = int64_t(p.r) * p.nb * p.nb;
  const int spb = cube_cap<N, double>();
  const int64_t blocks = (nslabs + spb - 1) / spb;
  hipLaunchKernelGGL((k_sigma_bwd_wc3<N>), dim3(unsigned(blocks)), dim3(spb * Cube<N>::LINES),
                     size_t(spb) * Cube<N>::SLAB * sizeof(zd), s, (const zd*)gt, (const zd*)sbar, (zd*)out, nslabs,
                     spb, p.no, p.nb, p.d_pairs, p.d_tw64);
  return hipGetLastError();
}

template <int N>
hipError_t contract_bwd3_n(const Plan& p, int mode, const void* xq, const void* y, void* out, hipStream_t s) {
  const TermTable& tt = (mode == 2) ? p.terms : p.terms_lj;
  const int cap = cube_cap<N, double>();
  const int spb = tt.max_terms < cap ? (tt.max_terms > 0 ? tt.max_terms : 1) : cap;
  const size_t lds = size_t(spb) * Cube<N>::SLAB * sizeof(zd);
  const unsigned blocks = unsigned(int64_t(p.r) * p.no * p.no);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(spb * Cube<N>::LINES), lds, s, (const zd*)xq, (const zd*)y,
                       (zd*)out, spb, p.no, p.nb, (const int4*)tt.d_terms, tt.d_off, p.d_tw64);
  };
  if (mode == 0) go(k_contract_bwd3<N, 0>);
  else if (mode == 1) go(k_contract_bwd3<N, 1>);
  else go(k_contract_bwd3<N, 2>);
  return hipGetLastError();
}

}  // namespace

#define QGW_CUBE_SWITCH(BODY)   \
  switch (p.n) {                \
    QGW_FOR_EACH_CUBE(BODY)     \
    default:                    \
      return hipErrorInvalidValue; \
  }

hipError_t launch_lattice_fft3(const Plan& p, int sign, double out_scale, int64_t batch, const void* in, void* out,
                               hipStream_t s) {
#define QGW_CASE(NN) \
  case NN:           \
    return p.prec == 0 ? fft3_n<NN, double>(p, sign, out_scale, batch, in, out, s) \
                       : fft3_n<NN, float>(p, sign, float(out_scale), batch, in, out, s);
  QGW_CUBE_SWITCH(QGW_CASE)
#undef QGW_CASE
}

hipError_t launch_bubble3(const Plan& p, const void* gt, const void* gr, int out_q, void* out, hipStream_t s) {
#define QGW_CASE(NN) \
  case NN:           \
    return p.prec == 0 ? bubble3_n<NN, double>(p, gt, gr, out_q, out, s) : bubble3_n<NN, float>(p, gt, gr, out_q, out, s);
  QGW_CUBE_SWITCH(QGW_CASE)
#undef QGW_CASE
}

hipError_t launch_sigma3(const Plan& p, const void* gt, const void* wc, int in_q, int out_k, void* sig, hipStream_t s) {
#define QGW_CASE(NN) \
  case NN:           \
    return p.prec == 0 ? sigma3_n<NN, double>(p, gt, wc, in_q, out_k, sig, s) \
                       : sigma3_n<NN, float>(p, gt, wc, in_q, out_k, sig, s);
  QGW_CUBE_SWITCH(QGW_CASE)
#undef QGW_CASE
}

hipError_t launch_sigma_bwd_wc3(const Plan& p, const void* gt, const void* sbar, void* out, hipStream_t s) {
#define QGW_CASE(NN) \
  case NN:           \
    return sigma_bwd_wc3_n<NN>(p, gt, sbar, out, s);
  QGW_CUBE_SWITCH(QGW_CASE)
#undef QGW_CASE
}

hipError_t launch_contract_bwd3(const Plan& p, int mode, const void* xq, const void* y, void* out, hipStream_t s) {
#define QGW_CASE(NN) \
  case NN:           \
    return contract_bwd3_n<NN>(p, mode, xq, y, out, s);
  QGW_CUBE_SWITCH(QGW_CASE)
#undef QGW_CASE
}

#undef QGW_CUBE_SWITCH

}  // namespace qgw
