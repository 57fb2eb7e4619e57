// Adjoints of the bubble (Eq. eq-polarizability), of the self-energy
// (Eq. eq-gw-self-energy) and of the density row, FP64.
//
// Cotangents follow zbar = dL/dRe z + i dL/dIm z: a complex-linear y = A x
// has xbar = A^H ybar and a product y = a b has abar = conj(b) ybar.
//
// Self-energy, S_ik(R, t) = -sum W^C_{(il),(jk)}(R, t) G_lj(R, t):
//   Wbar_{(il),(jk)}(R) = -conj(G_lj(R)) Sbar_ik(R)          (outer form)
//   Gbar_lj(R)         = -sum_{ik} conj(W^C_{(il),(jk)}(R)) Sbar_ik(R)
// Bubble, P_{(il),(jk)}(R, t) = -2 G_lj(R, t) G_ki(-R, beta - t):
//   Gbar_lj(R, t)          = -2 sum_{ik} conj(G_ki(-R, beta - t)) Pbar(R)
//   Gbar_ki(-R, beta - t) = -2 sum_{lj} conj(G_lj(R, t)) Pbar(R)
// The contractions reuse the layout of the forward self-energy kernel: one
// block per output slab, term lanes that each transform one pair slab from
// q to R in LDS, and a sum over lanes at the end.
#include "qgw_fft_reg.h"
#include "qgw_internal.h"

namespace qgw {

// ---------------------------------------------------------------------------
// density row: forward y[c] = s sum_t rho_t x[t][c] (with the Hermitian part
// of the input (herm 1) or of the output (herm 2) over the orbital pair)
// ---------------------------------------------------------------------------
__global__ void k_row_bwd(const zd* __restrict__ ybar, zd* __restrict__ xbar, const zd* __restrict__ rho,
                          int r, int64_t ncols, int no, int nk, double sre, double sim, int herm) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= int64_t(r) * ncols) return;
  const int t = int(gi / ncols);
  const int64_t c = gi - int64_t(t) * ncols;
  const cpx<double> w = conj(mk(sre, sim) * rho[t]);
  const cpx<double> y = ybar[c];
  cpx<double> x;
  if (herm == 0) {
    x = w * y;
  } else {
    const int64_t k = c % nk, ab = c / nk;
    const int a = int(ab / no), b = int(ab % no);
    const cpx<double> ys = ybar[(int64_t(b) * no + a) * nk + k];
    if (herm == 2)
      x = w * scale(y + conj(ys), 0.5);
    else
      x = scale(w * y + conj(w * ys), 0.5);
  }
  xbar[gi] = x;
}

// ---------------------------------------------------------------------------
// Wbar(q) = (1/N_k) sum_R e^{-iq.R} [-conj(G_lj(R)) Sbar_ik(R)], slab (t, alpha, beta)
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_sigma_bwd_wc(const zd* __restrict__ gt, const zd* __restrict__ sbar,
                                                      zd* __restrict__ out, int64_t nslabs, int spb, int no,
                                                      int nb, const int* __restrict__ pairs,
                                                      const zd* __restrict__ tw) {
  using M = MeshShape<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<double>* lds = reinterpret_cast<cpx<double>*>(smem_raw);
  const int64_t s0 = int64_t(blockIdx.x) * spb;
  const int nloc = int(nslabs - s0 < spb ? nslabs - s0 : spb);
  const int sl = threadIdx.x / N, line = threadIdx.x - sl * N;
  const bool act = sl < nloc;
  const double c = -1.0 / double(M::NN);
  cpx<double> x[N];
  if (act) {
    const int64_t s = s0 + sl;
    const int be = int(s % nb), al = int((s / nb) % nb);
    const int64_t t = s / (int64_t(nb) * nb);
    const int i = pairs[al], l = pairs[nb + al], j = pairs[be], k = pairs[nb + be];
    const zd* a = gt + ((t * no + l) * no + j) * M::NN;
    const zd* b = sbar + ((t * no + i) * no + k) * M::NN;
#pragma unroll
    for (int r1 = 0; r1 < N; ++r1) x[r1] = scale(conj(a[r1 * N + line]) * b[r1 * N + line], c);
    fft_reg<N, -1>(x, tw);  // R1 -> q1
    cpx<double>* slab = lds + sl * M::SLAB;
#pragma unroll
    for (int q1 = 0; q1 < N; ++q1) slab[q1 * M::LD + line] = x[q1];
  }
  __syncthreads();
  if (act) {
    cpx<double>* slab = lds + sl * M::SLAB;
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = slab[line * M::LD + j];
    fft_reg<N, -1>(x, tw);  // R2 -> q2
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
// contraction adjoints; one block per output slab (t, key), in the XCD-aware
// block order of the forward kernels (the outputs of one time node share an
// L2, which holds the Y slabs they all read)
//   MODE 0: key (l, j), terms (alpha, beta, i, k); X = conj(W^C(R)) with
//           W^C(R) = (1/N_k) sum_q e^{iq.R} W^C(q); Y = Sbar_ik(R); c = -1
//   MODE 1: key (l, j), terms (alpha, beta, i, k); X = Pbar(R) = sum_q e^{iq.R} Pbar(q);
//           Y = conj(G_ki(-R, beta - t)); c = -2
//   MODE 2: key (i, k), terms (alpha, beta, l, j); X = Pbar(R); Y = conj(G_lj(R, t)); c = -2;
//           the sum is the cotangent of G_ki(-R, beta - t), stored in slab (t, k, i) at -R
// Per term a lane loads one column of the X(q) slab straight into registers (N independent coalesced
// loads), transforms it along q1, passes it through LDS once to hold a row R1, transforms along q2 and
// accumulates X Y for that row; the lanes' rows are summed through LDS and stored coalesced.
// ---------------------------------------------------------------------------
template <int N, int MODE>
__global__ __launch_bounds__(256) void k_contract_bwd(const zd* __restrict__ xq, const zd* __restrict__ y,
                                                      zd* __restrict__ out, int spb, int no, int nb,
                                                      const int4* __restrict__ terms,
                                                      const int* __restrict__ term_off,
                                                      const zd* __restrict__ tw) {
  using M = MeshShape<N>;
  extern __shared__ unsigned char smem_raw[];
  cpx<double>* lds = reinterpret_cast<cpx<double>*>(smem_raw);
  const int out_slab = int(xcd_block(blockIdx.x, gridDim.x));  // t * no^2 + key
  const int key = out_slab % (no * no);
  const int64_t t = out_slab / (no * no);
  const int tb = term_off[key], te = term_off[key + 1];
  const int lane = threadIdx.x / N, line = threadIdx.x - lane * N;
  const bool act = lane < spb;
  cpx<double> acc[N];  // row R1 = line of this lane's partial sum
#pragma unroll
  for (int j = 0; j < N; ++j) acc[j] = mk(0.0, 0.0);
  cpx<double> x[N];
  cpx<double>* slab = lds + lane * M::SLAB;
  for (int c0 = tb; c0 < te; c0 += spb) {
    const bool mine = act && c0 + lane < te;
    int4 tm = make_int4(0, 0, 0, 0);
    if (mine) {
      tm = terms[c0 + lane];
      const zd* w = xq + ((t * nb + tm.x) * nb + tm.y) * M::NN;
#pragma unroll
      for (int j = 0; j < N; ++j) x[j] = w[j * N + line];  // column q2 = line
      fft_reg<N, +1>(x, tw);                                 // q1 -> R1
#pragma unroll
      for (int j = 0; j < N; ++j) slab[j * M::LD + line] = x[j];
    }
    __syncthreads();
    if (mine) {
#pragma unroll
      for (int j = 0; j < N; ++j) x[j] = slab[line * M::LD + j];  // row R1 = line
      fft_reg<N, +1>(x, tw);                                       // q2 -> R2; x[j] = X(R1 = line, R2 = j)
      if (MODE == 0) {
        const zd* g = y + ((t * no + tm.z) * no + tm.w) * M::NN + line * N;
#pragma unroll
        for (int j = 0; j < N; ++j) acc[j] = fma(acc[j], conj(x[j]), g[j]);
      } else if (MODE == 1) {
        const zd* g = y + ((t * no + tm.w) * no + tm.z) * M::NN + ((N - line) % N) * N;
#pragma unroll
        for (int j = 0; j < N; ++j) acc[j] = fma(acc[j], x[j], conj(g[(N - j) % N]));
      } else {
        const zd* g = y + ((t * no + tm.z) * no + tm.w) * M::NN + line * N;
#pragma unroll
        for (int j = 0; j < N; ++j) acc[j] = fma(acc[j], x[j], conj(g[j]));
      }
    }
    __syncthreads();  // the slab is free for the next term
  }
  // reduce the term lanes: lane partial rows -> LDS, the first lane's threads add them up in a fixed order
  if (act) {
#pragma unroll
    for (int j = 0; j < N; ++j) slab[line * M::LD + j] = acc[j];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    const double c = MODE == 0 ? -1.0 / double(M::NN) : -2.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cpx<double> s = lds[line * M::LD + j];
      for (int l2 = 1; l2 < spb; ++l2) s = s + lds[l2 * M::SLAB + line * M::LD + j];
      x[j] = scale(s, c);
    }
  }
  __syncthreads();  // every lane's partial row has been read
  if (threadIdx.x < N) {
    // MODE 2 stores at -R: row (N - line) % N, column (N - j) % N
    const int r1 = MODE == 2 ? (N - line) % N : line;
#pragma unroll
    for (int j = 0; j < N; ++j) lds[r1 * M::LD + (MODE == 2 ? (N - j) % N : j)] = x[j];
  }
  __syncthreads();
  int oslab = out_slab;
  if (MODE == 2) {
    const int i = key / no, k = key - i * no;
    oslab = int(t) * no * no + k * no + i;
  }
  zd* o = out + int64_t(oslab) * M::NN;
  for (int e = threadIdx.x; e < M::NN; e += blockDim.x) {
    const int r1 = e / N, r2 = e - r1 * N;
    o[e] = lds[r1 * M::LD + r2];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

constexpr int kLdsBudget = 64 * 1024;

template <int N>
hipError_t sigma_bwd_wc_n(const Plan& p, const void* gt, const void* sbar, void* out, hipStream_t s) {
  const int64_t nslabs = int64_t(p.r) * p.nb * p.nb;
  const int spb = slabs_per_block<double>(N, kLdsBudget);
  const int64_t blocks = (nslabs + spb - 1) / spb;
  const size_t lds = size_t(spb) * MeshShape<N>::SLAB * sizeof(zd);
  hipLaunchKernelGGL((k_sigma_bwd_wc<N>), dim3(unsigned(blocks)), dim3(spb * N), lds, s, (const zd*)gt,
                     (const zd*)sbar, (zd*)out, nslabs, spb, p.no, p.nb, p.d_pairs, p.d_tw64);
  return hipGetLastError();
}

template <int N>
hipError_t contract_bwd_n(const Plan& p, int mode, const void* xq, const void* y, void* out, hipStream_t s) {
  const TermTable& tt = (mode == 2) ? p.terms : p.terms_lj;
  // term lanes: the largest divisor of the per-output term count that fits (every lane gets the same count)
  const int cap = slabs_per_block<double>(N, kLdsBudget);
  int spb = 1;
  for (int d = 1; d <= tt.max_terms && d <= cap; ++d)
    if (tt.max_terms % d == 0) spb = d;
  const size_t lds = size_t(spb) * MeshShape<N>::SLAB * sizeof(zd);
  const unsigned blocks = unsigned(int64_t(p.r) * p.no * p.no);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(spb * N), lds, s, (const zd*)xq, (const zd*)y, (zd*)out, spb,
                       p.no, p.nb, (const int4*)tt.d_terms, tt.d_off, p.d_tw64);
  };
  if (mode == 0) go(k_contract_bwd<N, 0>);
  else if (mode == 1) go(k_contract_bwd<N, 1>);
  else go(k_contract_bwd<N, 2>);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_row_map_bwd(const Plan& p, int64_t ncols, double sre, double sim, int herm, const void* ybar,
                              void* xbar, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  const int64_t n = int64_t(p.r) * ncols;
  hipLaunchKernelGGL(k_row_bwd, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, (const zd*)ybar, (zd*)xbar,
                     (const zd*)p.dmaps64.m[5], p.r, ncols, p.no, p.nk, sre, sim, herm);
  return hipGetLastError();
}

hipError_t launch_sigma_bwd_wc(const Plan& p, const void* gt, const void* sbar, void* out, hipStream_t s) {
  if (p.dim == 3) return launch_sigma_bwd_wc3(p, gt, sbar, out, s);
  switch (p.n) {
#define QGW_CASE(NN) \
  case NN:           \
    return sigma_bwd_wc_n<NN>(p, gt, sbar, out, s);
    QGW_FOR_EACH_MESH(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_contract_bwd(const Plan& p, int mode, const void* xq, const void* y, void* out, hipStream_t s) {
  if (p.dim == 3) return launch_contract_bwd3(p, mode, xq, y, out, s);
  switch (p.n) {
#define QGW_CASE(NN) \
  case NN:           \
    return contract_bwd_n<NN>(p, mode, xq, y, out, s);
    QGW_FOR_EACH_MESH(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace qgw
