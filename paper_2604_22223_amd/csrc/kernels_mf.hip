// Transforms of the uniform-grid ("MF") form of the iteration: N = 2M
// Matsubara frequencies (fermionic w_n = (2n + 1) pi / beta, bosonic
// nu_n = 2 n pi / beta, n = -M .. M-1) and N midpoint times
// tau_j = (j + 1/2) beta / N, the conventional representation that the
// performance section compares the DLR with.
//
// Each transform along the node axis is a length-N DFT between two diagonal
// phase factors, out_k = post_k sum_j e^{s 2 pi i j k / N} pre_j in_j (+ an
// orbital-diagonal constant for iw -> tau, the exact transform of the 1/(iw)
// tail), so it runs as an FFT.  Arrays keep the library's layout, node axis
// slowest: a block owns C consecutive columns of all N nodes, loads them
// coalesced into LDS, and does the FFT in four steps, N = N1 N2:
//   1. N2 DFTs of length N1 (stride N2) in registers, one per thread, then the
//      twiddles e^{s 2 pi i j2 k1 / N};
//   2. N1 DFTs of length N2, one per thread, written to index k1 + N1 k2;
// then the output is scaled and stored coalesced.  N1, N2 <= 32 <= the
// threads per column, so every step is one round with no in-place hazard
// beyond the barrier between the reads and the writes of step 2.
#include "qgw.h"
#include "qgw_fft_reg.h"
#include "qgw_internal.h"

namespace qgw {

namespace {

template <int N1, int N2, int SIGN, int HERM>
__global__ __launch_bounds__(256) void k_mf_fft(const zd* __restrict__ in, zd* __restrict__ out,
                                                zd* __restrict__ out_rev, int64_t ncols, int no, int nk,
                                                const zd* __restrict__ tw, const zd* __restrict__ tw1,
                                                const zd* __restrict__ tw2, const zd* __restrict__ pre,
                                                const zd* __restrict__ post, const zd* __restrict__ diag, double sre,
                                                double sim) {
  constexpr int N = N1 * N2;
  constexpr int C = N <= 512 ? 8 : 4;  // columns per block (N C x 16 B of LDS <= 64 KB)
  constexpr int T = 256 / C;           // threads per column
  static_assert(N1 <= T && N2 <= T, "sub-transform longer than the threads of a column");
  __shared__ zd buf[N * C];
  const int64_t c0 = int64_t(blockIdx.x) * C;
  const int c = threadIdx.x % C, u = threadIdx.x / C;
  // load, with the input phase (and the Hermitian part over the orbital pair)
  for (int e = threadIdx.x; e < N * C; e += 256) {
    const int node = e / C, cc = e - node * C;
    const int64_t col = c0 + cc;
    cpx<double> v = mk(0.0, 0.0);
    if (col < ncols) {
      v = in[int64_t(node) * ncols + col];
      if (HERM) {
        const int64_t k = col % nk, ab = col / nk;
        const int a = int(ab / no), b = int(ab % no);
        const cpx<double> w = in[int64_t(node) * ncols + (int64_t(b) * no + a) * nk + k];
        v = scale(v + conj(w), 0.5);
      }
      v = v * pre[node];
    }
    buf[e] = v;
  }
  __syncthreads();
  if (u < N2) {
    const int j2 = u;
    cpx<double> x[N1];
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) x[j1] = buf[(j1 * N2 + j2) * C + c];
    fft_reg<N1, SIGN>(x, tw1);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      const int e = (j2 * k1) % N;
      const cpx<double> w = SIGN < 0 ? tw[e] : conj(tw[e]);
      buf[(k1 * N2 + j2) * C + c] = x[k1] * w;
    }
  }
  __syncthreads();
  cpx<double> y[N2];
  if (u < N1) {
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) y[j2] = buf[(u * N2 + j2) * C + c];
    fft_reg<N2, SIGN>(y, tw2);
  }
  __syncthreads();
  if (u < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) buf[(u + N1 * k2) * C + c] = y[k2];
  }
  __syncthreads();
  const cpx<double> sc = mk(sre, sim);
  for (int e = threadIdx.x; e < N * C; e += 256) {
    const int node = e / C, cc = e - node * C;
    const int64_t col = c0 + cc;
    if (col >= ncols) continue;
    cpx<double> v = buf[e] * post[node];
    if (diag) {
      const int64_t ab = col / nk;
      if (ab % (no + 1) == 0) v = v + diag[node];
    }
    v = sc * v;
    if (out) out[int64_t(node) * ncols + col] = v;
    if (out_rev) out_rev[int64_t(N - 1 - node) * ncols + col] = v;
  }
}

// per node, out[c][r] = in[r][c] for an R x CC matrix (the slab <-> matrix change of the pair arrays)
__global__ __launch_bounds__(256) void k_node_transpose(const zd* __restrict__ in, zd* __restrict__ out, int R, int CC) {
  __shared__ zd tile[32][33];
  const int64_t plane = int64_t(R) * CC;
  const zd* src = in + plane * blockIdx.z;
  zd* dst = out + plane * blockIdx.z;
  const int r0 = blockIdx.y * 32, cb = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + i, cc = cb + tx;
    if (r < R && cc < CC) tile[i][tx] = src[int64_t(r) * CC + cc];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int cc = cb + i, r = r0 + tx;
    if (r < R && cc < CC) dst[int64_t(cc) * R + r] = tile[tx][i];
  }
}

// y[col] += v on the orbital-diagonal columns (a == b) of an orbital array [no][no][nk]
__global__ __launch_bounds__(256) void k_diag_add(zd* __restrict__ y, int no, int nk, cpx<double> v) {
  const int64_t gi = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (gi >= int64_t(no) * nk) return;
  const int a = int(gi / nk), k = int(gi - int64_t(a) * nk);
  zd* p = y + (int64_t(a) * no + a) * nk + k;
  *p = *p + v;
}

struct MfTables {
  const zd *tw, *tw1, *tw2, *pre, *post, *diag;
};

// table offsets in Plan::d_mf: twiddles of N, N1, N2, then pre / post per transform, then the tail constant
MfTables mf_tables(const Plan& p, int t, bool with_diag) {
  const int N = p.r;
  const zd* b = p.d_mf;
  MfTables m;
  m.tw = b;
  m.tw1 = b + N;
  m.tw2 = b + N + p.mf_n1;
  const zd* ph = b + N + p.mf_n1 + p.mf_n2;
  m.pre = ph + size_t(2 * t) * N;
  m.post = ph + size_t(2 * t + 1) * N;
  m.diag = with_diag ? ph + size_t(8) * N : nullptr;
  return m;
}

template <int N1, int N2>
hipError_t mf_fft_n(const Plan& p, int t, int sign, int herm, int64_t ncols, const void* in, void* out, void* out_rev,
                    bool with_diag, double sre, double sim, hipStream_t s) {
  constexpr int N = N1 * N2;
  constexpr int C = N <= 512 ? 8 : 4;
  const MfTables m = mf_tables(p, t, with_diag);
  const unsigned blocks = unsigned((ncols + C - 1) / C);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, (const zd*)in, (zd*)out, (zd*)out_rev, ncols, p.no, p.nk,
                       m.tw, m.tw1, m.tw2, m.pre, m.post, m.diag, sre, sim);
  };
  if (sign < 0) go(k_mf_fft<N1, N2, -1, 0>);
  else if (herm) go(k_mf_fft<N1, N2, +1, 1>);
  else go(k_mf_fft<N1, N2, +1, 0>);
  return hipGetLastError();
}

// transform index t: 0 F_IW2TAU, 1 F_TAU2IW, 2 B_TAU2IW, 3 B_IW2TAU; sign of the DFT
constexpr int kMfSign[4] = {-1, +1, +1, -1};

hipError_t mf_fft(const Plan& p, int t, int herm, int64_t ncols, const void* in, void* out, void* out_rev,
                  bool with_diag, double sre, double sim, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  const int sign = kMfSign[t];
  switch (p.r) {
#define QGW_CASE(NN, A, B) \
  case NN:                 \
    return mf_fft_n<A, B>(p, t, sign, herm, ncols, in, out, out_rev, with_diag, sre, sim, s);
    QGW_FOR_EACH_MF_GRID(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

bool mf_grid_split(int n, int* n1, int* n2) {
  switch (n) {
#define QGW_CASE(NN, A, B) \
  case NN:                 \
    *n1 = A;               \
    *n2 = B;               \
    return true;
    QGW_FOR_EACH_MF_GRID(QGW_CASE)
#undef QGW_CASE
    default:
      return false;
  }
}

hipError_t launch_mf(const Plan& p, int map, int64_t ncols, double sre, double sim, const void* in, void* out,
                     hipStream_t s, int herm) {
  if (ncols <= 0) return hipSuccess;
  const int64_t norb = int64_t(p.no) * p.no * p.nk;
  switch (map) {
    case QGW_F_IW2TAU:
    case QGW_F_IW2TAUR:
      if (ncols != norb || herm) return hipErrorInvalidValue;
      return mf_fft(p, 0, 0, ncols, in, map == QGW_F_IW2TAU ? out : nullptr, map == QGW_F_IW2TAUR ? out : nullptr,
                    true, sre, sim, s);
    case QGW_F_TAU2IW:
      if (herm == 2 || (herm == 1 && ncols != norb)) return hipErrorInvalidValue;
      return mf_fft(p, 1, herm, ncols, in, out, nullptr, false, sre, sim, s);
    case QGW_B_TAU2IW:
      if (herm) return hipErrorInvalidValue;
      return mf_fft(p, 2, 0, ncols, in, out, nullptr, false, sre, sim, s);
    case QGW_B_IW2TAU:
      if (herm) return hipErrorInvalidValue;
      return mf_fft(p, 3, 0, ncols, in, out, nullptr, false, sre, sim, s);
    case QGW_F_IW2BETA: {
      // G(beta^-) = -(1/beta) sum_n G(i w_n) - delta_ab / 2: the density row, then the diagonal constant
      if (ncols != norb) return hipErrorInvalidValue;
      hipError_t e = launch_row_map(p, ncols, sre, sim, herm, in, out, s);
      if (e != hipSuccess) return e;
      const cpx<double> v = mk(-0.5 * sre, -0.5 * sim);
      hipLaunchKernelGGL(k_diag_add, dim3(unsigned((int64_t(p.no) * p.nk + 255) / 256)), dim3(256), 0, s, (zd*)out,
                         p.no, p.nk, v);
      return hipGetLastError();
    }
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_mf_g_tau(const Plan& p, const void* g_iw, void* g_tau, void* g_reflt, hipStream_t s) {
  return mf_fft(p, 0, 0, int64_t(p.no) * p.no * p.nk, g_iw, g_tau, g_reflt, true, 1.0, 0.0, s);
}

hipError_t launch_mf_pairs(const Plan& p, int map, int in_layout, int out_layout, const void* in, void* out,
                           hipStream_t s) {
  if (map != QGW_B_TAU2IW && map != QGW_B_IW2TAU) return hipErrorInvalidValue;
  const int t = map == QGW_B_TAU2IW ? 2 : 3;
  const int na = p.nb * p.nb;
  const int64_t ncols = int64_t(na) * p.nk;
  if (in_layout != out_layout) {
    // the layout change first, into out; then the transform in place (the node axis is slowest in both layouts)
    const int R = in_layout == QGW_LAYOUT_SLAB ? na : p.nk, CC = in_layout == QGW_LAYOUT_SLAB ? p.nk : na;
    hipLaunchKernelGGL(k_node_transpose, dim3(unsigned((CC + 31) / 32), unsigned((R + 31) / 32), unsigned(p.r)),
                       dim3(256), 0, s, (const zd*)in, (zd*)out, R, CC);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mf_fft(p, t, 0, ncols, out, out, nullptr, false, 1.0, 0.0, s);
  }
  return mf_fft(p, t, 0, ncols, in, out, nullptr, false, 1.0, 0.0, s);
}

}  // namespace qgw
