// DLR maps on the node axis: out[m][c] = s * sum_t T[m][t] in[t][c].
//
// The maps are r x r (r ~ 40-70) and the columns number up to ~10^6, so each
// thread owns one column and a chunk of MT output rows; the map entries are
// the same for every lane and are read through the scalar cache.  For pair
// arrays the kernel also changes the layout (slab <-> matrix) so that the
// Dyson-W solver reads whole matrices contiguously: the column read side is
// always coalesced, the write side goes out in 16-element runs.
//
// On orbital arrays (columns c = (a n_o + b) N_k + k) the plain map can also
// take the Hermitian part over (a, b) of its input (HERM = 1) or of its
// output (HERM = 2): the exact density matrix and the exact Sigma^C(k, tau)
// are Hermitian, and only their Hermitian parts are kept.
#include "qgw_internal.h"

namespace qgw {

enum { kPlain = 0, kSlabToMatrix = 1, kMatrixToSlab = 2 };

template <typename T, int MT, int MODE, int HERM>
__global__ __launch_bounds__(256) void k_dlr(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                             const cpx<T>* __restrict__ map, int r, int rows_out,
                                             int64_t ncols, int na, int nq, T sre, T sim) {
  const int tid = threadIdx.x;
  int64_t cin = 0, cout = 0, cswap = 0, plane = ncols;
  bool valid;
  if (MODE == kPlain) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + tid;
    valid = c < ncols;
    cin = cout = c;
    if (HERM) {  // na = n_o, nq = N_k: column of the transposed element
      const int64_t k = c % nq, ab = c / nq;
      const int a = int(ab / na), b = int(ab % na);
      cswap = (int64_t(b) * na + a) * nq + k;
    }
  } else {
    plane = int64_t(na) * nq;
    const int tq = (nq + 15) / 16;
    const int bq = int(blockIdx.x % tq), ba = int(blockIdx.x / tq);
    int qq, aa;
    if (MODE == kSlabToMatrix) {
      qq = tid & 15;
      aa = tid >> 4;
    } else {
      aa = tid & 15;
      qq = tid >> 4;
    }
    const int q = bq * 16 + qq, a = ba * 16 + aa;
    valid = (q < nq) && (a < na);
    if (MODE == kSlabToMatrix) {
      cin = int64_t(a) * nq + q;
      cout = int64_t(q) * na + a;
    } else {
      cin = int64_t(q) * na + a;
      cout = int64_t(a) * nq + q;
    }
  }
  const int m0 = blockIdx.y * MT;
  const cpx<T>* mp = map + int64_t(m0) * r;
  cpx<T> acc[MT];
#pragma unroll
  for (int mm = 0; mm < MT; ++mm) acc[mm] = mk(T(0), T(0));
  const cpx<T>* src = in + cin;
  const cpx<T>* srcs = in + cswap;
  if (HERM == 0) {
    cpx<T> x = valid ? src[0] : mk(T(0), T(0));
    for (int t = 0; t < r; ++t) {
      cpx<T> xn = (valid && t + 1 < r) ? src[int64_t(t + 1) * plane] : mk(T(0), T(0));
#pragma unroll
      for (int mm = 0; mm < MT; ++mm) acc[mm] = fma(acc[mm], mp[mm * r + t], x);
      x = xn;
    }
  } else if (HERM == 1) {
    const T h = T(0.5);
    for (int t = 0; t < r; ++t) {
      cpx<T> x = mk(T(0), T(0));
      if (valid) x = scale(src[int64_t(t) * plane] + conj(srcs[int64_t(t) * plane]), h);
#pragma unroll
      for (int mm = 0; mm < MT; ++mm) acc[mm] = fma(acc[mm], mp[mm * r + t], x);
    }
  } else {
    cpx<T> acc2[MT];
#pragma unroll
    for (int mm = 0; mm < MT; ++mm) acc2[mm] = mk(T(0), T(0));
    for (int t = 0; t < r; ++t) {
      cpx<T> x = mk(T(0), T(0)), y = mk(T(0), T(0));
      if (valid) {
        x = src[int64_t(t) * plane];
        y = srcs[int64_t(t) * plane];
      }
#pragma unroll
      for (int mm = 0; mm < MT; ++mm) {
        acc[mm] = fma(acc[mm], mp[mm * r + t], x);
        acc2[mm] = fma(acc2[mm], mp[mm * r + t], y);
      }
    }
    // (s A x)_ab / 2 + conj((s A x)_ba) / 2, applied below after the scale
    const cpx<T> sc0 = mk(sre, sim);
#pragma unroll
    for (int mm = 0; mm < MT; ++mm) acc[mm] = scale(sc0 * acc[mm] + conj(sc0 * acc2[mm]), T(0.5));
  }
  if (!valid) return;
  const cpx<T> sc = HERM == 2 ? mk(T(1), T(0)) : mk(sre, sim);
#pragma unroll
  for (int mm = 0; mm < MT; ++mm) {
    const int m = m0 + mm;
    if (m < rows_out) out[int64_t(m) * plane + cout] = sc * acc[mm];
  }
}

namespace {

template <typename T>
const cpx<T>* map_ptr(const Plan& p, int map) {
  const DeviceMaps& d = (sizeof(T) == 8) ? p.dmaps64 : p.dmaps32;
  return reinterpret_cast<const cpx<T>*>(d.m[map]);
}

template <typename T, int MODE, int HERM>
hipError_t dlr_launch(const Plan& p, int map, int64_t ncols, int na, int nq, double sre, double sim,
                      const void* in, void* out, hipStream_t s) {
  const DeviceMaps& d = (sizeof(T) == 8) ? p.dmaps64 : p.dmaps32;
  const int rows_out = (map == 5) ? 1 : p.r;
  // small column counts: 64-thread blocks and 8-row chunks for enough blocks
  const bool small = (MODE == kPlain) && ncols <= 65536;
  const int mt = small ? 8 : d.mt;
  const int bs = small ? 64 : 256;
  const unsigned chunks = unsigned((rows_out + mt - 1) / mt);
  unsigned bx;
  if (MODE == kPlain)
    bx = unsigned((ncols + bs - 1) / bs);
  else
    bx = unsigned(((nq + 15) / 16) * ((na + 15) / 16));
  if (bx == 0) return hipSuccess;
  const dim3 grid(bx, chunks);
#define QGW_DLR_MT(MTV)                                                                        \
  case MTV:                                                                                    \
    hipLaunchKernelGGL((k_dlr<T, MTV, MODE, HERM>), grid, dim3(bs), 0, s, (const cpx<T>*)in,   \
                       (cpx<T>*)out, map_ptr<T>(p, map), p.r, rows_out, ncols, na, nq, T(sre), \
                       T(sim));                                                                \
    break;
  switch (mt) {
    QGW_DLR_MT(8)
    QGW_DLR_MT(16)
    QGW_DLR_MT(20)
    QGW_DLR_MT(24)
    QGW_DLR_MT(28)
    QGW_DLR_MT(32)
    default:
      return hipErrorInvalidValue;
  }
#undef QGW_DLR_MT
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dlr(const Plan& p, int map, int64_t ncols, double sre, double sim, const void* in,
                      void* out, hipStream_t s, int herm) {
  if (herm) {
    if (ncols != int64_t(p.no) * p.no * p.nk) return hipErrorInvalidValue;
    if (p.prec == 0) {
      if (herm == 1) return dlr_launch<double, kPlain, 1>(p, map, ncols, p.no, p.nk, sre, sim, in, out, s);
      return dlr_launch<double, kPlain, 2>(p, map, ncols, p.no, p.nk, sre, sim, in, out, s);
    }
    if (herm == 1) return dlr_launch<float, kPlain, 1>(p, map, ncols, p.no, p.nk, sre, sim, in, out, s);
    return dlr_launch<float, kPlain, 2>(p, map, ncols, p.no, p.nk, sre, sim, in, out, s);
  }
  if (p.prec == 0) return dlr_launch<double, kPlain, 0>(p, map, ncols, 0, 0, sre, sim, in, out, s);
  return dlr_launch<float, kPlain, 0>(p, map, ncols, 0, 0, sre, sim, in, out, s);
}

hipError_t launch_dlr_pairs(const Plan& p, int map, int in_layout, int out_layout, const void* in,
                            void* out, hipStream_t s) {
  const int na = p.nb * p.nb, nq = p.nk;
  const int64_t ncols = int64_t(na) * nq;
  int mode = kPlain;
  if (in_layout == 0 && out_layout == 1) mode = kSlabToMatrix;
  if (in_layout == 1 && out_layout == 0) mode = kMatrixToSlab;
  if (p.prec == 0) {
    if (mode == kPlain) return dlr_launch<double, kPlain, 0>(p, map, ncols, na, nq, 1, 0, in, out, s);
    if (mode == kSlabToMatrix) return dlr_launch<double, kSlabToMatrix, 0>(p, map, ncols, na, nq, 1, 0, in, out, s);
    return dlr_launch<double, kMatrixToSlab, 0>(p, map, ncols, na, nq, 1, 0, in, out, s);
  }
  if (mode == kPlain) return dlr_launch<float, kPlain, 0>(p, map, ncols, na, nq, 1, 0, in, out, s);
  if (mode == kSlabToMatrix) return dlr_launch<float, kSlabToMatrix, 0>(p, map, ncols, na, nq, 1, 0, in, out, s);
  return dlr_launch<float, kMatrixToSlab, 0>(p, map, ncols, na, nq, 1, 0, in, out, s);
}

}  // namespace qgw
