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
#include "qgw_mfma.h"

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
#pragma unroll 4
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
#pragma unroll 4
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

// One-row maps (the density row G(beta^-) from G(i w_m)): out[c] = s sum_t row[t] in[t][c].  A block of
// kRowWaves waves takes 64 columns; wave w sums the nodes t = w, w + kRowWaves, ... for its lane's column
// (coalesced 64-column reads), and the partial sums are added in a fixed order.  HERM as for k_dlr.
constexpr int kRowWaves = 8;
template <typename T, int HERM>
__global__ __launch_bounds__(64 * kRowWaves) void k_dlr_row(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out,
                                                            const cpx<T>* __restrict__ row, int r, int64_t ncols,
                                                            int na, int nq, T sre, T sim) {
  __shared__ cpx<T> part[2][kRowWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c = int64_t(blockIdx.x) * 64 + lane;
  const bool valid = c < ncols;
  const int64_t cc = valid ? c : 0;
  int64_t cs = cc;
  if (HERM) {  // column (a na + b) nq + k -> (b na + a) nq + k
    const int64_t k = cc % nq, ab = cc / nq;
    const int a = int(ab / na), b = int(ab % na);
    cs = (int64_t(b) * na + a) * nq + k;
  }
  cpx<T> acc = mk(T(0), T(0)), acc2 = mk(T(0), T(0));
#pragma unroll 4
  for (int t = w; t < r; t += kRowWaves) {
    const cpx<T> m = row[t];
    const cpx<T> x = in[int64_t(t) * ncols + cc];
    if (HERM == 0) {
      acc = fma(acc, m, x);
    } else if (HERM == 1) {
      acc = fma(acc, m, scale(x + conj(in[int64_t(t) * ncols + cs]), T(0.5)));
    } else {
      acc = fma(acc, m, x);
      acc2 = fma(acc2, m, in[int64_t(t) * ncols + cs]);
    }
  }
  part[0][w][lane] = acc;
  part[1][w][lane] = acc2;
  __syncthreads();
  if (w != 0 || !valid) return;
  cpx<T> a = part[0][0][lane], b = part[1][0][lane];
#pragma unroll
  for (int i = 1; i < kRowWaves; ++i) {
    a = a + part[0][i][lane];
    b = b + part[1][i][lane];
  }
  const cpx<T> sc = mk(sre, sim);
  out[c] = HERM == 2 ? scale(sc * a + conj(sc * b), T(0.5)) : sc * a;
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
  int mt = small ? 8 : d.mt;
  if (MODE == kPlain && p.tune.orb_mt > 0) mt = p.tune.orb_mt;
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

// ---------------------------------------------------------------------------
// MFMA form for pair arrays (r <= 64): out = T in as a complex GEMM of an
// r x r map with ~10^5-10^6 columns, done as four real products per 4-deep
// slice on the 16x16x4 matrix cores (FP64 or FP32).  A block of 8 waves
// keeps Re T and Im T in LDS, zero padded and in operand order (the 64 values
// one MFMA takes are consecutive, so the reads are free of bank conflicts);
// each wave computes a strip of 16 columns for all rows.  When the layout
// changes, the 16 lanes of a strip run along the index that is contiguous in
// the output, so every wave writes whole 256-byte (FP64) runs per row; the 8
// waves of a block take 8 adjacent values of the other index, so together
// they read whole lines of the input.
// ---------------------------------------------------------------------------
// identity on a register value through a DPP move (quad_perm [0,1,2,3]); the
// compiler cannot see through it, which keeps a software-pipelined load from
// being folded back into its use
template <typename T>
__device__ __forceinline__ T dpp_identity(T v) {
  static_assert(sizeof(T) % 4 == 0, "32-bit words");
  int w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < int(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_update_dpp(w[i], w[i], 0xE4, 0xF, 0xF, false);
  __builtin_memcpy(&v, w, sizeof(T));
  return v;
}

// four waves per SIMD: two 512-thread blocks fit a CU.  TI, TO: element types of the input and the output when
// they differ from the arithmetic type T (an FP64 input rounded to FP32 as it is used, an FP32 result widened to
// FP64 as it is stored), which gives the same values as a separate conversion pass before or after the map
template <typename T, int MT, int MODE, bool HERM_IN, typename TI = T, typename TO = T>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_dlr_mfma(const cpx<TI>* __restrict__ in, cpx<TO>* __restrict__ out,
                                                  const cpx<T>* __restrict__ map, int r, int kp, int na,
                                                  int nq, int64_t nstrips, int no, T sre, T sim, int ysplit,
                                                  const cpx<T>* __restrict__ map2, cpx<TO>* __restrict__ out2,
                                                  int tiles_per_map) {
  static_assert(!HERM_IN || sizeof(TI) == sizeof(T), "the Hermitian part is taken in the arithmetic type");
  using M = Mfma<T>;
  using v4 = typename M::v4;
  extern __shared__ unsigned char smem_raw[];
  T* tre = reinterpret_cast<T*>(smem_raw);
  T* tim = tre + MT * 16 * kp;
  // With ysplit > 1 a block computes only the MT row tiles from tile ``tile`` MT on, and the ysplit blocks of
  // one group of strips are hardware blocks g 8 ysplit + 8 tile + x (x < 8): the same XCD (hardware blocks are
  // dealt round-robin to the 8 XCDs) at nearly the same time, so the group's inputs leave HBM once and the other
  // tiles read them from that XCD's L2.  The group count is a multiple of 8.
  int64_t group = blockIdx.x, ngroups = gridDim.x;
  int tile = 0;
  if (ysplit > 1) {
    const int64_t i = int64_t(blockIdx.x) >> 3;
    tile = int(i % ysplit);
    group = (i / ysplit) * 8 + (blockIdx.x & 7);
    ngroups = gridDim.x / ysplit;
  }
  // a second map of the same input (map2, out2): the tiles from tiles_per_map on are its row tiles
  if (map2 != nullptr && tile >= tiles_per_map) {
    map = map2;
    out = out2;
    tile -= tiles_per_map;
  }
  const int row0 = tile * MT * 16;
  // operand order: entry ((k / 4) MT + mt) 64 + lane holds T[row0 + mt 16 + lane % 16][4 (k / 4) + lane / 16],
  // so that the 64 lanes of one operand read 64 consecutive values
  for (int e = threadIdx.x; e < MT * 16 * kp; e += blockDim.x) {
    const int l = e & 63, g = e >> 6;
    const int kk = g / MT, mt = g - kk * MT;
    const int i = row0 + mt * 16 + (l & 15), k = 4 * kk + (l >> 4);
    const cpx<T> v = (i < r && k < r) ? map[int64_t(i) * r + k] : mk(T(0), T(0));
    tre[e] = v.re;
    tim[e] = v.im;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, lk = lane >> 4;
  const int64_t plane = int64_t(na) * nq;
  for (int64_t strip = group * 8 + wave; strip < nstrips; strip += ngroups * 8) {
    int64_t cin, cout;
    bool valid;
    if (MODE == kSlabToMatrix) {  // lanes along a (contiguous in the output), strips along q
      const int64_t ab = strip / nq;
      const int q = int(strip - ab * nq);
      const int a = int(ab) * 16 + lc;
      valid = a < na;
      cin = int64_t(a) * nq + q;
      cout = int64_t(q) * na + a;
    } else if (MODE == kMatrixToSlab) {  // lanes along q (contiguous in the output), strips along a
      const int64_t qb = strip / na;
      const int a = int(strip - qb * na);
      const int q = int(qb) * 16 + lc;
      valid = q < nq;
      cin = int64_t(q) * na + a;
      cout = int64_t(a) * nq + q;
    } else {
      cin = cout = strip * 16 + lc;
      valid = cin < plane;
    }
    int64_t cswap = cin;
    if (HERM_IN && valid) {  // orbital array: column (a n_o + b) N_k + k -> (b n_o + a) N_k + k
      const int64_t k = cin % nq, ab = cin / nq;
      const int a = int(ab / no), b = int(ab % no);
      cswap = (int64_t(b) * no + a) * nq + k;
    }
    v4 accr[MT], acci[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      accr[mt] = v4{T(0), T(0), T(0), T(0)};
      acci[mt] = v4{T(0), T(0), T(0), T(0)};
    }
    // Loads are unconditional, so that two stay in flight: the node index is
    // clamped to r - 1 (the map's zero padding for k >= r cancels what is
    // read there) and a column outside the array reads column 0 (its results
    // are not stored; every output column depends on its own input column only).
    const cpx<TI>* src = in + (valid ? cin : 0);
    const cpx<TI>* srcs = in + (valid ? cswap : 0);
    // the loaded values stay in the input type until their use, so that the conversion does not wait on the load
    auto load = [&](int t) -> cpx<TI> {
      const int64_t tc = t < r ? t : r - 1;
      cpx<TI> v = src[tc * plane];
      if (HERM_IN) v = scale(v + conj(srcs[tc * plane]), TI(0.5));
      return v;
    };
    // the input slice is read two steps ahead of its use
    cpx<TI> xi = dpp_identity(load(lk)), xn = dpp_identity(load(4 + lk));
    for (int kb = 0; kb < kp; kb += 4) {
      const cpx<TI> xnn = load(kb + 8 + lk);
      const cpx<T> x = cast<T>(xi);
      const int kk = kb >> 2;
      T ar[MT], ai[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        ar[mt] = tre[(kk * MT + mt) * 64 + lane];
        ai[mt] = tim[(kk * MT + mt) * 64 + lane];
      }
      // 2 MT independent accumulator chains per half-slice
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        accr[mt] = M::mac(ar[mt], x.re, accr[mt]);
        acci[mt] = M::mac(ar[mt], x.im, acci[mt]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        accr[mt] = M::mac(-ai[mt], x.im, accr[mt]);
        acci[mt] = M::mac(ai[mt], x.re, acci[mt]);
      }
      xi = xn;
      xn = xnn;
    }
    if (valid) {
      const cpx<T> sc = mk(sre, sim);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = row0 + mt * 16 + M::row(lane, v);
          if (m < r) out[int64_t(m) * plane + cout] = cast<TO>(sc * mk(accr[mt][v], acci[mt][v]));
        }
    }
  }
}

// Pair arrays with the slab <-> matrix layout change.  A block of 8 waves
// takes a tile of 16 x 8 columns: 16 values of the index L that is contiguous
// in the output (one per lane of a strip) and 8 values of the index W that is
// contiguous in the input (one per wave).  Per 4-deep slice of the node axis
// the block reads the 4 x 16 x 8 input values with one load per thread (eight
// threads cover 128 contiguous bytes), issued a slice ahead, and passes them
// through LDS (two buffers, alternating by slice); each wave then multiplies
// its 16-column strip on the matrix cores and writes whole 16-value runs of
// the output.  Slab -> matrix: L = pair index a, W = q; matrix -> slab:
// L = q, W = a.
// WT: W values per wave (tile 16 x 8 WT).  FP32 takes WT = 2, so that the eight threads' values of one row of the
// input (8 WT x 8 bytes) are a whole 128-byte line, as the 8 FP64 values of WT = 1 are; each barrier then also
// carries twice the matrix-core work.
template <typename T, int MT, int MODE, int WT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_dlr_mfma_pairs(
    const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, const cpx<T>* __restrict__ map, int r, int kp,
    int na, int nq, int tiles_l, int64_t ntiles, T sre, T sim, int64_t in_ld) {
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int TW = 8 * WT;         // W extent of a tile
  constexpr int SW = WT == 2 ? 4 : 3;  // log2(TW)
  constexpr int WP = TW + 1;         // padded W extent of the LDS tile
  constexpr int XT = 4 * 16 * WP;    // one tile buffer (complex values)
  extern __shared__ unsigned char smem_raw[];
  T* tre = reinterpret_cast<T*>(smem_raw);
  T* tim = tre + MT * 16 * kp;
  cpx<T>* xt = reinterpret_cast<cpx<T>*>(tim + MT * 16 * kp);
  for (int e = threadIdx.x; e < MT * 16 * kp; e += blockDim.x) {
    const int l = e & 63, g = e >> 6;
    const int kk = g / MT, mt = g - kk * MT;
    const int i = mt * 16 + (l & 15), k = 4 * kk + (l >> 4);
    const cpx<T> v = (i < r && k < r) ? map[int64_t(i) * r + k] : mk(T(0), T(0));
    tre[e] = v.re;
    tim[e] = v.im;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, lk = lane >> 4;
  // the values this thread loads per slice (j < WT): node lt[j], column (lL, lW) of the tile, from the index
  // threadIdx.x + 512 j over (node, L, W) with W fastest
  const int lW = threadIdx.x & (TW - 1), lL = (threadIdx.x >> SW) & 15;
  int lt[WT];
#pragma unroll
  for (int j = 0; j < WT; ++j) lt[j] = (threadIdx.x + 512 * j) >> (SW + 4);
  const int nL = MODE == kSlabToMatrix ? na : nq, nW = MODE == kSlabToMatrix ? nq : na;
  const int64_t plane = int64_t(na) * nq;
  // the input's rows (index L) are in_ld apart, its node planes nL in_ld (in_ld >= nW: padded rows)
  const int64_t in_plane = int64_t(nL) * in_ld;
  int buf = 0;  // slice parity, continued across tiles
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int tL = int(tile % tiles_l), tW = int(tile / tiles_l);
    // input column of this thread's loads (clamped into the array: values
    // outside it feed only columns that are not stored)
    const int Lld = min(tL * 16 + lL, nL - 1), Wld = min(tW * TW + lW, nW - 1);
    const cpx<T>* src = in + int64_t(Lld) * in_ld + Wld;
    // node index clamped to r - 1: the map's zero padding cancels it
    auto gload = [&](int kb, int j) -> cpx<T> { return src[int64_t(min(kb + lt[j], r - 1)) * in_plane]; };
    const int Lo = tL * 16 + lc;
    v4 accr[WT][MT], acci[WT][MT];
#pragma unroll
    for (int w = 0; w < WT; ++w)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        accr[w][mt] = v4{T(0), T(0), T(0), T(0)};
        acci[w][mt] = v4{T(0), T(0), T(0), T(0)};
      }
    cpx<T> g[WT];
#pragma unroll
    for (int j = 0; j < WT; ++j) g[j] = dpp_identity(gload(0, j));
    for (int kb = 0; kb < kp; kb += 4, buf ^= 1) {
      cpx<T>* xb = xt + buf * XT;
#pragma unroll
      for (int j = 0; j < WT; ++j) xb[(lt[j] * 16 + lL) * WP + lW] = g[j];
      __syncthreads();  // the slice is in LDS; the buffer written next was read two slices ago
#pragma unroll
      for (int j = 0; j < WT; ++j) g[j] = gload(kb + 4, j);
      cpx<T> x[WT];
#pragma unroll
      for (int w = 0; w < WT; ++w) x[w] = xb[(lk * 16 + lc) * WP + wave + 8 * w];
      const int kk = kb >> 2;
      T ar[MT], ai[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        ar[mt] = tre[(kk * MT + mt) * 64 + lane];
        ai[mt] = tim[(kk * MT + mt) * 64 + lane];
      }
#pragma unroll
      for (int w = 0; w < WT; ++w)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          accr[w][mt] = M::mac(ar[mt], x[w].re, accr[w][mt]);
          acci[w][mt] = M::mac(ar[mt], x[w].im, acci[w][mt]);
        }
#pragma unroll
      for (int w = 0; w < WT; ++w)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          accr[w][mt] = M::mac(-ai[mt], x[w].im, accr[w][mt]);
          acci[w][mt] = M::mac(ai[mt], x[w].re, acci[w][mt]);
        }
    }
    const cpx<T> sc = mk(sre, sim);
#pragma unroll
    for (int w = 0; w < WT; ++w) {
      const int Wo = tW * TW + wave + 8 * w;
      if (Lo < nL && Wo < nW) {
        const int64_t cout = int64_t(Wo) * nL + Lo;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = mt * 16 + M::row(lane, v);
            if (m < r) out[int64_t(m) * plane + cout] = sc * mk(accr[w][mt][v], acci[w][mt][v]);
          }
      }
    }
  }
}

// pair arrays with a layout change (MODE = kSlabToMatrix or kMatrixToSlab)
template <typename T, int MODE>
hipError_t dlr_mfma_pairs_launch(const Plan& p, int map, int na, int nq, double sre, double sim, const void* in,
                                 void* out, hipStream_t s, int64_t in_ld) {
  const int kp = (p.r + 3) / 4 * 4;
  const int mt = (p.r + 15) / 16;
  const int nL = MODE == kSlabToMatrix ? na : nq, nW = MODE == kSlabToMatrix ? nq : na;
  if (in_ld == 0) in_ld = nW;
  if (in_ld < nW) return hipErrorInvalidValue;
  constexpr int WT = sizeof(T) == 4 ? 2 : 1;  // W values per wave (see the kernel)
  const int tiles_l = (nL + 15) / 16;
  const int64_t ntiles = int64_t(tiles_l) * ((nW + 8 * WT - 1) / (8 * WT));
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int bpc = p.tune.mfma_bpc > 0 ? p.tune.mfma_bpc : 2;
  int64_t blocks = ntiles;
  if (blocks > int64_t(bpc) * ncu) blocks = int64_t(bpc) * ncu;
  const size_t lds = size_t(2) * mt * 16 * kp * sizeof(T) + size_t(2) * 4 * 16 * (8 * WT + 1) * sizeof(cpx<T>);
  const cpx<T>* mp = map_ptr<T>(p, map);
#define QGW_MFMA_MT(MTV)                                                                                       \
  case MTV:                                                                                                    \
    hipLaunchKernelGGL((k_dlr_mfma_pairs<T, MTV, MODE, WT>), dim3(unsigned(blocks)), dim3(512), lds, s,        \
                       (const cpx<T>*)in, (cpx<T>*)out, mp, p.r, kp, na, nq, tiles_l, ntiles, T(sre), T(sim), \
                       in_ld);                                                                                 \
    break;
  switch (mt) {
    QGW_MFMA_MT(1)
    QGW_MFMA_MT(2)
    QGW_MFMA_MT(3)
    QGW_MFMA_MT(4)
    default:
      return hipErrorInvalidValue;
  }
#undef QGW_MFMA_MT
  return hipGetLastError();
}

// na x nq columns; HERM_IN: orbital arrays (na = n_o^2, nq = N_k); TI, TO: input and output element types
template <typename T, int MODE, bool HERM_IN, typename TI = T, typename TO = T>
hipError_t dlr_mfma_launch(const Plan& p, int map, int na, int nq, double sre, double sim, const void* in,
                           void* out, hipStream_t s, int64_t in_ld = 0, int map2 = -1, void* out2 = nullptr) {
  const int kp = (p.r + 3) / 4 * 4;
  const int mt = (p.r + 15) / 16;
  if constexpr (MODE != kPlain) {
    static_assert(sizeof(TI) == sizeof(T) && sizeof(TO) == sizeof(T), "pair maps keep the arithmetic type");
    return dlr_mfma_pairs_launch<T, MODE>(p, map, na, nq, sre, sim, in, out, s, in_ld);
  }
  if (in_ld != 0) return hipErrorInvalidValue;
  int64_t nstrips;
  if (MODE == kSlabToMatrix)
    nstrips = int64_t((na + 15) / 16) * nq;
  else if (MODE == kMatrixToSlab)
    nstrips = int64_t((nq + 15) / 16) * na;
  else
    nstrips = (int64_t(na) * nq + 15) / 16;
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  int64_t blocks = (nstrips + 7) / 8;
  const int bpc = p.tune.mfma_bpc > 0 ? p.tune.mfma_bpc : 2;
  // too few strips for the GPU (the orbital-sized arrays): one block per row tile of a strip group, each
  // reading the same inputs (from L2) for its own 16 rows
  const int tiles = (blocks < 2 * int64_t(ncu)) ? mt : 1;  // row-tile blocks per strip group and map
  const int mtb = mt / tiles;
  if (map2 >= 0 && tiles == 1) {  // a second map of the same input: one launch only when the row tiles are split
    hipError_t e = dlr_mfma_launch<T, MODE, HERM_IN, TI, TO>(p, map, na, nq, sre, sim, in, out, s);
    return e == hipSuccess ? dlr_mfma_launch<T, MODE, HERM_IN, TI, TO>(p, map2, na, nq, sre, sim, in, out2, s) : e;
  }
  const int ysplit = map2 >= 0 ? 2 * tiles : tiles;
  if (blocks > int64_t(bpc) * ncu) blocks = int64_t(bpc) * ncu;
  if (ysplit > 1) blocks = (blocks + 7) / 8 * 8 * ysplit;  // groups rounded up to a multiple of 8, ysplit blocks each
  const size_t lds = size_t(2) * mtb * 16 * kp * sizeof(T);
  const cpx<T>* mp = map_ptr<T>(p, map);
  const cpx<T>* mp2 = map2 >= 0 ? map_ptr<T>(p, map2) : nullptr;
#define QGW_MFMA_MT(MTV)                                                                                  \
  case MTV:                                                                                               \
    hipLaunchKernelGGL((k_dlr_mfma<T, MTV, MODE, HERM_IN, TI, TO>), dim3(unsigned(blocks)), dim3(512), lds, s, \
                       (const cpx<TI>*)in, (cpx<TO>*)out, mp, p.r, kp, na, nq, nstrips, p.no, T(sre), T(sim),   \
                       ysplit, mp2, (cpx<TO>*)out2, tiles);                                                   \
    break;
  switch (mtb) {
    QGW_MFMA_MT(1)
    QGW_MFMA_MT(2)
    QGW_MFMA_MT(3)
    QGW_MFMA_MT(4)
    default:
      return hipErrorInvalidValue;
  }
#undef QGW_MFMA_MT
  return hipGetLastError();
}

}  // namespace

hipError_t launch_row_map(const Plan& p, int64_t ncols, double sre, double sim, int herm, const void* in, void* out,
                          hipStream_t s) {
  const int64_t ng = int64_t(p.no) * p.no * p.nk;
  if (herm && ncols != ng) return hipErrorInvalidValue;
  if (ncols <= 0) return hipSuccess;
  const unsigned blocks = unsigned((ncols + 63) / 64);
#define QGW_ROW(T, H)                                                                                     \
  hipLaunchKernelGGL((k_dlr_row<T, H>), dim3(blocks), dim3(64 * kRowWaves), 0, s, (const cpx<T>*)in, (cpx<T>*)out, \
                     map_ptr<T>(p, 5), p.r, ncols, p.no, p.nk, T(sre), T(sim))
  if (p.prec == 0) {
    if (herm == 0) QGW_ROW(double, 0);
    else if (herm == 1) QGW_ROW(double, 1);
    else QGW_ROW(double, 2);
  } else {
    if (herm == 0) QGW_ROW(float, 0);
    else if (herm == 1) QGW_ROW(float, 1);
    else QGW_ROW(float, 2);
  }
#undef QGW_ROW
  return hipGetLastError();
}

hipError_t launch_dlr(const Plan& p, int map, int64_t ncols, double sre, double sim, const void* in,
                      void* out, hipStream_t s, int herm) {
  if (p.grid == kGridMF) return launch_mf(p, map, ncols, sre, sim, in, out, s, herm);
  const int64_t ng = int64_t(p.no) * p.no * p.nk;
  if (p.r <= 64 && map != 5 && herm != 2 && (herm == 0 || ncols == ng) && p.tune.orb_valu != 1) {
    const int na = herm ? p.no * p.no : 1;
    const int nq = herm ? p.nk : int(ncols);
    if (herm == 0 && ncols > (int64_t(1) << 30)) return hipErrorInvalidValue;
    if (p.prec == 0) {
      if (herm) return dlr_mfma_launch<double, kPlain, true>(p, map, na, nq, sre, sim, in, out, s);
      return dlr_mfma_launch<double, kPlain, false>(p, map, na, nq, sre, sim, in, out, s);
    }
    if (herm) return dlr_mfma_launch<float, kPlain, true>(p, map, na, nq, sre, sim, in, out, s);
    return dlr_mfma_launch<float, kPlain, false>(p, map, na, nq, sre, sim, in, out, s);
  }
  if (map == 5) return launch_row_map(p, ncols, sre, sim, herm, in, out, s);  // one output row
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

hipError_t launch_dlr2(const Plan& p, int map1, int map2, int64_t ncols, const void* in, void* out1, void* out2,
                       hipStream_t s) {
  if (p.grid == kGridDLR && p.r <= 64 && map1 != 5 && map2 != 5 && p.tune.orb_valu != 1 && ncols <= (int64_t(1) << 30)) {
    if (p.prec == 0)
      return dlr_mfma_launch<double, kPlain, false>(p, map1, 1, int(ncols), 1, 0, in, out1, s, 0, map2, out2);
    return dlr_mfma_launch<float, kPlain, false>(p, map1, 1, int(ncols), 1, 0, in, out1, s, 0, map2, out2);
  }
  hipError_t e = launch_dlr(p, map1, ncols, 1.0, 0.0, in, out1, s);
  return e == hipSuccess ? launch_dlr(p, map2, ncols, 1.0, 0.0, in, out2, s) : e;
}

// An FP32 plan's two maps of an FP64 input (both time orders of G): the input is rounded to FP32 as the maps read
// it.  Where the matrix-core path does not apply, the input is first converted into `stage` (ncols r values).
hipError_t launch_dlr2_from_f64(const Plan& p, int map1, int map2, int64_t ncols, const void* in64, void* out1,
                                void* out2, void* stage, hipStream_t s) {
  if (p.prec != 1) return hipErrorInvalidValue;
  if (p.grid == kGridDLR && p.r <= 64 && map1 != 5 && map2 != 5 && p.tune.orb_valu != 1 && ncols <= (int64_t(1) << 30))
    return dlr_mfma_launch<float, kPlain, false, double, float>(p, map1, 1, int(ncols), 1, 0, in64, out1, s, 0, map2,
                                                               out2);
  hipError_t e = launch_convert(ncols * p.r, in64, stage, 1, s);
  return e == hipSuccess ? launch_dlr2(p, map1, map2, ncols, stage, out1, out2, s) : e;
}

// An FP32 plan's map of an orbital array (herm = 1: its Hermitian part) with the result widened to FP64 as it is
// stored.  Where the matrix-core path does not apply, the FP32 result goes to `stage` and is converted from there.
hipError_t launch_dlr_to_f64(const Plan& p, int map, int64_t ncols, double sre, double sim, const void* in,
                             void* out64, void* stage, hipStream_t s, int herm) {
  if (p.prec != 1) return hipErrorInvalidValue;
  const int64_t ng = int64_t(p.no) * p.no * p.nk;
  if (p.grid == kGridDLR && p.r <= 64 && map != 5 && herm != 2 && (herm == 0 || ncols == ng) &&
      p.tune.orb_valu != 1 && (herm != 0 || ncols <= (int64_t(1) << 30))) {
    const int na = herm ? p.no * p.no : 1;
    const int nq = herm ? p.nk : int(ncols);
    if (herm) return dlr_mfma_launch<float, kPlain, true, float, double>(p, map, na, nq, sre, sim, in, out64, s);
    return dlr_mfma_launch<float, kPlain, false, float, double>(p, map, na, nq, sre, sim, in, out64, s);
  }
  hipError_t e = launch_dlr(p, map, ncols, sre, sim, in, stage, s, herm);
  return e == hipSuccess ? launch_convert(ncols * p.r, stage, out64, 0, s) : e;
}

hipError_t launch_dlr_pairs(const Plan& p, int map, int in_layout, int out_layout, const void* in,
                            void* out, hipStream_t s, int64_t in_ld) {
  const int na = p.nb * p.nb, nq = p.nk;
  // padded input rows: only the matrix -> slab change of the matrix-core path reads them
  if (in_ld == (in_layout == 1 ? na : nq)) in_ld = 0;
  if (in_ld != 0 && !(p.grid == kGridDLR && p.r <= 64 && in_layout == 1 &&
                      out_layout == 0))
    return hipErrorInvalidValue;
  if (p.grid == kGridMF) return launch_mf_pairs(p, map, in_layout, out_layout, in, out, s);
  const int64_t ncols = int64_t(na) * nq;
  int mode = kPlain;
  if (in_layout == 0 && out_layout == 1) mode = kSlabToMatrix;
  if (in_layout == 1 && out_layout == 0) mode = kMatrixToSlab;
  if (p.r <= 64) {  // matrix-core path
    if (p.prec == 0) {
      if (mode == kPlain && in_ld == 0) return dlr_mfma_launch<double, kPlain, false>(p, map, na, nq, 1, 0, in, out, s);
      if (mode == kSlabToMatrix) return dlr_mfma_launch<double, kSlabToMatrix, false>(p, map, na, nq, 1, 0, in, out, s);
      if (mode == kMatrixToSlab)
        return dlr_mfma_launch<double, kMatrixToSlab, false>(p, map, na, nq, 1, 0, in, out, s, in_ld);
      return hipErrorInvalidValue;  // matrix -> matrix with padded rows
    }
    if (mode == kPlain && in_ld == 0) return dlr_mfma_launch<float, kPlain, false>(p, map, na, nq, 1, 0, in, out, s);
    if (mode == kSlabToMatrix) return dlr_mfma_launch<float, kSlabToMatrix, false>(p, map, na, nq, 1, 0, in, out, s);
    if (mode == kMatrixToSlab)
      return dlr_mfma_launch<float, kMatrixToSlab, false>(p, map, na, nq, 1, 0, in, out, s, in_ld);
    return hipErrorInvalidValue;
  }
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
