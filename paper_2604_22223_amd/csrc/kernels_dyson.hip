// Dyson equations.
//
// Screened interaction (Eq. eq-screened-coulomb): for every (bosonic node,
// q) solve (I - V P) W = V and return W^C = W - V.  Gauss-Jordan elimination
// with partial pivoting on the augmented system [I - V P | V], two lanes per
// row: lane (row, half 0) holds the row of I - V P, lane (row, half 1) the row
// of V, so a row costs 2 x N_b registers-worth of complex values spread over
// two lanes.  Both halves run the same instruction stream on different
// columns (no divergence): the pivot row is found by a segmented arg-max
// over the unused rows (ties go to the lower row) and broadcast through LDS;
// every row is updated as x <- x - f * pivot_row, with f = a_rs / a_ps for the
// other rows and f = 1 - 1 / a_ps for the pivot row itself (which normalises
// it).  At the end the half-1 lane of the row that pivoted column s holds row
// s of W.
//
// Green's function (Eq. full-green-freq): one thread per (fermionic node, k)
// inverts the n_o x n_o matrix (i w + mu) - H(k) - Sigma(k, i w) in registers
// (in-place Gauss-Jordan with partial pivoting).  The chemical potential for
// the target filling comes from a safeguarded Newton iteration on
// N_e(mu) = -2/N_k sum_{k,m} Re rho_m Tr G(k, i w_m), with
// dN_e/dmu = 2/N_k sum Re rho_m Tr G^2 (dG/dmu = -G^2): steps stay inside the
// sign-change bracket once one is known (bisection otherwise) and are capped
// before.  Each evaluation is one launch that writes per-block partial sums;
// a one-block launch sums them in a fixed order and takes the step, so the
// search is deterministic and needs no grid-wide barrier.
#include <cmath>
#include <utility>

#include "qgw_internal.h"
#include "qgw_mfma.h"

namespace qgw {

constexpr int pow2_ceil(int n) {
  int p = 1;
  while (p < n) p *= 2;
  return p;
}

// ---------------------------------------------------------------------------
// W^C = (I - V P)^{-1} V - V
// ---------------------------------------------------------------------------
template <int NB>
struct DysonWShape {
  static constexpr int SEG = pow2_ceil(NB);     // lanes per half
  static constexpr int LPM = 2 * SEG;           // lanes per matrix
  static constexpr int MPW = 64 / LPM;          // matrices per block (one wavefront)
  static constexpr int NN = NB * NB;
  static constexpr int SPLIT = (NB + 1) / 2;    // columns of I - V P formed by each half
};

template <typename T>
__device__ __forceinline__ cpx<T> shfl_cpx(cpx<T> v, int src, int width) {
  return mk(__shfl(v.re, src, width), __shfl(v.im, src, width));
}

// row shift by DPP; a lane whose source lies outside its row gets INT_MIN, the identity of the max it feeds, so the
// shift folds into the max instruction (no copy of the value first)
template <int CTRL>
__device__ __forceinline__ int dpp_shl_i(int v) {
  return __builtin_amdgcn_update_dpp(int(0x80000000u), v, CTRL, 0xF, 0xF, false);
}

// 1 / d by the hardware estimate and Newton-Raphson steps r <- r (2 - d r)
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp_nr(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return __builtin_fmaf(r, __builtin_fmaf(-d, r, 1.0f), r);
}

// |Re| + |Im| rounded to FP32, as bits; a larger value compares larger
template <typename T>
__device__ __forceinline__ int mag_bits(cpx<T> a) {
  return __float_as_int(float(fabs(a.re) + fabs(a.im)));
}

// ADJ: solve (I - V P)^H X = B instead, with B (pair matrix layout, dense) in place of V, and write X
template <int NB, typename T, bool ADJ = false>
__global__ __launch_bounds__(64) void k_dyson_w(const cpx<T>* __restrict__ vq,
                                                const cpx<T>* __restrict__ pnu,
                                                cpx<T>* __restrict__ wc, int64_t nmat, int nk, int64_t ld,
                                                int* __restrict__ cond, const cpx<T>* __restrict__ rhs = nullptr) {
  using S = DysonWShape<NB>;
  static_assert(S::SEG <= 32, "a row index must fit the five low bits of a pivot key");
  __shared__ cpx<T> sp[S::MPW * S::NN];
  __shared__ cpx<T> piv[2][S::MPW][2 * NB];
  const int lane = threadIdx.x;
  const int mw = lane / S::LPM;
  const int half = (lane / S::SEG) & 1;
  const int row = lane % S::SEG;
  const int64_t mat0 = int64_t(blockIdx.x) * S::MPW;
  const int64_t mat = mat0 + mw;
  const bool valid = (mat < nmat) && (row < NB);
  const int q = int(valid ? mat % nk : 0);
  const int64_t nload = (nmat - mat0 < S::MPW ? nmat - mat0 : S::MPW) * S::NN;
  for (int e = lane; e < S::MPW * S::NN; e += 64) sp[e] = e < nload ? pnu[mat0 * S::NN + e] : mk(T(0), T(0));
  __syncthreads();
  const cpx<T>* vrow = vq + (int64_t(q) * NB + (row < NB ? row : 0)) * NB;
  cpx<T>* pm = sp + mw * S::NN;
  // I - V P, formed in place of P: in round g, half h forms columns
  // [8 g + 4 h, 8 g + 4 h + 4) of its row; once every lane has read those
  // columns of P they are overwritten by the columns of I - V P.
  constexpr int CW = 4;
#pragma unroll
  for (int g = 0; g < (NB + 2 * CW - 1) / (2 * CW); ++g) {
    const int c0 = (2 * g + half) * CW;
    cpx<T> acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = mk(T(row == c0 + c ? 1 : 0), T(0));
    if (valid && c0 < NB) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const cpx<T> v = vrow[j];
#pragma unroll
        for (int c = 0; c < CW; ++c) {
          const int col = c0 + c < NB ? c0 + c : NB - 1;
          acc[c] = fms(acc[c], v, pm[j * NB + col]);
        }
      }
    }
    __syncthreads();
    if (valid) {
#pragma unroll
      for (int c = 0; c < CW; ++c)
        if (c0 + c < NB) pm[row * NB + c0 + c] = acc[c];
    }
  }
  __syncthreads();
  cpx<T> x[NB];
  if (valid) {
    if (half == 0) {
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = ADJ ? conj(pm[c * NB + row]) : pm[row * NB + c];
    } else if (ADJ) {
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = rhs[mat * S::NN + row * NB + c];
    } else {
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = vrow[c];
    }
  } else {
#pragma unroll
    for (int c = 0; c < NB; ++c) x[c] = mk(T(0), T(0));
  }
  bool used = false, singular = false;
  int my_step = 0;
  const int partner = lane - half * S::SEG;  // the half-0 lane of this row
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    // the candidates' keys (|Re| + |Im| in FP32 bits, low bits 31 - row: ties go to the lower row) reduced by DPP
    // row shifts over the SEG lanes of half 0 into its first lane (of each 16-lane DPP row), then sent to the
    // matrix's lanes
    int key = (valid && half == 0 && !used) ? ((mag_bits(x[s]) & ~31) | (31 - row)) : int(0x80000000u);
    if constexpr (S::SEG >= 16) key = max(key, dpp_shl_i<0x108>(key));
    if constexpr (S::SEG >= 8) key = max(key, dpp_shl_i<0x104>(key));
    if constexpr (S::SEG >= 4) key = max(key, dpp_shl_i<0x102>(key));
    if constexpr (S::SEG >= 2) key = max(key, dpp_shl_i<0x101>(key));
    if constexpr (S::SEG == 32)  // half 0 spans two DPP rows (one matrix per wave)
      key = max(__builtin_amdgcn_readlane(key, 0), __builtin_amdgcn_readlane(key, 16));
    else
      key = __shfl(key, mw * S::LPM, 64);
    const int idx = 31 - (key & 31);
    const bool is_p = valid && (row == idx);
    if (is_p) {
      if (half == 0) used = true;
      my_step = s;
#pragma unroll
      for (int c = 0; c < NB; ++c) piv[s & 1][mw][half * NB + c] = x[c];
    }
    __syncthreads();
    const cpx<T>* pr = piv[s & 1][mw] + half * NB;
    const cpx<T> pv = piv[s & 1][mw][s];
    const T pn = norm2(pv);
    singular |= !(pn > T(0)) || !isfinite(pn);  // exact zero, NaN or overflow
    const T d = rcp_nr(pn);
    const cpx<T> pinv = mk(pv.re * d, -pv.im * d);
    cpx<T> f = is_p ? mk(T(1), T(0)) - pinv : x[s] * pinv;  // meaningful on half 0
    f = shfl_cpx(f, partner, 64);
    if (valid) {
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = fms(x[c], f, pr[c]);
      if (half == 0) x[s] = mk(T(is_p ? 1 : 0), T(0));
    }
  }
  // a singular or non-finite system of an existing matrix raises the condition bit (the output is non-finite)
  if (singular && mat < nmat && row == 0 && half == 0) atomicOr(cond, kCondSingular);
  // W^C row my_step = (row of W) - (row of V); staged in LDS, stored contiguously
  __syncthreads();
  if (valid && half == 1) {
    const cpx<T>* vr = vq + (int64_t(q) * NB + my_step) * NB;
#pragma unroll
    for (int c = 0; c < NB; ++c) sp[mw * S::NN + my_step * NB + c] = ADJ ? x[c] : x[c] - vr[c];
  }
  __syncthreads();
  for (int e = lane; e < nload; e += 64) {
    const int mi = e / S::NN;
    wc[(mat0 + mi) * ld + (e - mi * S::NN)] = sp[e];
  }
}

// ---------------------------------------------------------------------------
// Register-blocked form of the same solve for N_b = 25 (the five-orbital
// product basis).  One wavefront per (node, q) matrix.  The augmented system
// [I - V P | V] is 25 x 50; its columns are numbered 0..24 for I - V P and
// 25..49 for V (56 with zero padding).  Lane = rg + 8 cg holds
//  * rows rg + 8 s (s < 3, rows 0..23) in columns cg + 8 t (t < 7), and
//  * one entry of row 24, column cg + 8 rg,
// so the last row costs one register pair per lane instead of a mostly empty
// fourth row slot.
//  * V P is formed in that layout: per summation index j a lane reads 3
//    values of V (rows rg + 8 s sit in distinct banks), V(24, j) (one
//    address) and 4 + 1 values of P, and does 13 complex multiply-adds.  P
//    is staged in LDS seven rows at a time, each chunk read into registers
//    while the previous one is used.
//  * Gauss-Jordan step K (a compile-time constant): the lanes holding column
//    K rank their unused rows by |Re| + |Im|, rounded to FP32 and packed with
//    31 - row into one 32-bit key (ties go to the lower row); three DPP
//    shifts inside the 8-lane group and one readlane give the pivot row p.
//    The owners of row p publish it, the owners of column K publish the
//    multipliers (the pivot's own entry less one), and every lane subtracts
//    f_r * (pivot row) with f_r = m_r / a_pK, which normalises the pivot
//    row and clears column K in every other row.
//  * Columns of I - V P left of K are never read again, so a slot whose
//    columns are all <= K drops out of the update.
// LDS holds V (10,000 bytes in FP64) and a 3,072-byte area shared by the P
// chunks and the pivot exchange (two buffers, alternating by step): twelve
// blocks fit a CU.
// ---------------------------------------------------------------------------
struct W25 {
  static constexpr int NB = 25, NS = 3, NT = 7;
  static constexpr int CH = 7;                   // rows of P per staged chunk
  static constexpr int NCH = (NB + CH - 1) / CH;
  static constexpr int ROW = 64;                 // pivot row: 56 columns and 8 zeros
  static constexpr int EX = ROW + 32;            // pivot row and multipliers of one step
  static constexpr int XS = 2 * EX;              // area shared by the P chunks and the pivot exchange
  static constexpr int MIN = int(0x80000000u);
};
static_assert(W25::CH * W25::NB <= W25::XS, "a chunk of P must fit the exchange area");

// The owners of pivot row p = rg + 8 S (S < 3) publish it from the slot
// holding column K on, mark the row as used and record the step; the owner
// of a_pK also stores a_pK - 1 as the pivot row's multiplier.
template <typename T, int K, int S>
__device__ __forceinline__ void gj25_publish(const cpx<T> (&x)[3][7], cpx<T>* xs, int cg, int p, int (&cs)[3],
                                             int (&kof)[3]) {
  constexpr int tk = K / 8;
  xs += (K & 1) * W25::EX;
#pragma unroll
  for (int t = tk; t < W25::NT; ++t) xs[cg + 8 * t] = x[S][t];
  if (cg == K % 8) xs[W25::ROW + p] = mk(x[S][tk].re - T(1), x[S][tk].im);
  cs[S] |= W25::MIN;
  kof[S] = K;
}

// cs[s] = 31 - row for a candidate row, with the sign bit set once the row
// has pivoted, so that a set sign drops it from the max
template <typename T, int K>
__device__ __forceinline__ void gj25_step(cpx<T> (&x)[3][7], cpx<T>& y, int (&cs)[3], int (&kof)[3], int& k24,
                                          int rg, int cg, cpx<T>* xs, bool& singular) {
  constexpr int NS = W25::NS, NT = W25::NT, ROW = W25::ROW, MIN = W25::MIN;
  constexpr int cgk = K % 8, tk = K / 8, t0 = (K + 1) / 8;
  const bool used24 = k24 >= 0;
  int key = (!used24 && rg == tk) ? ((mag_bits(y) & ~31) | (31 - 24)) : MIN;
#pragma unroll
  for (int s = 0; s < NS; ++s) key = max(key, (mag_bits(x[s][tk]) & ~31) | cs[s]);
  key = cg == cgk ? key : MIN;
  key = max(key, dpp_shl_i<0x104>(key));
  key = max(key, dpp_shl_i<0x102>(key));
  key = max(key, dpp_shl_i<0x101>(key));
  const int p = 31 - (__builtin_amdgcn_readlane(key, cgk * 8) & 31);
  const int rgp = p & 7, sp = p >> 3;
  cpx<T>* ex = xs + (K & 1) * W25::EX;  // exchange buffers alternate by step parity
  cpx<T>* mu = ex + ROW;
  if (cg == cgk) {
#pragma unroll
    for (int s = 0; s < NS; ++s) mu[rg + 8 * s] = x[s][tk];
    if (rg == tk) mu[24] = y;
  }
  if (p == 24) {
    if (rg < 7) ex[cg + 8 * rg] = y;
    if (rg == tk && cg == cgk) mu[24] = mk(y.re - T(1), y.im);
    k24 = K;
  } else if (rg == rgp) {
    if (sp == 0)
      gj25_publish<T, K, 0>(x, xs, cg, p, cs, kof);
    else if (sp == 1)
      gj25_publish<T, K, 1>(x, xs, cg, p, cs, kof);
    else
      gj25_publish<T, K, 2>(x, xs, cg, p, cs, kof);
  }
  __syncthreads();
  const cpx<T> pv = ex[K];
  const T pn = norm2(pv);
  singular |= !(pn > T(0)) || !isfinite(pn);  // exact zero, NaN or overflow (the same value in every lane)
  const T d = rcp_nr(pn);
  const cpx<T> pinv = mk(pv.re * d, -pv.im * d);
  cpx<T> f[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) f[s] = mu[rg + 8 * s] * pinv;
  y = fms(y, mu[24] * pinv, ex[cg + 8 * rg]);
#pragma unroll
  for (int t = t0; t < NT; ++t) {
    const cpx<T> pc = ex[cg + 8 * t];
#pragma unroll
    for (int s = 0; s < NS; ++s) x[s][t] = fms(x[s][t], f[s], pc);
  }
}

template <typename T, int... K>
__device__ __forceinline__ void gj25_all(cpx<T> (&x)[3][7], cpx<T>& y, int (&cs)[3], int (&kof)[3], int& k24, int rg,
                                         int cg, cpx<T>* xs, bool& singular, std::integer_sequence<int, K...>) {
  (gj25_step<T, K>(x, y, cs, kof, k24, rg, cg, xs, singular), ...);
}

// ADJ: solve (I - V P)^H X = B instead (A is formed as below, passed through the V area of LDS, which ADJ no
// longer needs, and read back conjugate-transposed), with B (pair matrix layout, dense) in place of V; writes X
// MVP: V P on the matrix cores (16x16x4, 2 x 2 tiles over the 25 x 25 product, 7 slices of 4 along the
// contraction; rows, columns and slices past 25 are zero), V from LDS as the A operand and P straight from memory
// as the B operand; I - V P then passes through the V area of LDS into the elimination layout, and the final
// W - V reads V(q) from memory again.  The matrix cores run beside the VALU elimination of the other waves of
// the SIMD and the product no longer streams V and P through LDS, but on gfx950 the FP64 matrix rate equals the
// VALU rate and the 32 x 32 x 28 padding costs 1.8x the product's flops: measured at 24 x 24, r = 53 it takes
// 0.46 ms (FP64) and 0.27 ms (FP32) against 0.42 and 0.25 for the VALU product, so it is an autotuner
// alternative and not the default.
// FP32 asks for five waves per SIMD: its elimination fits 96 VGPRs without spills (97 by default, four waves)
template <typename T, bool ADJ = false, bool MVP = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1))) void k_dyson_w25(const cpx<T>* __restrict__ vq, const cpx<T>* __restrict__ pnu,
                                                  cpx<T>* __restrict__ wc, int64_t nmat, int nk, int64_t ld,
                                                  int* __restrict__ cond, const cpx<T>* __restrict__ rhs = nullptr) {
  constexpr int NB = W25::NB, NN = NB * NB, NS = W25::NS, NT = W25::NT, CH = W25::CH, NCH = W25::NCH;
  __shared__ cpx<T> xs[W25::XS];  // a chunk of P rows; then the pivot exchange
  __shared__ cpx<T> sv[NN];       // V(q)
  const int lane = threadIdx.x;
  const int rg = lane & 7, cg = lane >> 3;
  const int c24 = cg + 8 * rg;  // this lane's column of row 24
  const int64_t mat = blockIdx.x;
  const int q = int(mat % nk);
  const cpx<T>* vm = vq + int64_t(q) * NN;
  const cpx<T>* pm = pnu + mat * NN;
  // chunk c of P (rows CH c ..) is read into registers one chunk ahead; a
  // chunk has at most 175 entries, three per lane
  static_assert(CH * NB <= 3 * 64, "a chunk of P must fit three entries per lane");
  cpx<T> x[NS][NT], y;
  if constexpr (MVP) {
    using M = Mfma<T>;
    using v4 = typename M::v4;
    const int l16 = lane & 15, l4 = lane >> 4;
    for (int e = lane; e < NN; e += 64) sv[e] = vm[e];
    // B operand of slice ks, column tile ct: P[4 ks + l4][16 ct + l16]
    auto ldp = [&](int ks, int ct) -> cpx<T> {
      const int k = 4 * ks + l4, n = 16 * ct + l16;
      return (k < NB && n < NB) ? pm[k * NB + n] : mk(T(0), T(0));
    };
    v4 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cr[a][b] = v4{T(0), T(0), T(0), T(0)};
        ci[a][b] = v4{T(0), T(0), T(0), T(0)};
      }
    cpx<T> b0 = ldp(0, 0), b1 = ldp(0, 1);
    __syncthreads();  // V(q) is in LDS
#pragma unroll 1
    for (int ks = 0; ks < 7; ++ks) {
      const cpx<T> pb[2] = {b0, b1};
      if (ks + 1 < 7) {
        b0 = ldp(ks + 1, 0);
        b1 = ldp(ks + 1, 1);
      }
      const int k = 4 * ks + l4;
      cpx<T> a[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int m = 16 * rt + l16;
        a[rt] = (k < NB && m < NB) ? sv[m * NB + k] : mk(T(0), T(0));
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          cr[rt][ct] = M::mac(a[rt].re, pb[ct].re, cr[rt][ct]);
          ci[rt][ct] = M::mac(a[rt].re, pb[ct].im, ci[rt][ct]);
        }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          cr[rt][ct] = M::mac(-a[rt].im, pb[ct].im, cr[rt][ct]);
          ci[rt][ct] = M::mac(a[rt].im, pb[ct].re, ci[rt][ct]);
        }
    }
    __syncthreads();  // every lane has finished reading V: its area takes A = I - V P
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * rt + M::row(lane, v), col = 16 * ct + l16;
          if (row < NB && col < NB)
            sv[row * NB + col] = mk(T(row == col ? 1 : 0) - cr[rt][ct][v], -ci[rt][ct][v]);
        }
    __syncthreads();
    // A (ADJ: A^H) from LDS and the right-hand side (V, or Wbar for ADJ) from memory into the elimination layout
    const cpx<T>* bm = ADJ ? rhs + mat * NN : vm;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int row = rg + 8 * s;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = cg + 8 * t;
        cpx<T> val = mk(T(0), T(0));
        if (t < 4 && c < NB)
          val = ADJ ? conj(sv[c * NB + row]) : sv[row * NB + c];
        else if (c >= NB && c < 2 * NB)
          val = bm[row * NB + c - NB];
        x[s][t] = val;
      }
    }
    y = mk(T(0), T(0));
    if (c24 < NB)
      y = ADJ ? conj(sv[c24 * NB + 24]) : sv[24 * NB + c24];
    else if (c24 < 2 * NB)
      y = bm[24 * NB + c24 - NB];
  } else {
  cpx<T> pre0 = mk(T(0), T(0)), pre1 = pre0, pre2 = pre0;
  auto load_chunk = [&](int c) {
    const int n = min(CH, NB - CH * c) * NB;
    const cpx<T>* src = pm + CH * c * NB;
    if (lane < n) pre0 = src[lane];
    if (lane + 64 < n) pre1 = src[lane + 64];
    if (lane + 128 < n) pre2 = src[lane + 128];
  };
  load_chunk(0);
  for (int e = lane; e < NN; e += 64) sv[e] = vm[e];
  {
    // V P on the columns of I - V P: slots t < 3, t = 3 where cg = 0 (column
    // 24), and row 24 at column c24 < 25
    cpx<T> acc[NS][4], a24 = mk(T(0), T(0));
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[s][t] = mk(T(0), T(0));
    const int j24 = min(c24, NB - 1);
#pragma unroll 1
    for (int c = 0; c < NCH; ++c) {
      const int rows = min(CH, NB - CH * c);
      __syncthreads();  // the previous chunk has been read
      if (lane < rows * NB) xs[lane] = pre0;
      if (lane + 64 < rows * NB) xs[lane + 64] = pre1;
      if (lane + 128 < rows * NB) xs[lane + 128] = pre2;
      if (c + 1 < NCH) load_chunk(c + 1);
      __syncthreads();
#pragma unroll
      for (int jj = 0; jj < CH; ++jj) {
        if (jj < rows) {
          const int j = CH * c + jj;
          cpx<T> v[NS], pj[4];
#pragma unroll
          for (int s = 0; s < NS; ++s) v[s] = sv[(rg + 8 * s) * NB + j];
#pragma unroll
          for (int t = 0; t < 4; ++t) pj[t] = xs[jj * NB + min(cg + 8 * t, NB - 1)];
#pragma unroll
          for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[s][t] = fma(acc[s][t], v[s], pj[t]);
          a24 = fma(a24, sv[24 * NB + j], xs[jj * NB + j24]);
        }
      }
    }
    if (ADJ) {
      // A = I - V P through the V area (every lane has finished reading V), then back as A^H
      __syncthreads();
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int row = rg + 8 * s, c = cg + 8 * t;
          if (c < NB) sv[row * NB + c] = mk(T(row == c ? 1 : 0) - acc[s][t].re, -acc[s][t].im);
        }
      if (c24 < NB) sv[24 * NB + c24] = mk(T(c24 == 24 ? 1 : 0) - a24.re, -a24.im);
      __syncthreads();
    }
    const cpx<T>* bm = ADJ ? rhs + mat * NN : nullptr;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int row = rg + 8 * s;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = cg + 8 * t;
        cpx<T> val = mk(T(0), T(0));
        if (t < 4 && c < NB)
          val = ADJ ? conj(sv[c * NB + row]) : mk(T(row == c ? 1 : 0) - acc[s][t < 4 ? t : 0].re,
                                                   -acc[s][t < 4 ? t : 0].im);
        else if (c >= NB && c < 2 * NB)
          val = ADJ ? bm[row * NB + c - NB] : sv[row * NB + c - NB];
        x[s][t] = val;
      }
    }
    y = mk(T(0), T(0));
    if (c24 < NB)
      y = ADJ ? conj(sv[c24 * NB + 24]) : mk(T(c24 == 24 ? 1 : 0) - a24.re, -a24.im);
    else if (c24 < 2 * NB)
      y = ADJ ? bm[24 * NB + c24 - NB] : sv[24 * NB + c24 - NB];
  }
  }
  __syncthreads();  // the last chunk has been read: its area takes the pivot exchange
  if (lane < 16) xs[(lane >> 3) * W25::EX + 56 + (lane & 7)] = mk(T(0), T(0));  // pivot-row padding columns
  int cs[NS], kof[NS], k24 = -1;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    cs[s] = 31 - (rg + 8 * s);
    kof[s] = 0;
  }
  bool singular = false;
  gj25_all<T>(x, y, cs, kof, k24, rg, cg, xs, singular, std::make_integer_sequence<int, NB>{});
  if (singular && lane == 0) atomicOr(cond, kCondSingular);
  // row r of the V part is row kof of W; W^C = W - V (ADJ: row kof of X)
  cpx<T>* wm = wc + mat * ld;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int k = kof[s];
#pragma unroll
    for (int t = 3; t < NT; ++t) {
      const int col = cg + 8 * t - NB;
      if (col >= 0 && col < NB) wm[k * NB + col] = ADJ ? x[s][t] : x[s][t] - (MVP ? vm : sv)[k * NB + col];
    }
  }
  if (c24 >= NB && c24 < 2 * NB) wm[k24 * NB + c24 - NB] = ADJ ? y : y - (MVP ? vm : sv)[k24 * NB + c24 - NB];
}

// ---------------------------------------------------------------------------
// Register-blocked form for 8 < N_b <= 16 (three orbitals, four orbitals): one wavefront per (node, q) matrix,
// the layout and elimination of the N_b = 25 kernel without its spread last row.  Lane = rg + 8 cg holds rows
// rg + 8 s (s < 2) in columns cg + 8 t (t < NT) of [I - V P | V] (columns 0..N_b-1, then N_b..2 N_b-1; rows and
// columns past them are zero).  V(q) and P are staged in LDS; V P is formed in that layout; step K searches column
// K by packed keys in the 8-lane group holding it, the owners of the pivot row and of column K publish them through
// LDS, and every lane subtracts f_r * (pivot row).  Slots whose columns are all in I - V P and left of K drop out of
// the update at compile time.  With ADJ it solves the conjugate-transposed system of the adjoint.
// ---------------------------------------------------------------------------
template <int NB>
struct WR {
  static_assert(NB > 8 && NB <= 16, "two row slots of eight");
  static constexpr int NS = 2, NT = (2 * NB + 7) / 8, NN = NB * NB;
  static constexpr int ROW = 8 * NT;      // pivot row (all column slots)
  static constexpr int EX = ROW + 16;     // pivot row and the multipliers of one step
  static constexpr int TA = (NB + 7) / 8;  // slots holding columns of I - V P
  static_assert(2 * EX <= NN, "the exchange area reuses the P area");
};

template <typename T, int NB, int K, int S>
__device__ __forceinline__ void wr_publish(const cpx<T> (&x)[2][WR<NB>::NT], cpx<T>* ex, int cg, int p, int (&cs)[2],
                                           int (&kof)[2]) {
  constexpr int tk = K / 8;
#pragma unroll
  for (int t = tk; t < WR<NB>::NT; ++t) ex[cg + 8 * t] = x[S][t];
  if (cg == K % 8) ex[WR<NB>::ROW + p] = mk(x[S][tk].re - T(1), x[S][tk].im);
  cs[S] |= int(0x80000000u);
  kof[S] = K;
}

template <typename T, int NB, int K>
__device__ __forceinline__ void wr_step(cpx<T> (&x)[2][WR<NB>::NT], int (&cs)[2], int (&kof)[2], int rg, int cg,
                                        cpx<T>* xs, bool& singular) {
  constexpr int NT = WR<NB>::NT, ROW = WR<NB>::ROW, MIN = int(0x80000000u);
  constexpr int cgk = K % 8, tk = K / 8;
  constexpr int t0 = (K + 1) / 8 < NB / 8 ? (K + 1) / 8 : NB / 8;  // slots left of t0 hold dead columns only
  int key = MIN;
#pragma unroll
  for (int s = 0; s < 2; ++s) key = max(key, (mag_bits(x[s][tk]) & ~31) | cs[s]);
  key = cg == cgk ? key : MIN;
  key = max(key, dpp_shl_i<0x104>(key));
  key = max(key, dpp_shl_i<0x102>(key));
  key = max(key, dpp_shl_i<0x101>(key));
  const int p = 31 - (__builtin_amdgcn_readlane(key, cgk * 8) & 31);
  cpx<T>* ex = xs + (K & 1) * WR<NB>::EX;  // exchange buffers alternate by step parity
  cpx<T>* mu = ex + ROW;
  if (cg == cgk) {
#pragma unroll
    for (int s = 0; s < 2; ++s) mu[rg + 8 * s] = x[s][tk];
  }
  if (rg == (p & 7)) {
    if ((p >> 3) == 0)
      wr_publish<T, NB, K, 0>(x, ex, cg, p, cs, kof);
    else
      wr_publish<T, NB, K, 1>(x, ex, cg, p, cs, kof);
  }
  __syncthreads();
  const cpx<T> pv = ex[K];
  const T pn = norm2(pv);
  singular |= !(pn > T(0)) || !isfinite(pn);  // exact zero, NaN or overflow (the same value in every lane)
  const T d = rcp_nr(pn);
  const cpx<T> pinv = mk(pv.re * d, -pv.im * d);
  cpx<T> f[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) f[s] = mu[rg + 8 * s] * pinv;
#pragma unroll
  for (int t = t0; t < NT; ++t) {
    const cpx<T> pc = ex[cg + 8 * t];
#pragma unroll
    for (int s = 0; s < 2; ++s) x[s][t] = fms(x[s][t], f[s], pc);
  }
}

template <typename T, int NB, int... K>
__device__ __forceinline__ void wr_all(cpx<T> (&x)[2][WR<NB>::NT], int (&cs)[2], int (&kof)[2], int rg, int cg,
                                       cpx<T>* xs, bool& singular, std::integer_sequence<int, K...>) {
  (wr_step<T, NB, K>(x, cs, kof, rg, cg, xs, singular), ...);
}

// ADJ: solve (I - V P)^H X = B instead, with B (pair matrix layout, dense) in place of V, and write X; A = I - V P
// passes through the P area of LDS and is read back conjugate-transposed
template <typename T, int NB, bool ADJ = false>
__global__ __launch_bounds__(64) void k_dyson_wr(const cpx<T>* __restrict__ vq, const cpx<T>* __restrict__ pnu,
                                                 cpx<T>* __restrict__ wc, int64_t nmat, int nk, int64_t ld,
                                                 int* __restrict__ cond, const cpx<T>* __restrict__ rhs = nullptr) {
  using S = WR<NB>;
  constexpr int NT = S::NT, NN = S::NN, TA = S::TA;
  __shared__ cpx<T> sv[NN];  // V(q)
  __shared__ cpx<T> sp[NN];  // P; then the pivot exchange
  const int lane = threadIdx.x;
  const int rg = lane & 7, cg = lane >> 3;
  const int64_t mat = blockIdx.x;
  const int q = int(mat % nk);
  const cpx<T>* vm = vq + int64_t(q) * NN;
  const cpx<T>* pm = pnu + mat * NN;
  for (int e = lane; e < NN; e += 64) {
    sv[e] = vm[e];
    sp[e] = pm[e];
  }
  __syncthreads();
  // I - V P in the columns of slots t < TA, V in the right-hand-side columns
  cpx<T> acc[2][TA];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < TA; ++t) acc[s][t] = mk(T(0), T(0));
  const int r1 = min(rg + 8, NB - 1);  // row of slot 1 (clamped: rows past N_b are not kept)
#pragma unroll 4
  for (int j = 0; j < NB; ++j) {
    const cpx<T> v0 = sv[rg * NB + j], v1 = sv[r1 * NB + j];
#pragma unroll
    for (int t = 0; t < TA; ++t) {
      const cpx<T> pj = sp[j * NB + min(cg + 8 * t, NB - 1)];
      acc[0][t] = fma(acc[0][t], v0, pj);
      acc[1][t] = fma(acc[1][t], v1, pj);
    }
  }
  if constexpr (ADJ) {
    __syncthreads();  // every lane has read P: its area takes A = I - V P
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < TA; ++t) {
        const int row = rg + 8 * s, c = cg + 8 * t;
        if (row < NB && c < NB) sp[row * NB + c] = mk(T(row == c ? 1 : 0) - acc[s][t].re, -acc[s][t].im);
      }
    __syncthreads();
  }
  const cpx<T>* bm = ADJ ? rhs + mat * NN : nullptr;
  cpx<T> x[2][NT];
  int cs[2], kof[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int row = rg + 8 * s;
    const bool rv = row < NB;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = cg + 8 * t;
      cpx<T> val = mk(T(0), T(0));
      if (rv && c < NB)
        val = ADJ ? conj(sp[c * NB + row])
                  : mk(T(row == c ? 1 : 0) - acc[s][t < TA ? t : 0].re, -acc[s][t < TA ? t : 0].im);
      else if (rv && c < 2 * NB)
        val = ADJ ? bm[row * NB + c - NB] : sv[row * NB + c - NB];
      x[s][t] = val;
    }
    cs[s] = rv ? 31 - row : int(0x80000000u);  // rows past N_b never pivot
    kof[s] = 0;
  }
  __syncthreads();  // every lane has read P (ADJ: A): its area takes the pivot exchange
  bool singular = false;
  wr_all<T, NB>(x, cs, kof, rg, cg, sp, singular, std::make_integer_sequence<int, NB>{});
  if (singular && lane == 0) atomicOr(cond, kCondSingular);
  // row r of the right-hand side is row kof of the solution; W^C = W - V (ADJ: X)
  cpx<T>* wm = wc + mat * ld;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int k = kof[s];
    if (rg + 8 * s < NB) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int col = cg + 8 * t - NB;
        if (col >= 0 && col < NB) wm[k * NB + col] = ADJ ? x[s][t] : x[s][t] - sv[k * NB + col];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// n_o x n_o inverse in registers, Gauss-Jordan with partial pivoting
// ---------------------------------------------------------------------------
template <int NO>
__device__ __forceinline__ void invert_inplace(cpx<double> (&a)[NO][NO]) {
  int perm[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    int p = k;
    double best = norm2(a[k][k]);
#pragma unroll
    for (int i = k + 1; i < NO; ++i) {
      const double v = norm2(a[i][k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    perm[k] = p;
    // row swap k <-> p as exact 0/1-weighted blends (w x + (1 - w) y is exact
    // for w in {0, 1}); keeps the matrix in registers, unlike a select chain
#pragma unroll
    for (int i = k + 1; i < NO; ++i) {
      const double w = (p == i) ? 1.0 : 0.0, v = 1.0 - w;
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        const cpx<double> t = a[k][j], u = a[i][j];
        a[k][j] = mk(w * u.re + v * t.re, w * u.im + v * t.im);
        a[i][j] = mk(w * t.re + v * u.re, w * t.im + v * u.im);
      }
    }
    const cpx<double> pinv = inv(a[k][k]);
    a[k][k] = mk(1.0, 0.0);
#pragma unroll
    for (int j = 0; j < NO; ++j) a[k][j] = a[k][j] * pinv;
#pragma unroll
    for (int i = 0; i < NO; ++i) {
      if (i == k) continue;
      const cpx<double> f = a[i][k];
      a[i][k] = mk(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < NO; ++j) a[i][j] = fms(a[i][j], f, a[k][j]);
    }
  }
#pragma unroll
  for (int k = NO - 1; k >= 0; --k) {
#pragma unroll
    for (int c = k + 1; c < NO; ++c) {
      const double w = (perm[k] == c) ? 1.0 : 0.0, v = 1.0 - w;
#pragma unroll
      for (int i = 0; i < NO; ++i) {
        const cpx<double> t = a[i][k], u = a[i][c];
        a[i][k] = mk(w * u.re + v * t.re, w * u.im + v * t.im);
        a[i][c] = mk(w * t.re + v * u.re, w * t.im + v * u.im);
      }
    }
  }
}

struct DysonGArgs {
  const zd* hk;       // [no][no][nk]
  const zd* sig;      // [r][no][no][nk] or null
  const double* wn;   // [r]
  const zd* rho;      // [r]: G(beta^-) = sum_m rho_m G(i w_m)
  zd* g;              // [r][no][no][nk]
  double* scal;       // [0] mu (in: start / fixed; out), [1] n_target, [2] evaluations, [3] final N_e,
                      // [8] status (copy), [9] the value at ``extra`` (copy), so one read returns all
  double* partials;   // [2][4][max blocks]
  int* status;        // 0 ok, 2 not converged
  const double* extra;  // optional scalar copied to scal[9] by the final pass
  int* fail_word;       // optional: raised to the search's failing status by the final pass, never lowered here
  int r, nk, mode, max_evals;
  double beta, tol_mu, tol_n;
  double ne_offset;   // added to -(2/N_k) sum Re rho_m Tr G_m (the uniform grid's 1/2 per spin-orbital)
};

template <int NO>
__device__ __forceinline__ void load_base(const DysonGArgs& A, int64_t gi, cpx<double> (&bm)[NO][NO]) {
  const int m = int(gi / A.nk), k = int(gi - int64_t(m) * A.nk);
  const double w = A.wn[m];
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const zd h = A.hk[(int64_t(i) * NO + j) * A.nk + k];
      cpx<double> v = mk(-h.re, -h.im);
      if (A.sig) {
        const zd sg = A.sig[((int64_t(m) * NO + i) * NO + j) * A.nk + k];
        v = v - sg;
      }
      if (i == j) v.im += w;
      bm[i][j] = v;
    }
}

// block-level deterministic reductions (one wavefront per block); the xor
// butterfly leaves the same value in every lane
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// ---------------------------------------------------------------------------
// The search as a chain of launches.  Its state lives in the scalar block:
//   [0] mu  [1] n_target  [2] evaluations  [3] last N_e  [4] lo  [5] hi
//   [6] step cap  [7] done flag
// Each k_dg_eval launch first takes the Newton step of the previous
// evaluation (every block takes the same step from the same partial sums),
// then evaluates; the final pass takes the last step.  Once the search has
// converged the remaining launches return at once, so a caller may queue a
// fixed number of steps (graph capture) or queue a few, read the done flag
// and continue.
// ---------------------------------------------------------------------------

// per-block partials of H(k): Gershgorin bounds (used when no starting point is given) and the sum of the
// diagonal (the mean level, whose change between two searches of a state shifts the start)
template <int NO>
__global__ __launch_bounds__(64) void k_dg_gersh(DysonGArgs A) {
  double glo = 1e300, ghi = -1e300, dsum = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 64 + threadIdx.x; k < A.nk; k += int64_t(gridDim.x) * 64) {
#pragma unroll
    for (int i = 0; i < NO; ++i) {
      double rad = 0.0;
#pragma unroll
      for (int j = 0; j < NO; ++j)
        if (j != i) rad += sqrt(norm2(A.hk[(int64_t(i) * NO + j) * A.nk + k]));
      const double d = A.hk[(int64_t(i) * NO + i) * A.nk + k].re;
      glo = fmin(glo, d - rad);
      ghi = fmax(ghi, d + rad);
      dsum += d;
    }
  }
  glo = wave_min(glo);
  ghi = wave_max(ghi);
  dsum = wave_sum(dsum);
  if (threadIdx.x == 0) {
    A.partials[blockIdx.x] = glo;
    A.partials[gridDim.x + blockIdx.x] = ghi;
    A.partials[2 * gridDim.x + blockIdx.x] = dsum;
  }
}

// mu <- centre of the Gershgorin bounds if no finite start was given; otherwise, with ``track``, the start moves
// by the change of the mean diagonal of H since the previous search (scal[10]), the shift of a level by a change
// of Sigma_HF (so that a Hartree shift of many eV does not cost a chain of capped steps); resets the search
// set: the start point (mu0, n_target) comes as arguments instead of a copy into scal[0..1]
// diag_only: partials holds only nblk diagonal sums (a14's), no Gershgorin bounds
// bmax (optional): a14's nbmax block maxima of |Delta Sigma| (non-finite ones already +inf); their maximum goes to
// *dsig, so that a14 needs no reduction launch of its own (the maximum is exact, so the order does not matter)
__global__ __launch_bounds__(64) void k_dg_begin(double* __restrict__ scal, int* __restrict__ status,
                                                 const double* __restrict__ partials, int nblk, double inv_count,
                                                 int track, int set, double mu0, double nt, int diag_only,
                                                 const double* __restrict__ bmax, int nbmax,
                                                 double* __restrict__ dsig) {
  if (bmax) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nbmax; b += 64) v = fmax(v, bmax[b]);
    v = wave_max(v);
    if (threadIdx.x == 0) *dsig = v;
  }
  double glo = 1e300, ghi = -1e300, dsum = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) {
    if (diag_only) {
      dsum += partials[b];
    } else {
      glo = fmin(glo, partials[b]);
      ghi = fmax(ghi, partials[nblk + b]);
      dsum += partials[2 * nblk + b];
    }
  }
  if (diag_only) glo = ghi = NAN;  // no bounds: a start that is not finite stays so (status 1)
  glo = wave_min(glo);
  ghi = wave_max(ghi);
  const double mean = wave_sum(dsum) * inv_count;
  if (threadIdx.x != 0) return;
  if (set) {
    scal[0] = mu0;
    scal[1] = nt;
  }
  if (!isfinite(scal[0])) {
    scal[0] = 0.5 * (glo + ghi);
  } else if (track && isfinite(scal[10]) && isfinite(mean)) {
    scal[0] += mean - scal[10];
  }
  scal[10] = mean;
  const bool ok = isfinite(scal[0]);
  scal[2] = 0.0;
  scal[3] = 0.0;
  scal[4] = -INFINITY;
  scal[5] = INFINITY;
  scal[6] = 1.0;
  scal[7] = ok ? 0.0 : 1.0;
  status[0] = ok ? 0 : 1;
}

// The search state after j Newton steps: mu, n_target, steps taken, N_e at the last evaluation, bracket lo / hi,
// step cap, done.  The host-visible words scal[0..7] hold it between rounds; inside a round the state after step
// j sits in slot j % 2 (scal[16 + 8 (j % 2) ..]) and the partial sums of evaluation j in half j % 2 of the
// partials, so that a launch reads the previous launch's slot and half while its block 0 writes the other ones.
constexpr int kDgSlot = 16;

// one Newton step of the search from the summed partials (s: sum of rho Tr G, sd: of rho Tr G^2)
__device__ __forceinline__ void dg_newton_update(const DysonGArgs& A, double s, double sd, double (&st)[8]) {
  const double ne = -2.0 * s / double(A.nk) + A.ne_offset, dne = 2.0 * sd / double(A.nk);
  double mu = st[0], lo = st[4], hi = st[5], cap = st[6];
  const double nt = st[1];
  const double f = ne - nt;
  st[2] += 1.0;
  st[3] = ne;
  if (f < 0.0) lo = fmax(lo, mu);
  if (f > 0.0) hi = fmin(hi, mu);
  bool done = false;
  if (fabs(f) <= A.tol_n) {
    done = true;
  } else {
    double nxt = (dne > 0.0) ? mu - f / dne : NAN;
    const bool bracket = isfinite(lo) && isfinite(hi);
    if (bracket) {
      if (!(nxt > lo && nxt < hi)) nxt = 0.5 * (lo + hi);
    } else {
      if (!isfinite(nxt)) nxt = mu + (f < 0.0 ? cap : -cap);
      if (fabs(nxt - mu) > cap) {
        nxt = mu + (nxt > mu ? cap : -cap);
        cap *= 4.0;
      }
    }
    const double tol = A.tol_mu * fmax(1.0, fabs(mu));
    if (fabs(nxt - mu) <= tol || (bracket && hi - lo <= tol)) done = true;
    mu = nxt;
  }
  st[0] = mu;
  st[4] = lo;
  st[5] = hi;
  st[6] = cap;
  st[7] = done ? 1.0 : 0.0;
}

// the state after j steps of this round: step j (j >= 1) is taken from the state after j - 1 steps and the
// partial sums of evaluation j - 1.  Every lane of every block sums the partials in the same order (the
// butterfly reduction leaves the same bits in every lane), so all take the same step.
__device__ __forceinline__ void dg_state(const DysonGArgs& A, int j, int nblk, double (&st)[8]) {
  const double* src = (j == 0) ? A.scal : A.scal + kDgSlot + 8 * ((j - 1) & 1);
#pragma unroll
  for (int i = 0; i < 8; ++i) st[i] = src[i];
  if (j >= 1 && st[7] == 0.0) {
    const double* part = A.partials + int64_t(2) * nblk * ((j - 1) & 1);
    double s = 0.0, sd = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) {
      s += part[b];
      sd += part[nblk + b];
    }
    s = wave_sum(s);
    sd = wave_sum(sd);
    dg_newton_update(A, s, sd, st);
  }
}

// evaluation j of a round: N_e(mu) and dN_e/dmu at the state after j steps, as per-block partial sums
template <int NO>
__global__ __launch_bounds__(64) void k_dg_eval(DysonGArgs A, int j, int nblk) {
  double st[8];
  dg_state(A, j, nblk, st);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* dst = A.scal + kDgSlot + 8 * (j & 1);
#pragma unroll
    for (int i = 0; i < 8; ++i) dst[i] = st[i];
  }
  if (st[7] != 0.0) return;
  const double mu = st[0];
  const int64_t total = int64_t(A.r) * A.nk;
  const int64_t stride = int64_t(gridDim.x) * 64;
  double acc = 0.0, accd = 0.0;
  for (int64_t gi = int64_t(blockIdx.x) * 64 + threadIdx.x; gi < total; gi += stride) {
    cpx<double> a[NO][NO];
    load_base<NO>(A, gi, a);
#pragma unroll
    for (int i = 0; i < NO; ++i) a[i][i].re += mu;
    invert_inplace<NO>(a);
    cpx<double> tr = mk(0.0, 0.0), tr2 = mk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < NO; ++i) {
      tr = tr + a[i][i];
#pragma unroll
      for (int jj = 0; jj < NO; ++jj) tr2 = fma(tr2, a[i][jj], a[jj][i]);
    }
    const zd rh = A.rho[int(gi / A.nk)];
    acc += rh.re * tr.re - rh.im * tr.im;
    accd += rh.re * tr2.re - rh.im * tr2.im;
  }
  acc = wave_sum(acc);
  accd = wave_sum(accd);
  if (threadIdx.x == 0) {
    double* part = A.partials + int64_t(2) * nblk * (j & 1);
    part[blockIdx.x] = acc;
    part[nblk + blockIdx.x] = accd;
  }
}

// G at the search's result: with n >= 1 evaluations in this round the last step (from evaluation n - 1) is
// taken here, and block 0 writes the state back to the host-visible words
template <int NO>
__global__ __launch_bounds__(64) void k_dg_final(DysonGArgs A, int n, int nblk) {
  double st[8];
  if (A.mode == 1 && n >= 1) {
    dg_state(A, n, nblk, st);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) st[i] = A.scal[i];
  }
  const double mu = st[0];
  const int64_t total = int64_t(A.r) * A.nk;
  const int64_t stride = int64_t(gridDim.x) * 64;
  for (int64_t gi = int64_t(blockIdx.x) * 64 + threadIdx.x; gi < total; gi += stride) {
    cpx<double> a[NO][NO];
    load_base<NO>(A, gi, a);
#pragma unroll
    for (int i = 0; i < NO; ++i) a[i][i].re += mu;
    invert_inplace<NO>(a);
    const int m = int(gi / A.nk), k = int(gi - int64_t(m) * A.nk);
#pragma unroll
    for (int i = 0; i < NO; ++i)
#pragma unroll
      for (int j = 0; j < NO; ++j) A.g[((int64_t(m) * NO + i) * NO + j) * A.nk + k] = a[i][j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (A.mode == 1 && n >= 1) {
#pragma unroll
      for (int i = 0; i < 8; ++i) A.scal[i] = st[i];
    }
    if (A.mode == 1 && A.status[0] == 0) {
      const bool conv = st[7] != 0.0 || fabs(st[3] - st[1]) <= A.tol_n;
      if (!conv || !isfinite(mu)) A.status[0] = 2;
    }
    if (A.fail_word && A.status[0] > *A.fail_word) *A.fail_word = A.status[0];
    A.scal[8] = double(A.status[0]);
    if (A.extra) A.scal[9] = *A.extra;
  }
}

// ---------------------------------------------------------------------------
// adjoint of Dyson W (FP64).  With A = I - V P and W = A^{-1} V,
// dW = A^{-1} dV (I + P W) + W dP W.  For a cotangent Wbar of W^C = W - V:
//   X = A^{-H} Wbar,  Y = X W^H,  Pbar = W^H Wbar W^H = V^H Y,
//   Vbar = A^{-H} Wbar (I + P W)^H - Wbar = X + Y P^H - Wbar.
// W^C and X come from the register Gauss-Jordan kernels above (the forward
// solve, and its ADJ form on A^H with Wbar as the right-hand side); this
// kernel forms the products.  Block (q, chunk of nodes), 256 threads: thread
// (i, g) owns row i and the columns g, g + G, g + 2G of every product, so
// each LDS value it loads serves three multiply-adds.  V(q) is static, so
// Vbar(q) sums over the nodes: each block sums its chunk in a fixed order and
// writes a partial.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(256) void k_dyson_w_bwd_prod(const zd* __restrict__ vq, const zd* __restrict__ pnu,
                                                          const zd* __restrict__ wbar, const zd* __restrict__ wcm,
                                                          const zd* __restrict__ xm, zd* __restrict__ pbar,
                                                          zd* __restrict__ vpart, int r, int nk, int chunks) {
  constexpr int NN = NB * NB;
  constexpr int CPT = 3;                        // columns per thread
  constexpr int G = (NB + CPT - 1) / CPT;       // column groups
  static_assert(NB * G <= 256, "one thread per (row, column group)");
  __shared__ cpx<double> sV[NN], sP[NN], sX[NN], sW[NN], sY[NN];
  const int q = blockIdx.x, ch = blockIdx.y, tid = threadIdx.x;
  const int m0 = int(int64_t(r) * ch / chunks), m1 = int(int64_t(r) * (ch + 1) / chunks);
  const bool own = tid < NB * G;
  const int i = own ? tid / G : 0, g = tid - (tid / G) * G;
  for (int e = tid; e < NN; e += 256) sV[e] = vq[int64_t(q) * NN + e];
  cpx<double> vacc[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) vacc[c] = mk(0.0, 0.0);
  for (int m = m0; m < m1; ++m) {
    const int64_t base = (int64_t(m) * nk + q) * NN;
    __syncthreads();  // the previous node's products are done with the LDS tiles
    for (int e = tid; e < NN; e += 256) {
      sP[e] = pnu[base + e];
      sX[e] = xm[base + e];
      sW[e] = wcm[base + e] + sV[e];  // W = W^C + V
    }
    __syncthreads();
    // Y = X W^H
    if (own) {
      cpx<double> y[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) y[c] = mk(0.0, 0.0);
      // one k per step: an unrolled loop hoists the operand loads and runs out of registers
#pragma unroll 1
      for (int k = 0; k < NB; ++k) {
        const cpx<double> a = sX[i * NB + k];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const int j = g + c * G;
          if (j < NB) y[c] = fma(y[c], a, conj(sW[j * NB + k]));
        }
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int j = g + c * G;
        if (j < NB) sY[i * NB + j] = y[c];
      }
    }
    __syncthreads();
    // Pbar = V^H Y;  Vbar += X + Y P^H - Wbar
    if (own) {
      cpx<double> pb[CPT], vy[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) pb[c] = vy[c] = mk(0.0, 0.0);
#pragma unroll 1
      for (int k = 0; k < NB; ++k) {
        const cpx<double> vki = conj(sV[k * NB + i]), yik = sY[i * NB + k];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const int j = g + c * G;
          if (j < NB) {
            pb[c] = fma(pb[c], vki, sY[k * NB + j]);
            vy[c] = fma(vy[c], yik, conj(sP[j * NB + k]));
          }
        }
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int j = g + c * G;
        if (j < NB) {
          pbar[base + i * NB + j] = pb[c];
          vacc[c] = vacc[c] + (sX[i * NB + j] - wbar[base + i * NB + j]) + vy[c];
        }
      }
    }
  }
  if (own) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int j = g + c * G;
      if (j < NB) vpart[(int64_t(ch) * nk + q) * NN + i * NB + j] = vacc[c];
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint of Dyson G with the chemical potential.  G = [(i w + mu) - X]^{-1}
// with X = H + Sigma; dG = G (dX - dmu) G, so the direct cotangent of X is
// S = G^H Gbar G^H and dL/dmu = mubar - Re sum tr S.  With the filling held,
// N_e(mu, X) = N_target moves mu by -dN_X / N_mu, with
// N_mu = 2/N_k Re sum rho_m tr G^2 and the X-cotangent of N_e equal to
// -2/N_k conj(rho_m) (G^2)^H; the second pass adds that term.
// ---------------------------------------------------------------------------
template <int NO>
__global__ __launch_bounds__(64) void k_dyson_g_bwd1(DysonGArgs A, double mu, const zd* __restrict__ gbar,
                                                     zd* __restrict__ sbar, double* __restrict__ part) {
  const int64_t total = int64_t(A.r) * A.nk;
  const int64_t gi = int64_t(blockIdx.x) * 64 + threadIdx.x;
  double acc = 0.0, acc2 = 0.0;
  if (gi < total) {
    cpx<double> g[NO][NO];
    load_base<NO>(A, gi, g);
#pragma unroll
    for (int i = 0; i < NO; ++i) g[i][i].re += mu;
    invert_inplace<NO>(g);
    const int m = int(gi / A.nk), k = int(gi - int64_t(m) * A.nk);
    cpx<double> t1[NO][NO];
#pragma unroll
    for (int i = 0; i < NO; ++i)
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        cpx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < NO; ++c) s = fma(s, conj(g[c][i]), gbar[((int64_t(m) * NO + c) * NO + j) * A.nk + k]);
        t1[i][j] = s;
      }
    cpx<double> tr2 = mk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < NO; ++i)
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        cpx<double> s = mk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < NO; ++c) s = fma(s, t1[i][c], conj(g[j][c]));
        sbar[((int64_t(m) * NO + i) * NO + j) * A.nk + k] = s;
        if (i == j) acc += s.re;
        tr2 = fma(tr2, g[i][j], g[j][i]);
      }
    const zd rh = A.rho[m];
    acc2 = rh.re * tr2.re - rh.im * tr2.im;
  }
  acc = wave_sum(acc);
  acc2 = wave_sum(acc2);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = acc;
    part[gridDim.x + blockIdx.x] = acc2;
  }
}

template <int NO>
__global__ __launch_bounds__(64) void k_dyson_g_bwd2(DysonGArgs A, double mu, double mubar,
                                                     const double* __restrict__ part, int nblk,
                                                     zd* __restrict__ sbar) {
  double s = 0.0, s2 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) {
    s += part[b];
    s2 += part[nblk + b];
  }
  s = wave_sum(s);
  s2 = wave_sum(s2);
  const double n_mu = 2.0 * s2 / double(A.nk);
  const double coef = (mubar - s) / n_mu * 2.0 / double(A.nk);
  const int64_t total = int64_t(A.r) * A.nk;
  const int64_t gi = int64_t(blockIdx.x) * 64 + threadIdx.x;
  if (gi >= total) return;
  cpx<double> g[NO][NO];
  load_base<NO>(A, gi, g);
#pragma unroll
  for (int i = 0; i < NO; ++i) g[i][i].re += mu;
  invert_inplace<NO>(g);
  const int m = int(gi / A.nk), k = int(gi - int64_t(m) * A.nk);
  const cpx<double> w = scale(conj(A.rho[m]), coef);
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      cpx<double> g2ji = mk(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < NO; ++c) g2ji = fma(g2ji, g[j][c], g[c][i]);
      const int64_t o = ((int64_t(m) * NO + i) * NO + j) * A.nk + k;
      sbar[o] = sbar[o] + w * conj(g2ji);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

template <int NB, typename T>
hipError_t dyson_w_nb(const Plan& p, const void* v_q, const void* p_nu, void* wc_nu, hipStream_t s, int64_t ld) {
  constexpr int MPW = DysonWShape<NB>::MPW;
  const int64_t nmat = int64_t(p.r) * p.nk;
  if (ld == 0) ld = int64_t(NB) * NB;
  if (ld < int64_t(NB) * NB) return hipErrorInvalidValue;
  if (NB == 25) {
    if (p.tune.w25_mfma == 1)
      hipLaunchKernelGGL((k_dyson_w25<T, false, true>), dim3(unsigned(nmat)), dim3(64), 0, s, (const cpx<T>*)v_q,
                         (const cpx<T>*)p_nu, (cpx<T>*)wc_nu, nmat, p.nk, ld, p.d_status + kCondWord, nullptr);
    else
      hipLaunchKernelGGL((k_dyson_w25<T, false, false>), dim3(unsigned(nmat)), dim3(64), 0, s, (const cpx<T>*)v_q,
                         (const cpx<T>*)p_nu, (cpx<T>*)wc_nu, nmat, p.nk, ld, p.d_status + kCondWord, nullptr);
    return hipGetLastError();
  }
  if constexpr (NB > 8 && NB <= 16) {
    hipLaunchKernelGGL((k_dyson_wr<T, NB>), dim3(unsigned(nmat)), dim3(64), 0, s, (const cpx<T>*)v_q,
                       (const cpx<T>*)p_nu, (cpx<T>*)wc_nu, nmat, p.nk, ld, p.d_status + kCondWord);
    return hipGetLastError();
  }
  const unsigned blocks = unsigned((nmat + MPW - 1) / MPW);
  hipLaunchKernelGGL((k_dyson_w<NB, T>), dim3(blocks), dim3(64), 0, s, (const cpx<T>*)v_q,
                     (const cpx<T>*)p_nu, (cpx<T>*)wc_nu, nmat, p.nk, ld, p.d_status + kCondWord);
  return hipGetLastError();
}

template <int NO>
DysonGArgs dyson_g_args(const Plan& p, const void* h_k, const void* sig_iw, int mode, void* g_iw, double* scal,
                        double* partials, int* status) {
  DysonGArgs A;
  A.hk = (const zd*)h_k;
  A.sig = (const zd*)sig_iw;
  A.wn = p.d_wn;
  A.rho = (const zd*)p.dmaps64.m[5];
  A.g = (zd*)g_iw;
  A.scal = scal;
  A.partials = partials;
  A.status = status;
  A.r = p.r;
  A.nk = p.nk;
  A.mode = mode;
  A.max_evals = 200;
  A.beta = p.beta;
  A.tol_mu = 1e-13;
  A.tol_n = 1e-13;
  A.extra = nullptr;
  A.fail_word = nullptr;
  A.ne_offset = p.ne_offset;
  return A;
}

// grid of the search: one block per 64 (node, k) points, at most max_blocks (grid-stride beyond)
// one-wave blocks over the (node, k) points, at most 1024: every evaluation re-sums the previous one's per-block
// partials in each block, so that work grows with the square of the block count
static int dyson_g_blocks(const Plan& p) {
  const int64_t need = (int64_t(p.r) * p.nk + 63) / 64;
  const int64_t cap = p.max_blocks < 1024 ? p.max_blocks : 1024;
  return int(need < cap ? need : cap);
}

}  // namespace

int dyson_g_partials_needed(const Plan& p) {
  const int64_t gb = (p.nk + 63) / 64 < 1024 ? (p.nk + 63) / 64 : 1024;  // start: three partials per block
  const int nb = dyson_g_blocks(p);                                      // evaluations: two halves of two
  return int(3 * gb > 4 * int64_t(nb) ? 3 * gb : 4 * int64_t(nb));
}

namespace {

template <int NO>
hipError_t dyson_g_begin_no(const Plan& p, const void* h_k, double* scal, double* partials, int* status, int track,
                            int set, double mu0, double nt, const double* dpart, int dnblk, const double* bmax,
                            int nbmax, double* dsig, hipStream_t s) {
  if (dpart) {
    hipLaunchKernelGGL(k_dg_begin, dim3(1), dim3(64), 0, s, scal, status, dpart, dnblk, 1.0 / (double(NO) * p.nk),
                       track, set, mu0, nt, 1, bmax, nbmax, dsig);
    return hipGetLastError();
  }
  DysonGArgs A = dyson_g_args<NO>(p, h_k, nullptr, 1, nullptr, scal, partials, status);
  const int gb = int((p.nk + 63) / 64 < 1024 ? (p.nk + 63) / 64 : 1024);
  hipLaunchKernelGGL((k_dg_gersh<NO>), dim3(gb), dim3(64), 0, s, A);
  hipLaunchKernelGGL(k_dg_begin, dim3(1), dim3(64), 0, s, scal, status, (const double*)partials, gb,
                     1.0 / (double(NO) * p.nk), track, set, mu0, nt, 0, bmax, nbmax, dsig);
  return hipGetLastError();
}

template <int NO>
hipError_t dyson_g_steps_no(const Plan& p, const void* h_k, const void* sig_iw, double* scal, double* partials,
                            int* status, int steps, hipStream_t s) {
  DysonGArgs A = dyson_g_args<NO>(p, h_k, sig_iw, 1, nullptr, scal, partials, status);
  const int blocks = dyson_g_blocks(p);
  for (int i = 0; i < steps; ++i) hipLaunchKernelGGL((k_dg_eval<NO>), dim3(blocks), dim3(64), 0, s, A, i, blocks);
  return hipGetLastError();
}

template <int NO>
hipError_t dyson_g_final_no(const Plan& p, const void* h_k, const void* sig_iw, int mode, void* g_iw,
                            double* scal, double* partials, int* status, const double* extra, int steps,
                            int* fail_word, hipStream_t s) {
  DysonGArgs A = dyson_g_args<NO>(p, h_k, sig_iw, mode, g_iw, scal, partials, status);
  A.extra = extra;
  A.fail_word = fail_word;
  const int blocks = dyson_g_blocks(p);
  hipLaunchKernelGGL((k_dg_final<NO>), dim3(blocks), dim3(64), 0, s, A, mode == 1 ? steps : 0, blocks);
  return hipGetLastError();
}

// workspace: W^C and X (pair matrix layout, dense), then the Vbar partials [chunks][N_k][N_b][N_b]
template <int NB>
hipError_t dyson_w_bwd_nb(const Plan& p, const void* v_q, const void* p_nu, const void* wbar, void* pbar,
                          void* ws, int chunks, hipStream_t s) {
  constexpr int64_t NN = int64_t(NB) * NB;
  const int64_t nmat = int64_t(p.r) * p.nk;
  zd* wcm = (zd*)ws;
  zd* xm = wcm + nmat * NN;
  zd* vpart = xm + nmat * NN;
  int* cond = p.d_status + kCondWord;
  if (NB == 25 && p.tune.w25_mfma == 1) {
    hipLaunchKernelGGL((k_dyson_w25<double, false, true>), dim3(unsigned(nmat)), dim3(64), 0, s, (const zd*)v_q,
                       (const zd*)p_nu, wcm, nmat, p.nk, NN, cond, nullptr);
    hipLaunchKernelGGL((k_dyson_w25<double, true, true>), dim3(unsigned(nmat)), dim3(64), 0, s, (const zd*)v_q,
                       (const zd*)p_nu, xm, nmat, p.nk, NN, cond, (const zd*)wbar);
  } else if (NB == 25) {
    hipLaunchKernelGGL((k_dyson_w25<double, false, false>), dim3(unsigned(nmat)), dim3(64), 0, s, (const zd*)v_q,
                       (const zd*)p_nu, wcm, nmat, p.nk, NN, cond, nullptr);
    hipLaunchKernelGGL((k_dyson_w25<double, true, false>), dim3(unsigned(nmat)), dim3(64), 0, s, (const zd*)v_q,
                       (const zd*)p_nu, xm, nmat, p.nk, NN, cond, (const zd*)wbar);
  } else if constexpr (NB > 8 && NB <= 16) {
    hipLaunchKernelGGL((k_dyson_wr<double, NB, false>), dim3(unsigned(nmat)), dim3(64), 0, s, (const zd*)v_q,
                       (const zd*)p_nu, wcm, nmat, p.nk, NN, cond, nullptr);
    hipLaunchKernelGGL((k_dyson_wr<double, NB, true>), dim3(unsigned(nmat)), dim3(64), 0, s, (const zd*)v_q,
                       (const zd*)p_nu, xm, nmat, p.nk, NN, cond, (const zd*)wbar);
  } else {
    constexpr int MPW = DysonWShape<NB>::MPW;
    const unsigned blocks = unsigned((nmat + MPW - 1) / MPW);
    hipLaunchKernelGGL((k_dyson_w<NB, double, false>), dim3(blocks), dim3(64), 0, s, (const zd*)v_q,
                       (const zd*)p_nu, wcm, nmat, p.nk, NN, cond, nullptr);
    hipLaunchKernelGGL((k_dyson_w<NB, double, true>), dim3(blocks), dim3(64), 0, s, (const zd*)v_q,
                       (const zd*)p_nu, xm, nmat, p.nk, NN, cond, (const zd*)wbar);
  }
  hipLaunchKernelGGL((k_dyson_w_bwd_prod<NB>), dim3(unsigned(p.nk), unsigned(chunks)), dim3(256), 0, s,
                     (const zd*)v_q, (const zd*)p_nu, (const zd*)wbar, (const zd*)wcm, (const zd*)xm, (zd*)pbar,
                     vpart, p.r, p.nk, chunks);
  return hipGetLastError();
}

template <int NO>
hipError_t dyson_g_bwd_no(const Plan& p, const void* h_k, const void* sig_iw, double mu, double n_target,
                          double mubar, const void* gbar, void* sbar, hipStream_t s) {
  DysonGArgs A;
  A.hk = (const zd*)h_k;
  A.sig = (const zd*)sig_iw;
  A.wn = p.d_wn;
  A.rho = (const zd*)p.dmaps64.m[5];
  A.g = nullptr;
  A.scal = p.d_scalars;
  A.partials = p.d_partials;
  A.status = p.d_status;
  A.r = p.r;
  A.nk = p.nk;
  A.mode = 0;
  A.max_evals = 0;
  A.beta = p.beta;
  A.tol_mu = A.tol_n = 0.0;
  A.extra = nullptr;
  A.fail_word = nullptr;
  A.ne_offset = p.ne_offset;
  const int64_t total = int64_t(p.r) * p.nk;
  const int nblk = int((total + 63) / 64);
  if (2 * int64_t(nblk) > 8 * int64_t(p.max_blocks)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_dyson_g_bwd1<NO>), dim3(unsigned(nblk)), dim3(64), 0, s, A, mu, (const zd*)gbar, (zd*)sbar,
                     p.d_partials);
  if (std::isfinite(n_target))
    hipLaunchKernelGGL((k_dyson_g_bwd2<NO>), dim3(unsigned(nblk)), dim3(64), 0, s, A, mu, mubar,
                       (const double*)p.d_partials, nblk, (zd*)sbar);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dyson_w_bwd(const Plan& p, const void* v_q, const void* p_nu, const void* wbar, void* pbar,
                              void* vpart, int chunks, hipStream_t s) {
  switch (p.nb) {
#define QGW_CASE(NBV) \
  case NBV:           \
    return dyson_w_bwd_nb<NBV>(p, v_q, p_nu, wbar, pbar, vpart, chunks, s);
    QGW_FOR_EACH_NB(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_dyson_g_bwd(const Plan& p, const void* h_k, const void* sig_iw, double mu, double n_target,
                              double mubar, const void* gbar, void* sbar, hipStream_t s) {
  switch (p.no) {
#define QGW_CASE(NOV) \
  case NOV:           \
    return dyson_g_bwd_no<NOV>(p, h_k, sig_iw, mu, n_target, mubar, gbar, sbar, s);
    QGW_FOR_EACH_NO(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_dyson_w(const Plan& p, const void* v_q, const void* p_nu, void* wc_nu,
                          hipStream_t s, int64_t out_ld) {
  switch (p.nb) {
#define QGW_CASE(NBV)                                                                     \
  case NBV:                                                                               \
    return p.prec == 0 ? dyson_w_nb<NBV, double>(p, v_q, p_nu, wc_nu, s, out_ld)          \
                       : dyson_w_nb<NBV, float>(p, v_q, p_nu, wc_nu, s, out_ld);
    QGW_FOR_EACH_NB(QGW_CASE)
#undef QGW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

#define QGW_NO_SWITCH(CALL)    \
  switch (p.no) {              \
    case 1: { constexpr int NOV = 1; return CALL; } \
    case 2: { constexpr int NOV = 2; return CALL; } \
    case 3: { constexpr int NOV = 3; return CALL; } \
    case 4: { constexpr int NOV = 4; return CALL; } \
    case 5: { constexpr int NOV = 5; return CALL; } \
    case 6: { constexpr int NOV = 6; return CALL; } \
    case 7: { constexpr int NOV = 7; return CALL; } \
    case 8: { constexpr int NOV = 8; return CALL; } \
    default: return hipErrorInvalidValue;          \
  }

hipError_t launch_dyson_g_begin(const Plan& p, const void* h_k, double* scal, double* partials, int* status,
                                int track, hipStream_t s, int set, double mu0, double nt, const double* dpart,
                                int dnblk, const double* bmax, int nbmax, double* dsig) {
  QGW_NO_SWITCH((dyson_g_begin_no<NOV>(p, h_k, scal, partials, status, track, set, mu0, nt, dpart, dnblk, bmax, nbmax,
                                       dsig, s)))
}

hipError_t launch_dyson_g_steps(const Plan& p, const void* h_k, const void* sig_iw, double* scal, double* partials,
                                int* status, int steps, hipStream_t s) {
  QGW_NO_SWITCH((dyson_g_steps_no<NOV>(p, h_k, sig_iw, scal, partials, status, steps, s)))
}

hipError_t launch_dyson_g_final(const Plan& p, const void* h_k, const void* sig_iw, int mode, void* g_iw,
                                double* scal, double* partials, int* status, hipStream_t s, const double* extra,
                                int steps, int* fail_word) {
  QGW_NO_SWITCH((dyson_g_final_no<NOV>(p, h_k, sig_iw, mode, g_iw, scal, partials, status, extra, steps, fail_word,
                                       s)))
}

hipError_t launch_dyson_g_chain(const Plan& p, const void* h_k, const void* sig_iw, int mode, void* g_iw,
                                double* scal, double* partials, int* status, int steps, int* fail_word,
                                hipStream_t s, const double* dpart, int dnblk, const double* bmax, int nbmax,
                                double* dsig) {
  hipError_t e = hipSuccess;
  if (mode == 1) {
    e = launch_dyson_g_begin(p, h_k, scal, partials, status, 1, s, 0, 0.0, 0.0, dpart, dnblk, bmax, nbmax, dsig);
    if (e == hipSuccess) e = launch_dyson_g_steps(p, h_k, sig_iw, scal, partials, status, steps, s);
  }
  if (e == hipSuccess) e = launch_dyson_g_final(p, h_k, sig_iw, mode, g_iw, scal, partials, status, s, nullptr,
                                                mode == 1 ? steps : 0, fail_word);
  return e;
}

#undef QGW_NO_SWITCH

}  // namespace qgw
