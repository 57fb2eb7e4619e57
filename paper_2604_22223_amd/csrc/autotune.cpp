// Launch-shape autotuner.  For one plan it times the candidate shapes of the
// kernels whose best shape depends on the instance (mesh side, orbital count,
// product basis, DLR rank) on scratch arrays of the plan's real sizes, with
// HIP events on the caller's stream, and keeps the fastest in the plan:
//   lattice transform:  slabs per block
//   bubble:             slabs per block
//   self-energy:        term lanes per block
//   pair DLR maps:      resident blocks per CU of the matrix-core kernel
//   orbital DLR maps:   matrix cores, or the VALU kernel with 8 / 16 / 32 rows per chunk
//   Dyson W (N_b = 25): V P on the matrix cores or on the VALU
// Every candidate computes the same thing; only the self-energy lane count
// and the orbital-map kernel change the order of floating-point sums.  An
// FP64 plan is also tuned for its FP32 kernels (the single-precision
// iterations of a state's mixed schedule), whose best shapes differ.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <string>
#include <vector>

#include "../../include/qgw.h"
#include "qgw_internal.h"

using namespace qgw;

namespace {

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t init() {
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    return e;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// best of `reps` timed runs after one warm-up; +inf if a launch fails
double time_launch(Timer& t, hipStream_t s, const std::function<hipError_t()>& f, int reps = 3) {
  if (f() != hipSuccess) return 1e30;
  double best = 1e30;
  for (int i = 0; i < reps; ++i) {
    if (hipEventRecord(t.a, s) != hipSuccess) return 1e30;
    if (f() != hipSuccess) return 1e30;
    if (hipEventRecord(t.b, s) != hipSuccess) return 1e30;
    if (hipEventSynchronize(t.b) != hipSuccess) return 1e30;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) return 1e30;
    best = std::min(best, double(ms));
  }
  return best;
}

template <typename F>
int pick(Timer& t, hipStream_t s, const std::vector<int>& cands, int& knob, F run) {
  int best = cands.empty() ? 0 : cands[0];
  double tb = 1e30;
  for (int c : cands) {
    knob = c;
    const double ms = time_launch(t, s, run);
    if (ms < tb) {
      tb = ms;
      best = c;
    }
  }
  knob = best;
  return best;
}

}  // namespace

extern "C" {

qgw_status qgw_plan_autotune(qgw_plan h, int32_t* choices, void* stream) {
  if (!h) {
    set_error("qgw_plan_autotune: null plan");
    return QGW_ERR_INVALID_ARG;
  }
  Plan& p = h->p;
  if (p.grid != kGridDLR) {
    set_error("qgw_plan_autotune: DLR plans only");
    return QGW_ERR_UNSUPPORTED;
  }
  const bool dev_ok = hipSetDevice(p.device) == hipSuccess;
  (void)hipGetLastError();  // a stale error of an earlier call must not fail the trial launches
  if (!dev_ok) {
    set_error("qgw_plan_autotune: hipSetDevice failed");
    return QGW_ERR_DEVICE;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t c = 16;  // sized for FP64, large enough for the FP32 trials too
  const size_t sg = size_t(p.r) * p.no * p.no * p.nk * c;
  const size_t sp = size_t(p.r) * p.nb * p.nb * p.nk * c;
  const size_t sv = size_t(p.nb) * p.nb * p.nk * c;
  void *gt = nullptr, *gr = nullptr, *og = nullptr, *pa = nullptr, *pb = nullptr, *vv = nullptr;
  hipError_t e = hipMalloc(&gt, sg);
  if (e == hipSuccess && p.nb == 25) e = hipMalloc(&vv, sv);
  if (e == hipSuccess && p.nb == 25) e = hipMemsetAsync(vv, 0x3f, sv, s);
  if (e == hipSuccess) e = hipMalloc(&gr, sg);
  if (e == hipSuccess) e = hipMalloc(&og, sg);
  if (e == hipSuccess) e = hipMalloc(&pa, sp);
  if (e == hipSuccess) e = hipMalloc(&pb, sp);
  // finite, non-zero test data (every byte 0x3f)
  if (e == hipSuccess) e = hipMemsetAsync(gt, 0x3f, sg, s);
  if (e == hipSuccess) e = hipMemsetAsync(gr, 0x3f, sg, s);
  if (e == hipSuccess) e = hipMemsetAsync(pa, 0x3f, sp, s);
  Timer t;
  if (e == hipSuccess) e = t.init();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    for (void* q : {gt, gr, og, pa, pb, vv})
      if (q) (void)hipFree(q);
    set_error(std::string("qgw_plan_autotune: ") + hipGetErrorString(e));
    return QGW_ERR_DEVICE;
  }
  const int64_t no2 = int64_t(p.no) * p.no;
  const int lane_cap = std::max(1, 256 / lines_per_slab(p));
  std::vector<int> spb;
  for (int v = 1; v <= lane_cap; v *= 2) spb.push_back(v);
  if (spb.back() != lane_cap) spb.push_back(lane_cap);
  // every knob of q.tune, timed with q's precision
  auto tune_one = [&](Plan& q) {
    Tune& tn = q.tune;
    pick(t, s, spb, tn.fft_spb, [&] { return launch_lattice_fft(q, QGW_K_TO_R, no2 * q.r, gt, og, s); });
    pick(t, s, spb, tn.bubble_spb, [&] { return launch_bubble(q, gt, gr, 1, pa, s); });
    std::vector<int> lanes;
    for (int v = 1; v <= std::min(lane_cap, std::max(1, q.terms.max_terms)); ++v) lanes.push_back(v);
    pick(t, s, lanes, tn.sigma_spb, [&] { return launch_sigma(q, gt, pa, 1, 1, og, s); });
    if (q.r <= 64) {
      pick(t, s, {1, 2, 3, 4, 6, 8}, tn.mfma_bpc, [&] {
        hipError_t r = launch_dlr_pairs(q, QGW_B_TAU2IW, QGW_LAYOUT_SLAB, QGW_LAYOUT_MATRIX, pa, pb, s);
        if (r == hipSuccess) r = launch_dlr_pairs(q, QGW_B_IW2TAU, QGW_LAYOUT_MATRIX, QGW_LAYOUT_SLAB, pb, pa, s);
        return r;
      });
    }
    // orbital maps: code 0 = matrix cores, 8 / 16 / 32 = VALU kernel with that chunk
    std::vector<int> orb = {8, 16, 32};
    if (q.r <= 64) orb.insert(orb.begin(), 0);
    int code = 0;
    pick(t, s, orb, code, [&] {
      tn.orb_valu = code == 0 ? 0 : 1;
      tn.orb_mt = code;
      return launch_dlr(q, QGW_F_IW2TAU, no2 * q.nk, 1.0, 0.0, gt, og, s);
    });
    tn.orb_valu = code == 0 ? 0 : 1;
    tn.orb_mt = code;
    if (q.nb == 25) pick(t, s, {0, 1}, tn.w25_mfma, [&] { return launch_dyson_w(q, vv, pa, pb, s, 0); });
  };
  tune_one(p);
  if (p.prec == QGW_F64) {
    Plan q = p;  // the same device data read by the FP32 kernels
    q.prec = QGW_F32;
    q.tune = Tune();
    tune_one(q);
    p.tune32 = q.tune;
    p.has_tune32 = true;
  }
  const Tune& tn = p.tune;
  // the trial data are arbitrary: a condition the Dyson-W trials raised is not the caller's
  if (p.nb == 25) (void)hipMemsetAsync(p.d_status + kCondWord, 0, sizeof(int), s);
  e = hipStreamSynchronize(s);
  for (void* q : {gt, gr, og, pa, pb, vv}) (void)hipFree(q);
  if (e != hipSuccess) {
    set_error(std::string("qgw_plan_autotune: ") + hipGetErrorString(e));
    return QGW_ERR_DEVICE;
  }
  if (choices) {
    choices[0] = tn.fft_spb;
    choices[1] = tn.bubble_spb;
    choices[2] = tn.sigma_spb;
    choices[3] = tn.mfma_bpc;
    choices[4] = tn.orb_valu;
    choices[5] = tn.orb_mt;
    choices[6] = tn.w25_mfma;
  }
  return QGW_OK;
}

qgw_status qgw_plan_set_tuning(qgw_plan h, int32_t precision, const int32_t* choices) {
  if (!h || !choices) {
    set_error("qgw_plan_set_tuning: null argument");
    return QGW_ERR_INVALID_ARG;
  }
  Plan& p = h->p;
  if (precision != QGW_F64 && precision != QGW_F32) {
    set_error("qgw_plan_set_tuning: precision must be QGW_F64 or QGW_F32");
    return QGW_ERR_INVALID_ARG;
  }
  if (precision == QGW_F32 && p.prec != QGW_F64) {
    set_error("qgw_plan_set_tuning: the FP32 shapes belong to an FP64 plan (an FP32 plan takes QGW_F64's slot)");
    return QGW_ERR_INVALID_ARG;
  }
  const int lane_cap = std::max(1, 256 / lines_per_slab(p));
  const bool ok = choices[0] >= 0 && choices[0] <= lane_cap && choices[1] >= 0 && choices[1] <= lane_cap &&
                  choices[2] >= 0 && choices[2] <= lane_cap && choices[3] >= 0 && choices[3] <= 8 &&
                  choices[4] >= -1 && choices[4] <= 1 &&
                  (choices[5] == 0 || choices[5] == 8 || choices[5] == 16 || choices[5] == 32) &&
                  choices[6] >= -1 && choices[6] <= 1;
  if (!ok) {
    set_error("qgw_plan_set_tuning: a choice is outside its range");
    return QGW_ERR_INVALID_ARG;
  }
  Tune tn;
  tn.fft_spb = choices[0];
  tn.bubble_spb = choices[1];
  tn.sigma_spb = choices[2];
  tn.mfma_bpc = choices[3];
  tn.orb_valu = choices[4];
  tn.orb_mt = choices[5];
  tn.w25_mfma = choices[6];
  if (precision == QGW_F32 && p.prec == QGW_F64) {
    p.tune32 = tn;
    p.has_tune32 = true;
  } else {
    p.tune = tn;
  }
  return QGW_OK;
}

}  // extern "C"
