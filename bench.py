"""GW iterations per second on one MI355X (five-orbital model, 24 x 24 k-mesh).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one full GW iteration through libqgw (Fig. fig-self (b): density
and Hartree-Fock, G(i w) -> G(tau), bubble, P(i nu), Dyson W, W^C(tau),
self-energy, Sigma(i w), Delta Sigma, Dyson G with the chemical-potential
search).  Inputs are seeded and synthetic and resident in HBM before timing.

The timed work is back-to-back self-consistent solves from G0 to
max |Delta Sigma| <= 1e-6 (a converged solve restarts from G0), under two
precision schedules: plain FP64, and the chosen one (the bulk steps a1-a11
in FP32 while |Delta Sigma| is large, FP64 to finish, so every solve ends on
an FP64 fixed point).  For each, W untimed iterations run first, then exactly
K iterations are timed between two device synchronisations; `value` is the
chosen schedule's iterations/s.  Per-step durations come from HIP events the
library records on the same stream inside the timed region.  One solve per
schedule is also timed on its own (iterations and time to solution).  The
oracle is timed on the host for one iteration of the same workload (the CPU
baseline).  Further legs, reported beside the headline line: quasiparticle
post-processing, the Hartree-Fock solve, the paper's own five-orbital
benchmark on its 8 x 8 x 8 cubic mesh (per-iteration times grouped into the
quantities of the paper's timing table), both workloads on a uniform
Matsubara grid of the same cutoff (the MF axis of the paper's table), and the
batched sweep.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector = matrix), TFLOP/s
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 (vector = matrix), TFLOP/s
SWITCH_FACTOR = 3.0            # the mixed solve leaves FP32 at |Delta Sigma| <= SWITCH_FACTOR x the solve tolerance

WORKLOAD = "five_orbital_24"
METRIC = "GW iterations/sec (5-orb, 24^2 k), chosen vs plain FP64, at |dSigma|<=1e-6"


_TOL = [1e-6]


def switch_tol():
    """|Delta Sigma| at which the chosen schedule leaves its FP32 phase: a few times the solve tolerance, so the
    FP32 iterations carry the solve close to it and FP64 iterations make the end point an FP64 fixed point."""
    return SWITCH_FACTOR * _TOL[0]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload():
    """Five orbitals on a 24 x 24 square lattice, beta = 50/eV, filling 6/10,
    omega_max = 25 eV (Lambda = 1250), eps = 1e-10, N_b = 25; interaction of
    the paper's five-orbital benchmark (U = 1, J = 0.1, V = 0.2 eV)."""
    from paper_2604_22223_amd import workloads as wl
    return wl.workload(WORKLOAD)


def step_model(r, n_o, n_b, n_k, prec="f64"):
    """Algorithmic HBM bytes and flops of each timed step.

    FP64 iterations hold complex128 arrays (16 bytes); the FP32 iterations run
    a1-a11 on complex64 arrays (8 bytes) and start from / end in the FP64
    G(i w) and Sigma(i w) of the solve; a12, a13 and a14 are FP64 in both."""
    c = 16.0 if prec == "f64" else 8.0
    ng = r * n_o * n_o * n_k                 # elements of one fermionic array
    npair = r * n_b * n_b * n_k              # elements of one pair array
    stat_o = n_o * n_o * n_k * 16.0
    fft_flops = 5.0 * n_k * math.log2(max(n_k, 2))   # per slab (complex 2-D FFT)
    return {
        "a12_density_hf": {"bytes": 16.0 * ng + 6 * stat_o + n_b * n_b * n_k * 16.0, "flops": 8.0 * r * n_o * n_o * n_k},
        # read G(i w) once (FP64), write G(tau) and G(beta - tau)
        "a1_dlr_g": {"bytes": 16.0 * ng + 2 * c * ng, "flops": 2 * 8.0 * r * r * n_o * n_o * n_k},
        "a2_fft_g": {"bytes": 4 * c * ng, "flops": 2 * r * n_o * n_o * fft_flops},
        "a3a4_bubble": {"bytes": 2 * c * ng + c * npair, "flops": r * n_b * n_b * (fft_flops + 12.0 * n_k)},
        "a5_dlr_p": {"bytes": 2 * c * npair, "flops": 8.0 * r * r * n_b * n_b * n_k},
        "a6_dyson_w": {"bytes": 2 * c * npair + n_b * n_b * n_k * c, "flops": (8.0 + 8.0 / 3.0 + 8.0) * n_b ** 3 * r * n_k},
        "a7_dlr_w": {"bytes": 2 * c * npair, "flops": 8.0 * r * r * n_b * n_b * n_k},
        "a8a9a10_sigma": {"bytes": c * npair + 2 * c * ng, "flops": r * n_b * n_b * (fft_flops + 8.0 * n_k) + r * n_o * n_o * fft_flops},
        # read Sigma^C(k, tau), write the FP64 Sigma^C(k, i w)
        "a11_dlr_sigma": {"bytes": c * ng + 16.0 * ng, "flops": 8.0 * r * r * n_o * n_o * n_k},
        # Sigma^C new and old read, old written (at mixing 1, as timed, the new values are not rewritten); Sigma_HF
        # new and old read, old written, H0 read and H0 + Sigma_HF written
        "a14_delta_mix": {"bytes": 3 * 16.0 * ng + 5 * stat_o, "flops": 0.0},
        "a13_dyson_g": {"bytes": 2 * 16.0 * ng, "flops": 0.0},
    }


PEAK_TFLOPS = {"f64": FP64_PEAK_TFLOPS, "f32": FP32_PEAK_TFLOPS}

# Measured HBM bytes per launch of the kernels that carry a step (rocprofv3 FETCH_SIZE and WRITE_SIZE runs of
# `bench.py --steps 3 --warmup 1 --no-cpu-baseline --batch 0 --paper-steps 0 --mf-steps 0 --copy-calibration 256`, each
# counter scaled by what it reads for a 256 MiB device copy: FETCH x 1.9997, WRITE x 1.0000;
# profiles/hbm_traffic_gw_iteration_five_orbital_24.md).
# Valid for the kernels as they were profiled; a changed kernel drops its entry until it is profiled again.
MEASURED_TRAFFIC = {
    "a3a4_bubble:f64": 332.3e6, "a5_dlr_p:f64": 671.9e6, "a6_dyson_w:f64": 629.4e6, "a7_dlr_w:f64": 655.2e6,
    "a8a9a10_sigma:f64": 333.8e6, "a14_delta_mix:f64": 37.8e6,
    "a3a4_bubble:f32": 166.2e6, "a5_dlr_p:f32": 334.9e6, "a6_dyson_w:f32": 314.9e6, "a7_dlr_w:f32": 309.2e6,
    "a8a9a10_sigma:f32": 166.0e6, "a14_delta_mix:f32": 37.8e6,
}
FP64_STEPS = ("a12_density_hf", "a14_delta_mix", "a13_dyson_g")


def bound_of(entry, prec):
    """HBM-bound if the arithmetic intensity is below the ridge point of the step's precision."""
    ridge = PEAK_TFLOPS[prec] * 1e12 / (HBM_PEAK_GBS * 1e9)
    return "alu" if entry["flops"] / max(entry["bytes"], 1.0) > ridge else "hbm"


def roof(entry, prec, ms):
    b = bound_of(entry, prec)
    if b == "hbm":
        ach, peak, unit = entry["bytes"] / (ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        ach, peak, unit = entry["flops"] / (ms * 1e-3) / 1e12, PEAK_TFLOPS[prec], "TFLOP/s"
    return {"ms": round(ms, 5), "bound": b, "achieved": round(ach, 3), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4)}


def cpu_baseline(w, min_seconds=10.0, max_iter=8):
    """The oracle's GW iterations of the same workload from G0 on the host CPU,
    until at least min_seconds have passed (at most max_iter iterations)."""
    from oracle import gw
    from oracle.dlr import DLR
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    st = gw.initial_state(m, d)
    t0 = time.perf_counter()
    k = 0
    while k < max_iter and (k == 0 or time.perf_counter() - t0 < min_seconds):
        st = gw.gw_iteration(m, d, st)
        k += 1
    dt = time.perf_counter() - t0
    res = {"value": k / dt, "unit": "GW iterations/sec", "cores": int(threads), "kind": "oracle",
           "sample": "the first %d GW iterations from G0 of the same 24x24 five-orbital workload "
                     "(NumPy FP64, %s BLAS threads, %d host CPUs visible), %.1f s" % (k, threads, os.cpu_count(), dt)}
    # the same oracle on one thread: the first two iterations from G0 with every BLAS pool limited to one thread
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        return res
    st = gw.initial_state(m, d)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(2):
            st = gw.gw_iteration(m, d, st)
        dt1 = time.perf_counter() - t0
    res["single_thread"] = {"value": 2 / dt1, "cores": 1, "sample": "the first 2 GW iterations from G0, %.1f s" % dt1}
    return res


def solve(st, mode, tol, max_iter=60):
    """One self-consistent solve from G0 under a precision schedule."""
    st.set_precision(mode, switch_tol())
    st.init_g0()
    hist = []
    for _ in range(max_iter):
        _, dsig, mu = st.iterate(1)
        hist.append((dsig, st.info()[0], st.mu_evals()))
        if dsig <= tol and hist[-1][1] == 0:
            break
    return hist, mu


def timed_solves(torch, st, mode, tol, steps):
    """Exactly `steps` GW iterations of back-to-back solves from G0 (a converged
    solve restarts from G0), between two device synchronisations."""
    st.set_precision(mode, switch_tol())
    st.init_g0()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        # the library runs iterations back to back and stops at a converged FP64 iteration
        n, dsig, _ = st.iterate(steps - done, tol)
        done += n
        if dsig <= tol and st.info()[0] == 0:
            st.init_g0()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def quasiparticle_leg(torch, qgw, plan, st, H_R, mu, reps=20):
    """Post-processing of the converged state: Sigma(k, 0), Z(k), H_QP(k) and its bands (qgw_quasiparticle),
    timed with HIP events over ``reps`` calls (the call waits for its stream, so each one is whole)."""
    h_k = torch.empty_like(H_R)
    plan.lattice_fft(qgw.R_TO_K, H_R, h_k)
    shf, sig = st.array(2), st.array(1)
    plan.quasiparticle(h_k, shf, sig, mu=mu)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        sig0, z, hqp, bands = plan.quasiparticle(h_k, shf, sig, mu=mu)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    zr = np.linalg.eigvalsh(np.moveaxis(z.cpu().numpy(), -1, 0))
    return {"ms_per_call": round(ms, 4), "z_min": round(float(zr.min()), 6), "z_max": round(float(zr.max()), 6),
            "band_min_eV": round(float(bands.min()), 6), "band_max_eV": round(float(bands.max()), 6),
            "note": "bands relative to the chemical potential of the converged solve; includes the call's wait"}


def hf_leg(torch, qgw, plan, H_R, V_R, n_target, tol=1e-10, reps=3):
    """Hartree-Fock self-consistency (Fig. fig-self (a)) on the same model: passes to max |dSigma_HF| <= tol,
    wall time per solve (each pass waits once for the device) over ``reps`` solves after one warm-up."""
    st = qgw.State(plan, H_R, V_R, n_target=n_target, mixing=0.7)
    passes, ds, mu = st.hf_solve(tol=tol, max_iter=500)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        passes, ds, mu = st.hf_solve(tol=tol, max_iter=500)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    st.close()
    return {"passes": passes, "final_dsigma_hf": ds, "mu": mu, "mixing": 0.7, "tol": tol,
            "time_to_solution_s": round(el, 6), "passes_per_s": round(passes / el, 1)}


# The paper's own timing of one GW iteration of its five-orbital benchmark (8 x 8 x 8 mesh, beta = 100,
# Lambda = 25 eV), DLR + vectorised NumPy on an unstated CPU, seconds per iteration by quantity (table
# tab:performance_5orb).  Context only: other hardware, unstated precision and DLR accuracy.
PAPER_DLR_VEC_S = {"G": 2.21, "P": 137.55, "W": 65.48, "Sigma": 27.32}
# the library's steps grouped into the table's four quantities
PAPER_COLUMNS = {"G": ("a13_dyson_g", "a14_delta_mix"),
                 "P": ("a1_dlr_g", "a2_fft_g", "a3a4_bubble", "a5_dlr_p"),
                 "W": ("a6_dyson_w", "a7_dlr_w"),
                 "Sigma": ("a12_density_hf", "a8a9a10_sigma", "a11_dlr_sigma")}


def paper_workload_leg(torch, qgw, steps, tol, warmup=3, mixing=0.5):
    """The paper's five-orbital benchmark model on its 8 x 8 x 8 cubic mesh (t = 1, U = 1, J = 0.1,
    V = 0.2 eV, beta = 100/eV, omega_max = 25 eV, half filling; DLR eps = 1e-10): exactly ``steps``
    iterations from G0 in each schedule (FP64 throughout; FP32 bulk steps then FP64), per-step times from
    the library's HIP events grouped into the table's G, P, W and Sigma, and one solve to ``tol`` per
    schedule (linear mixing ``mixing``: the undamped loop oscillates on this model)."""
    from paper_2604_22223_amd import workloads as wl
    w = wl.workload("cubic_five_orbital_8")
    nodes = qgw.dlr_build(w["beta"] * w["omega_max"], w["eps"])
    nodes["omega"] = nodes["x"] / w["beta"]
    plan = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], nodes, dim=3)
    flat = lambda x: torch.from_numpy(np.ascontiguousarray(x.reshape(x.shape[:2] + (-1,)))).to("cuda:0")
    st = qgw.State(plan, flat(w["H_R"]), flat(w["V_R"]), n_target=w["n_target"], mixing=mixing)
    res = {"workload": "cubic_five_orbital_8", "mesh": "8x8x8", "n_orb": plan.n_o, "n_pair": plan.n_b,
           "beta": w["beta"], "omega_max": w["omega_max"], "dlr_eps": w["eps"], "dlr_rank": plan.r,
           "t": 1.0, "U": 1.0, "J": 0.1, "V_nn": 0.2, "filling": w["n_target"], "mixing": mixing,
           "paper_dlr_vec_s_per_iteration": dict(PAPER_DLR_VEC_S, total=round(sum(PAPER_DLR_VEC_S.values()), 2))}
    for name, mode in (("fp64", 0), ("mixed", 1)):
        st.set_precision(mode, switch_tol())
        st.init_g0()
        st.iterate(warmup)
        st.init_g0()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, _, _ = st.iterate(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # the per-step breakdown: the same iterations again, every step timed, a12 in line
        st.init_g0()
        st.profile_select(None, in_line=True)
        st.profile(1)
        st.iterate(steps)
        torch.cuda.synchronize()
        prof = st.profile(0, per_precision=True)
        st.profile_select(None, in_line=False)
        entry = {"iterations": done, "ms_per_iteration": round(1e3 * el / max(done, 1), 4)}
        for prec in ("f64", "f32"):
            ms_tot, iters = prof[prec]
            if iters == 0:
                continue
            cols = {c: round(sum(ms_tot[s] for s in ss) / iters, 4) for c, ss in PAPER_COLUMNS.items()}
            entry["%s_ms_by_quantity" % prec] = cols
            entry["%s_iterations" % prec] = iters
        # one solve to the tolerance from G0
        st.init_g0()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = []
        for _ in range(200):
            _, dsig, mu = st.iterate(1)
            hist.append((dsig, st.info()[0]))
            if dsig <= tol and hist[-1][1] == 0:
                break
        torch.cuda.synchronize()
        entry["solve"] = {"iterations": len(hist), "fp32_iterations": sum(1 for _, p in hist if p == 1),
                          "final_dsigma": hist[-1][0], "mu": mu,
                          "time_to_solution_s": round(time.perf_counter() - t0, 5)}
        res[name] = entry
        log("[bench] cubic 8^3 %-5s: %.3f ms/iteration; solve %d iterations in %.4f s"
            % (name, entry["ms_per_iteration"], len(hist), entry["solve"]["time_to_solution_s"]))
    res["speedup_vs_paper_dlr_vec_fp64"] = round(sum(PAPER_DLR_VEC_S.values())
                                                 / (1e-3 * res["fp64"]["ms_per_iteration"]), 1)
    st.close()
    plan.close()
    return res


def mf_leg(torch, qgw, w, steps, tol, warmup=2, mixing=1.0, dlr_ms=None, name=""):
    """The same workload on a uniform Matsubara grid reaching the same omega_max (qgw_plan_create_mf): exactly
    ``steps`` FP64 iterations from G0 with per-step HIP events, and one solve to ``tol``; ``dlr_ms`` is the DLR
    plan's FP64 ms per iteration on the workload, for the ratio."""
    n_nodes = qgw.mf_nodes_for(w["beta"], w["omega_max"])
    d = len(w["mesh"])
    plan = qgw.Plan.uniform(w["mesh"][0], w["site_norb"], w["beta"], n_nodes, dim=d)
    flat = lambda x: torch.from_numpy(np.ascontiguousarray(x.reshape(x.shape[:2] + (-1,)))).to("cuda:0")
    st = qgw.State(plan, flat(w["H_R"]), flat(w["V_R"]), n_target=w["n_target"], mixing=mixing)
    st.init_g0()
    st.iterate(warmup)
    st.init_g0()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, _, _ = st.iterate(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the per-step breakdown: the same iterations again, every step timed, a12 in line
    st.init_g0()
    st.profile_select(None, in_line=True)
    st.profile(1)
    st.iterate(steps)
    torch.cuda.synchronize()
    ms_tot, iters = st.profile(0)
    st.profile_select(None, in_line=False)
    ms = 1e3 * el / max(done, 1)
    res = {"workload": name, "nodes": n_nodes, "omega_max": w["omega_max"], "iterations": done,
           "ms_per_iteration": round(ms, 4),
           "ms_by_quantity": {c: round(sum(ms_tot[s] for s in ss) / max(iters, 1), 4)
                              for c, ss in PAPER_COLUMNS.items()},
           "pair_array_GB": round(n_nodes * plan.n_b ** 2 * plan.n_k * 16 / 1e9, 3)}
    if dlr_ms:
        res["dlr_ms_per_iteration"] = round(dlr_ms, 4)
        res["mf_over_dlr"] = round(ms / dlr_ms, 2)
    st.init_g0()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = []
    for _ in range(200):
        _, dsig, mu = st.iterate(1)
        hist.append(dsig)
        if dsig <= tol:
            break
    torch.cuda.synchronize()
    res["solve"] = {"iterations": len(hist), "final_dsigma": hist[-1], "mu": mu, "mixing": mixing,
                    "time_to_solution_s": round(time.perf_counter() - t0, 5)}
    log("[bench] uniform grid %s: N = %d, %.3f ms/iteration (%s); solve %d iterations in %.4f s"
        % (name, n_nodes, ms, ("%.1fx the DLR plan" % res["mf_over_dlr"]) if dlr_ms else "", len(hist),
           res["solve"]["time_to_solution_s"]))
    st.close()
    plan.close()
    return res


def adjoint_model(r, n_o, n_b, n_k):
    """Algorithmic HBM bytes and flops of one call of each adjoint step (FP64; S_P and S_G are one pair and one
    orbital array with nodes).  Only what the adjoint must read and write once is counted."""
    sp = 16.0 * r * n_b * n_b * n_k
    sg = 16.0 * r * n_o * n_o * n_k
    so = 16.0 * n_o * n_o * n_k
    stat_p = 16.0 * n_b * n_b * n_k
    fft_flops = 5.0 * n_k * math.log2(max(n_k, 2))
    return {
        # Pbar (read once), G(tau), G(beta - tau) read, both cotangents written
        "bubble_bwd": {"bytes": sp + 4 * sg, "flops": r * n_b * n_b * (fft_flops + 16.0 * n_k)},
        # W^C read, W^C-bar written, G and Sigma-bar read, G-bar written
        "sigma_bwd": {"bytes": 2 * sp + 3 * sg, "flops": 2 * r * n_b * n_b * (fft_flops + 8.0 * n_k)},
        # P and W-bar read, P-bar written; per matrix V P, the inverse and five products of N_b^3 complex MACs
        "dyson_W_bwd": {"bytes": 3 * sp + 2 * stat_p, "flops": 7 * 8.0 * n_b ** 3 * r * n_k},
        "dlr_transform_pairs_bwd": {"bytes": 2 * sp, "flops": 8.0 * r * r * n_b * n_b * n_k},
        "dlr_transform_bwd": {"bytes": 2 * sg, "flops": 8.0 * r * r * n_o * n_o * n_k},
        "lattice_fft_bwd": {"bytes": 2 * sg, "flops": r * n_o * n_o * fft_flops},
        # G-bar, Sigma, H read, Sigma-bar written (the implicit-mu pass rereads and rewrites it)
        "dyson_G_bwd": {"bytes": 5 * sg + so, "flops": 0.0},
        "hartree_fock_bwd": {"bytes": 2 * stat_p + 4 * so, "flops": 0.0},
        "energy_bwd": {"bytes": 6 * sg, "flops": 8.0 * r * r * n_o * n_o * n_k},
    }


class _CallTimer:
    """HIP events on torch's current stream (the stream every library call here is queued on) around each call of
    the wrapped plan methods; durations are read after the timed region's final synchronisation."""

    def __init__(self, torch, plan, names):
        self.torch, self.plan, self.names = torch, plan, names
        self.pending = {n: [] for n in names}
        self.orig = {n: getattr(plan, n) for n in names}
        for n in names:
            setattr(plan, n, self._wrap(n, self.orig[n]))

    def _wrap(self, name, f):
        def g(*a, **k):
            e0 = self.torch.cuda.Event(enable_timing=True)
            e1 = self.torch.cuda.Event(enable_timing=True)
            e0.record()
            r = f(*a, **k)
            e1.record()
            self.pending[name].append((e0, e1))
            return r
        return g

    def reset(self):
        for n in self.names:
            self.pending[n] = []

    def totals(self):
        return {n: (sum(a.elapsed_time(b) for a, b in v), len(v)) for n, v in self.pending.items() if v}

    def close(self):
        for n in self.names:
            setattr(self.plan, n, self.orig[n])


def adjoint_leg(torch, qgw, steps, warmup=1):
    """The five-orbital model at 48 x 48, beta = 100 (r = 59), benchmark interaction: one GW iteration from G0
    through the autograd layer with per-iteration checkpointing, then the backward pass of
    L = Re sum conj(C) Sigma^C(k, i w_0) + E (w_0 = pi / beta, C seeded), i.e. the gradients of Sigma(k, i w_0) and of
    the total energy with respect to H0(R) and V(R) (through them the hoppings, U, J and V).  HIP events time the
    whole forward + backward and each adjoint call."""
    from paper_2604_22223_amd import autograd as qa
    from paper_2604_22223_amd import workloads as wl
    w = wl.workload("five_orbital_48")
    nodes = qgw.dlr_build(w["beta"] * w["omega_max"], w["eps"])
    nodes["omega"] = nodes["x"] / w["beta"]
    plan = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], nodes)
    flat = lambda x: torch.from_numpy(np.ascontiguousarray(x.reshape(x.shape[:-2] + (-1,)))).to("cuda:0")
    m0 = int(np.nonzero(nodes["n_f"] == 0)[0][0])
    rng = np.random.default_rng(48)
    shp = (plan.n_o, plan.n_o, plan.n_k)
    cs = torch.from_numpy(rng.standard_normal(shp) + 1j * rng.standard_normal(shp)).to("cuda:0")
    H0, V0 = flat(w["H_R"]), flat(w["V_R"])

    def step():
        H_R = H0.clone().requires_grad_(True)
        V_R = V0.clone().requires_grad_(True)
        G, mu, Siw, shf = qa.run(plan, H_R, V_R, w["n_target"], n_iter=1, checkpointed=True)[-1]
        H_k = qa.FFT.apply(plan, qgw.R_TO_K, H_R)
        loss = (cs.conj() * Siw[m0]).real.sum() + qa.energy(plan, H_k, shf, Siw, G).to(cs.device)
        loss.backward()
        return H_R.grad, V_R.grad

    names = sorted(adjoint_model(1, 1, 1, 1))
    timer = _CallTimer(torch, plan, names)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    timer.reset()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        gh, gv = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    tot = timer.totals()
    timer.close()
    model = adjoint_model(plan.r, plan.n_o, plan.n_b, plan.n_k)
    calls = {}
    for n, (t, c) in tot.items():
        per = t / c
        e = model[n]
        b = bound_of(e, "f64")
        calls[n] = dict(roof(e, "f64", per), calls_per_step=c // steps,
                        per_call={"bytes": e["bytes"], "flops": e["flops"]})
        log("[bench]   adjoint %-24s %8.4f ms x %d per step  %-3s %9.2f %-7s (%.1f%% of peak)"
            % (n, per, c // steps, b, calls[n]["achieved"], calls[n]["unit"], 100 * calls[n]["frac"]))
    res = {"workload": "five_orbital_48", "mesh": "48x48", "beta": w["beta"], "dlr_rank": plan.r,
           "U": w["interaction"]["U"], "J": w["interaction"]["J"], "V_nn": w["interaction"]["V_nn"],
           "steps": steps, "ms_per_forward_backward": round(ms, 4),
           "adjoint_ms_per_step": round(sum(t for t, _ in tot.values()) / steps, 4),
           "loss": "Re sum conj(C) Sigma^C(k, i pi/beta) + E_GM, gradients in H0(R) and V(R)",
           "grad_norms": {"H_R": float(gh.abs().max()), "V_R": float(gv.abs().max())},
           "calls": calls}
    log("[bench] adjoint leg 48x48: %.3f ms per forward + backward (%.3f ms in adjoint calls)"
        % (ms, res["adjoint_ms_per_step"]))
    plan.close()
    return res


def batch_leg(torch, qgw, count, launches, warmup, mu_steps, solve_replays=100):
    """Seeded instances of uneven size (1-5 orbitals, 12^2-48^2 meshes, beta 10-100) advanced by one
    graph launch per iteration, FP64 and FP32 bulk steps, against the same states iterated one by one."""
    from paper_2604_22223_amd import workloads as wl
    t0 = time.perf_counter()
    ws = wl.batch_sweep(count)
    plans, states, n_f, t_tune = [], [], [], 0.0
    flat = lambda x: torch.from_numpy(np.ascontiguousarray(x.reshape(x.shape[:-2] + (-1,)))).to("cuda:0")
    for w in ws:
        nodes = qgw.dlr_build(w["beta"] * w["omega_max"], w["eps"])
        nodes["omega"] = nodes["x"] / w["beta"]
        n_f.append(nodes["n_f"])
        pl = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], nodes)
        t1 = time.perf_counter()
        pl.autotune()
        t_tune += time.perf_counter() - t1
        # linear mixing 0.5: at U up to 6 eV many sweep instances oscillate undamped, so that the solves of the
        # batch reach a fixed point (the per-sweep rates do not depend on it)
        st = qgw.State(pl, flat(w["H_R"]), flat(w["V_R"]), n_target=w["n_target"], mixing=0.5)
        st.init_g0()
        plans.append(pl)
        states.append(st)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    log("[bench] batch: %d instances built in %.1f s (autotuning %.1f s)" % (count, setup, t_tune))
    res = {"instances": count, "launches": launches, "setup_s": round(setup, 2), "autotune_s": round(t_tune, 2),
           "mu_steps_per_iteration": mu_steps,
           "recipe": "workloads.batch_sweep(%d): n_o 1-5, meshes 12^2-48^2, beta 10-100/eV, U 1-6 eV; mixing 0.5"
                     % count,
           "legs": "each leg restarts every instance from G0 and times iterations 2 .. launches + 1 (one untimed)"}

    def restart():
        for st in states:
            st.set_precision(0)
            st.init_g0()
        torch.cuda.synchronize()

    # one by one (eager), FP64
    restart()
    for st in states:
        st.iterate(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = 0
    for _ in range(launches):
        for st in states:
            st.iterate(1)
            evals = max(evals, st.mu_evals())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res["eager_fp64"] = {"instance_iterations_per_s": round(count * launches / el, 2), "s_per_sweep": round(el / launches, 5),
                         "max_mu_evaluations": int(evals)}
    log("[bench] batch eager FP64: %.4f s per sweep of %d instances" % (el / launches, count))
    # GPU time of the steps alone: one more sweep per precision with every state's step events on, summed over the
    # instances (each instance's kernels back to back with no host gaps; the floor of any launch scheme that does not
    # run two instances' kernels at once)
    for key, mode in (("fp64", 0), ("fp32", 2)):
        for st in states:
            st.set_precision(mode)
            st.profile_select(None, in_line=True)      # a12 in line: every step's time is its own
            st.profile(1)
            st.iterate(1)
        torch.cuda.synchronize()
        tot = 0.0
        for st in states:
            ms, _ = st.profile(2)
            tot += sum(ms.values())
            st.profile(0)
            st.profile_select(None, in_line=False)
        res["step_time_sum_%s_s_per_sweep" % key] = round(tot / 1e3, 5)
    log("[bench] batch: summed step time per sweep %.4f s (FP64), %.4f s (FP32)"
        % (res["step_time_sum_fp64_s_per_sweep"], res["step_time_sum_fp32_s_per_sweep"]))
    labels = {"graph_fp64": "FP64 iterations", "graph_fp32": "single-precision bulk steps a1-a11 in every iteration "
              "(the FP32 phase of the mixed schedule, without its FP64 finish: not a refined end point)"}
    for name, prec in (("graph_fp64", qgw.F64), ("graph_fp32", qgw.F32)):
        restart()
        b = qgw.Batch(states, precision=prec, n_iter=1, mu_steps=mu_steps)
        for _ in range(warmup):
            b.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(launches):
            b.launch()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ds, mu, status, evs = b.read(with_evals=True)
        res[name] = {"instance_iterations_per_s": round(count * launches / el, 2), "s_per_sweep": round(el / launches, 5),
                     "unconverged_mu_searches": int(np.count_nonzero(status)), "max_mu_evaluations": int(evs.max()),
                     "arithmetic": labels[name]}
        log("[bench] batch %s: %.4f s per sweep (%d unconverged mu searches, at most %d evaluations)"
            % (name, el / launches, int(np.count_nonzero(status)), int(evs.max())))
        b.close()
    # solves to the tolerance from G0: FP64 replays alone, and the mixed schedule (FP32 replays until every
    # instance is at the switch tolerance or stalled, then FP64 replays); per instance the time at which its
    # max |Delta Sigma| first met the tolerance after an FP64 replay
    tol = _TOL[0]
    if solve_replays <= 0:  # (a profiling run of the sweep alone)
        for st in states:
            st.close()
        res["backward"] = batch_backward(torch, qgw, plans, ws, n_f, launches)
        for pl in plans:
            pl.close()
        return res
    b64 = qgw.Batch(states, precision=qgw.F64, n_iter=1, mu_steps=mu_steps)
    b32 = qgw.Batch(states, precision=qgw.F32, n_iter=1, mu_steps=mu_steps)
    runs = {}
    for name, kw in (("solve_fp64", {}), ("solve_mixed", {"b32": b32, "switch_tol": switch_tol()})):
        restart()
        runs[name] = qgw.batch_solve(b64, tol, max_replays=solve_replays, **kw)
    b32.close()
    b64.close()
    both = np.ones(count, dtype=bool)
    for r in runs.values():
        both &= r["fp64_replays_to_tol"] >= 0
    for name, r in runs.items():
        conv = r["fp64_replays_to_tol"] >= 0
        t = r["seconds_to_tol"][both]
        res[name] = {"tol": tol, "converged_instances": int(conv.sum()), "fp32_replays": int(r["fp32_replays"]),
                     "fp64_replays": int(r["fp64_replays"]), "failed_searches": int(np.count_nonzero(r["status"])),
                     "instances_converged_in_both_solves": int(both.sum()),
                     "median_s_to_tol_over_those": round(float(np.median(t)), 4) if both.any() else None,
                     "s_until_the_last_of_those": round(float(t.max()), 4) if both.any() else None}
        log("[bench] batch %s: %d of %d instances at |dSigma| <= %.0e (%d FP32 + %d FP64 replays); over the %d "
            "converged in both solves: median %s s, last %s s"
            % (name, int(conv.sum()), count, tol, r["fp32_replays"], r["fp64_replays"], int(both.sum()),
               res[name]["median_s_to_tol_over_those"], res[name]["s_until_the_last_of_those"]))
    for st in states:
        st.close()
    res["backward"] = batch_backward(torch, qgw, plans, ws, n_f, launches)
    for pl in plans:
        pl.close()
    return res


def batch_backward(torch, qgw, plans, ws, n_f, launches, nstreams=4):
    """The sweep's backward: per instance one GW iteration from G0 through the autograd layer (no checkpointing), loss
    Re sum conj(C) Sigma^C(k, i w_0) with a seeded C, gradients in H0(R) and V(R).  The instances are dealt to four
    streams by estimated work, as in the forward graph.  The backward of all instances is timed as eager autograd (one call per
    stream) and as one captured graph; the graph's gradients must equal the eager ones."""
    from paper_2604_22223_amd import autograd as qa
    rng = np.random.default_rng(64)
    flat = lambda x: torch.from_numpy(np.ascontiguousarray(x.reshape(x.shape[:-2] + (-1,)))).to("cuda:0")
    groups = [(torch.cuda.Stream(), []) for _ in range(nstreams)]
    # instances to streams by longest estimated work first, with the per-iteration estimate the batch graph uses
    # (Dyson W ~ N_k r N_b^3, pair maps ~ N_k N_b^2 r^2, bubble and self-energy ~ N_k N_b^2 r; ns)
    cost = [pl.n_k * pl.r * (0.8e-3 * pl.n_b ** 3 + 1.5 + 4.5e-4 * pl.n_b ** 2 * pl.r + 0.0105 * pl.n_b ** 2) + 1e5
            for pl in plans]
    load, stream_of = [0.0] * nstreams, [0] * len(plans)
    for i in sorted(range(len(plans)), key=lambda k: -cost[k]):
        k = load.index(min(load))
        stream_of[i] = k
        load[k] += cost[i]
    leaves = []
    t0 = time.perf_counter()
    for i, (pl, w, nf) in enumerate(zip(plans, ws, n_f)):
        s, losses = groups[stream_of[i]]
        with torch.cuda.stream(s):
            H = flat(w["H_R"]).requires_grad_(True)
            V = flat(w["V_R"]).requires_grad_(True)
            G, mu, Siw, shf = qa.run(pl, H, V, w["n_target"], n_iter=1, checkpointed=False)[-1]
            m0 = int(np.nonzero(np.asarray(nf) == 0)[0][0])
            shp = tuple(Siw[m0].shape)
            C = torch.from_numpy(rng.standard_normal(shp) + 1j * rng.standard_normal(shp)).to("cuda:0")
            losses.append((C.conj() * Siw[m0]).real.sum())
        leaves.append((H, V))
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0

    def eager():
        for H, V in leaves:
            H.grad, V.grad = None, None
        for s, losses in groups:
            with torch.cuda.stream(s):
                torch.autograd.backward(losses, retain_graph=True)

    eager()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(launches):
        eager()
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / launches
    ref = [(H.grad.clone(), V.grad.clone()) for H, V in leaves]
    for H, V in leaves:
        H.grad, V.grad = None, None
    g = qa.backward_graph(groups)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(launches):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / launches
    diff = 0.0
    for (H, V), (rh, rv) in zip(leaves, ref):
        for a, b in ((H.grad, rh), (V.grad, rv)):
            diff = max(diff, float((a - b).abs().max()) / max(float(b.abs().max()), 1e-300))
    del g
    res = {"loss": "Re sum conj(C) Sigma^C(k, i pi/beta) after one iteration from G0; gradients in H0(R) and V(R)",
           "streams": nstreams, "forward_s": round(t_fwd, 4), "eager_backward_s_per_sweep": round(t_eager, 5),
           "graph_backward_s_per_sweep": round(t_graph, 5), "graph_vs_eager_max_rel_diff": diff}
    log("[bench] batch backward: forward of %d instances (autograd, one iteration from G0) %.3f s; backward per "
        "sweep %.4f s eager, %.4f s as one graph on %d streams (max rel. difference %.1e)"
        % (len(plans), t_fwd, t_eager, t_graph, nstreams, diff))
    return res

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--batch", type=int, default=64, metavar="N",
                    help="instances of the batched leg (0 skips it)")
    ap.add_argument("--batch-launches", type=int, default=5)
    ap.add_argument("--mf-steps", type=int, default=10, metavar="K",
                    help="timed iterations of the uniform-Matsubara-grid plans (0 skips them)")
    ap.add_argument("--paper-steps", type=int, default=20, metavar="K",
                    help="timed iterations of the paper's 8x8x8 five-orbital workload per schedule (0 skips it)")
    ap.add_argument("--batch-mu-steps", type=int, default=64)
    ap.add_argument("--batch-solve-replays", type=int, default=100, metavar="K",
                    help="replays per batched solve to the tolerance (0 skips the solves)")
    ap.add_argument("--adjoint-steps", type=int, default=3, metavar="K",
                    help="timed forward + backward steps of the 48x48 adjoint leg (0 skips it)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-MiB device buffer three times (a plain copy kernel of known size "
                         "that scales the HBM byte counters of a profiler run)")
    a = ap.parse_args()
    _TOL[0] = a.tol
    if a.gpus != 1:
        print("bench.py measures one GPU: the GW iteration here runs on a single MI355X "
              "(multi-GPU sharding is a design note only); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_22223_amd import qgw

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if a.copy_calibration > 0:
        src = torch.ones(a.copy_calibration << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 copies of %d MiB" % a.copy_calibration)
        del src, dst
    w = make_workload()
    lam = w["beta"] * w["omega_max"]
    t0 = time.perf_counter()
    nodes = qgw.dlr_build(lam, w["eps"])
    nodes["omega"] = nodes["x"] / w["beta"]
    n = w["mesh"][0]
    plan = qgw.Plan.from_nodes(n, w["site_norb"], w["beta"], nodes)
    flat = lambda x: torch.from_numpy(np.ascontiguousarray(x.reshape(x.shape[:-2] + (-1,)))).to(dev)
    H_R, V_R = flat(w["H_R"]), flat(w["V_R"])
    setup_s = time.perf_counter() - t0
    log("[bench] plan: r=%d n_o=%d N_b=%d N_k=%d (setup %.2fs)" % (plan.r, plan.n_o, plan.n_b, plan.n_k, setup_s))
    st = qgw.State(plan, H_R, V_R, n_target=w["n_target"])

    # self-consistent solves from G0 to the tolerance under both schedules
    solves = {}
    for name, mode in (("fp64", 0), ("mixed", 1)):
        solve(st, mode, a.tol)                 # first solve: warm caches and code paths
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist, mu = solve(st, mode, a.tol)
        torch.cuda.synchronize()
        tts = time.perf_counter() - t0
        sig = st.array(1).cpu().numpy()
        n32 = sum(1 for _, p, _ in hist if p == 1)
        solves[name] = {"iterations": len(hist), "fp32_iterations": n32, "time_to_solution_s": round(tts, 6),
                        "final_dsigma": hist[-1][0], "converged": bool(hist[-1][0] <= a.tol), "mu": mu, "sigma": sig,
                        "mu_evaluations_per_iteration": [int(e) for _, _, e in hist]}
        log("[bench] %-5s solve from G0: %d iterations (%d FP32) to |dSigma| = %.2e in %.4f s, mu = %.10f"
            % (name, len(hist), n32, hist[-1][0], tts, mu))
    sig_diff = float(np.max(np.abs(solves["mixed"]["sigma"] - solves["fp64"]["sigma"])))
    log("[bench] max |Sigma_mixed - Sigma_fp64| at convergence: %.2e" % sig_diff)
    for v in solves.values():
        del v["sigma"]

    # per-step breakdown of the chosen schedule: a pass of its own (same length), with a12 on the caller's stream
    # ahead of a1 so that every step's time is its own
    timed_solves(torch, st, 1, a.tol, a.warmup)
    st.profile_select(None, in_line=True)
    st.profile(1)
    el_detail = timed_solves(torch, st, 1, a.tol, a.steps)
    detail = st.profile(0, per_precision=True)
    log("[bench] step breakdown pass (every step timed, a12 in line): %.3f ms/iteration" % (1e3 * el_detail / a.steps))
    steps, totals = {}, {}
    for prec in ("f64", "f32"):
        ms_tot, iters = detail[prec]
        if iters == 0:
            continue
        model = step_model(plan.r, plan.n_o, plan.n_b, plan.n_k, prec)
        for name, tot in ms_tot.items():
            key = "%s:%s" % (name, prec)
            kprec = "f64" if name in FP64_STEPS else prec
            steps[key] = dict(roof(model[name], kprec, tot / iters), iterations=iters)
            steps[key]["per_launch"] = {"bytes": model[name]["bytes"], "flops": model[name]["flops"]}
            steps[key]["traffic"] = MEASURED_TRAFFIC.get(key)
            totals[key] = tot
            log("[bench]   %-22s %8.4f ms x %3d  %-3s %9.2f %-7s (%.1f%% of peak)"
                % (key, tot / iters, iters, steps[key]["bound"], steps[key]["achieved"], steps[key]["unit"],
                   100 * steps[key]["frac"]))
    dom = max(totals, key=totals.get)
    dom_step, dom_prec = dom.split(":")

    # plain FP64 and chosen (mixed) schedules: W untimed, then exactly K timed iterations each, with HIP events
    # around the dominant step only (two per iteration)
    timed = {}
    for name, mode in (("fp64", 0), ("mixed", 1)):
        timed_solves(torch, st, mode, a.tol, a.warmup)
        st.profile_select([dom_step], in_line=False)
        st.profile(1)
        el = timed_solves(torch, st, mode, a.tol, a.steps)
        timed[name] = {"elapsed": el, "prof": st.profile(0, per_precision=True)}
        log("[bench] %-5s: %d timed iterations in %.4f s: %.3f ms/iteration, %.1f iterations/s"
            % (name, a.steps, el, 1e3 * el / a.steps, a.steps / el))
    st.profile_select(None, in_line=False)
    value = a.steps / timed["mixed"]["elapsed"]
    ms_per_step = 1e3 * timed["mixed"]["elapsed"] / a.steps
    value64 = a.steps / timed["fp64"]["elapsed"]

    # the dominant kernel's roofline from the events inside the chosen schedule's timed region
    ms_tot, iters = timed["mixed"]["prof"][dom_prec]
    model = step_model(plan.r, plan.n_o, plan.n_b, plan.n_k, dom_prec)
    kprec = "f64" if dom_step in FP64_STEPS else dom_prec
    dd = roof(model[dom_step], kprec, ms_tot[dom_step] / iters)
    log("[bench] dominant step %s: %.4f ms x %d in the timed region (%.4f ms in the breakdown pass)"
        % (dom, dd["ms"], iters, steps[dom]["ms"]))
    roofline = {"bound": dd["bound"], "achieved": dd["achieved"], "peak": dd["peak"], "unit": dd["unit"],
                "frac": dd["frac"], "traffic": MEASURED_TRAFFIC.get(dom), "kernel": dom,
                "per_launch": {"bytes": model[dom_step]["bytes"], "flops": model[dom_step]["flops"], "ms": dd["ms"],
                               "launches_timed": iters}}

    _, mu_conv = solve(st, 1, a.tol)           # a converged state for the post-processing leg
    qpl = quasiparticle_leg(torch, qgw, plan, st, H_R, mu_conv)
    log("[bench] quasiparticle post-processing: %.4f ms per call, Z in [%.4f, %.4f]"
        % (qpl["ms_per_call"], qpl["z_min"], qpl["z_max"]))

    hfl = hf_leg(torch, qgw, plan, H_R, V_R, w["n_target"])
    log("[bench] Hartree-Fock solve: %d passes to |dSigma_HF| = %.1e in %.4f s (%.0f passes/s)"
        % (hfl["passes"], hfl["final_dsigma_hf"], hfl["time_to_solution_s"], hfl["passes_per_s"]))

    paper = None
    if a.paper_steps > 0:
        paper = paper_workload_leg(torch, qgw, a.paper_steps, a.tol)
    mf = None
    if a.mf_steps > 0:
        from paper_2604_22223_amd import workloads as wl
        mf = [mf_leg(torch, qgw, w, a.mf_steps, a.tol, dlr_ms=1e3 * timed["fp64"]["elapsed"] / a.steps,
                     name=WORKLOAD)]
        if paper is not None:
            mf.append(mf_leg(torch, qgw, wl.workload("cubic_five_orbital_8"), a.mf_steps, a.tol, mixing=0.5,
                             dlr_ms=paper["fp64"]["ms_per_iteration"], name="cubic_five_orbital_8"))
    batch = (batch_leg(torch, qgw, a.batch, a.batch_launches, 1, a.batch_mu_steps, a.batch_solve_replays)
             if a.batch > 0 else None)
    adjoint = adjoint_leg(torch, qgw, a.adjoint_steps) if a.adjoint_steps > 0 else None

    cpu = None
    if not a.no_cpu_baseline:
        log("[bench] CPU baseline: oracle iterations on the host ...")
        cpu = cpu_baseline(w)
        log("[bench] CPU baseline: %.4f iterations/s" % cpu["value"])

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GW iterations/sec", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic (seeded five-orbital model)",
        "config": {"workload": WORKLOAD, "mesh": "24x24", "n_orb": plan.n_o, "n_pair": plan.n_b,
                   "beta": w["beta"], "omega_max": w["omega_max"], "dlr_eps": w["eps"], "dlr_rank": plan.r,
                   "U": w["interaction"]["U"], "J": w["interaction"]["J"], "V_nn": w["interaction"]["V_nn"],
                   "filling": w["n_target"], "tol": a.tol,
                   "path": "chosen: FP32 a1-a11 while |dSigma| > %g and falling, then FP64" % switch_tol(),
                   "timed_work": "back-to-back self-consistent solves from G0 to |dSigma| <= tol"},
        "plain_fp64": {"value": round(value64, 3), "ms_per_step": round(1e3 * timed["fp64"]["elapsed"] / a.steps, 4)},
        "chosen_vs_fp64": round(value / value64, 4),
        "solves": solves,
        "time_to_solution_fp64_over_chosen": round(solves["fp64"]["time_to_solution_s"]
                                                   / solves["mixed"]["time_to_solution_s"], 4),
        "sigma_diff_chosen_vs_fp64": sig_diff,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batch": batch,
        "adjoint": adjoint,
        "quasiparticle": qpl,
        "hartree_fock": hfl,
        "paper_workload": paper,
        "uniform_grid": mf,
        "steps_detail": steps,
        "steps_detail_pass": {"iterations": a.steps, "schedule": "chosen", "a12": "in line (caller's stream)",
                              "ms_per_iteration": round(1e3 * el_detail / a.steps, 4)},
    }
    print(json.dumps(out), flush=True)
    st.close()
    plan.close()


if __name__ == "__main__":
    main()
