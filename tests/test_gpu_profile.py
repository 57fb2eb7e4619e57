"""Step timing of the GW iteration (qgw_state_profile, qgw_state_profile_select).

Timing changes where a12 is queued (the state's second stream, or the caller's stream ahead of a1) and which
events are recorded; the kernels and their inputs stay the same, so the state after a few iterations must be
bitwise equal with and without timing, in both precisions.  A selection times its steps only.
"""
import ctypes

import numpy as np
import pytest

from paper_2604_22223_amd import qgw
from paper_2604_22223_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def flat(x):
    return np.ascontiguousarray(x.reshape(x.shape[:-2] + (-1,)))


@pytest.fixture(scope="module")
def case():
    torch = _torch()
    print("\n[profile case] five orbitals, 8 x 8, beta = 20", flush=True)
    w = wl.five_orbital(n=8, U=1.0, J=0.1, Vnn=0.2, beta=20.0, omega_max=25.0, eps=1e-10, scale_mesh=8)
    nodes = qgw.dlr_build(w["beta"] * w["omega_max"], w["eps"])
    nodes["omega"] = nodes["x"] / w["beta"]
    plan = qgw.Plan.from_nodes(8, w["site_norb"], w["beta"], nodes)
    st = qgw.State(plan, torch.from_numpy(flat(w["H_R"])).to("cuda:0"),
                   torch.from_numpy(flat(w["V_R"])).to("cuda:0"), n_target=w["n_target"])
    yield st
    st.close()
    plan.close()


def _run(st, per_call):
    """Two FP32 iterations from G0, then two FP64 ones, per_call iterations per call."""
    torch = _torch()
    st.set_precision(2, 1e-3)
    st.init_g0()
    for prec in (2, 0):
        st.set_precision(prec, 1e-3)
        for _ in range(2 // per_call):
            st.iterate(per_call)
    torch.cuda.synchronize()
    _, n32, n64 = st.info()
    return [st.array(k).cpu().numpy().copy() for k in (0, 1, 2)], (n32, n64)


@pytest.mark.parametrize("per_call", [2, 1])
def test_timing_leaves_the_iteration_bitwise_unchanged(case, per_call):
    st = case
    ref, counts = _run(st, per_call)
    assert counts == (2, 2), counts
    names = st.STEP_NAMES
    for steps, in_line in ((None, True), (["a6_dyson_w"], False), (None, False)):
        st.profile_select(steps, in_line=in_line)
        st.profile(1)
        got, c2 = _run(st, per_call)
        rows = st.profile(0, per_precision=True)
        assert c2 == counts
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (steps, in_line)
        for prec, n_it in (("f32", counts[0]), ("f64", counts[1])):
            ms, iters = rows[prec]
            assert iters == n_it
            for name in names:
                if steps is None or name in steps:
                    assert ms[name] > 0.0, (prec, name)
                else:
                    assert ms[name] == 0.0, (prec, name)
    st.profile_select(None, in_line=False)


def test_selection_is_checked(case):
    st = case
    L = qgw.lib()
    assert L.qgw_state_profile_select(st.handle, ctypes.c_uint32(1 << len(st.STEP_NAMES)), 0) != qgw.QGW_OK
    st.profile(1)
    with pytest.raises(qgw.QGWError):
        st.profile_select(["a6_dyson_w"])       # timing is on: select first, then enable
    st.profile(0)
    st.profile_select(["a13_dyson_g", "a12_density_hf"], in_line=True)
    st.profile_select(None, in_line=False)


def _solve(st, per_call, n, tol):
    """The mixed schedule from G0 (FP64 once |dSigma| <= 5e-2): n iterations, or to tol, per_call per call."""
    torch = _torch()
    st.set_precision(1, 5e-2)
    st.init_g0()
    done = 0
    while done < n:
        k, ds, _ = st.iterate(min(per_call, n - done), tol)
        done += k
        if ds <= tol and st.info()[0] == 0:
            break
    torch.cuda.synchronize()
    return [st.array(k).cpu().numpy().copy() for k in (0, 1, 2)], st.info(), done


@pytest.mark.parametrize("tol", [0.0, 1e-8])
def test_next_a1_queued_ahead_changes_nothing(case, tol):
    """Within one call each iteration queues the next one's a1 while the host waits for its search; a call of one
    iteration queues nothing ahead.  Both must give the same states bit for bit, across the FP32 -> FP64 switch
    and, with a tolerance, at the stop."""
    st = case
    one, info1, n1 = _solve(st, 1, 40, tol)
    many, info2, n2 = _solve(st, 40, 40, tol)
    assert info1 == info2 and n1 == n2, (info1, info2, n1, n2)
    assert info1[1] >= 1 and info1[2] >= 1, info1        # both precisions ran
    if tol > 0.0:
        assert n1 < 40
    for a, b in zip(one, many):
        assert np.array_equal(a, b)


def test_g0_warm_start_gives_the_same_g0(case):
    """qgw_state_init_g0 without a start begins the search at the state's previous G0 mu: the search stops at
    its first evaluation, so mu and G0 come out bit for bit as from the cold start."""
    torch = _torch()
    st = case
    st.set_precision(0)
    mu_cold = st.init_g0(0.0)
    torch.cuda.synchronize()
    g_cold = st.array(0).cpu().numpy().copy()
    for _ in range(2):
        mu_warm = st.init_g0()
        torch.cuda.synchronize()
        assert mu_warm == mu_cold
        assert np.array_equal(st.array(0).cpu().numpy(), g_cold)


@pytest.mark.parametrize("per_call", [1, 40])
def test_searches_in_several_rounds_give_the_same_states(case, per_call):
    """With one Newton evaluation queued per iteration (qgw_state_set_search_steps(1)) nearly every search
    continues in a second round after a read-back, and within a call the next iteration's a1, queued during the
    first read-back, is queued again.  The evaluations are the same as with the adaptive count, so the states are
    bit for bit the same, across the FP32 -> FP64 switch and at the stop."""
    st = case
    ref, info_ref, n_ref = _solve(st, per_call, 40, 1e-8)
    try:
        st.set_search_steps(1)
        got, info, n = _solve(st, per_call, 40, 1e-8)
    finally:
        st.set_search_steps(0)
    assert (info, n) == (info_ref, n_ref)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_search_steps_are_checked(case):
    with pytest.raises(qgw.QGWError):
        case.set_search_steps(65)
    with pytest.raises(qgw.QGWError):
        case.set_search_steps(-1)
    case.set_search_steps(0)
