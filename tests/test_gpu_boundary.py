"""The C-ABI boundary: caller-provided scratch, the device status word, non-finite
self-energies, restarts after a failed iteration, and graph capture of the
adjoint calls on their first use.

* qgw_workspace_size reports each call's scratch; a call given less (or none)
  is refused before anything is queued.
* A Dyson-W system I - V P with an exact zero pivot (Eq. eq-screened-coulomb
  has no solution there) raises QGW_ERR_SINGULAR through qgw_sync_status,
  in the 1 x 1 kernel and the 25 x 25 kernel, FP64 and FP32; the other
  matrices of the same call are the plain solve (numpy reference).
* A NaN in the model reaches Sigma; the iteration reports it instead of a
  finite max |Delta Sigma|, and the state refuses further iterations until it
  is restarted.
* The adjoint calls allocate nothing, so a chain of them captured into a HIP
  graph on the plan's first use replays to the eager result (every replay,
  with eager work and synchronisation between replays).
"""
import numpy as np
import pytest

from conftest import rel_err
from oracle import gw
from oracle.dlr import DLR
from paper_2604_22223_amd import qgw
from paper_2604_22223_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(x, dtype=np.complex128):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def flat(x):
    return np.ascontiguousarray(x.reshape(x.shape[:-2] + (-1,)))


def crand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _plan(n, site_norb, precision=qgw.F64, beta=10.0, omega_max=20.0, eps=1e-10):
    d = DLR(beta, omega_max, eps)
    return d, qgw.Plan.from_nodes(n, site_norb, beta, d.nodes(), precision=precision)


def test_workspace_sizes_and_refusals():
    torch = _torch()
    d, p = _plan(6, [5])
    r, no, nb, nk = p.r, p.n_o, p.n_b, p.n_k
    so, se = no * no * nk * 16, no * nk * 8
    expect = {qgw.OP_SIGMA_BWD: r * so, qgw.OP_DYSON_W_BWD: (2 * r + min(r, 8)) * nb * nb * nk * 16,
              qgw.OP_HARTREE_FOCK_BWD: nb * nb * 16, qgw.OP_ENERGY: 2 * so + r * so + 2 * 4096 * 8 + 64,
              qgw.OP_ENERGY_BWD: 2 * so + 2 * r * so, qgw.OP_HF_DENSITY: so + se + 64 * 8,
              qgw.OP_QUASIPARTICLE: 64}
    for op, b in expect.items():
        assert p.workspace_size(op) == b, (op, p.workspace_size(op), b)
    with pytest.raises(qgw.QGWError) as e:
        p.workspace_size(99)
    assert e.value.status == qgw.QGW_ERR_INVALID_ARG
    rng = np.random.default_rng(1)
    gt = dev(crand(rng, (r, no, no, nk)))
    wc = dev(crand(rng, (r, nb, nb, nk)))
    sb = dev(crand(rng, (r, no, no, nk)))
    a, b = torch.empty_like(gt), torch.empty_like(wc)
    small = torch.empty(expect[qgw.OP_SIGMA_BWD] - 16, dtype=torch.uint8, device="cuda:0")
    for ws in (small, None):
        with pytest.raises(qgw.QGWError) as e:
            qgw._check(qgw.lib().qgw_sigma_bwd(p.handle, qgw._ptr(gt), qgw._ptr(wc), 1, qgw._ptr(sb), qgw._ptr(a),
                                               qgw._ptr(b), qgw._ptr(ws), qgw._nbytes(ws), qgw._stream()))
        assert e.value.status == qgw.QGW_ERR_INVALID_ARG
    # out_k = 0 needs no scratch; the exact size is accepted
    p.sigma_bwd(gt, wc, sb, a, b, out_k=False, workspace=None)
    p.sigma_bwd(gt, wc, sb, a, b, out_k=True, workspace=p.workspace(qgw.OP_SIGMA_BWD))
    torch.cuda.synchronize()
    p.close()


def _dyson_ref(vq, pnu, mask):
    """W^C = (I - V P)^{-1} V - V (numpy solve) at the (node, q) where mask is set; vq [N_k, A, B],
    pnu [r, N_k, A, B]; returns the selected matrices."""
    nb = vq.shape[-1]
    v = np.broadcast_to(vq[None], pnu.shape)[mask]
    a = np.eye(nb) - v @ pnu[mask]
    return np.linalg.solve(a, v) - v


@pytest.mark.parametrize("site_norb", [[1], [3], [4], [5]])
@pytest.mark.parametrize("precision", [qgw.F64, qgw.F32])
def test_singular_dyson_w_sets_status(site_norb, precision):
    """One (node, q) matrix has V(q) = I and P = I, so I - V P = 0 exactly (every pivot is zero): the call sets
    the device status word; the other matrices match the numpy solve; reading the word clears it."""
    torch = _torch()
    d, p = _plan(4, site_norb, precision)
    r, nb, nk = p.r, p.n_b, p.n_k
    rng = np.random.default_rng(2)
    v = crand(rng, (nk, nb, nb))
    vq = 0.5 * (v + np.conj(np.swapaxes(v, 1, 2)))
    pnu = 0.05 * crand(rng, (r, nk, nb, nb))
    q0, m0 = 3, r // 2
    vq[q0] = np.eye(nb)
    pnu[m0, q0] = np.eye(nb)
    cdt = np.complex128 if precision == qgw.F64 else np.complex64
    vq_d, pnu_d = dev(vq, cdt), dev(pnu, cdt)
    out = torch.empty_like(pnu_d)
    p.sync_status()                               # a fresh plan has a clear word
    print("\n[boundary] singular Dyson W, N_b = %d, precision %d" % (nb, precision), flush=True)
    p.dyson_W(vq_d, pnu_d, out)
    with pytest.raises(qgw.QGWError) as e:
        p.sync_status()
    assert e.value.status == qgw.QGW_ERR_SINGULAR
    p.sync_status()                               # cleared by the read
    w = host(out).astype(np.complex128)
    assert not np.all(np.isfinite(w[m0, q0]))
    mask = np.ones((r, nk), dtype=bool)
    mask[m0, q0] = False
    ref = _dyson_ref(vq, pnu, mask)
    # rounding bar of a partially pivoted solve: a few N_b cond(I - V P) units of the precision
    v = np.broadcast_to(vq[None], pnu.shape)[mask]
    cond = float(np.linalg.cond(np.eye(nb) - v @ pnu[mask]).max())
    unit = 2.0 ** -53 if precision == qgw.F64 else 2.0 ** -24
    tol = 4.0 * nb * cond * unit
    # W^C = W - V: the difference is measured against the larger of |W^C| and |V| (the cancellation in W - V)
    err = float(np.abs(w[mask] - ref).max()) / max(float(np.abs(ref).max()), float(np.abs(v).max()))
    assert err < tol, (err, tol, cond)
    # a regular call leaves the word clear
    pnu[m0, q0] = 0.0
    p.dyson_W(vq_d, dev(pnu, cdt), out)
    p.sync_status()
    p.close()


def test_nan_in_model_is_reported_and_state_needs_restart():
    """A NaN in one hopping entry spreads through G into Sigma.  The fixed-mu iteration (no chemical-potential
    search to trip over it) reports the error: max |Delta Sigma| counts the NaN as infinite, and the singular
    Dyson-W word names the first place it surfaced.  The state then refuses further iterations."""
    w = wl.random_model((4, 4), [2, 1], seed=3, beta=6.0, omega_max=12.0, eps=1e-10, U=0.7, J=0.1, Vnn=0.1)
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    p = qgw.Plan.from_nodes(4, w["site_norb"], w["beta"], d.nodes())
    h = w["H_R"].copy()
    h[0, 1, 1, 0] = np.nan
    st = qgw.State(p, dev(flat(h)), dev(flat(w["V_R"])), n_target=None)
    st.init_g0(mu=0.1)
    with pytest.raises(qgw.QGWError) as e:
        st.iterate(1)
    assert e.value.status in (qgw.QGW_ERR_NONFINITE, qgw.QGW_ERR_SINGULAR), e.value
    with pytest.raises(qgw.QGWError) as e:
        st.iterate(1)
    assert e.value.status == qgw.QGW_ERR_INVALID_ARG
    st.close()
    # the same model without the NaN iterates normally at the same mu, and a restart clears a failed state
    st = qgw.State(p, dev(flat(w["H_R"])), dev(flat(w["V_R"])), n_target=None)
    st.init_g0(mu=0.1)
    done, ds, mu = st.iterate(2)
    assert done == 2 and np.isfinite(ds) and mu == 0.1
    st.close()
    p.sync_status()
    p.close()


def _bwd_chain(p, t, ws):
    """A chain of adjoint calls on fixed inputs (t) into fixed outputs; ws: dict op -> workspace tensor."""
    p.sigma_bwd(t["gt"], t["wc"], t["sb"], t["o_g1"], t["o_wc"], out_k=True, workspace=ws[qgw.OP_SIGMA_BWD])
    p.dyson_W_bwd(t["vq"], t["pnu"], t["o_wc"], t["o_p"], t["o_v"], workspace=ws[qgw.OP_DYSON_W_BWD])
    p.hartree_fock_bwd(t["vr"], t["nr"], t["shf"], t["o_n"], t["o_vr"], workspace=ws[qgw.OP_HARTREE_FOCK_BWD])
    p.bubble_bwd(t["gt"], t["gr"], t["o_wc"], t["o_g2"], t["o_g3"])
    p.dyson_G_bwd(t["hk"], t["siw"], 0.3, t["o_g1"], t["o_s"], t["o_h"], n_target=t["n_target"], mubar=0.7)
    p.dlr_transform_bwd(qgw.F_TAU2IW, t["o_s"], t["o_g4"], hermitian=1)


def test_bwd_chain_captured_on_first_use_replays_to_eager():
    torch = _torch()
    w = wl.random_model((4, 4), [2, 1], seed=5, beta=6.0, omega_max=12.0, eps=1e-10, U=0.7, J=0.1, Vnn=0.1)
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    st = gw.initial_state(m, d)
    r, no, nb, nk = d.r, m.n_o, m.n_b, m.n_k
    rng = np.random.default_rng(9)
    t = {"gt": dev(crand(rng, (r, no, no, nk))), "gr": dev(crand(rng, (r, no, no, nk))),
         "wc": dev(crand(rng, (r, nb, nb, nk))), "sb": dev(crand(rng, (r, no, no, nk))),
         "vq": dev(np.ascontiguousarray(np.moveaxis(flat(m.V_q), -1, 0))),
         "pnu": dev(0.05 * crand(rng, (r, nk, nb, nb))), "vr": dev(flat(m.V_R)),
         "nr": dev(crand(rng, (no, no, nk))), "shf": dev(crand(rng, (no, no, nk))),
         "hk": dev(flat(m.H_k)), "siw": dev(0.1 * flat(st["sig_iw"]) + 0.01 * crand(rng, (r, no, no, nk))),
         "n_target": w["n_target"]}
    for k, like in (("o_g1", "gt"), ("o_g2", "gt"), ("o_g3", "gt"), ("o_g4", "gt"), ("o_s", "gt"),
                    ("o_wc", "wc"), ("o_n", "nr"), ("o_vr", "vr"), ("o_h", "nr")):
        t[k] = torch.zeros_like(t[like])
    t["o_p"] = torch.zeros_like(t["pnu"])
    t["o_v"] = torch.zeros_like(t["vq"])
    outs = ["o_g1", "o_g2", "o_g3", "o_g4", "o_s", "o_wc", "o_n", "o_vr", "o_h", "o_p", "o_v"]
    # eager on one plan
    pe = qgw.Plan.from_nodes(4, w["site_norb"], w["beta"], d.nodes())
    ws_e = {op: pe.workspace(op) for op in (qgw.OP_SIGMA_BWD, qgw.OP_DYSON_W_BWD, qgw.OP_HARTREE_FOCK_BWD)}
    _bwd_chain(pe, t, ws_e)
    torch.cuda.synchronize()
    ref = {k: host(t[k]).copy() for k in outs}
    assert all(np.all(np.isfinite(v)) for v in ref.values())
    # captured on a fresh plan's first use (scratch from the graph's pool)
    pc = qgw.Plan.from_nodes(4, w["site_norb"], w["beta"], d.nodes())
    for k in outs:
        t[k].zero_()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print("\n[boundary] capturing the adjoint chain", flush=True)
    with torch.cuda.graph(g):
        ws_c = {op: pc.workspace(op) for op in (qgw.OP_SIGMA_BWD, qgw.OP_DYSON_W_BWD, qgw.OP_HARTREE_FOCK_BWD)}
        _bwd_chain(pc, t, ws_c)
    for rep in range(3):
        for k in outs:
            t[k].fill_(float(rep + 1))        # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in outs:
            assert rel_err(host(t[k]), ref[k]) < 1e-14, (rep, k)
    del g
    pe.close()
    pc.close()
