"""Batched instances in one graph launch against the same instances run one by one (forward), and the
backward of every instance captured in one graph against the eager backward.

Six instances of uneven size (orbitals 1-5, product bases 1-25, 2-D meshes
5-8 and one 4 x 4 x 4 mesh, different beta and DLR rank) are started twice: one copy is iterated by
qgw_gw_iteration, the other by replaying a captured batch graph.  Every
replay is followed by eager work and a synchronisation, and every replay's
Sigma, G and mu must equal the eager ones (the graph runs the same kernels
with the same grids, so the agreement is to rounding; the bar is 1e-13).
One instance is also held against the oracle.
"""
import numpy as np
import pytest

from conftest import rel_err
from oracle import gw
from oracle.dlr import DLR
from paper_2604_22223_amd import qgw
from paper_2604_22223_amd import workloads as wl

pytestmark = pytest.mark.gpu

SPECS = [
    lambda: wl.random_model((4, 4), [2, 1], seed=3, beta=6.0, omega_max=12.0, eps=1e-10, U=0.7, J=0.1, Vnn=0.1),
    lambda: wl.five_orbital(n=6, norb=2, n_target=2.0, U=1.0, J=0.1, Vnn=0.2, beta=10.0, omega_max=20.0,
                            eps=1e-10, scale_mesh=6),
    lambda: wl.graphene(n=6, U=3.0, beta=10.0, omega_max=40.0, eps=1e-8),
    lambda: wl.five_orbital(n=5, norb=5, U=1.0, J=0.1, Vnn=0.2, beta=8.0, omega_max=25.0, eps=1e-10,
                            scale_mesh=5),
    lambda: wl.five_orbital(n=8, norb=1, n_target=1.0, U=2.0, J=0.0, Vnn=0.3, beta=20.0, omega_max=10.0,
                            eps=1e-10, scale_mesh=8),
    # a cubic mesh in the same graph
    lambda: wl.random_model_3d((4, 4, 4), [2, 1], seed=3, beta=8.0, omega_max=20.0, eps=1e-10, U=1.0, J=0.1,
                               Vnn=0.2),
]


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(x, dim=2):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x.reshape(x.shape[:-dim] + (-1,)), dtype=np.complex128)).to("cuda:0")


class Inst:
    def __init__(self, w):
        self.w = w
        self.d = DLR(w["beta"], w["omega_max"], w["eps"])
        self.dim = len(w["mesh"])
        self.plan = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], self.d.nodes(), dim=self.dim)
        self.H, self.V = dev(w["H_R"], self.dim), dev(w["V_R"], self.dim)

    def state(self):
        st = qgw.State(self.plan, self.H, self.V, n_target=self.w["n_target"])
        st.init_g0()
        return st


@pytest.fixture(scope="module")
def insts():
    print("\n[batch] building %d instances" % len(SPECS), flush=True)
    return [Inst(f()) for f in SPECS]


def _same(a, b):
    return rel_err(a.array(1).cpu().numpy(), b.array(1).cpu().numpy()) < 1e-13 and \
        rel_err(a.array(0).cpu().numpy(), b.array(0).cpu().numpy()) < 1e-13


@pytest.mark.parametrize("precision", [qgw.F64, qgw.F32])
def test_batch_replays_match_eager_iterations(insts, precision):
    torch = _torch()
    eager = [i.state() for i in insts]
    batched = [i.state() for i in insts]
    if precision == qgw.F32:
        for st in eager:
            st.set_precision(2)                 # every eager iteration in single precision
    b = qgw.Batch(batched, precision=precision, n_iter=1, mu_steps=12)
    for rep in range(3):
        print("[batch] precision %d replay %d" % (precision, rep), flush=True)
        mus = [st.iterate(1)[2] for st in eager]
        b.launch()
        ds, mu, status = b.read()
        torch.cuda.synchronize()
        assert list(status) == [0] * len(insts)
        for k, (e, s) in enumerate(zip(eager, batched)):
            assert abs(mu[k] - mus[k]) <= 1e-13 * max(1.0, abs(mus[k])), (rep, k, mu[k], mus[k])
            assert _same(e, s), (rep, k)
    b.close()
    for st in eager + batched:
        st.close()


def test_batch_with_two_iterations_per_launch(insts):
    eager = [i.state() for i in insts]
    batched = [i.state() for i in insts]
    b = qgw.Batch(batched, n_iter=2)
    for st in eager:
        st.iterate(1)
        st.iterate(1)
    b.launch()
    ds, mu, status = b.read()
    assert list(status) == [0] * len(insts)
    for e, s in zip(eager, batched):
        assert _same(e, s)
    b.close()
    for st in eager + batched:
        st.close()


def test_batch_instance_against_oracle(insts):
    """The multi-orbital instance after one batched iteration, at the FP64 parity bar."""
    inst = insts[3]
    w, d = inst.w, inst.d
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    ref = gw.gw_iteration(m, d, gw.initial_state(m, d))
    st = inst.state()
    b = qgw.Batch([st])
    b.launch()
    ds, mu, status = b.read()
    assert status[0] == 0
    assert abs(mu[0] - ref["mu"]) <= 1e-10 * max(1.0, abs(ref["mu"]))
    assert rel_err(st.array(1).cpu().numpy(), ref["sig_iw"].reshape(st.array(1).shape)) < 1e-10
    assert rel_err(st.array(0).cpu().numpy(), ref["G_iw"].reshape(st.array(0).shape)) < 1e-10
    b.close()
    st.close()


def test_batch_rejects_bad_arguments(insts):
    st = insts[0].state()
    with pytest.raises(qgw.QGWError):
        qgw.Batch([st, st])
    with pytest.raises(qgw.QGWError):
        qgw.Batch([st], n_iter=0)
    st.close()


def test_autotuned_plan_matches_default(insts):
    """The tuned launch shapes change only the order of some sums."""
    inst = insts[3]
    w = inst.w
    tuned = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], inst.d.nodes())
    ch = tuned.autotune()
    print("[batch] tuned shapes", ch, flush=True)
    assert ch["fft_slabs_per_block"] >= 1 and ch["bubble_slabs_per_block"] >= 1 and ch["sigma_term_lanes"] >= 1
    assert ch["orbital_map_valu"] in (0, 1)
    a = inst.state()
    b = qgw.State(tuned, inst.H, inst.V, n_target=w["n_target"])
    b.init_g0()
    for _ in range(2):
        da, _, ma = a.iterate(1)
        db, _, mb = b.iterate(1)
        assert abs(ma - mb) <= 1e-12 * max(1.0, abs(ma))
    assert rel_err(b.array(1).cpu().numpy(), a.array(1).cpu().numpy()) < 1e-12
    a.close()
    b.close()
    tuned.close()


def test_autotuned_cubic_plan_matches_default(insts):
    """The autotuner on a cubic-mesh plan (line counts of n^2 per slab) changes only the order of some sums."""
    inst = insts[5]
    w = inst.w
    tuned = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], inst.d.nodes(), dim=3)
    ch = tuned.autotune()
    print("[batch] tuned shapes (cubic)", ch, flush=True)
    a = inst.state()
    b = qgw.State(tuned, inst.H, inst.V, n_target=w["n_target"])
    b.init_g0()
    for _ in range(2):
        da, _, ma = a.iterate(1)
        db, _, mb = b.iterate(1)
        assert abs(ma - mb) <= 1e-12 * max(1.0, abs(ma))
    assert rel_err(b.array(1).cpu().numpy(), a.array(1).cpu().numpy()) < 1e-12
    a.close()
    b.close()
    tuned.close()


def test_batch_rejects_uniform_grid_states(insts):
    w = insts[0].w
    p = qgw.Plan.uniform(w["mesh"][0], w["site_norb"], w["beta"], 32)
    st = qgw.State(p, insts[0].H, insts[0].V, n_target=w["n_target"])
    with pytest.raises(qgw.QGWError) as e:
        qgw.Batch([st])
    assert e.value.status == 3
    with pytest.raises(qgw.QGWError) as e:
        p.autotune()
    assert e.value.status == 3
    st.close()
    p.close()


def test_batched_mixed_schedule_reaches_the_fixed_point(insts):
    """Solves of four 2-D instances in one batch from G0 to max |Delta Sigma| <= 1e-9: FP32 graph replays until
    every instance is at 3e-9 or stalled, then FP64 replays.  Every end point is the oracle's FP64 fixed point
    (converged to 1e-11) within the mixed schedule's 1e-6, and the FP64-only replays land on it too."""
    torch = _torch()
    sel = [insts[k] for k in (0, 1, 3, 4)]
    refs = []
    for inst in sel:
        w = inst.w
        m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
        ref, hist = gw.scf(m, inst.d, tol=1e-11, max_iter=200)
        assert hist[-1][0] <= 1e-11
        refs.append(ref)
    for mixed in (True, False):
        states = [inst.state() for inst in sel]
        b64 = qgw.Batch(states, precision=qgw.F64, n_iter=1, mu_steps=16)
        b32 = qgw.Batch(states, precision=qgw.F32, n_iter=1, mu_steps=16) if mixed else None
        print("[batch] batched solve, mixed=%s" % mixed, flush=True)
        r = qgw.batch_solve(b64, 1e-9, b32=b32, switch_tol=3e-9, max_replays=120)
        torch.cuda.synchronize()
        assert np.all(r["fp64_replays_to_tol"] >= 0), r
        assert np.all(r["status"] == 0)
        if mixed:
            assert r["fp32_replays"] >= 2
        for st, ref in zip(states, refs):
            sig = st.array(1).cpu().numpy()
            sref = ref["sig_iw"].reshape(sig.shape)
            assert np.max(np.abs(sig - sref)) <= 1e-6 * max(1.0, np.max(np.abs(sref)))
            hf = st.array(2).cpu().numpy()
            assert np.max(np.abs(hf - ref["sig_hf_k"].reshape(hf.shape))) <= 1e-6
        for b in (b64, b32):
            if b is not None:
                b.close()
        for st in states:
            st.close()


def test_backward_of_every_instance_in_one_graph(insts):
    """The adjoint chains of every instance in one captured graph.  Per instance: one GW iteration from G0 through
    the autograd layer (no checkpointing), loss Re sum conj(C) Sigma^C(k, i w_0) with a seeded C, gradients in
    H0(R) and V(R).  The instances are dealt to three streams, so the graph runs three chains side by side.  The
    eager backward gives the reference; the captured backward is replayed three times, with eager work and a
    synchronisation between replays, and every replay must give the same gradients."""
    torch = _torch()
    from paper_2604_22223_amd import autograd as qa
    rng = np.random.default_rng(17)
    streams = [torch.cuda.Stream() for _ in range(3)]
    groups = [(s, []) for s in streams]
    leaves = []
    print("\n[batch] forward of %d instances for the batched backward" % len(insts), flush=True)
    for i, inst in enumerate(insts):
        s, losses = groups[i % len(groups)]
        with torch.cuda.stream(s):
            H = inst.H.clone().requires_grad_(True)
            V = inst.V.clone().requires_grad_(True)
            G, mu, Siw, shf = qa.run(inst.plan, H, V, inst.w["n_target"], n_iter=1, checkpointed=False)[-1]
            m0 = int(np.nonzero(inst.d.nodes()["n_f"] == 0)[0][0])
            shp = tuple(Siw[m0].shape)
            C = torch.from_numpy(rng.standard_normal(shp) + 1j * rng.standard_normal(shp)).to("cuda:0")
            losses.append((C.conj() * Siw[m0]).real.sum())
        leaves.append((H, V))
    torch.cuda.synchronize()
    for s, losses in groups:
        with torch.cuda.stream(s):
            torch.autograd.backward(losses, retain_graph=True)
    torch.cuda.synchronize()
    ref = [(H.grad.cpu().numpy().copy(), V.grad.cpu().numpy().copy()) for H, V in leaves]
    for rh, rv in ref:
        assert np.all(np.isfinite(rh)) and np.all(np.isfinite(rv))
        assert np.max(np.abs(rh)) > 0 and np.max(np.abs(rv)) > 0
    for H, V in leaves:
        H.grad, V.grad = None, None
    print("[batch] capturing the backward of %d instances on %d streams" % (len(insts), len(groups)), flush=True)
    g = qa.backward_graph(groups)
    for rep in range(3):
        for H, V in leaves:
            H.grad.fill_(float(rep + 1))
            V.grad.fill_(-float(rep + 1))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, ((H, V), (rh, rv)) in enumerate(zip(leaves, ref)):
            assert rel_err(H.grad.cpu().numpy(), rh) < 1e-13, (rep, k)
            assert rel_err(V.grad.cpu().numpy(), rv) < 1e-13, (rep, k)
    del g
