"""The benchmark workloads at their full sizes, in the launch configuration
bench.py times (an untuned plan, the library's own iteration entry point).

* five_orbital_24 (the headline workload, r = 53): one GW iteration from G0
  against the oracle, every element, at the FP64 bar 1e-10; the plain FP64
  solve and the chosen one (FP32 iterations, then FP64) to |dSigma| <= 1e-6
  agree to 1e-6 (mu to 2e-6), and the oracle's iteration from the converged state changes
  Sigma by no more than the tolerance (the end point is a fixed point).
* graphene_ohno_36 (r = 63) as specified (U = 3 eV): past the charge
  instability of the bare bubble (1 - P0 V has a negative eigenvalue, so the
  first W^C has a pole on the imaginary axis and is no DLR-representable
  function); the well-posed part of the first iteration -- G0 and mu, G(tau),
  the density, Hartree-Fock, G(tau, R), the bubble in tau and i nu -- against
  the oracle at 1e-10.  The same mesh, beta and DLR with U = 1 eV, where
  1 - P0 V stays positive: one iteration at 1e-10 and the chosen solve
  confirmed as a fixed point by the oracle.
* five_orbital_24 with the stronger U = 4, J = 0.7, V = 1 eV: past the same
  bare-bubble instability (1 - P0 V has eigenvalues with negative real part),
  so again the first iteration through the bubble at 1e-10.
* five_orbital_48 (r = 59, beta = 100): one iteration against the oracle at
  1e-10.  With U = 4, J = 0.7, V = 1 eV on the same mesh, forward and adjoint:
  the gradient of a loss of Sigma, mu and the total energy with respect to
  H0(R) and V(R) along seeded directions against central differences of the
  GPU forward (1e-5 relative), a check that holds at any size.
* The 64-instance sweep: one graph launch per precision against the same
  states iterated one by one (1e-13), with every chemical-potential search
  converged, and three instances (smallest, one-orbital, largest) against the
  oracle (1e-10 FP64; 2e-4 for the single-precision bulk steps).
"""
import numpy as np
import pytest

from conftest import directional_fd, rel_err
from oracle import gw, lattice
from oracle.dlr import DLR
from paper_2604_22223_amd import qgw
from paper_2604_22223_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def flat(x):
    return np.ascontiguousarray(x.reshape(x.shape[:-2] + (-1,)))


def dev(x):
    torch = _torch()
    return torch.from_numpy(flat(np.asarray(x, dtype=np.complex128))).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


class Full:
    def __init__(self, name, w=None, keep=False, iterate=True):
        print("\n[full size] %s: oracle ..." % name, flush=True)
        self.w = w = wl.workload(name) if w is None else w
        self.d = DLR(w["beta"], w["omega_max"], w["eps"])
        self.m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
        self.st0 = gw.initial_state(self.m, self.d)
        self.st1 = gw.gw_iteration(self.m, self.d, self.st0, keep=keep) if iterate else None
        self.plan = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], self.d.nodes())
        print("[full size] %s: r = %d, N_k = %d" % (name, self.plan.r, self.plan.n_k), flush=True)

    def state(self):
        return qgw.State(self.plan, dev(self.m.H_R), dev(self.m.V_R), n_target=self.m.n_target)


def _one_iteration(c):
    """Sigma and |dSigma| are unique and compared directly.  The new chemical potential is unique only where
    N_e(mu) is not flat; where the spectrum of H0 + Sigma has a gap at the filling every mu in it is a root, so the
    library's mu is checked as a root (its filling from the oracle's density) and G is compared with the oracle's
    Dyson equation at that mu."""
    st = c.state()
    mu0 = st.init_g0()
    assert abs(mu0 - c.st0["mu"]) <= 1e-10 * max(1.0, abs(c.st0["mu"]))
    done, dsig, mu = st.iterate(1)
    ref, d, m = c.st1, c.d, c.m
    assert abs(dsig - ref["d_sigma"]) <= 1e-10 * max(1.0, ref["d_sigma"])
    assert rel_err(host(st.array(2)), flat(ref["sig_hf_k"])) < TOL
    assert rel_err(host(st.array(1)), flat(ref["sig_iw"])) < TOL
    g_at_mu = gw.dyson_G(m.H_k, ref["sig_hf_k"], ref["sig_iw"], d.iw, mu)
    assert abs(gw.electron_count(gw.density_k(g_at_mu, d)) - m.n_target) <= 1e-10
    print("[full size] mu: library %.14f, oracle bisection %.14f" % (mu, ref["mu"]), flush=True)
    assert rel_err(host(st.array(0)), flat(g_at_mu)) < TOL
    st.close()


def _solve(c, mode, tol=1e-6, max_iter=60):
    st = c.state()
    st.set_precision(mode, 1e-4)
    st.init_g0()
    for _ in range(max_iter):
        done, dsig, mu = st.iterate(1)
        if dsig <= tol and st.info()[0] == 0:
            break
    assert dsig <= tol and st.info()[0] == 0
    return st, mu


def _oracle_fixed_point(c, st, mu, tol=1e-6):
    d, m = c.d, c.m
    shape = (d.r, m.n_o, m.n_o) + m.mesh
    state = {"G_iw": host(st.array(0)).reshape(shape), "mu": mu,
             "sig_hf_k": host(st.array(2)).reshape((m.n_o, m.n_o) + m.mesh),
             "sig_iw": host(st.array(1)).reshape(shape), "iteration": 0}
    nxt = gw.gw_iteration(m, d, state)
    assert nxt["d_sigma"] <= tol, nxt["d_sigma"]


@pytest.fixture(scope="module")
def five24():
    return Full("five_orbital_24")


def test_headline_one_iteration(five24):
    _one_iteration(five24)


def test_headline_chosen_solve_reaches_fixed_point(five24):
    st64, mu64 = _solve(five24, 0)
    st32, mu32 = _solve(five24, 1)
    assert st32.info()[1] >= 2                    # the chosen schedule ran FP32 iterations
    assert np.max(np.abs(host(st64.array(1)) - host(st32.array(1)))) <= 1e-6
    assert abs(mu64 - mu32) <= 2e-6               # a shift of Sigma moves mu by as much: mu agrees to Sigma's order
    _oracle_fixed_point(five24, st32, mu32)
    st64.close()
    st32.close()


def _through_the_bubble(c):
    """The first iteration from G0 up to P(q, i nu), each step from the oracle's input to it."""
    torch = _torch()
    I, p, m = c.st1["intermediates"], c.plan, c.m
    r, nb, nk = c.d.r, m.n_b, m.n_k
    st = c.state()
    mu0 = st.init_g0()
    assert abs(mu0 - c.st0["mu"]) <= 1e-10 * max(1.0, abs(c.st0["mu"]))
    assert rel_err(host(st.array(0)), flat(c.st0["G_iw"])) < TOL
    g = st.array(0)
    out = torch.empty_like(g)
    p.dlr_transform(qgw.F_IW2TAU, g, out)
    assert rel_err(host(out), flat(I["G_tau"])) < TOL
    n_out = torch.empty_like(g[0])
    p.dlr_transform(qgw.F_IW2BETA, g, n_out, scale=-1.0, hermitian=2)
    assert rel_err(host(n_out), flat(I["n_k"])) < TOL
    hf = torch.empty_like(g[0])
    p.hartree_fock(dev(m.V_R), dev(I["n_R"]), hf)
    assert rel_err(host(hf), flat(I["sig_hf_R"])) < TOL
    gt = torch.empty_like(g)
    p.lattice_fft(qgw.K_TO_R, dev(I["G_tau"]), gt)
    assert rel_err(host(gt), flat(I["G_tau_R"])) < TOL
    pq = torch.empty((r, nb, nb, nk), dtype=torch.complex128, device="cuda:0")
    p.bubble(gt, dev(I["G_reflt_R"]), pq, out_q=True)
    assert rel_err(host(pq), flat(I["P_tau_q"])) < TOL
    p_nu = torch.empty_like(pq)
    p.dlr_transform_pairs(qgw.B_TAU2IW, qgw.LAYOUT_SLAB, qgw.LAYOUT_SLAB, dev(I["P_tau_q"]), p_nu)
    assert rel_err(host(p_nu), flat(I["P_nu_q"])) < TOL
    st.close()


def test_headline_model_with_strong_interaction_through_the_bubble():
    _through_the_bubble(Full("five_orbital_24 (U = 4)", wl.five_orbital(n=24, beta=50.0, omega_max=25.0, eps=1e-10),
                             keep=True))


def test_graphene_ohno_36_through_the_bubble():
    _through_the_bubble(Full("graphene_ohno_36", keep=True))


def test_graphene_ohno_36_weak_interaction_solve():
    c = Full("graphene_ohno_36 (U = 1)", wl.graphene(n=36, U=1.0, ohno=True, beta=40.0, omega_max=100.0, eps=1e-10))
    _one_iteration(c)
    st, mu = _solve(c, 1)
    _oracle_fixed_point(c, st, mu)
    st.close()


@pytest.fixture(scope="module")
def five48():
    return Full("five_orbital_48")


def test_five_orbital_48_one_iteration(five48):
    _one_iteration(five48)


def test_five_orbital_48_gradient_by_gpu_finite_differences():
    torch = _torch()
    from paper_2604_22223_amd import autograd as qa
    c = Full("five_orbital_48", iterate=False)
    m, p = c.m, c.plan
    rng = np.random.default_rng(48)
    shp = (c.d.r, m.n_o, m.n_o) + m.mesh
    cs = dev(rng.standard_normal(shp) + 1j * rng.standard_normal(shp))

    def loss(res, H_R):
        G, mu, Siw, shf = res
        H_k = qa.FFT.apply(p, qgw.R_TO_K, H_R)
        return (cs.conj() * Siw).real.sum() + 0.9 * mu.to(cs.device) + 1.7 * qa.energy(p, H_k, shf, Siw, G).to(cs.device)

    H_R = dev(m.H_R).requires_grad_(True)
    V_R = dev(m.V_R).requires_grad_(True)
    loss(qa.run(p, H_R, V_R, m.n_target, n_iter=1)[-1], H_R).backward()

    def L(h, v):
        with torch.no_grad():
            hh = dev(h)
            return float(loss(qa.run(p, hh, dev(v), m.n_target, n_iter=1)[-1], hh))

    def sym(x):
        x = x + np.conj(np.swapaxes(lattice.reflect(x), 0, 1))
        return x / np.linalg.norm(x)

    for name, x0, g in (("H", m.H_R, host(H_R.grad)), ("V", m.V_R, host(V_R.grad))):
        dirn = sym(rng.standard_normal(x0.shape) + 1j * rng.standard_normal(x0.shape))
        f = (lambda t: L(t, m.V_R)) if name == "H" else (lambda t: L(m.H_R, t))
        num = directional_fd(f, x0, dirn)
        ana = float(np.sum(np.conj(g) * flat(dirn)).real)
        print("[full size] 48x48 d/d%s: analytic %.10e, central differences %.10e" % (name, ana, num), flush=True)
        assert abs(num - ana) <= 1e-5 * abs(num) + 1e-9 * np.linalg.norm(g), (name, num, ana)


# sweep instances held against the oracle after one batched iteration from G0: the smallest (12 x 12, two
# orbitals), a one-orbital instance and the largest (48 x 48, five orbitals, r = 58).  Seven sweep instances start
# past the bare-bubble instability (1 - P0 V has eigenvalues with negative real part: 1, 4, 36, 45, 47, 49, 53),
# where two FP64 builds of the bosonic maps disagree far above 1e-10 (see the graphene and U = 4 cases above);
# none of the sampled three is among them.  Their searches must converge like every other instance's.
SWEEP_ORACLE_SAMPLE = (9, 42, 31)
_SWEEP_REF = {}


def _sweep_oracle(w, nodes):
    key = w["name"]
    if key not in _SWEEP_REF:
        d = DLR(w["beta"], w["omega_max"], w["eps"], nodes=nodes)
        m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
        _SWEEP_REF[key] = gw.gw_iteration(m, d, gw.initial_state(m, d))
    return _SWEEP_REF[key]


@pytest.mark.parametrize("precision", [qgw.F64, qgw.F32])
def test_batched_sweep_64(precision):
    """One graph launch of all 64 instances from G0 (the iteration with the largest chemical-potential moves:
    the Hartree shift of up to ~50 eV) against the same states iterated one by one (1e-13), every search
    converged; the oracle sample at 1e-10 (FP64) or within the FP32 iteration's 2e-4 (single-precision bulk)."""
    torch = _torch()
    ws = wl.batch_sweep(64)
    print("\n[full size] batch sweep: 64 instances, precision %d" % precision, flush=True)
    plans, eager, batched, node_sets = [], [], [], []
    for w in ws:
        nodes = qgw.dlr_build(w["beta"] * w["omega_max"], w["eps"])
        nodes["omega"] = nodes["x"] / w["beta"]
        node_sets.append(nodes)
        pl = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], nodes)
        plans.append(pl)
        for lst in (eager, batched):
            st = qgw.State(pl, dev(w["H_R"]), dev(w["V_R"]), n_target=w["n_target"])
            st.init_g0()
            lst.append(st)
    if precision == qgw.F32:
        for st in eager:
            st.set_precision(2)
    b = qgw.Batch(batched, precision=precision, n_iter=1, mu_steps=48)
    mus = []
    evals_eager = []
    for st in eager:
        mus.append(st.iterate(1)[2])
        evals_eager.append(st.mu_evals())
    b.launch()
    ds, mu, status, evals = b.read(with_evals=True)
    torch.cuda.synchronize()
    print("[full size] search evaluations: eager max %d, graph max %d; statuses %s"
          % (max(evals_eager), int(evals.max()), np.unique(status).tolist()), flush=True)
    assert int(np.count_nonzero(status)) == 0, [(k, int(status[k])) for k in np.nonzero(status)[0]]
    for k, (e, s) in enumerate(zip(eager, batched)):
        assert abs(mu[k] - mus[k]) <= 1e-13 * max(1.0, abs(mus[k])), (k, mu[k], mus[k])
        assert rel_err(host(s.array(1)), host(e.array(1))) < 1e-13, k
        assert rel_err(host(s.array(0)), host(e.array(0))) < 1e-13, k
    for k in SWEEP_ORACLE_SAMPLE:
        w = ws[k]
        print("[full size] sweep instance %s against the oracle" % w["name"], flush=True)
        ref = _sweep_oracle(w, node_sets[k])
        s = batched[k]
        sig = host(s.array(1)) + host(s.array(2))[None]
        sig_ref = flat(ref["sig_iw"]) + flat(ref["sig_hf_k"])[None]
        tol = TOL if precision == qgw.F64 else 2e-4
        assert rel_err(sig, sig_ref) < tol, (k, rel_err(sig, sig_ref))
        assert abs(mu[k] - ref["mu"]) <= tol * max(1.0, abs(ref["mu"])), (k, mu[k], ref["mu"])
        if precision == qgw.F64:
            assert rel_err(host(s.array(0)), flat(ref["G_iw"])) < TOL, k
    b.close()
    for st in eager + batched:
        st.close()
    for pl in plans:
        pl.close()
