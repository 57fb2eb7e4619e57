"""Hartree-Fock mode (Fig. fig-self (a)) against the oracle.

qgw_hf_density is held against the oracle's Fermi-function density and
bisection for mu; qgw_state_hf_solve against the oracle's HF loop for the same
number of passes (a negative tol), with and without mixing, and at convergence; a GW
iteration continued from the HF solution against the oracle's GW iteration from
the same state.  The bar is the FP64 parity bar, 1e-10 (mu: 1e-10 relative).
"""
import numpy as np
import pytest

from conftest import rel_err
from oracle import gw, hf
from oracle.dlr import DLR
from paper_2604_22223_amd import qgw
from paper_2604_22223_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES = {
    "random_2+1_6x6": lambda: wl.random_model((6, 6), [2, 1], seed=3, beta=10.0, omega_max=20.0, eps=1e-10),
    "five_orbital_10x10": lambda: wl.five_orbital(n=10, U=1.0, J=0.1, Vnn=0.2, beta=20.0, omega_max=25.0,
                                                  eps=1e-10, scale_mesh=10),
    "graphene_12": lambda: wl.graphene(n=12, U=3.0, beta=10.0, omega_max=100.0, eps=1e-8),
    "random3d_2+1_4x4x4": lambda: wl.random_model_3d((4, 4, 4), [2, 1], seed=3, beta=10.0, omega_max=20.0,
                                                     eps=1e-10, U=1.0, J=0.1, Vnn=0.2),
}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


# number of mesh axes of the current case (2, or 3 on a cubic mesh); set by the ``case`` fixture
_MESH_DIM = [2]


def flat(x):
    return np.ascontiguousarray(x.reshape(x.shape[:-_MESH_DIM[0]] + (-1,)))


def dev(x):
    torch = _torch()
    return torch.from_numpy(flat(np.asarray(x, dtype=np.complex128))).to("cuda:0")


def host(t):
    return t.cpu().numpy()


class Case:
    def __init__(self, w):
        self.w = w
        self.d = DLR(w["beta"], w["omega_max"], w["eps"])
        self.m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
        self.dim = len(w["mesh"])
        self.plan = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], self.d.nodes(), dim=self.dim)
        self.H_R, self.V_R = dev(w["H_R"]), dev(w["V_R"])

    def state(self, mixing=1.0):
        return qgw.State(self.plan, self.H_R, self.V_R, n_target=self.w["n_target"], mixing=mixing)


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print("\n[hf case] %s" % request.param, flush=True)
    c = Case(CASES[request.param]())
    _MESH_DIM[0] = c.dim
    return c


def test_hf_density(case):
    m = case.m
    rng = np.random.default_rng(11)
    x = rng.standard_normal(m.H_k.shape) + 1j * rng.standard_normal(m.H_k.shape)
    h = m.H_k + 0.3 * gw.hermitian_part(x)
    mu_ref, n_ref = hf.fermi_density(h, m.beta, n_target=m.n_target)
    mu, n = case.plan.hf_density(dev(h), n_target=m.n_target)
    assert abs(mu - mu_ref) <= TOL * max(1.0, abs(mu_ref))
    assert rel_err(host(n), flat(n_ref)) < TOL
    # fixed mu
    mu2, n2 = case.plan.hf_density(dev(h), mu=mu_ref + 0.2)
    _, n2_ref = hf.fermi_density(h, m.beta, mu=mu_ref + 0.2)
    assert mu2 == mu_ref + 0.2
    assert rel_err(host(n2), flat(n2_ref)) < TOL


@pytest.mark.parametrize("mixing", [1.0, 0.5])
def test_hf_passes_match_oracle(case, mixing):
    m = case.m
    st = case.state(mixing)
    passes, ds, mu = st.hf_solve(tol=-1.0, max_iter=4)   # a negative tol runs exactly max_iter passes
    assert passes == 4
    ref = hf.initial_state(m)
    for _ in range(4):
        ref = hf.hf_iteration(m, ref, mixing)
    assert abs(mu - ref["mu"]) <= TOL * max(1.0, abs(ref["mu"]))
    assert abs(ds - ref["d_sigma"]) <= 1e-9 * max(1.0, ref["d_sigma"])
    assert rel_err(host(st.array(2)), flat(ref["sig_hf_k"])) < TOL
    assert rel_err(host(st.array(5)), flat(ref["n_k"])) < TOL
    st.close()


def test_hf_converged(case):
    m = case.m
    st = case.state(0.7)
    passes, ds, mu = st.hf_solve(tol=1e-10, max_iter=300)
    ref, hist = hf.scf(m, tol=1e-10, max_iter=300, mixing=0.7)
    assert ds <= 1e-10 and hist[-1] <= 1e-10
    assert abs(passes - len(hist)) <= 1
    assert abs(mu - ref["mu"]) <= 1e-9 * max(1.0, abs(ref["mu"]))
    assert rel_err(host(st.array(2)), flat(ref["sig_hf_k"])) < 1e-9
    st.close()


def test_gw_continues_from_hf(case):
    """After the HF solve the state holds G = [(i w + mu) - H0 - Sigma_HF]^{-1}; one GW iteration from there."""
    m, d = case.m, case.d
    st = case.state()
    passes, ds, mu = st.hf_solve(tol=-1.0, max_iter=3)
    sig_hf = host(st.array(2)).reshape(m.H_k.shape)
    g_hf = gw.dyson_G(m.H_k, sig_hf, None, d.iw, mu)
    assert rel_err(host(st.array(0)), flat(g_hf)) < TOL
    ref = gw.gw_iteration(m, d, {"G_iw": g_hf, "mu": mu, "sig_hf_k": sig_hf,
                                 "sig_iw": np.zeros_like(g_hf), "iteration": 0})
    _, ds_gw, mu_gw = st.iterate(1)
    assert abs(mu_gw - ref["mu"]) <= TOL * max(1.0, abs(ref["mu"]))
    assert rel_err(host(st.array(1)), flat(ref["sig_iw"])) < TOL
    assert rel_err(host(st.array(0)), flat(ref["G_iw"])) < TOL
    st.close()
