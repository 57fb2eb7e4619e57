"""qgw_dyson_G_noalloc (the Dyson G solve with its search scratch in the library's
static device array) against qgw_dyson_G on the same inputs.

Two calls in a row share the GPU's one copy of the array, the second on a
smaller plan (fewer orbitals, smaller mesh, other DLR rank), each at the
target filling (the chemical-potential search) and at a fixed mu.  The two
entry points run the same kernels with the same grids and summation order,
so mu and G agree bit for bit; the bar written here is 1e-13 relative.
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


def dev(x):
    torch = _torch()
    x = np.asarray(x, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(x.reshape(x.shape[:-2] + (-1,)))).to("cuda:0")


def _case(w, seed):
    """plan, H(k) = H0(k) + a static shift, and a Sigma(k, i w) with the structure of a self-energy (the oracle's
    first-iteration Sigma scaled, plus small noise), so the search moves mu away from G0's."""
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    st = gw.gw_iteration(m, d, gw.initial_state(m, d))
    rng = np.random.default_rng(seed)
    noise = 1e-3 * (rng.standard_normal(st["sig_iw"].shape) + 1j * rng.standard_normal(st["sig_iw"].shape))
    plan = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], d.nodes())
    return plan, dev(m.H_k + st["sig_hf_k"]), dev(st["sig_iw"] + noise), w["n_target"]


def _compare(plan, hk, sig, n_target):
    torch = _torch()
    g_ref, g_na = torch.empty_like(sig), torch.empty_like(sig)
    g_ref.fill_(1.0)
    g_na.fill_(2.0)
    mu_ref = plan.dyson_G(hk, sig, g_ref, n_target=n_target, mu=float("nan"))
    mu_na = plan.dyson_G_noalloc(hk, sig, g_na, n_target=n_target, mu=float("nan"))
    torch.cuda.synchronize()
    assert abs(mu_na - mu_ref) <= 1e-13 * max(1.0, abs(mu_ref)), (mu_na, mu_ref)
    assert rel_err(g_na.cpu().numpy(), g_ref.cpu().numpy()) < 1e-13
    # fixed mu (no search), away from the root
    mu_fix = mu_ref + 0.25
    plan.dyson_G(hk, sig, g_ref, n_target=None, mu=mu_fix)
    out = plan.dyson_G_noalloc(hk, sig, g_na, n_target=None, mu=mu_fix)
    torch.cuda.synchronize()
    assert out == mu_fix
    assert rel_err(g_na.cpu().numpy(), g_ref.cpu().numpy()) < 1e-13
    return mu_ref


def test_dyson_g_noalloc_matches_dyson_g_two_calls_second_smaller():
    big = wl.five_orbital(n=8, U=1.0, J=0.1, Vnn=0.2, beta=20.0, omega_max=25.0, eps=1e-10, scale_mesh=8)
    small = wl.random_model((4, 4), [1, 1], seed=7, beta=6.0, omega_max=12.0, eps=1e-8, U=0.7, J=0.0, Vnn=0.1)
    cases = [_case(big, 1), _case(small, 2)]
    assert cases[1][0].r < cases[0][0].r and cases[1][0].n_k < cases[0][0].n_k and cases[1][0].n_o < cases[0][0].n_o
    mus = []
    for k, (plan, hk, sig, nt) in enumerate(cases):
        print("\n[no-alloc] call %d: n_o %d, N_k %d, r %d" % (k, plan.n_o, plan.n_k, plan.r), flush=True)
        mus.append(_compare(plan, hk, sig, nt))
    # the first plan again, after the smaller call left its contents in the array
    _compare(*cases[0])
    for plan, *_ in cases:
        plan.close()
    assert all(np.isfinite(mus))
