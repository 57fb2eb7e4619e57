"""Pins of the uniform-grid (MF) oracle -- not GPU.

Expected values come from outside the oracle's code: the discrete
orthogonality of the exponentials on the grids (closed form: identity), the
exact imaginary-time Green's function of one pole with a remainder bound
derived by hand, the Lindhard bubble summed over bands and k, the DLR
iteration (pinned by its own tests) as the grid grows, and the atomic limit.
"""
import math

import numpy as np
import pytest

from oracle import gw, mf
from oracle.dlr import DLR
from paper_2604_22223_amd import workloads as wl


def fermi(x):
    return 0.5 * (1.0 - np.tanh(0.5 * x))


@pytest.mark.parametrize("n", [16, 64, 100])
def test_discrete_orthogonality(n):
    """tau -> iw after iw -> tau is the identity on the grid's N frequencies (sum_j e^{2 pi i (m - m')(j + 1/2) / N}
    = N delta_mm' for |m - m'| < N), fermionic and bosonic."""
    g = mf.MatsubaraGrid(7.0, n)
    eye = np.eye(n)
    assert np.abs(g.F_tau2iw @ g.F_iw2tau - eye).max() < 1e-12
    assert np.abs(g.B_tau2iw @ g.B_iw2tau - eye).max() < 1e-12
    # the reflected time is on the grid
    assert np.abs(g.beta - g.tau - g.tau[::-1]).max() < 1e-13


@pytest.mark.parametrize("eps", [0.0, 0.7, -2.3])
def test_single_pole_within_remainder_bound(eps):
    """G(iw) = 1/(iw - eps): G(tau) = -e^{-eps tau} (1 - f(eps)) and n = f(eps).  With the 1/(iw) tail exact the
    truncated sum misses (1/beta) sum_{|n| outside} e^{-iwt} eps / (iw (iw - eps)), each term at most |eps| / w^2
    once w > |eps|, so the error is at most |eps| beta / (2 pi^2 M)."""
    beta = 10.0
    for n in (64, 256):
        g = mf.MatsubaraGrid(beta, n)
        assert g.w[-1] > 4 * abs(eps)
        G = (1.0 / (g.iw - eps)).reshape(-1, 1, 1, 1, 1)
        gt = mf.g_tau(g, G)[:, 0, 0, 0, 0]
        exact = -np.exp(-eps * g.tau) * fermi(-beta * eps) if eps >= 0 else \
            -np.exp(-eps * (g.tau - beta)) * fermi(beta * eps)
        bound = abs(eps) * beta / (2 * math.pi ** 2 * g.M)
        assert np.abs(gt - exact).max() <= bound + 1e-13, (n, np.abs(gt - exact).max(), bound)
        dens = mf.density_k(g, G)[0, 0, 0, 0].real
        assert abs(dens - fermi(beta * eps)) <= bound + 1e-13
    # one pole at zero energy: exact on any grid (-1/2 and 1/2)
    if eps == 0.0:
        assert np.abs(gt + 0.5).max() < 1e-14 and abs(dens - 0.5) < 1e-14


def test_bubble_of_g0_converges_to_lindhard():
    """The grid bubble of G0 at bosonic frequency nu_m against the Lindhard sum over bands and k,
    P(q, i nu) = (2 / N_k) sum_{k, a, b} |<a k|b k+q>|^2 (f(e_a) - f(e_b)) / (i nu + e_a - e_b) (orbital-summed
    density response, the (ii),(jj) trace); the error falls at least 3x from N = 64 to 256."""
    w = wl.random_model((4, 4), [2], seed=5, beta=6.0, omega_max=20.0, eps=1e-10)
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], 2.0)
    mu = 0.3
    h = np.moveaxis(m.H_k, (0, 1), (-2, -1))
    ev, U = np.linalg.eigh(h)
    f = fermi(m.beta * (ev - mu))
    n1, n2 = m.mesh
    errs = []
    for n in (64, 256):
        g = mf.MatsubaraGrid(m.beta, n)
        G = gw.dyson_G(m.H_k, np.zeros_like(m.H_k), None, g.iw, mu)
        st = {"G_iw": G, "mu": mu, "sig_hf_k": np.zeros_like(m.H_k), "sig_iw": np.zeros_like(G), "iteration": 0}
        out = mf.mf_iteration(m, g, st, keep=True)
        P = out["intermediates"]["P_nu_q"]                    # [nu, A, B, q1, q2]
        dens = [a * 2 + a for a in range(2)]                  # pair indices (a, a)
        Pd = P[:, dens][:, :, dens].sum(axis=(1, 2))          # sum over (aa),(bb)
        err = 0.0
        for mi in (g.M, g.M + 1, g.M + 3):                    # nu = 0, 2 pi / beta, 6 pi / beta
            inu = g.inu[mi]
            for q1 in range(n1):
                for q2 in range(n2):
                    s = 0.0
                    for k1 in range(n1):
                        for k2 in range(n2):
                            kq = ((k1 + q1) % n1, (k2 + q2) % n2)
                            ov = np.abs(np.conj(U[k1, k2]).T @ U[kq]) ** 2      # [a, b]
                            num = f[k1, k2][:, None] - f[kq][None, :]
                            den = inu + ev[k1, k2][:, None] - ev[kq][None, :]
                            with np.errstate(invalid="ignore", divide="ignore"):
                                term = np.where(np.abs(den) < 1e-12,
                                                -m.beta * f[k1, k2][:, None] * (1 - f[k1, k2][:, None]), num / den)
                            s += np.sum(ov * term)
                    lind = 2.0 * s / (n1 * n2)
                    err = max(err, abs(Pd[mi, q1, q2] - lind))
        errs.append(err)
    assert errs[1] <= errs[0] / 3.0, errs
    assert errs[1] < 5e-3, errs


def test_iteration_approaches_dlr_iteration():
    """One GW iteration on the grid converges to the DLR iteration (pinned by its own tests) as N grows:
    Sigma^C at the DLR's Matsubara nodes inside the grid, error falling at least 3x from N = 128 to 512."""
    w = wl.random_model((3, 3), [2, 1], seed=3, beta=5.0, omega_max=40.0, eps=1e-12, U=1.0, J=0.1, Vnn=0.2)
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    ref = gw.gw_iteration(m, d, gw.initial_state(m, d))
    nodes = np.rint((np.imag(d.iw) * w["beta"] / math.pi - 1) / 2).astype(int)
    errs, dmus = [], []
    inside = [k for k, nn in enumerate(nodes) if -64 <= nn < 64]      # nodes inside both grids
    assert len(inside) >= 30
    for n in (128, 512):
        g = mf.MatsubaraGrid(w["beta"], n)
        out = mf.mf_iteration(m, g, mf.initial_state(m, g))
        sel = [(k, int(nodes[k] + g.M)) for k in inside]
        a = np.stack([out["sig_iw"][j] for _, j in sel])
        b = np.stack([ref["sig_iw"][k] for k, _ in sel])
        errs.append(np.abs(a - b).max() / np.abs(b).max())
        dmus.append(abs(out["mu"] - ref["mu"]))
    assert errs[1] <= errs[0] / 3.0 and errs[1] < 2e-3, errs
    assert dmus[1] < dmus[0] and dmus[1] < 1e-3, dmus


def test_atomic_limit_half_filling():
    """Flat band at e0 with on-site U at half filling: particle-hole symmetry on the symmetric grid gives
    n = 1/2, Sigma_HF = U / 2 and mu = e0 + U / 2 after every iteration, on 2-D and 3-D meshes."""
    e0, U = -0.4, 1.3
    for mesh in ((2, 2), (2, 2, 2)):
        w = wl.local_model(mesh, [1], [e0], np.array([[U]]), 8.0, 20.0, 1e-10, n_target=1.0)
        m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], 1.0)
        g = mf.MatsubaraGrid(8.0, 64)
        st = mf.initial_state(m, g)
        assert abs(st["mu"] - e0) < 1e-12
        for _ in range(2):
            st = mf.mf_iteration(m, g, st)
            assert abs(st["mu"] - (e0 + U / 2)) < 1e-11
            assert np.abs(st["sig_hf_k"] - U / 2).max() < 1e-12
