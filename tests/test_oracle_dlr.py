"""Pins of the oracle's DLR (not GPU).

Closed forms used (the Lehmann representation of one pole, convention
X(i w) = int_0^beta e^{i w tau} X(tau) dtau):
  fermionic  G(tau) = -e^{-w0 tau} / (1 + e^{-beta w0})  <->  1 / (i w_n - w0)
  bosonic    B(tau) = same function                       <->  tanh(beta w0 / 2) / (i nu_n - w0)
  G(beta^-) = -1 / (1 + e^{beta w0}),  G(0^+) + G(beta^-) = -1.
A pole placed on a DLR frequency is represented exactly, so every map must
reproduce it to round-off; an off-grid pole to the DLR accuracy.
"""
import math

import numpy as np
import pytest

from oracle.dlr import DLR

CASES = [(10.0, 100.0, 1e-8), (50.0, 25.0, 1e-10), (10.0, 20.0, 1e-10)]


def g_tau_exact(tau, w0, beta):
    tau = np.asarray(tau, dtype=float)
    if w0 >= 0:
        return -np.exp(-w0 * tau) / (1.0 + math.exp(-beta * w0))
    return -np.exp(w0 * (beta - tau)) / (1.0 + math.exp(beta * w0))


def fermi(x):
    """1 / (1 + e^x) without overflow."""
    if x > 0:
        return math.exp(-x) / (1.0 + math.exp(-x))
    return 1.0 / (1.0 + math.exp(x))


def iw_f(n, beta):
    return 1j * (2 * np.asarray(n) + 1) * math.pi / beta


def inu_b(n, beta):
    return 1j * 2 * np.asarray(n) * math.pi / beta


@pytest.fixture(scope="module", params=CASES, ids=lambda c: "b%g_w%g_e%g" % c)
def dlr(request):
    beta, wmax, eps = request.param
    return DLR(beta, wmax, eps)


def test_rank_sizes(dlr):
    # ranks of the construction for these cutoffs (checked against the
    # library's independent host builder in test_lib_abi)
    assert 20 <= dlr.r <= 70
    assert np.all(np.diff(dlr.omega) > 0) and np.all(np.diff(dlr.tau_t) > 0)
    assert np.all(dlr.tau_t > 0) and np.all(dlr.tau_t < 1)
    assert len(set(dlr.n_f)) == dlr.r and len(set(dlr.n_b)) == dlr.r


def test_on_grid_pole_fermionic_exact(dlr):
    b = dlr.beta
    tau = dlr.tau_t * b
    for l in [0, dlr.r // 3, dlr.r // 2, dlr.r - 1]:
        w0 = dlr.omega[l]
        giw = 1.0 / (iw_f(dlr.n_f, b) - w0)
        gt = g_tau_exact(tau, w0, b)
        gtr = g_tau_exact(b - tau, w0, b) if w0 < 0 else -np.exp(-w0 * (b - tau)) / (1 + math.exp(-b * w0))
        scale = max(1.0, np.abs(gt).max())
        assert np.abs(dlr.F_iw2tau @ giw - gt).max() / scale < 1e-12
        assert np.abs(dlr.F_iw2taur @ giw - gtr).max() / scale < 1e-12
        assert np.abs(dlr.F_tau2iw @ gt - giw).max() / np.abs(giw).max() < 1e-12
        assert abs(dlr.F_iw2beta @ giw - (-fermi(b * w0))) < 1e-12


def test_on_grid_pole_bosonic_exact(dlr):
    b = dlr.beta
    tau = dlr.tau_t * b
    for l in [0, dlr.r // 4, dlr.r // 2 + 1, dlr.r - 1]:
        w0 = dlr.omega[l]
        bt = g_tau_exact(tau, w0, b)
        nu = inu_b(dlr.n_b, b)
        biw = np.where((nu == 0) & (w0 == 0), -0.5 * b, np.tanh(0.5 * b * w0) / (nu - w0))
        assert np.abs(dlr.B_tau2iw @ bt - biw).max() / np.abs(biw).max() < 1e-11
        assert np.abs(dlr.B_iw2tau @ biw - bt).max() / np.abs(bt).max() < 1e-11


def test_off_grid_poles(dlr):
    """Random off-grid poles: tau values from Matsubara values to ~1e-6, the
    reverse (well conditioned) direction to ~1e-8, and the sum rule
    G(0+) + G(beta-) = -1 through the DLR coefficients."""
    b = dlr.beta
    tau = dlr.tau_t * b
    rng = np.random.default_rng(7)
    wmax = dlr.lam / b
    w0 = rng.uniform(-0.9 * wmax, 0.9 * wmax, 12)
    wt = rng.uniform(0.0, 1.0, 12)
    wt /= wt.sum()
    giw = sum(c / (iw_f(dlr.n_f, b) - w) for c, w in zip(wt, w0))
    gt = sum(c * g_tau_exact(tau, w, b) for c, w in zip(wt, w0))
    assert np.abs(dlr.F_iw2tau @ giw - gt).max() < 1e-6
    assert np.abs(dlr.F_tau2iw @ gt - giw).max() / np.abs(giw).max() < 100 * dlr.eps
    g_beta = sum(c * (-fermi(b * w)) for c, w in zip(wt, w0))
    assert abs(dlr.F_iw2beta @ giw - g_beta) < 1e-6
    coeff = dlr.coeffs_from_iw_f(giw)
    assert abs(coeff.sum() - 1.0) < 1e-5      # = -(G(0+) + G(beta-))


def test_given_nodes_reproduce_maps(dlr):
    d2 = DLR(dlr.beta, lam=dlr.lam, eps=dlr.eps, nodes=dlr.nodes())
    for name in ["F_iw2tau", "F_iw2taur", "F_tau2iw", "B_tau2iw", "B_iw2tau", "F_iw2beta"]:
        assert np.array_equal(getattr(d2, name), getattr(dlr, name))
