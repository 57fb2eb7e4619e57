"""Pins of the oracle on a 3-D k-mesh (the cubic benchmark model of the
performance section) -- not GPU.

Expected values come from outside the oracle's code: DFT sums written out
term by term, the index map R -> -R done by hand, the cubic tight-binding
dispersion, the 2-D oracle (already pinned by its own tests) on a mesh with a
trivial third axis, the atomic limit, and the cubic symmetry of the model.
"""
import itertools
import math

import numpy as np
import pytest

from conftest import rel_err
from oracle import adjoint, gw, hf, lattice
from oracle.dlr import DLR
from paper_2604_22223_amd import workloads as wl


def model_of(w):
    return gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])


def test_lattice_3d_brute_force():
    """X(k) = sum_R X(R) exp(-2 pi i sum_a k_a R_a / n_a) on a 2 x 3 x 5 mesh, summed term by term;
    X(R) = (1/N_k) sum_k X(k) exp(+...), and X(-R) by the explicit index map."""
    mesh = (2, 3, 5)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2,) + mesh) + 1j * rng.standard_normal((2,) + mesh)
    want = np.zeros_like(x)
    for k in itertools.product(*map(range, mesh)):
        for r in itertools.product(*map(range, mesh)):
            ph = sum(ka * ra / na for ka, ra, na in zip(k, r, mesh))
            want[(slice(None),) + k] += x[(slice(None),) + r] * np.exp(-2j * math.pi * ph)
    assert np.abs(lattice.k_from_R(x, 3) - want).max() < 1e-12
    back = np.zeros_like(x)
    for r in itertools.product(*map(range, mesh)):
        for k in itertools.product(*map(range, mesh)):
            ph = sum(ka * ra / na for ka, ra, na in zip(k, r, mesh))
            back[(slice(None),) + r] += want[(slice(None),) + k] * np.exp(2j * math.pi * ph) / 30.0
    assert np.abs(lattice.R_from_k(want, 3) - back).max() < 1e-12
    assert np.abs(back - x).max() < 1e-12
    refl = np.empty_like(x)
    for r in itertools.product(*map(range, mesh)):
        mr = tuple((-ra) % na for ra, na in zip(r, mesh))
        refl[(slice(None),) + r] = x[(slice(None),) + mr]
    assert np.array_equal(lattice.reflect(x, 3), refl)


def test_cubic_dispersion_and_g0():
    """The cubic model has H0(k) = -2t (cos k1 + cos k2 + cos k3) I, and G0 = 1 / (i w + mu - eps(k))."""
    n, t = 4, 1.0
    w = wl.cubic_five_orbital(n=n, t=t, beta=10.0, omega_max=20.0, eps=1e-10, norb=2)
    m = model_of(w)
    k = 2.0 * np.pi * np.arange(n) / n
    c = np.cos(k)
    eps_k = -2.0 * t * (c[:, None, None] + c[None, :, None] + c[None, None, :])
    want = eps_k[None, None] * np.eye(2)[:, :, None, None, None]
    assert np.abs(m.H_k - want).max() < 1e-14
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    mu = 0.37
    g = gw.dyson_G(m.H_k, np.zeros_like(m.H_k), None, d.iw, mu)
    g_exact = 1.0 / (d.iw[:, None, None, None] + mu - eps_k[None])
    assert np.abs(g[:, 0, 0] - g_exact).max() < 1e-14
    assert np.abs(g[:, 0, 1]).max() == 0.0
    # half filling of a particle-hole symmetric band: mu = 0 (up to the DLR error of the density)
    st = gw.initial_state(m, d)
    assert abs(st["mu"]) < 1e-8          # within the DLR accuracy of the density


def test_bubble_3d_brute_force():
    """P_{(il),(jk)}(R) = -2 G_lj(R, tau) G_ki(-R, beta - tau), the reflection done per axis by hand."""
    mesh = (2, 3, 4)
    rng = np.random.default_rng(2)
    pairs = lattice.pair_list([2])
    gt = rng.standard_normal((3, 2, 2) + mesh) + 1j * rng.standard_normal((3, 2, 2) + mesh)
    gr = rng.standard_normal((3, 2, 2) + mesh) + 1j * rng.standard_normal((3, 2, 2) + mesh)
    p = gw.bubble(gt, gr, pairs)
    for a, (i, l) in enumerate(pairs):
        for b, (j, k) in enumerate(pairs):
            for r in itertools.product(*map(range, mesh)):
                mr = tuple((-x) % n for x, n in zip(r, mesh))
                want = -2.0 * gt[(slice(None), l, j) + r] * gr[(slice(None), k, i) + mr]
                assert np.abs(p[(slice(None), a, b) + r] - want).max() < 1e-15


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_trivial_axis_reduces_to_2d(axis):
    """A 3-D mesh with one axis of length 1 is the 2-D model: one GW iteration, its total energy and the
    adjoint's gradient agree with the 2-D oracle (which its own tests pin) wherever the unit axis sits."""
    w2 = wl.random_model((3, 4), [2, 1], seed=7, beta=8.0, omega_max=20.0, eps=1e-10)
    w3 = dict(w2)
    w3["mesh"] = tuple(np.insert(np.array(w2["mesh"]), axis, 1))
    w3["H_R"] = np.expand_dims(w2["H_R"], 2 + axis)
    w3["V_R"] = np.expand_dims(w2["V_R"], 2 + axis)
    d = DLR(w2["beta"], w2["omega_max"], w2["eps"])
    m2, m3 = model_of(w2), model_of(w3)
    s2 = gw.gw_iteration(m2, d, gw.initial_state(m2, d), keep=True)
    s3 = gw.gw_iteration(m3, d, gw.initial_state(m3, d), keep=True)
    sq = lambda x, lead: np.squeeze(x, axis=lead + axis)
    assert abs(s3["mu"] - s2["mu"]) < 1e-12
    assert rel_err(sq(s3["G_iw"], 3), s2["G_iw"]) < 1e-12
    assert rel_err(sq(s3["sig_iw"], 3), s2["sig_iw"]) < 1e-12
    assert rel_err(sq(s3["sig_hf_k"], 2), s2["sig_hf_k"]) < 1e-12
    i2, i3 = s2["intermediates"], s3["intermediates"]
    assert rel_err(sq(i3["P_tau_q"], 3), i2["P_tau_q"]) < 1e-12
    e2, e3 = gw.total_energy(m2, d, s2)[0], gw.total_energy(m3, d, s3)[0]
    assert abs(e3 - e2) < 1e-12 * max(1.0, abs(e2))
    rng = np.random.default_rng(4)
    cot2 = {"sig_iw": rng.standard_normal(s2["sig_iw"].shape) + 0j, "energy": 0.3}
    cot3 = {"sig_iw": np.expand_dims(cot2["sig_iw"], 3 + axis), "energy": 0.3}
    _, g2 = adjoint.one_iteration_grad(m2, d, cot2)
    _, g3 = adjoint.one_iteration_grad(m3, d, cot3)
    assert rel_err(sq(g3["H_R"], 2), g2["H_R"]) < 1e-11
    assert rel_err(sq(g3["V_R"], 2), g2["V_R"]) < 1e-11


def test_cubic_atomic_limit_hf():
    """Flat band at e0 with on-site U on a 2 x 2 x 2 mesh at half filling: Sigma_HF = U / 2, mu = e0 + U / 2."""
    e0, U = -0.4, 1.3
    w = wl.local_model((2, 2, 2), [1], [e0], np.array([[U]]), 7.0, 20.0, 1e-10, n_target=1.0)
    m = model_of(w)
    st, hist = hf.scf(m, tol=1e-12)
    assert abs(st["mu"] - (e0 + U / 2)) < 1e-12
    assert np.abs(st["sig_hf_k"] - U / 2).max() < 1e-12


def test_cubic_symmetry_of_sigma():
    """The cubic model is invariant under every permutation of the three axes (and under k -> -k), so one GW
    iteration gives Sigma(k) and P(q) with the same symmetry; an axis mixed up anywhere breaks it."""
    w = wl.cubic_five_orbital(n=4, beta=10.0, omega_max=20.0, eps=1e-10, norb=2, n_target=1.6)
    m = model_of(w)
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    st = gw.gw_iteration(m, d, gw.initial_state(m, d), keep=True)
    sig, p = st["sig_iw"], st["intermediates"]["P_tau_q"]
    assert np.abs(sig).max() > 1e-3
    for perm in itertools.permutations(range(3)):
        axes = (0, 1, 2) + tuple(3 + x for x in perm)
        assert np.abs(np.transpose(sig, axes) - sig).max() < 1e-12
        assert np.abs(np.transpose(p, axes) - p).max() < 1e-12
    assert np.abs(lattice.reflect(sig, 3) - sig).max() < 1e-12
