"""Pins of the Hartree-Fock oracle (Fig. fig-self (a), H class paragraph)."""
import numpy as np
import pytest

from conftest import rel_err
from oracle import gw, hf
from oracle.dlr import DLR
from paper_2604_22223_amd import workloads as wl


@pytest.fixture(scope="module")
def model():
    w = wl.random_model((4, 4), [2, 1], seed=3, beta=10.0, omega_max=20.0, eps=1e-10, U=0.7, J=0.1, Vnn=0.1)
    return w, gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])


def test_fermi_density_spectrum(model):
    """n commutes with H, its eigenvalues are f(beta (eps - mu)) and the filling is the target."""
    w, m = model
    mu, n = hf.fermi_density(m.H_k, m.beta, n_target=m.n_target)
    h = np.moveaxis(m.H_k, (0, 1), (-2, -1))
    nn = np.moveaxis(n, (0, 1), (-2, -1))
    assert np.abs(h @ nn - nn @ h).max() < 1e-13
    eps = np.linalg.eigvalsh(h)
    occ = np.sort(np.linalg.eigvalsh(nn), axis=-1)
    want = np.sort(1.0 / (np.exp(m.beta * (eps - mu)) + 1.0), axis=-1)
    assert np.abs(occ - want).max() < 1e-13
    assert abs(gw.electron_count(n) - m.n_target) < 1e-11


def test_fermi_density_equals_dlr_density_of_g0(model):
    """Two independent routes to the density of H0: the Fermi function of H0, and -G0(beta^-) from the DLR
    expansion of G0(i w) = [(i w + mu) - H0]^{-1} on the Matsubara nodes."""
    w, m = model
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    mu = 0.31
    _, n_f = hf.fermi_density(m.H_k, m.beta, mu=mu)
    g0 = gw.dyson_G(m.H_k, np.zeros_like(m.H_k), None, d.iw, mu)
    n_dlr = gw.density_k(g0, d)
    assert rel_err(n_f, n_dlr) < 1e-8


def test_atom_at_half_filling():
    """One orbital, flat band at e0, on-site U: Sigma_H + Sigma_F = U n, and at half filling n = 1/2, so the loop
    lands on Sigma_HF = U/2 and mu = e0 + U/2 after one pass (particle-hole symmetry)."""
    mesh, e0, U, beta = (4, 4), -0.4, 1.3, 7.0
    H_R = np.zeros((1, 1) + mesh, dtype=np.complex128)
    H_R[0, 0, 0, 0] = e0
    V_R = np.zeros((1, 1) + mesh, dtype=np.complex128)
    V_R[0, 0, 0, 0] = U
    m = gw.Model(mesh, [1], H_R, V_R, beta, 1.0)
    st, hist = hf.scf(m, tol=1e-12)
    assert abs(st["mu"] - (e0 + U / 2)) < 1e-12
    assert np.abs(st["sig_hf_k"] - U / 2).max() < 1e-12
    assert np.abs(st["n_k"] - 0.5).max() < 1e-12


def test_fixed_point(model):
    w, m = model
    st, hist = hf.scf(m, tol=1e-12, max_iter=300)
    assert hist[-1] <= 1e-12
    nxt = hf.hf_iteration(m, st)
    assert nxt["d_sigma"] <= 1e-11
    assert abs(gw.electron_count(st["n_k"]) - m.n_target) < 1e-11
    # Sigma_HF(k) and n(k) are Hermitian
    assert np.abs(st["sig_hf_k"] - np.conj(np.swapaxes(st["sig_hf_k"], 0, 1))).max() < 1e-13
