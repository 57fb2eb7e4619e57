"""Hartree-Fock self-consistency (Fig. fig-self (a): the H0, V, SigH, SigF and H classes), plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): not for the product path.

The H class paragraph: with H = H0 + Sigma^H + Sigma^F (frequency independent),
the chemical potential is set by the target filling and the density matrix is
the Fermi function of H,
    n(k) = 1 / (e^{beta (H(k) - mu)} + 1) = U f(beta (eps - mu)) U^H,
H(k) = U diag(eps) U^H.  Sigma^H and Sigma^F follow from n and V as in the GW
loop (Eqs. eq-hartree-self-energy, eq-fock-self-energy; ``gw.hartree_fock_R``).
The loop starts from the density of H0 at the target filling and stops when
max |Delta Sigma_HF| <= tol over k and orbital pairs.
"""
import numpy as np

from . import lattice
from .gw import hartree_fock_R


def fermi(x):
    """1 / (e^x + 1), written with tanh so that it stays finite for any real x."""
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def eigen_k(H_k):
    """Eigenvalues [*mesh, band] and eigenvectors [*mesh, a, band] of the Hermitian part of H(k)."""
    h = np.moveaxis(H_k, (0, 1), (-2, -1))
    h = 0.5 * (h + np.conj(np.swapaxes(h, -1, -2)))
    return np.linalg.eigh(h)


def electron_count(eps, mu, beta):
    """N_e(mu) = (2 / N_k) sum_{k, n} f(beta (eps_n(k) - mu)) (two spins)."""
    n_k = int(np.prod(eps.shape[:-1]))
    return 2.0 * float(np.sum(fermi(beta * (eps - mu)))) / n_k


def solve_mu(eps, beta, n_target, tol=1e-13, max_steps=400):
    """mu with N_e(mu) = n_target, by bisection (N_e increases with mu)."""
    lo = float(eps.min()) - 50.0 / beta - 1.0
    hi = float(eps.max()) + 50.0 / beta + 1.0
    for _ in range(max_steps):
        mid = 0.5 * (lo + hi)
        if hi - lo <= tol * max(1.0, abs(mid)):
            break
        if electron_count(eps, mid, beta) < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def fermi_density(H_k, beta, n_target=None, mu=None):
    """(mu, n(k)) for the static Hamiltonian H(k): n = U f(beta (eps - mu)) U^H, [a, b, *mesh]."""
    eps, u = eigen_k(H_k)
    if n_target is not None:
        mu = solve_mu(eps, beta, n_target)
    occ = fermi(beta * (eps - mu))
    n = np.einsum("...an,...n,...bn->...ab", u, occ, np.conj(u))
    return mu, np.moveaxis(n, (-2, -1), (0, 1))


def hf_self_energy_k(model, n_k):
    """Sigma_HF(k) from the density (SigH and SigF classes)."""
    n_R = lattice.R_from_k(n_k, model.dim)
    return lattice.k_from_R(hartree_fock_R(n_R, model.V_R, model.pairs), model.dim)


def initial_state(model):
    """The density of H0 at the target filling, with Sigma_HF = 0."""
    mu, n_k = fermi_density(model.H_k, model.beta, n_target=model.n_target)
    return {"n_k": n_k, "sig_hf_k": np.zeros_like(model.H_k), "mu": mu, "iteration": 0}


def hf_iteration(model, state, mixing=1.0):
    """One pass of the HF loop: n -> Sigma_H + Sigma_F -> H -> mu, n."""
    sig = hf_self_energy_k(model, state["n_k"])
    d_sigma = float(np.max(np.abs(sig - state["sig_hf_k"])))
    if mixing != 1.0:
        sig = (1.0 - mixing) * state["sig_hf_k"] + mixing * sig
    mu, n_k = fermi_density(model.H_k + sig, model.beta, n_target=model.n_target)
    return {"n_k": n_k, "sig_hf_k": sig, "mu": mu, "d_sigma": d_sigma, "iteration": state["iteration"] + 1}


def scf(model, tol=1e-8, max_iter=200, mixing=1.0, state=None):
    """HF self-consistency from the density of H0 until max |Delta Sigma_HF| <= tol."""
    if state is None:
        state = initial_state(model)
    history = []
    for _ in range(max_iter):
        state = hf_iteration(model, state, mixing)
        history.append(state["d_sigma"])
        if state["d_sigma"] <= tol:
            break
    return state, history
