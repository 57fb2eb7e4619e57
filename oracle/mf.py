"""The GW iteration on uniform Matsubara and imaginary-time grids (the "MF"
representation the performance section compares the DLR with), plain FP64
NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): not for the product path.

The paper names the conventional Matsubara-frequency grid with a cutoff
Lambda but gives no formulas for its transforms; the reading here is the
textbook one:

* N = 2M nodes, M chosen so that the grid reaches Lambda: fermionic
  w_n = (2n + 1) pi / beta and bosonic nu_n = 2 n pi / beta for
  n = -M .. M-1, and midpoint times tau_j = (j + 1/2) beta / N, j < N.  The
  reflected time beta - tau_j is tau_{N-1-j}, on the same grid.
* iw -> tau (fermionic) is the truncated Matsubara sum with the 1/(iw) tail
  of the orbital diagonal treated exactly: G(tau) = (1/beta) sum_n
  e^{-i w_n tau} [G(i w_n) - delta_ab / (i w_n)] - delta_ab / 2, the second
  term being the exact transform of 1/(iw) on 0 < tau < beta.
* iw -> tau (bosonic) is the truncated sum (1/beta) sum_n e^{-i nu_n tau} W(i nu_n)
  (W^C decays like 1/nu^2: no tail term).
* tau -> iw (both) is the midpoint rule (beta / N) sum_j e^{i w tau_j} X(tau_j).
* The density is n = -G(beta^-) = 1/2 delta_ab + (1/beta) sum_n G(i w_n)
  (the symmetric sum of 1/(i w_n) over the grid vanishes), Hermitian part.

Everything else -- Hartree-Fock, bubble, Dyson W, self-energy, Dyson G and the
chemical potential -- is the DLR iteration's own step from ``gw`` on these
nodes.
"""
import math

import numpy as np

from . import lattice
from .dlr import apply_map
from .gw import bubble, dyson_G, dyson_W, hartree_fock_R, hermitian_part, sigma


class MatsubaraGrid:
    """Uniform grids of N = 2M nodes and the transforms between them, as dense matrices from their definitions."""

    def __init__(self, beta, n_nodes):
        if n_nodes % 2:
            raise ValueError("the node count must be even")
        self.beta = float(beta)
        self.N = int(n_nodes)
        self.M = self.N // 2
        n = np.arange(-self.M, self.M)
        self.n = n
        self.w = (2 * n + 1) * math.pi / self.beta          # fermionic frequencies
        self.nu = 2 * n * math.pi / self.beta               # bosonic frequencies
        self.iw = 1j * self.w
        self.inu = 1j * self.nu
        self.tau = (np.arange(self.N) + 0.5) * self.beta / self.N
        b, N = self.beta, self.N
        # [out, in] matrices
        self.F_iw2tau = np.exp(-1j * np.outer(self.tau, self.w)) / b
        self.F_tau2iw = np.exp(1j * np.outer(self.w, self.tau)) * (b / N)
        self.B_iw2tau = np.exp(-1j * np.outer(self.tau, self.nu)) / b
        self.B_tau2iw = np.exp(1j * np.outer(self.nu, self.tau)) * (b / N)
        # orbital-diagonal constant of the fermionic iw -> tau transform: -(t_j + 1/2) with
        # t_j = (1/beta) sum_n e^{-i w_n tau_j} / (i w_n) the grid's own sum of the tail
        self.tail = -(self.F_iw2tau @ (1.0 / self.iw) + 0.5)

    @classmethod
    def for_cutoff(cls, beta, omega_max, sizes=None):
        """The smallest grid (from ``sizes`` if given) whose last fermionic frequency reaches omega_max."""
        m = max(1, math.ceil(omega_max * beta / (2.0 * math.pi) + 0.5))      # (2M - 1) pi / beta >= omega_max
        n = 2 * m
        if sizes is not None:
            n = min(s for s in sizes if s >= n)
        return cls(beta, n)


def _diag_mask(n_o, mesh):
    return np.eye(n_o).reshape((n_o, n_o) + (1,) * len(mesh))


def g_tau(grid, G_iw):
    """G(tau_j) from G(i w_n) [node, a, b, *mesh] with the orbital-diagonal tail exact."""
    n_o, mesh = G_iw.shape[1], G_iw.shape[3:]
    out = apply_map(grid.F_iw2tau, G_iw)
    return out + grid.tail.reshape((-1, 1, 1) + (1,) * len(mesh)) * _diag_mask(n_o, mesh)[None]


def density_k(grid, G_iw):
    """n(k) = 1/2 + (1/beta) sum_n G(k, i w_n), Hermitian part."""
    n_o, mesh = G_iw.shape[1], G_iw.shape[3:]
    s = np.sum(G_iw, axis=0) / grid.beta
    return hermitian_part(s + 0.5 * _diag_mask(n_o, mesh))


def electron_count(n_k):
    """N_e = (2 / N_k) sum_k Re Tr n(k)."""
    n_kpts = int(np.prod(n_k.shape[2:]))
    return 2.0 * float(np.sum(np.einsum("aa...->...", n_k).real)) / n_kpts


def solve_mu(H_k, sig_hf_k, sig_iw, grid, n_target, tol=1e-13, max_steps=200):
    """Chemical potential by bisection on the grid's density (the same search as the DLR iteration's)."""
    h = np.moveaxis(H_k + sig_hf_k, (0, 1), (-2, -1))
    ev = np.linalg.eigvalsh(0.5 * (h + np.conj(np.swapaxes(h, -1, -2))))
    smax = 0.0 if sig_iw is None else float(np.max(np.abs(sig_iw)))
    pad = 10.0 / grid.beta + smax + 1.0
    lo, hi = float(ev.min()) - pad, float(ev.max()) + pad

    def count(mu):
        return electron_count(density_k(grid, dyson_G(H_k, sig_hf_k, sig_iw, grid.iw, mu)))

    for _ in range(60):
        if count(lo) < n_target < count(hi):
            break
        w = hi - lo
        lo, hi = lo - w, hi + w
    else:
        raise RuntimeError("chemical potential not bracketed")
    steps = 0
    while hi - lo > tol and steps < max_steps:
        mid = 0.5 * (lo + hi)
        if count(mid) < n_target:
            lo = mid
        else:
            hi = mid
        steps += 1
    mu = 0.5 * (lo + hi)
    return mu, dyson_G(H_k, sig_hf_k, sig_iw, grid.iw, mu)


def initial_state(model, grid):
    """G0 on the grid at the chemical potential of the target filling."""
    zero = np.zeros_like(model.H_k)
    mu, g = solve_mu(model.H_k, zero, None, grid, model.n_target)
    return {"G_iw": g, "mu": mu, "sig_hf_k": zero, "sig_iw": np.zeros_like(g), "iteration": 0}


def mf_iteration(model, grid, state, mixing=1.0, keep=False):
    """One GW iteration on the uniform grids, in the order of the DLR iteration (Fig. fig-self (b))."""
    G_iw = state["G_iw"]
    pairs, d = model.pairs, model.dim
    n_k = density_k(grid, G_iw)
    n_R = lattice.R_from_k(n_k, d)
    sig_hf_R = hartree_fock_R(n_R, model.V_R, pairs)
    sig_hf_k = lattice.k_from_R(sig_hf_R, d)
    G_tau = g_tau(grid, G_iw)
    G_reflt = G_tau[::-1]                                      # G(beta - tau_j) = G(tau_{N-1-j})
    G_tau_R = lattice.R_from_k(G_tau, d)
    G_reflt_R = lattice.R_from_k(G_reflt, d)
    P_tau_R = bubble(G_tau_R, G_reflt_R, pairs)
    P_tau_q = lattice.k_from_R(P_tau_R, d)
    P_nu_q = apply_map(grid.B_tau2iw, P_tau_q)
    Wc_nu_q = dyson_W(model.V_q, P_nu_q)
    Wc_tau_q = apply_map(grid.B_iw2tau, Wc_nu_q)
    Wc_tau_R = lattice.R_from_k(Wc_tau_q, d)
    sig_tau_R = sigma(G_tau_R, Wc_tau_R, pairs, model.n_o)
    sig_tau_k = hermitian_part(lattice.k_from_R(sig_tau_R, d), axes=(1, 2))
    sig_iw = apply_map(grid.F_tau2iw, sig_tau_k)
    old_total = state["sig_hf_k"][None] + state["sig_iw"]
    d_sigma = float(np.max(np.abs(sig_hf_k[None] + sig_iw - old_total)))
    if mixing != 1.0:
        sig_hf_k = (1.0 - mixing) * state["sig_hf_k"] + mixing * sig_hf_k
        sig_iw = (1.0 - mixing) * state["sig_iw"] + mixing * sig_iw
    mu, G_new = solve_mu(model.H_k, sig_hf_k, sig_iw, grid, model.n_target)
    out = {"G_iw": G_new, "mu": mu, "sig_hf_k": sig_hf_k, "sig_iw": sig_iw, "d_sigma": d_sigma,
           "iteration": state["iteration"] + 1}
    if keep:
        out["intermediates"] = {"n_k": n_k, "G_tau": G_tau, "G_reflt": G_reflt, "P_tau_q": P_tau_q,
                                "P_nu_q": P_nu_q, "Wc_nu_q": Wc_nu_q, "Wc_tau_q": Wc_tau_q, "sig_tau_k": sig_tau_k}
    return out
