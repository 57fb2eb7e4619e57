"""One GW iteration and the GW self-consistency loop, plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): not for the product path.

Conventions (where the paper leaves a choice open):

* Arrays carry the DLR node axis first, then orbital or pair indices, then
  the d mesh axes: G[node, a, b, n1, n2], P[node, alpha, beta, n1, n2] on a
  2-D mesh, G[node, a, b, n1, n2, n3] on a 3-D one.
* Orbital indices a = (p, i) are global; pair indices alpha = (p; i, l) come
  from ``lattice.pair_list`` and X_{(il),(jk)} stands for the paper's X_{ijkl}
  (Eq. eq:many-body-hamiltonian pairs c+_i ... c_l at one site and
  c+_j ... c_k at the other).  With that labelling the Dyson equation for W
  (Eq. eq-screened-coulomb) is a plain matrix product in the pair index.
* G(R, tau) is the (R, 0) block of -<T c(R, tau) c+(0, 0)>; the density
  matrix is n = -G(beta^-) (G class paragraph of Fig. fig-self (b)).
* Paramagnetic and spin-independent V: the spin sum of the bubble gives a
  factor 2, the Hartree term a factor 2, and the electron count per cell is
  2/N_k sum_k Tr n(k).
"""
import numpy as np

from . import lattice
from .dlr import apply_map


# ----------------------------------------------------------------------------
# model container (inputs only; no arithmetic of the method)
# ----------------------------------------------------------------------------

class Model:
    """Lattice model: mesh, orbitals per site, H0(R), V(R), beta, filling."""

    def __init__(self, mesh, site_norb, H_R, V_R, beta, n_target):
        self.mesh = tuple(int(x) for x in mesh)
        self.site_norb = list(site_norb)
        self.H_R = np.asarray(H_R, dtype=np.complex128)
        self.V_R = np.asarray(V_R, dtype=np.complex128)
        self.beta = float(beta)
        self.n_target = n_target
        self.n_o = int(sum(self.site_norb))
        self.pairs = lattice.pair_list(self.site_norb)
        self.n_b = len(self.pairs)
        assert self.H_R.shape == (self.n_o, self.n_o) + self.mesh
        assert self.V_R.shape == (self.n_b, self.n_b) + self.mesh
        self.dim = len(self.mesh)
        self.n_k = int(np.prod(self.mesh))
        self.H_k = lattice.k_from_R(self.H_R, self.dim)           # H0(k), Eq. eq:fourier-transform-kr
        self.V_q = lattice.k_from_R(self.V_R, self.dim)           # V(q)


# ----------------------------------------------------------------------------
# a13: Dyson equation for G, density, chemical potential
# ----------------------------------------------------------------------------

def dyson_G(H_k, sig_hf_k, sig_iw, iw, mu):
    """G(k, i w_m) = [(i w_m + mu) I - H0(k) - Sigma_HF(k) - Sigma_C(k, i w_m)]^{-1}.

    Eq. full-green-freq rearranged as G^{-1} = G0^{-1} - Sigma with
    G0(k, i w)^{-1} = (i w + mu) - H0(k) (Eq. eq:bare-green-freq evaluated
    for the quadratic H0).  ``sig_iw`` may be None (Sigma_C = 0).
    """
    n_o = H_k.shape[0]
    r = len(iw)
    h = np.moveaxis(H_k + sig_hf_k, (0, 1), (-2, -1))           # [n1, n2, a, b]
    a = np.empty((r,) + h.shape, dtype=np.complex128)
    eye = np.eye(n_o)
    for m in range(r):
        a[m] = (iw[m] + mu) * eye - h
        if sig_iw is not None:
            a[m] -= np.moveaxis(sig_iw[m], (0, 1), (-2, -1))
    g = np.linalg.inv(a)
    return np.moveaxis(g, (-2, -1), (1, 2))                     # [m, a, b, n1, n2]


def hermitian_part(x, axes=(0, 1)):
    """(X + X^dagger) / 2 over the two orbital axes."""
    return 0.5 * (x + np.conj(np.swapaxes(x, *axes)))


def density_k(G_iw, dlr):
    """n(k) = -G(k, beta^-) from the DLR expansion of G(k, i w) (a12).

    The density matrix n_ab(k) = <c+_b c_a> is Hermitian; the DLR evaluation
    at beta^- carries an anti-Hermitian error of the size of the DLR
    accuracy, which the self-consistency would amplify (the filling fixes
    only Re Tr n), so the Hermitian part is kept.
    """
    return hermitian_part(-apply_map(dlr.F_iw2beta[None, :], G_iw)[0])


def electron_count(n_k):
    """N_e = (2 / N_k) sum_k Re Tr n(k)  (two spins)."""
    n_kpts = int(np.prod(lattice.mesh_of(n_k, 2)))
    tr = np.einsum("aa...->...", n_k)
    return 2.0 * float(np.sum(tr.real)) / n_kpts


def mu_bracket(H_k, sig_hf_k, sig_iw, beta):
    """A bracket [lo, hi] containing the chemical potential: the spectrum of H0 + Sigma_HF padded by
    10 / beta + max|Sigma^C| + 1."""
    h = np.moveaxis(H_k + sig_hf_k, (0, 1), (-2, -1))
    h = 0.5 * (h + np.conj(np.swapaxes(h, -1, -2)))
    ev = np.linalg.eigvalsh(h)
    smax = 0.0 if sig_iw is None else float(np.max(np.abs(sig_iw)))
    pad = 10.0 / beta + smax + 1.0
    return float(ev.min()) - pad, float(ev.max()) + pad


def solve_mu(H_k, sig_hf_k, sig_iw, dlr, n_target, tol=1e-13, max_steps=200):
    """Chemical potential by bisection on N_e(mu) = n_target, to |d mu| <= 1e-13 max(1, |mu|).

    N_e(mu) is evaluated through the same Dyson equation and the DLR density.
    Returns (mu, G_iw at mu, number of evaluations).
    """
    lo, hi = mu_bracket(H_k, sig_hf_k, sig_iw, dlr.beta)

    def count(mu):
        g = dyson_G(H_k, sig_hf_k, sig_iw, dlr.iw, mu)
        return electron_count(density_k(g, dlr))

    evals = 0
    for _ in range(60):                      # widen until the bracket holds
        n_lo, n_hi = count(lo), count(hi)
        evals += 2
        if n_lo < n_target < n_hi:
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
        evals += 1
    mu = 0.5 * (lo + hi)
    return mu, dyson_G(H_k, sig_hf_k, sig_iw, dlr.iw, mu), evals


# ----------------------------------------------------------------------------
# a12: Hartree and Fock self-energies
# ----------------------------------------------------------------------------

def hartree_fock_R(n_R, V_R, pairs):
    """Sigma_HF(R) = Sigma_F(R) + delta_{R,0} Sigma_H.

    Fock (Eq. eq-fock-self-energy, indices from Wick's theorem on
    Eq. eq:many-body-hamiltonian):
        Sigma_F_{ik}(R) = - sum_{(il),(jk)} V_{(il),(jk)}(R) n_{lj}(R)
    Hartree (Eq. eq-hartree-self-energy, two spins):
        Sigma_H_{il} = 2 sum_{(jk)} V_{(il),(jk)}(q = 0) n_{kj}(R = 0)
    """
    n_o = n_R.shape[0]
    mesh = lattice.mesh_of(n_R, 2)
    r0 = (0,) * len(mesh)                                       # R = 0
    sig = np.zeros((n_o, n_o) + mesh, dtype=np.complex128)
    v_q0 = np.sum(V_R, axis=lattice.mesh_axes(len(mesh)))
    for al, (i, l) in enumerate(pairs):
        for be, (j, k) in enumerate(pairs):
            sig[i, k] -= V_R[al, be] * n_R[l, j]
            sig[(i, l) + r0] += 2.0 * v_q0[al, be] * n_R[(k, j) + r0]
    return sig


# ----------------------------------------------------------------------------
# a3: polarizability bubble
# ----------------------------------------------------------------------------

def bubble(G_tau_R, G_reflt_R, pairs, spin_factor=2.0):
    """P_{(il),(jk)}(R, tau) = -s G_{lj}(R, tau) G_{ki}(-R, beta - tau).

    Eq. eq-polarizability takes G_{ki}(-R, -tau) G_{lj}(R, tau); with the
    fermionic antiperiodicity G(-tau) = -G(beta - tau) for 0 < tau < beta
    and the spin sum s = 2 this is the expression above.  ``G_reflt_R`` holds
    G(R, beta - tau_k) at the DLR time nodes (unreflected in R).
    """
    r = G_tau_R.shape[0]
    mesh = lattice.mesh_of(G_tau_R, 3)
    nb = len(pairs)
    g_minus_r = lattice.reflect(G_reflt_R, len(mesh))           # G(-R, beta - tau)
    p = np.empty((r, nb, nb) + mesh, dtype=np.complex128)
    for al, (i, l) in enumerate(pairs):
        for be, (j, k) in enumerate(pairs):
            p[:, al, be] = -spin_factor * G_tau_R[:, l, j] * g_minus_r[:, k, i]
    return p


# ----------------------------------------------------------------------------
# a6: screened interaction
# ----------------------------------------------------------------------------

def dyson_W(V_q, P_nu):
    """W^C = W - V with W = V + V P W (Eq. eq-screened-coulomb), per (q, i nu).

    W = (I - V P)^{-1} V by a linear solve for every q and bosonic node.
    """
    nb = V_q.shape[0]
    v = np.moveaxis(V_q, (0, 1), (-2, -1))                      # [n1, n2, A, B]
    eye = np.eye(nb)
    out = np.empty_like(P_nu)
    for m in range(P_nu.shape[0]):
        p = np.moveaxis(P_nu[m], (0, 1), (-2, -1))
        w = np.linalg.solve(eye - v @ p, v)
        out[m] = np.moveaxis(w - v, (-2, -1), (0, 1))
    return out


# ----------------------------------------------------------------------------
# a9: GW self-energy
# ----------------------------------------------------------------------------

def sigma(G_tau_R, Wc_tau_R, pairs, n_o):
    """Sigma^C_{ik}(R, tau) = - sum_{(il),(jk)} W^C_{(il),(jk)}(R, tau) G_{lj}(R, tau).

    Eq. eq-gw-self-energy with the orbital labels fixed by Wick's theorem on
    Eq. eq:many-body-hamiltonian (the same contraction as the Fock term).
    """
    r = G_tau_R.shape[0]
    mesh = lattice.mesh_of(G_tau_R, 3)
    sig = np.zeros((r, n_o, n_o) + mesh, dtype=np.complex128)
    for al, (i, l) in enumerate(pairs):
        for be, (j, k) in enumerate(pairs):
            sig[:, i, k] -= Wc_tau_R[:, al, be] * G_tau_R[:, l, j]
    return sig


# ----------------------------------------------------------------------------
# a14: total energy
# ----------------------------------------------------------------------------

def total_energy(model, dlr, state):
    """Galitskii-Migdal energy per cell (two spins); the paper names no formula, this is the standard one.

    E = 2/N_k sum_k Re Tr[(H0(k) + Sigma_HF(k) / 2) n(k)]
        + 1/N_k sum_k Re (1/beta) sum_n Tr[Sigma^C(k, i w_n) G(k, i w_n)]

    with n = -G(beta^-) from the state's G (Hermitian part) and the Matsubara
    sum over all n taken exactly from the DLR expansions of Sigma^C and G:
    (1/beta) sum_n A(i w_n) B(i w_n) = sum_{l l'} a_l b_l' D[l, l'] with
    D the divided differences of the Fermi function (fermi_divided_differences).
    Returns (E, E_HF part, correlation part).
    """
    G = state["G_iw"]
    n_k = density_k(G, dlr)
    nk = model.n_k
    a = model.H_k + 0.5 * state["sig_hf_k"]
    e_hf = 2.0 / nk * float(np.sum(np.einsum("ab...,ba...->...", a, n_k)).real)
    sig_c = dlr.coeffs_from_iw_f(state["sig_iw"])          # [l, a, b, n1, n2]
    g_c = dlr.coeffs_from_iw_f(G)
    flat = lambda x: x.reshape(x.shape[:3] + (-1,))           # mesh axes as one k axis
    tr = np.einsum("labk,mbak->lm", flat(sig_c), flat(g_c))  # sum_k Tr[sigma_l g_m]
    e_c = float(np.sum(dlr.D_sum * tr).real) / nk
    return e_hf + e_c, e_hf, e_c


# ----------------------------------------------------------------------------
# the iteration (Fig. fig-self (b))
# ----------------------------------------------------------------------------

def initial_state(model, dlr):
    """G0 at the chemical potential that gives the target filling (the iteration starts from G0, with no prior HF loop)."""
    zero = np.zeros_like(model.H_k)
    if model.n_target is None:
        raise ValueError("initial_state needs a target filling; use g0_fixed_mu")
    mu, g, _ = solve_mu(model.H_k, zero, None, dlr, model.n_target)
    return {"G_iw": g, "mu": mu, "sig_hf_k": zero,
            "sig_iw": np.zeros_like(g), "iteration": 0}


def g0_fixed_mu(model, dlr, mu):
    zero = np.zeros_like(model.H_k)
    g = dyson_G(model.H_k, zero, None, dlr.iw, mu)
    return {"G_iw": g, "mu": mu, "sig_hf_k": zero,
            "sig_iw": np.zeros_like(g), "iteration": 0}


def gw_iteration(model, dlr, state, mixing=1.0, keep=False):
    """One pass of the GW cycle, steps a1 .. a14, from the incoming G.

    Returns the new state; with ``keep`` every intermediate array is returned
    under its step name for the parity tests.
    """
    G_iw = state["G_iw"]
    pairs = model.pairs
    d = model.dim
    inter = {}
    # a12: density of the incoming G, then Hartree + Fock
    n_k = density_k(G_iw, dlr)
    n_R = lattice.R_from_k(n_k, d)
    sig_hf_R = hartree_fock_R(n_R, model.V_R, pairs)
    sig_hf_k = lattice.k_from_R(sig_hf_R, d)
    # a1: Matsubara -> tau and beta - tau
    G_tau = apply_map(dlr.F_iw2tau, G_iw)
    G_reflt = apply_map(dlr.F_iw2taur, G_iw)
    # a2: k -> R
    G_tau_R = lattice.R_from_k(G_tau, d)
    G_reflt_R = lattice.R_from_k(G_reflt, d)
    # a3: bubble
    P_tau_R = bubble(G_tau_R, G_reflt_R, pairs)
    # a4: R -> q
    P_tau_q = lattice.k_from_R(P_tau_R, d)
    # a5: tau -> i nu (bosonic)
    P_nu_q = apply_map(dlr.B_tau2iw, P_tau_q)
    # a6: Dyson W, W^C = W - V
    Wc_nu_q = dyson_W(model.V_q, P_nu_q)
    # a7: i nu -> tau (bosonic)
    Wc_tau_q = apply_map(dlr.B_iw2tau, Wc_nu_q)
    # a8: q -> R
    Wc_tau_R = lattice.R_from_k(Wc_tau_q, d)
    # a9: self-energy
    sig_tau_R = sigma(G_tau_R, Wc_tau_R, pairs, model.n_o)
    # a10: R -> k; Sigma^C(k, tau) is Hermitian (Lehmann form), keep that part
    sig_tau_k = hermitian_part(lattice.k_from_R(sig_tau_R, d), axes=(1, 2))
    # a11: tau -> i omega (fermionic)
    sig_iw = apply_map(dlr.F_tau2iw, sig_tau_k)
    # a14 (part): linear mixing of the total self-energy
    old_total = state["sig_hf_k"][None] + state["sig_iw"]
    new_total = sig_hf_k[None] + sig_iw
    d_sigma = float(np.max(np.abs(new_total - old_total)))
    if mixing != 1.0:
        sig_hf_k = (1.0 - mixing) * state["sig_hf_k"] + mixing * sig_hf_k
        sig_iw = (1.0 - mixing) * state["sig_iw"] + mixing * sig_iw
    # a13: Dyson G with the chemical potential for the target filling
    if model.n_target is None:
        mu = state["mu"]
        G_new = dyson_G(model.H_k, sig_hf_k, sig_iw, dlr.iw, mu)
    else:
        mu, G_new, _ = solve_mu(model.H_k, sig_hf_k, sig_iw, dlr, model.n_target)
    if keep:
        inter = {"n_k": n_k, "n_R": n_R, "sig_hf_R": sig_hf_R, "G_tau": G_tau,
                 "G_reflt": G_reflt, "G_tau_R": G_tau_R, "G_reflt_R": G_reflt_R,
                 "P_tau_R": P_tau_R, "P_tau_q": P_tau_q, "P_nu_q": P_nu_q,
                 "Wc_nu_q": Wc_nu_q, "Wc_tau_q": Wc_tau_q, "Wc_tau_R": Wc_tau_R,
                 "sig_tau_R": sig_tau_R, "sig_tau_k": sig_tau_k}
    out = {"G_iw": G_new, "mu": mu, "sig_hf_k": sig_hf_k, "sig_iw": sig_iw,
           "d_sigma": d_sigma, "iteration": state["iteration"] + 1}
    if keep:
        out["intermediates"] = inter
    return out


def scf(model, dlr, tol=1e-6, max_iter=100, mixing=1.0, state=None, callback=None):
    """GW self-consistency from G0 until max|Delta Sigma| <= tol, where Delta Sigma is the change of
    Sigma_HF + Sigma^C(k, i w_m) over k, node and orbital pair in one iteration."""
    if state is None:
        state = initial_state(model, dlr)
    history = []
    for _ in range(max_iter):
        state = gw_iteration(model, dlr, state, mixing=mixing)
        history.append((state["d_sigma"], state["mu"]))
        if callback is not None:
            callback(state)
        if state["d_sigma"] <= tol:
            break
    return state, history
