"""Reverse-mode derivative of the GW iteration, plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): not for the product path.

The paper has no gradients; this module differentiates the forward steps of
``gw`` as written: a fixed number of iterations from G0, with the chemical
potential differentiated through the implicit function
N_e(mu, H, Sigma) = N_target.

Convention for a real loss L of complex arrays: the cotangent of z is
    zbar = dL/dRe z + i dL/dIm z,
so that dL = Re sum conj(zbar) dz.  Then a complex-linear y = A x has
xbar = A^H ybar, a product y = x1 x2 has x1bar = conj(x2) ybar, and the
Hermitian part (X + X^H)/2 is its own adjoint.
"""
import numpy as np

from . import lattice
from .dlr import apply_map
from .gw import density_k, dyson_G, hermitian_part


# ----------------------------------------------------------------------------
# linear steps
# ----------------------------------------------------------------------------

def apply_map_adj(mat, ybar):
    """Adjoint of out = mat @ x over the node axis: xbar = mat^H @ ybar."""
    return apply_map(np.conj(mat.T), ybar)


def k_from_R_adj(xbar_k, d=2):
    """Adjoint of X(k) = sum_R X(R) e^{-ik.R}: Xbar(R) = sum_k Xbar(k) e^{+ik.R}."""
    n_k = int(np.prod(xbar_k.shape[-d:]))
    return n_k * lattice.R_from_k(xbar_k, d)


def R_from_k_adj(xbar_r, d=2):
    """Adjoint of X(R) = (1/N_k) sum_k X(k) e^{+ik.R}: Xbar(k) = (1/N_k) sum_R Xbar(R) e^{-ik.R}."""
    n_k = int(np.prod(xbar_r.shape[-d:]))
    return lattice.k_from_R(xbar_r, d) / n_k


def density_k_adj(nbar_k, dlr):
    """Adjoint of n(k) = Herm(-rho_beta . G(k, i w)): Gbar[m] = -conj(rho_m) Herm(nbar)."""
    h = hermitian_part(nbar_k)
    rho = np.conj(dlr.F_iw2beta).reshape((-1,) + (1,) * h.ndim)
    return -rho * h[None]


# ----------------------------------------------------------------------------
# bilinear steps
# ----------------------------------------------------------------------------

def hartree_fock_R_adj(sbar_R, n_R, V_R, pairs):
    """Adjoint of gw.hartree_fock_R in both arguments: returns (nbar_R, Vbar_R).

    Fock: S_ik(R) -= V_ab(R) n_lj(R) for a = (i, l), b = (j, k).
    Hartree: S_il(0) += 2 V_ab(q = 0) n_kj(0), V(q = 0) = sum_R V(R).
    """
    nbar = np.zeros_like(n_R)
    vbar = np.zeros_like(V_R)
    d = n_R.ndim - 2
    r0 = (0,) * d                                               # R = 0
    vq0 = np.sum(V_R, axis=lattice.mesh_axes(d))
    vq0bar = np.zeros_like(vq0)
    for al, (i, l) in enumerate(pairs):
        for be, (j, k) in enumerate(pairs):
            vbar[al, be] -= np.conj(n_R[l, j]) * sbar_R[i, k]
            nbar[l, j] -= np.conj(V_R[al, be]) * sbar_R[i, k]
            vq0bar[al, be] += 2.0 * np.conj(n_R[(k, j) + r0]) * sbar_R[(i, l) + r0]
            nbar[(k, j) + r0] += 2.0 * np.conj(vq0[al, be]) * sbar_R[(i, l) + r0]
    vbar += vq0bar.reshape(vq0bar.shape + (1,) * d)
    return nbar, vbar


def bubble_adj(pbar, G_tau_R, G_reflt_R, pairs, spin_factor=2.0):
    """Adjoint of gw.bubble: returns (G_tau_R bar, G_reflt_R bar).

    P_ab(R) = -s G_lj(R, tau) G_ki(-R, beta - tau) for a = (i, l), b = (j, k).
    """
    d = G_tau_R.ndim - 3
    g_minus_r = lattice.reflect(G_reflt_R, d)
    gt_bar = np.zeros_like(G_tau_R)
    gm_bar = np.zeros_like(G_reflt_R)
    for al, (i, l) in enumerate(pairs):
        for be, (j, k) in enumerate(pairs):
            gt_bar[:, l, j] -= spin_factor * np.conj(g_minus_r[:, k, i]) * pbar[:, al, be]
            gm_bar[:, k, i] -= spin_factor * np.conj(G_tau_R[:, l, j]) * pbar[:, al, be]
    return gt_bar, lattice.reflect(gm_bar, d)   # the reflection is its own inverse and adjoint


def sigma_adj(sbar, G_tau_R, Wc_tau_R, pairs):
    """Adjoint of gw.sigma: returns (G_tau_R bar, Wc_tau_R bar).

    S_ik(R, tau) = -sum W^C_ab(R, tau) G_lj(R, tau) for a = (i, l), b = (j, k).
    """
    g_bar = np.zeros_like(G_tau_R)
    w_bar = np.zeros_like(Wc_tau_R)
    for al, (i, l) in enumerate(pairs):
        for be, (j, k) in enumerate(pairs):
            w_bar[:, al, be] -= np.conj(G_tau_R[:, l, j]) * sbar[:, i, k]
            g_bar[:, l, j] -= np.conj(Wc_tau_R[:, al, be]) * sbar[:, i, k]
    return g_bar, w_bar


# ----------------------------------------------------------------------------
# Dyson equations
# ----------------------------------------------------------------------------

def dyson_W_adj(wbar, V_q, P_nu):
    """Adjoint of gw.dyson_W: returns (V_q bar, P_nu bar).

    With A = I - V P and W = A^{-1} V:  dW = A^{-1} dV (I + P W) + W dP W, so
    Pbar = W^H Wbar W^H and Vbar = A^{-H} Wbar (I + P W)^H; W^C = W - V adds
    -Wbar to Vbar.  V(q) is static, so its cotangent sums over the nodes.
    """
    nb = V_q.shape[0]
    v = np.moveaxis(V_q, (0, 1), (-2, -1))
    eye = np.eye(nb)
    vbar = np.zeros_like(v)
    pbar = np.empty_like(P_nu)
    for m in range(P_nu.shape[0]):
        p = np.moveaxis(P_nu[m], (0, 1), (-2, -1))
        wb = np.moveaxis(wbar[m], (0, 1), (-2, -1))
        a = eye - v @ p
        w = np.linalg.solve(a, v)
        ainv_h = np.conj(np.swapaxes(np.linalg.inv(a), -1, -2))
        wh = np.conj(np.swapaxes(w, -1, -2))
        pbar[m] = np.moveaxis(wh @ wb @ wh, (-2, -1), (0, 1))
        vbar += ainv_h @ wb @ np.conj(np.swapaxes(eye + p @ w, -1, -2)) - wb
    return np.moveaxis(vbar, (-2, -1), (0, 1)), pbar


def dyson_G_adj(gbar, H_k, sig_hf_k, sig_iw, dlr, mu, n_target, mubar=0.0):
    """Adjoint of G = [(i w + mu) - H - Sigma_HF - Sigma_C]^{-1} with mu at the filling.

    Returns (Xbar[m, a, b, n1, n2]) with X = H + Sigma_HF + Sigma_C(i w_m):
    H and Sigma_HF receive sum_m Xbar[m], Sigma_C receives Xbar.

    dG = G (dX - dmu) G gives the direct part S = G^H Gbar G^H and
    dL/dmu = mubar - Re sum tr S.  With n_target the chemical potential moves
    with X: N_e(mu, X) = N_target gives dmu = -dN_X / N_mu with
    N_mu = (2/N_k) Re sum rho_m tr G^2 and the X-cotangent of N_e equal to
    -(2/N_k) conj(rho_m) (G^2)^H (the Hermitian part in n does not change
    Re tr n).  Without n_target mu is held fixed.
    """
    g = dyson_G(H_k, sig_hf_k, sig_iw, dlr.iw, mu)
    gm = np.moveaxis(g, (1, 2), (-2, -1))                       # [m, n1, n2, a, b]
    gb = np.moveaxis(gbar, (1, 2), (-2, -1))
    gmh = np.conj(np.swapaxes(gm, -1, -2))
    s = gmh @ gb @ gmh
    if n_target is not None:
        d = g.ndim - 3
        n_kpts = int(np.prod(g.shape[3:]))
        rho = dlr.F_iw2beta.reshape((-1,) + (1,) * d)
        g2 = gm @ gm
        n_mu = 2.0 / n_kpts * float(np.sum((rho * np.trace(g2, axis1=-2, axis2=-1)).real))
        mu_bar_total = mubar - float(np.sum(np.trace(s, axis1=-2, axis2=-1).real))
        n_x = -2.0 / n_kpts * np.conj(rho)[..., None, None] * np.conj(np.swapaxes(g2, -1, -2))
        s = s - (mu_bar_total / n_mu) * n_x
    return np.moveaxis(s, (-2, -1), (1, 2))


# ----------------------------------------------------------------------------
# a14: total energy
# ----------------------------------------------------------------------------

def energy_vjp(model, dlr, state, ebar):
    """Cotangents of ebar * gw.total_energy(model, dlr, state)[0].

    E_HF = 2/N_k Re sum A_ab n_ba with A = H0 + Sigma_HF / 2 gives
    Abar = c conj(n^T), nbar = c conj(A^T) (c = 2 ebar / N_k), and n = Herm(-rho G);
    E_c = 1/N_k Re sum S_m,ab F_gm[m, m'] G_m',ba gives
    Sbar = ebar/N_k conj((F_gm G)^T), Gbar += ebar/N_k conj((F_gm^T S)^T).
    Returns cotangents of H_k, sig_hf_k, sig_iw and G_iw.
    """
    G = state["G_iw"]
    n_k = density_k(G, dlr)
    c = 2.0 * ebar / model.n_k
    a = model.H_k + 0.5 * state["sig_hf_k"]
    abar = c * np.conj(np.swapaxes(n_k, 0, 1))
    gbar = density_k_adj(c * np.conj(np.swapaxes(a, 0, 1)), dlr)
    qg = apply_map(dlr.F_gm, G)
    sq = apply_map(dlr.F_gm.T, state["sig_iw"])
    sbar = ebar / model.n_k * np.conj(np.swapaxes(qg, 1, 2))
    gbar = gbar + ebar / model.n_k * np.conj(np.swapaxes(sq, 1, 2))
    return {"H_k": abar, "sig_hf_k": 0.5 * abar, "sig_iw": sbar, "G_iw": gbar}


# ----------------------------------------------------------------------------
# one iteration, and the parameter chain from G0
# ----------------------------------------------------------------------------

def iteration_vjp(model, dlr, state_in, out, cot):
    """Cotangents of one gw.gw_iteration (mixing 1) through all its steps.

    ``out`` is the iteration's result with ``keep=True``.  ``cot`` holds the
    cotangents of the outputs: "G_iw", "sig_iw", "sig_hf_k" (arrays or None),
    "mu" and "energy" (floats; the energy is that of the output state).  Returns a dict with the cotangents of the incoming
    G_iw and of the model inputs H_k and V_R (V enters as V(R) in
    Hartree-Fock and as V(q) = FT V(R) in Dyson W).
    """
    inter = out["intermediates"]
    pairs = model.pairs
    d = model.dim
    G_iw = state_in["G_iw"]
    gbar_new = cot.get("G_iw")
    if gbar_new is None:
        gbar_new = np.zeros_like(G_iw)
    ev = None
    if cot.get("energy"):
        ev = energy_vjp(model, dlr, out, cot["energy"])
        gbar_new = gbar_new + ev["G_iw"]
    # a13
    xbar = dyson_G_adj(gbar_new, model.H_k, out["sig_hf_k"], out["sig_iw"], dlr, out["mu"], model.n_target,
                       mubar=cot.get("mu", 0.0))
    hbar_k = np.sum(xbar, axis=0)
    shf_bar = np.sum(xbar, axis=0)
    if cot.get("sig_hf_k") is not None:
        shf_bar = shf_bar + cot["sig_hf_k"]
    sc_bar = xbar.copy()
    if cot.get("sig_iw") is not None:
        sc_bar = sc_bar + cot["sig_iw"]
    if ev is not None:
        hbar_k = hbar_k + ev["H_k"]
        shf_bar = shf_bar + ev["sig_hf_k"]
        sc_bar = sc_bar + ev["sig_iw"]
    # a11, a10 (Hermitian part), a9
    stk_bar = hermitian_part(apply_map_adj(dlr.F_tau2iw, sc_bar), axes=(1, 2))
    str_bar = k_from_R_adj(stk_bar, d)
    gt_bar, wct_r_bar = sigma_adj(str_bar, inter["G_tau_R"], inter["Wc_tau_R"], pairs)
    # a8, a7, a6
    wct_q_bar = R_from_k_adj(wct_r_bar, d)
    wcn_bar = apply_map_adj(dlr.B_iw2tau, wct_q_bar)
    vq_bar, pn_bar = dyson_W_adj(wcn_bar, model.V_q, inter["P_nu_q"])
    # a5, a4, a3
    ptq_bar = apply_map_adj(dlr.B_tau2iw, pn_bar)
    ptr_bar = k_from_R_adj(ptq_bar, d)
    gt2, gr_bar = bubble_adj(ptr_bar, inter["G_tau_R"], inter["G_reflt_R"], pairs)
    gt_bar = gt_bar + gt2
    # a2, a1
    gin_bar = (apply_map_adj(dlr.F_iw2tau, R_from_k_adj(gt_bar, d))
               + apply_map_adj(dlr.F_iw2taur, R_from_k_adj(gr_bar, d)))
    # a12: Hartree-Fock from the density of the incoming G
    shf_r_bar = k_from_R_adj(shf_bar, d)
    n_r_bar, vr_bar = hartree_fock_R_adj(shf_r_bar, inter["n_R"], model.V_R, pairs)
    gin_bar = gin_bar + density_k_adj(R_from_k_adj(n_r_bar, d), dlr)
    vr_bar = vr_bar + k_from_R_adj(vq_bar, d)
    return {"G_iw": gin_bar, "H_k": hbar_k, "V_R": vr_bar}


def g0_vjp(model, dlr, state0, gbar):
    """Cotangent of H_k through G0 = [(i w + mu0) - H0(k)]^{-1} with mu0 at the filling."""
    zero = np.zeros_like(model.H_k)
    xbar = dyson_G_adj(gbar, model.H_k, zero, None, dlr, state0["mu"], model.n_target)
    return np.sum(xbar, axis=0)


def one_iteration_grad(model, dlr, cot):
    """Gradient of L(one GW iteration from G0) with respect to H0(R) and V(R).

    Returns (out, {"H_R": Hbar_R, "V_R": Vbar_R}) where ``out`` is the forward
    result and the cotangents follow the module's convention.
    """
    from . import gw
    st0 = gw.initial_state(model, dlr)
    out = gw.gw_iteration(model, dlr, st0, keep=True)
    c = iteration_vjp(model, dlr, st0, out, cot)
    hbar_k = c["H_k"] + g0_vjp(model, dlr, st0, c["G_iw"])
    return out, {"H_R": k_from_R_adj(hbar_k, model.dim), "V_R": c["V_R"]}


def n_iteration_grad(model, dlr, cot, n_iter):
    """Gradient of L(state after n GW iterations from G0) with respect to H0(R) and V(R).

    The forward keeps every iteration's input state (the checkpoints); the
    backward runs the iterations' adjoints in reverse, passing the incoming-G
    cotangent of one iteration to the G output of the one before, and adds
    up the H and V cotangents of all of them and of G0.
    """
    from . import gw
    states = [gw.initial_state(model, dlr)]
    outs = []
    for _ in range(n_iter):
        o = gw.gw_iteration(model, dlr, states[-1], keep=True)
        outs.append(o)
        states.append(o)
    hbar_k = np.zeros_like(model.H_k)
    vbar_r = np.zeros_like(model.V_R)
    c = dict(cot)
    for it in range(n_iter - 1, -1, -1):
        res = iteration_vjp(model, dlr, states[it], outs[it], c)
        hbar_k = hbar_k + res["H_k"]
        vbar_r = vbar_r + res["V_R"]
        c = {"G_iw": res["G_iw"]}
    hbar_k = hbar_k + g0_vjp(model, dlr, states[0], c["G_iw"])
    return outs[-1], {"H_R": k_from_R_adj(hbar_k, model.dim), "V_R": vbar_r}
