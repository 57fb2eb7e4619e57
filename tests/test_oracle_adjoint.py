"""Pins of the oracle's reverse-mode derivative (not GPU).

Linear steps: the dot-product identity Re<ybar, A x> = Re<A^H ybar, x> for
random x, ybar.  Nonlinear steps and the whole iteration: central finite
differences of the oracle's forward along random unit directions with one
Richardson step (h = 3e-5, truncation ~h^4), held to the 1e-5 relative bar
for gradients.  The cotangent convention is zbar = dL/dRe z + i dL/dIm z, so
a directional derivative is Re sum conj(zbar) d.
"""
import numpy as np
import pytest

from conftest import directional_fd
from oracle import adjoint as ad
from oracle import gw, lattice
from oracle.dlr import DLR, apply_map
from paper_2604_22223_amd import workloads as wl

GRAD_TOL = 1e-5


def crand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rdot(a, b):
    return float(np.sum(np.conj(a) * b).real)


def check(g, f, x, d):
    """Directional derivative along the unit direction d / |d| against Re<g, d / |d|>."""
    d = d / np.linalg.norm(d)
    num = directional_fd(f, x, d)
    ana = rdot(g, d)
    assert abs(num - ana) <= GRAD_TOL * abs(num) + 1e-9 * np.linalg.norm(g), (num, ana)


@pytest.fixture(scope="module")
def small():
    w = wl.random_model((3, 3), [2, 1], seed=5, beta=8.0, omega_max=12.0, eps=1e-10, U=1.5, J=0.2, Vnn=0.3)
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    return w, d, m


# ----------------------------------------------------------------------------
# linear steps: dot-product identities
# ----------------------------------------------------------------------------

def test_linear_adjoints_dot_product(small):
    w, d, m = small
    rng = np.random.default_rng(1)
    shape = (d.r, 3, 3, 3, 3)
    x, yb = crand(rng, shape), crand(rng, shape)
    for mat in (d.F_iw2tau, d.F_iw2taur, d.F_tau2iw, d.B_tau2iw, d.B_iw2tau):
        assert abs(rdot(yb, apply_map(mat, x)) - rdot(ad.apply_map_adj(mat, yb), x)) < 1e-9 * np.abs(yb).sum()
    assert abs(rdot(yb, lattice.k_from_R(x)) - rdot(ad.k_from_R_adj(yb), x)) < 1e-10 * np.abs(yb).sum()
    assert abs(rdot(yb, lattice.R_from_k(x)) - rdot(ad.R_from_k_adj(yb), x)) < 1e-10 * np.abs(yb).sum()
    nb = crand(rng, (3, 3, 3, 3))
    assert abs(rdot(nb, gw.density_k(x, d)) - rdot(ad.density_k_adj(nb, d), x)) < 1e-9 * np.abs(nb).sum()
    # reflection and Hermitian part are self-adjoint
    assert abs(rdot(yb, lattice.reflect(x)) - rdot(lattice.reflect(yb), x)) < 1e-10 * np.abs(yb).sum()
    assert abs(rdot(yb, gw.hermitian_part(x, (1, 2))) - rdot(gw.hermitian_part(yb, (1, 2)), x)) < 1e-10 * np.abs(yb).sum()


# ----------------------------------------------------------------------------
# bilinear and nonlinear steps: finite differences
# ----------------------------------------------------------------------------

def test_bubble_and_sigma_adjoints(small):
    w, d, m = small
    rng = np.random.default_rng(2)
    shp_g = (d.r, m.n_o, m.n_o) + m.mesh
    shp_p = (d.r, m.n_b, m.n_b) + m.mesh
    gt, gr, wc = crand(rng, shp_g), crand(rng, shp_g), crand(rng, shp_p)
    c_p, c_s = crand(rng, shp_p), crand(rng, shp_g)
    gtb, grb = ad.bubble_adj(c_p, gt, gr, m.pairs)
    check(gtb, lambda x: rdot(c_p, gw.bubble(x, gr, m.pairs)), gt, crand(rng, shp_g))
    check(grb, lambda x: rdot(c_p, gw.bubble(gt, x, m.pairs)), gr, crand(rng, shp_g))
    gb, wb = ad.sigma_adj(c_s, gt, wc, m.pairs)
    check(gb, lambda x: rdot(c_s, gw.sigma(x, wc, m.pairs, m.n_o)), gt, crand(rng, shp_g))
    check(wb, lambda x: rdot(c_s, gw.sigma(gt, x, m.pairs, m.n_o)), wc, crand(rng, shp_p))


def test_hartree_fock_adjoint(small):
    w, d, m = small
    rng = np.random.default_rng(3)
    n_r = crand(rng, (m.n_o, m.n_o) + m.mesh)
    c = crand(rng, (m.n_o, m.n_o) + m.mesh)
    nb, vb = ad.hartree_fock_R_adj(c, n_r, m.V_R, m.pairs)
    check(nb, lambda x: rdot(c, gw.hartree_fock_R(x, m.V_R, m.pairs)), n_r, crand(rng, n_r.shape))
    check(vb, lambda x: rdot(c, gw.hartree_fock_R(n_r, x, m.pairs)), m.V_R, crand(rng, m.V_R.shape))


def test_dyson_w_adjoint(small):
    w, d, m = small
    rng = np.random.default_rng(4)
    p = 0.1 * crand(rng, (d.r, m.n_b, m.n_b) + m.mesh)
    c = crand(rng, p.shape)
    vb, pb = ad.dyson_W_adj(c, m.V_q, p)
    check(pb, lambda x: rdot(c, gw.dyson_W(m.V_q, x)), p, crand(rng, p.shape))
    check(vb, lambda x: rdot(c, gw.dyson_W(x, p)), m.V_q, crand(rng, m.V_q.shape))


@pytest.mark.parametrize("with_mu", [False, True])
def test_dyson_g_adjoint(small, with_mu):
    """Fixed mu, and mu at the filling (implicit function), with a mu cotangent."""
    w, d, m = small
    rng = np.random.default_rng(5)
    sig = 0.05 * crand(rng, (d.r, m.n_o, m.n_o) + m.mesh)
    sig = gw.hermitian_part(sig, (1, 2))
    hf = np.zeros_like(m.H_k)
    c = crand(rng, sig.shape)
    c_mu = 0.7
    nt = m.n_target if with_mu else None
    mu0, g0, _ = gw.solve_mu(m.H_k, hf, sig, d, m.n_target)

    def fwd(h, s):
        if nt is None:
            return rdot(c, gw.dyson_G(h, hf, s, d.iw, mu0))
        mu, g, _ = gw.solve_mu(h, hf, s, d, nt)
        return rdot(c, g) + c_mu * mu

    xb = ad.dyson_G_adj(c, m.H_k, hf, sig, d, mu0, nt, mubar=c_mu if with_mu else 0.0)
    dh = gw.hermitian_part(crand(rng, m.H_k.shape))
    ds = crand(rng, sig.shape)
    check(np.sum(xb, axis=0), lambda x: fwd(x, sig), m.H_k, dh)
    check(xb, lambda x: fwd(m.H_k, x), sig, ds)


# ----------------------------------------------------------------------------
# the whole iteration from G0, by parameters
# ----------------------------------------------------------------------------

def _loss_parts(rng, m, d):
    shp = (d.r, m.n_o, m.n_o) + m.mesh
    return {"sig_iw": crand(rng, shp), "sig_hf_k": crand(rng, (m.n_o, m.n_o) + m.mesh),
            "G_iw": crand(rng, shp), "mu": 0.9, "energy": 1.7}


def _loss(out, cot, m=None, d=None):
    val = (rdot(cot["sig_iw"], out["sig_iw"]) + rdot(cot["sig_hf_k"], out["sig_hf_k"])
           + rdot(cot["G_iw"], out["G_iw"]) + cot["mu"] * out["mu"])
    if m is not None:
        val += cot["energy"] * gw.total_energy(m, d, out)[0]
    return val


def _sym_dir(rng, shape):
    """A direction X with X(-R) = X(R)^dagger (keeps H0 Hermitian in k)."""
    x = crand(rng, shape)
    return x + np.conj(np.swapaxes(lattice.reflect(x), 0, 1))


def test_one_iteration_gradient_by_finite_differences(small):
    w, d, m = small
    rng = np.random.default_rng(6)
    cot = _loss_parts(rng, m, d)
    out, g = ad.one_iteration_grad(m, d, cot)

    def L(H_R, V_R):
        mm = gw.Model(m.mesh, m.site_norb, H_R, V_R, m.beta, m.n_target)
        st0 = gw.initial_state(mm, d)
        return _loss(gw.gw_iteration(mm, d, st0), cot, mm, d)

    assert abs(L(m.H_R, m.V_R) - _loss(out, cot, m, d)) < 1e-12 * abs(_loss(out, cot, m, d))
    for trial in range(2):
        dh = _sym_dir(rng, m.H_R.shape)
        check(g["H_R"], lambda x: L(x, m.V_R), m.H_R, dh)
        dv = _sym_dir(rng, m.V_R.shape)
        check(g["V_R"], lambda x: L(m.H_R, x), m.V_R, dv)


def test_energy_adjoint(small):
    """The energy alone, in every argument, by finite differences."""
    w, d, m = small
    rng = np.random.default_rng(9)
    st = gw.gw_iteration(m, d, gw.initial_state(m, d))
    ev = ad.energy_vjp(m, d, st, 1.0)

    def E(**over):
        s2 = dict(st)
        mm = m
        if "H_k" in over:
            mm = gw.Model(m.mesh, m.site_norb, m.H_R, m.V_R, m.beta, m.n_target)
            mm.H_k = over.pop("H_k")
        s2.update(over)
        return gw.total_energy(mm, d, s2)[0]

    for key in ("G_iw", "sig_iw", "sig_hf_k"):
        check(ev[key], lambda x, key=key: E(**{key: x}), st[key], crand(rng, st[key].shape))
    check(ev["H_k"], lambda x: E(H_k=x), m.H_k, crand(rng, m.H_k.shape))


def test_one_iteration_gradient_in_U_J_V():
    """Scalar interaction parameters of the five-orbital model (V is linear in U, J, V_nn)."""
    kw = dict(n=3, beta=6.0, omega_max=10.0, eps=1e-10, scale_mesh=3, norb=2, n_target=2.0)
    base = dict(U=1.0, J=0.1, Vnn=0.2)
    w = wl.five_orbital(**kw, **base)
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    rng = np.random.default_rng(7)
    cot = _loss_parts(rng, m, d)
    out, g = ad.one_iteration_grad(m, d, cot)

    def L(**p):
        ww = wl.five_orbital(**kw, **p)
        mm = gw.Model(ww["mesh"], ww["site_norb"], ww["H_R"], ww["V_R"], ww["beta"], ww["n_target"])
        return _loss(gw.gw_iteration(mm, d, gw.initial_state(mm, d)), cot, mm, d)

    for name in ("U", "J", "Vnn"):
        def f(t):
            p = dict(base)
            p[name] += float(t)
            return L(**p)
        num = directional_fd(f, 0.0, 1.0)
        up = dict(base); up[name] += 1.0
        dv = wl.five_orbital(**kw, **up)["V_R"] - wl.five_orbital(**kw, **base)["V_R"]   # V is linear in U, J, V_nn
        ana = rdot(g["V_R"], dv)
        assert abs(num - ana) <= GRAD_TOL * abs(num) + 1e-9, (name, num, ana)


def test_two_iteration_gradient_by_finite_differences(small):
    w, d, m = small
    rng = np.random.default_rng(8)
    cot = _loss_parts(rng, m, d)
    out, g = ad.n_iteration_grad(m, d, cot, 2)

    def L(H_R, V_R):
        mm = gw.Model(m.mesh, m.site_norb, H_R, V_R, m.beta, m.n_target)
        st = gw.initial_state(mm, d)
        for _ in range(2):
            st = gw.gw_iteration(mm, d, st)
        return _loss(st, cot, mm, d)

    check(g["H_R"], lambda x: L(x, m.V_R), m.H_R, _sym_dir(rng, m.H_R.shape))
    check(g["V_R"], lambda x: L(m.H_R, x), m.V_R, _sym_dir(rng, m.V_R.shape))
