"""Parity of every adjoint entry point with the oracle's reverse mode, and
gradients of whole iterations through torch.autograd (FP64).

Each ``*_bwd`` call gets a seeded random cotangent and the oracle's forward
arrays, and is compared element by element with the oracle's adjoint at the
FP64 bar (max |gpu - oracle| / max |oracle| <= 1e-10; 1e-9 for the chains).

The DLR maps are the exception: the library and the oracle build them
independently in FP64, and as matrices they agree only to what their
conditioning allows (1e-5; applied to representable data, to rounding).  A
random cotangent is not representable data, so the map adjoints are pinned
twice: as exact adjoints of the library's own forward maps (the dot-product
identity Re<ybar, T x> = Re<T^H ybar, x> to 1e-12), and against the oracle's
adjoint at the matrices' 1e-5.

The autograd gradients are also checked against central finite differences
of the GPU forward itself (unit directions, one Richardson step, relative
1e-5).
"""
import numpy as np
import pytest

from conftest import directional_fd, rel_err
from oracle import adjoint as ad
from oracle import gw, lattice
from oracle.dlr import DLR, apply_map
from paper_2604_22223_amd import qgw
from paper_2604_22223_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(x):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


# number of mesh axes of the current case (2, or 3 on a cubic mesh); set by the ``case`` fixture
_MESH_DIM = [2]


def flat(x):
    """oracle [..., n1, n2] (or [..., n1, n2, n3]) -> library [..., N_k]"""
    return np.ascontiguousarray(x.reshape(x.shape[:-_MESH_DIM[0]] + (-1,)))


def crand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def to_matrix(x):
    """oracle pair slab [r, A, B, n1, n2] -> library matrix layout [r, N_k, A, B]"""
    f = flat(x)
    return np.ascontiguousarray(np.moveaxis(f, -1, 1))


def from_matrix(x, mesh):
    """library matrix layout [r, N_k, A, B] -> oracle pair slab [r, A, B, n1, n2]"""
    s = np.moveaxis(x, 1, -1)
    return s.reshape(s.shape[:-1] + tuple(mesh))


class Case:
    def __init__(self, w):
        self.w = w
        self.d = DLR(w["beta"], w["omega_max"], w["eps"])
        self.m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
        self.st0 = gw.initial_state(self.m, self.d)
        self.out = gw.gw_iteration(self.m, self.d, self.st0, keep=True)
        self.inter = self.out["intermediates"]
        self.mesh = tuple(w["mesh"])
        self.dim = len(self.mesh)
        self.plan = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], self.d.nodes(), dim=self.dim)


CASES = {
    # a contracting coupling (the loop damps differences between iterations)
    "random_2+1_5x5": lambda: wl.random_model((5, 5), [2, 1], seed=11, beta=8.0, omega_max=15.0, eps=1e-10,
                                              U=0.7, J=0.1, Vnn=0.1),
    "five_orbital_6x6": lambda: wl.five_orbital(n=6, U=1.0, J=0.1, Vnn=0.2, beta=10.0, omega_max=20.0, eps=1e-10,
                                                scale_mesh=6),
    "random3d_2+1_4x4x4": lambda: wl.random_model_3d((4, 4, 4), [2, 1], seed=11, beta=8.0, omega_max=15.0,
                                                     eps=1e-10, U=0.7, J=0.1, Vnn=0.1),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print("\n[adjoint case] %s" % request.param, flush=True)
    c = Case(CASES[request.param]())
    _MESH_DIM[0] = c.dim
    return c


def _rdot(a, b):
    return float(np.sum(np.conj(a) * b).real)


def _dot_identity(fwd_out, ybar, bwd_out, x):
    """|Re<ybar, T x> - Re<T^H ybar, x>| relative to the sum of the products' magnitudes."""
    ybar, fwd_out, bwd_out, x = (np.ravel(v) for v in (ybar, fwd_out, bwd_out, x))
    lhs = _rdot(ybar, fwd_out)
    rhs = _rdot(bwd_out, x)
    scale = float(np.sum(np.abs(ybar) * np.abs(fwd_out)))
    return abs(lhs - rhs) / scale


MAP_TOL = 1e-5


def test_dlr_bwd(case):
    torch = _torch()
    d, m, p = case.d, case.m, case.plan
    rng = np.random.default_rng(1)
    shp = (d.r, m.n_o, m.n_o) + case.mesh
    yb, x = crand(rng, shp), crand(rng, shp)
    s = 0.5 - 0.25j
    for which, mat in [(qgw.F_IW2TAU, d.F_iw2tau), (qgw.F_IW2TAUR, d.F_iw2taur), (qgw.F_TAU2IW, d.F_tau2iw),
                       (qgw.B_TAU2IW, d.B_tau2iw), (qgw.B_IW2TAU, d.B_iw2tau), (qgw.F_IW2GM, d.F_gm)]:
        for herm in (0, 1, 2):
            fwd = torch.empty_like(dev(flat(x)))
            p.dlr_transform(which, dev(flat(x)), fwd, scale=s, hermitian=herm)
            out = torch.empty_like(fwd)
            p.dlr_transform_bwd(which, dev(flat(yb)), out, scale=s, hermitian=herm)
            assert _dot_identity(host(fwd), flat(yb), host(out), flat(x)) < 1e-12, (which, herm)
        out = torch.empty_like(dev(flat(yb)))
        if which == qgw.F_IW2GM:
            # The Matsubara-sum map is meaningful only as a bilinear form on representable
            # data (its entries carry the square of the kernel's condition number): pair
            # the adjoint of conj(K c1) with K c2, which must give s c1^T D c2.
            c1, c2 = crand(rng, shp), crand(rng, shp)
            y_rep, x_rep = np.conj(apply_map(d.K_f, c1)), apply_map(d.K_f, c2)
            p.dlr_transform_bwd(which, dev(flat(y_rep)), out, scale=s)
            got = np.sum(np.conj(host(out)) * flat(x_rep))
            want = s * np.einsum("lm,lx,mx->", d.D_sum, c1.reshape(d.r, -1), c2.reshape(d.r, -1))
            assert abs(got - want) <= 1e-9 * abs(want), (got, want)
            continue
        p.dlr_transform_bwd(which, dev(flat(yb)), out, scale=s)
        assert rel_err(host(out), flat(np.conj(s) * ad.apply_map_adj(mat, yb))) < MAP_TOL, which
    # a11 with the Hermitian part of its input
    out = torch.empty_like(dev(flat(yb)))
    p.dlr_transform_bwd(qgw.F_TAU2IW, dev(flat(yb)), out, hermitian=1)
    ref = gw.hermitian_part(ad.apply_map_adj(d.F_tau2iw, yb), axes=(1, 2))
    assert rel_err(host(out), flat(ref)) < MAP_TOL
    # density row (one output row), every Hermitian mode; the oracle's form is scale -1, herm 2
    nb = crand(rng, (m.n_o, m.n_o) + case.mesh)
    for herm in (0, 1, 2):
        fwd = torch.empty_like(dev(flat(nb)))
        p.dlr_transform(qgw.F_IW2BETA, dev(flat(x)), fwd, scale=s, hermitian=herm)
        out = torch.empty_like(dev(flat(yb)))
        p.dlr_transform_bwd(qgw.F_IW2BETA, dev(flat(nb)), out, scale=s, hermitian=herm)
        assert _dot_identity(host(fwd), flat(nb), host(out), flat(x)) < 1e-12, herm
    out = torch.empty_like(dev(flat(yb)))
    p.dlr_transform_bwd(qgw.F_IW2BETA, dev(flat(nb)), out, scale=-1.0, hermitian=2)
    assert rel_err(host(out), flat(ad.density_k_adj(nb, d))) < MAP_TOL


def test_dlr_pairs_and_fft_bwd(case):
    torch = _torch()
    d, m, p = case.d, case.m, case.plan
    rng = np.random.default_rng(2)
    shp = (d.r, m.n_b, m.n_b) + case.mesh
    yb, x = crand(rng, shp), crand(rng, shp)
    for which, mat in [(qgw.B_TAU2IW, d.B_tau2iw), (qgw.B_IW2TAU, d.B_iw2tau)]:
        for lin, lout in [(qgw.LAYOUT_SLAB, qgw.LAYOUT_MATRIX), (qgw.LAYOUT_MATRIX, qgw.LAYOUT_SLAB)]:
            xin = dev(flat(x) if lin == qgw.LAYOUT_SLAB else to_matrix(x))
            ybi = dev(flat(yb) if lout == qgw.LAYOUT_SLAB else to_matrix(yb))
            fwd = torch.empty_like(xin)
            p.dlr_transform_pairs(which, lin, lout, xin, fwd)
            out = torch.empty_like(xin)
            p.dlr_transform_pairs_bwd(which, lin, lout, ybi, out)
            assert _dot_identity(host(fwd), host(ybi), host(out), host(xin)) < 1e-12, (which, lin)
            got = host(out)
            if lin == qgw.LAYOUT_MATRIX:
                got = flat(from_matrix(got.reshape(d.r, m.n_k, m.n_b, m.n_b), case.mesh))
            assert rel_err(got, flat(ad.apply_map_adj(mat, yb))) < MAP_TOL, (which, lin)
    # lattice transforms, both directions, in place allowed: exact to rounding
    for direction, fn in [(qgw.K_TO_R, ad.R_from_k_adj), (qgw.R_TO_K, ad.k_from_R_adj)]:
        xx = dev(flat(yb))
        p.lattice_fft_bwd(direction, xx, xx)
        assert rel_err(host(xx), flat(fn(yb, case.dim))) < TOL


def test_bubble_bwd(case):
    torch = _torch()
    d, m, p, it = case.d, case.m, case.plan, case.inter
    rng = np.random.default_rng(3)
    pb = crand(rng, (d.r, m.n_b, m.n_b) + case.mesh)
    gt, gr = dev(flat(it["G_tau_R"])), dev(flat(it["G_reflt_R"]))
    a, b = torch.empty_like(gt), torch.empty_like(gr)
    p.bubble_bwd(gt, gr, dev(flat(pb)), a, b)
    ra, rb = ad.bubble_adj(ad.k_from_R_adj(pb, case.dim), it["G_tau_R"], it["G_reflt_R"], m.pairs)
    assert rel_err(host(a), flat(ra)) < TOL
    assert rel_err(host(b), flat(rb)) < TOL


def test_sigma_bwd(case):
    torch = _torch()
    d, m, p, it = case.d, case.m, case.plan, case.inter
    rng = np.random.default_rng(4)
    sb = crand(rng, (d.r, m.n_o, m.n_o) + case.mesh)
    gt, wc = dev(flat(it["G_tau_R"])), dev(flat(it["Wc_tau_q"]))
    a, b = torch.empty_like(gt), torch.empty_like(wc)
    p.sigma_bwd(gt, wc, dev(flat(sb)), a, b, out_k=True)
    ga, wr = ad.sigma_adj(ad.k_from_R_adj(sb, case.dim), it["G_tau_R"], it["Wc_tau_R"], m.pairs)
    assert rel_err(host(a), flat(ga)) < TOL
    assert rel_err(host(b), flat(ad.R_from_k_adj(wr, case.dim))) < TOL


def test_dyson_w_bwd(case):
    torch = _torch()
    d, m, p, it = case.d, case.m, case.plan, case.inter
    rng = np.random.default_rng(5)
    wb = crand(rng, (d.r, m.n_b, m.n_b) + case.mesh)
    vq = dev(np.ascontiguousarray(np.moveaxis(flat(m.V_q), -1, 0)))
    pnu = dev(to_matrix(it["P_nu_q"]))
    pbar, vbar = torch.empty_like(pnu), torch.empty_like(vq)
    p.dyson_W_bwd(vq, pnu, dev(to_matrix(wb)), pbar, vbar)
    rv, rp = ad.dyson_W_adj(wb, m.V_q, it["P_nu_q"])
    assert rel_err(from_matrix(host(pbar), case.mesh), rp) < TOL
    assert rel_err(np.moveaxis(host(vbar), 0, -1).reshape(rv.shape), rv) < TOL


def test_hartree_fock_bwd(case):
    torch = _torch()
    d, m, p, it = case.d, case.m, case.plan, case.inter
    rng = np.random.default_rng(6)
    sb = crand(rng, (m.n_o, m.n_o) + case.mesh)
    nr, vr = dev(flat(it["n_R"])), dev(flat(m.V_R))
    nb, vb = torch.empty_like(nr), torch.empty_like(vr)
    p.hartree_fock_bwd(vr, nr, dev(flat(sb)), nb, vb)
    rn, rv = ad.hartree_fock_R_adj(sb, it["n_R"], m.V_R, m.pairs)
    assert rel_err(host(nb), flat(rn)) < TOL
    assert rel_err(host(vb), flat(rv)) < TOL


@pytest.mark.parametrize("with_mu", [False, True])
def test_dyson_g_bwd(case, with_mu):
    """Fixed mu: against the oracle at the FP64 bar.  Mu at the filling: the
    implicit term weighs the cotangent with the density row rho_beta, which
    the library and the oracle build independently (as vectors they agree to
    1e-5, see the map test); it is held against the oracle at 1e-7 and
    against central differences of the library's own Dyson-G solve at 1e-6."""
    torch = _torch()
    d, m, p, out = case.d, case.m, case.plan, case.out
    rng = np.random.default_rng(7)
    gb = crand(rng, (d.r, m.n_o, m.n_o) + case.mesh)
    hs_np = flat(m.H_k + out["sig_hf_k"])
    hs = dev(hs_np)
    sig = dev(flat(out["sig_iw"]))
    sb, hb = torch.empty_like(sig), torch.empty_like(hs)
    nt = m.n_target if with_mu else None
    mubar = 0.3 if with_mu else 0.0
    p.dyson_G_bwd(hs, sig, out["mu"], dev(flat(gb)), sb, hb, n_target=nt, mubar=mubar)
    ref = ad.dyson_G_adj(gb, m.H_k, out["sig_hf_k"], out["sig_iw"], d, out["mu"], nt, mubar=mubar)
    tol = 1e-7 if with_mu else 1e-9
    assert rel_err(host(sb), flat(ref)) < tol
    assert rel_err(host(hb), flat(np.sum(ref, axis=0))) < tol
    if not with_mu:
        return
    g_out = torch.empty_like(sig)

    def L(h):
        mu = p.dyson_G(dev(h), sig, g_out, n_target=nt, mu=out["mu"])
        return _rdot(flat(gb), host(g_out)) + mubar * mu

    dh = crand(rng, hs_np.shape)
    dh = dh + np.conj(np.swapaxes(dh, 0, 1))        # Hermitian at every k
    dh /= np.linalg.norm(dh)
    num = directional_fd(L, hs_np, dh)
    ana = _rdot(host(hb), dh)
    assert abs(num - ana) <= 1e-6 * abs(num), (num, ana)


# ----------------------------------------------------------------------------
# whole iterations through torch.autograd
# ----------------------------------------------------------------------------

def _cotangents(case, seed):
    rng = np.random.default_rng(seed)
    d, m = case.d, case.m
    shp = (d.r, m.n_o, m.n_o) + case.mesh
    return {"sig_iw": crand(rng, shp), "sig_hf_k": crand(rng, (m.n_o, m.n_o) + case.mesh),
            "G_iw": crand(rng, shp), "mu": 0.9, "energy": 1.7}


def _torch_loss(res, cot, plan=None, H_R=None):
    """Projections of the outputs, plus the total energy of the output state when H_R is given."""
    from paper_2604_22223_amd import autograd as qa
    G, mu, Siw, shf = res
    tot = 0.0
    for t, c in ((Siw, cot["sig_iw"]), (shf, cot["sig_hf_k"]), (G, cot["G_iw"])):
        tot = tot + (dev(flat(c)).conj() * t).real.sum()
    tot = tot + cot["mu"] * mu.to(tot.device)
    if H_R is not None:
        H_k = qa.FFT.apply(plan, qgw.R_TO_K, H_R)
        tot = tot + cot["energy"] * qa.energy(plan, H_k, shf, Siw, G).to(tot.device)
    return tot


@pytest.mark.parametrize("n_iter", [1, 2])
def test_iteration_gradients_match_oracle_adjoint(case, n_iter):
    torch = _torch()
    from paper_2604_22223_amd import autograd as qa
    m, d, p = case.m, case.d, case.plan
    cot = _cotangents(case, 8 + n_iter)
    H_R = dev(flat(m.H_R)).requires_grad_(True)
    V_R = dev(flat(m.V_R)).requires_grad_(True)
    res = qa.run(p, H_R, V_R, m.n_target, n_iter=n_iter, checkpointed=True)[-1]
    loss = _torch_loss(res, cot, p, H_R)
    loss.backward()
    ref_out, ref = ad.n_iteration_grad(m, d, cot, n_iter)
    assert rel_err(host(res[2]), flat(ref_out["sig_iw"])) < TOL
    assert abs(float(res[1].detach()) - ref_out["mu"]) <= 1e-10 * max(1.0, abs(ref_out["mu"]))
    assert rel_err(host(H_R.grad), flat(ref["H_R"])) < 1e-9
    assert rel_err(host(V_R.grad), flat(ref["V_R"])) < 1e-9


def test_checkpointing_changes_nothing(case):
    torch = _torch()
    from paper_2604_22223_amd import autograd as qa
    m, p = case.m, case.plan
    cot = _cotangents(case, 20)
    grads = []
    for ck in (True, False):
        H_R = dev(flat(m.H_R)).requires_grad_(True)
        V_R = dev(flat(m.V_R)).requires_grad_(True)
        _torch_loss(qa.run(p, H_R, V_R, m.n_target, n_iter=2, checkpointed=ck)[-1], cot, p, H_R).backward()
        grads.append((host(H_R.grad), host(V_R.grad)))
    assert rel_err(grads[0][0], grads[1][0]) < 1e-13
    assert rel_err(grads[0][1], grads[1][1]) < 1e-13


def test_gradient_against_gpu_finite_differences(case):
    """Central differences of the GPU forward along seeded Hermitian-consistent unit directions."""
    torch = _torch()
    from paper_2604_22223_amd import autograd as qa
    m, p = case.m, case.plan
    cot = _cotangents(case, 30)
    rng = np.random.default_rng(31)
    H_R = dev(flat(m.H_R)).requires_grad_(True)
    V_R = dev(flat(m.V_R)).requires_grad_(True)
    _torch_loss(qa.run(p, H_R, V_R, m.n_target, n_iter=1)[-1], cot, p, H_R).backward()

    def L(h, v):
        with torch.no_grad():
            hh = dev(flat(h))
            return float(_torch_loss(qa.run(p, hh, dev(flat(v)), m.n_target, n_iter=1)[-1], cot, p, hh))

    def sym(shape):
        x = crand(rng, shape)
        x = x + np.conj(np.swapaxes(lattice.reflect(x, case.dim), 0, 1))
        return x / np.linalg.norm(x)

    for name, x0, g in (("H", m.H_R, host(H_R.grad)), ("V", m.V_R, host(V_R.grad))):
        dirn = sym(x0.shape)
        f = (lambda t: L(t, m.V_R)) if name == "H" else (lambda t: L(m.H_R, t))
        num = directional_fd(f, x0, dirn)
        ana = float(np.sum(np.conj(g) * flat(dirn)).real)
        assert abs(num - ana) <= 1e-5 * abs(num) + 1e-9 * np.linalg.norm(g), (name, num, ana)


def test_energy_and_its_adjoint(case):
    torch = _torch()
    m, d, p, out = case.m, case.d, case.plan, case.out
    ref = gw.total_energy(m, d, out)
    args = [dev(flat(m.H_k)), dev(flat(out["sig_hf_k"])), dev(flat(out["sig_iw"])), dev(flat(out["G_iw"]))]
    e = p.energy(*args)
    for got, want in zip(e, ref):
        assert abs(got - want) <= 1e-10 * max(1.0, abs(ref[0])), (e, ref)
    outs = [torch.empty_like(t) for t in args]
    p.energy_bwd(*args, 0.8, *outs)
    rv = ad.energy_vjp(m, d, out, 0.8)
    for key, got in zip(("H_k", "sig_hf_k"), outs[:2]):
        assert rel_err(host(got), flat(rv[key])) < 1e-9, key
    # The Sigma and G cotangents pass through the Matsubara-sum map K^{-T} D K^{-1}, which
    # the two sides build independently; entry by entry they agree only to what the
    # kernel's conditioning allows.  Paired with representable directions K c (the
    # derivative of the energy along a DLR-representable change) they agree to rounding.
    rng = np.random.default_rng(7)
    for key, got in zip(("sig_iw", "G_iw"), outs[2:]):
        assert rel_err(host(got), flat(rv[key])) < MAP_TOL, key
        for _ in range(3):
            x_rep = apply_map(d.K_f, crand(rng, rv[key].shape))
            a = float(np.sum(np.conj(host(got)) * flat(x_rep)).real)
            b = float(np.sum(np.conj(rv[key]) * x_rep).real)
            assert abs(a - b) <= 1e-9 * abs(b), (key, a, b)


def test_adjoints_reject_fp32_plans(case):
    torch = _torch()
    d = case.d
    p32 = qgw.Plan.from_nodes(case.mesh[0], case.w["site_norb"], d.beta, d.nodes(), precision=qgw.F32,
                              dim=case.dim)
    x = torch.zeros((d.r, case.m.n_o, case.m.n_o, case.m.n_k), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(qgw.QGWError) as e:
        p32.dlr_transform_bwd(qgw.F_IW2TAU, x, x.clone())
    assert e.value.status == 3
    p32.close()
