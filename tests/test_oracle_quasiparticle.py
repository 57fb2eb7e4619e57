"""Pins of the quasiparticle oracle (Z class, SigStc class, Eq. eq-z-factor,
Eq. eq-quasi-particle-Hamiltonian) against closed forms and invariants.

For a self-energy with one pole, Sigma^C(i w) = A / (i w - e) with A Hermitian,
the values at +-i pi/beta are known exactly:
  Sigma(k, 0) = Sigma_HF - A e / (w0^2 + e^2),  Z^{-1} = 1 + A / (w0^2 + e^2),
with w0 = pi / beta (the w0 -> 0 limits are the analytic -A/e and 1 + A/e^2).
"""
import numpy as np
import pytest

from conftest import rel_err
from oracle import gw, quasiparticle as qp
from oracle.dlr import DLR
from paper_2604_22223_amd import workloads as wl


def herm(rng, shape):
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return 0.5 * (x + np.conj(np.swapaxes(x, 0, 1)))


@pytest.fixture(scope="module")
def d():
    return DLR(8.0, 12.0, 1e-10)


def one_pole(d, a, e):
    """A / (i w_m - e) on the fermionic nodes: [node, a, b, n1, n2]."""
    return a[None] / (d.iw[:, None, None, None, None] - e)


@pytest.mark.parametrize("on_node", [True, False])
def test_single_pole_closed_form(d, on_node):
    rng = np.random.default_rng(5)
    n_o, mesh = 3, (2, 3)
    a = herm(rng, (n_o, n_o) + mesh)
    e = d.omega[len(d.omega) // 3] if on_node else 0.37
    sig = one_pole(d, a, e)
    hf = herm(rng, (n_o, n_o) + mesh)
    w0 = np.pi / d.beta
    want0 = hf - a * e / (w0 ** 2 + e ** 2)
    wantz = np.eye(n_o)[:, :, None, None] + a / (w0 ** 2 + e ** 2)
    tol = 1e-12 if on_node else 1e-8
    assert rel_err(qp.static_self_energy(d, hf, sig), want0) < tol
    assert rel_err(qp.z_inverse(d, sig), wantz) < tol


def test_zero_self_energy(d):
    rng = np.random.default_rng(6)
    n_o, mesh = 4, (3, 3)
    h = herm(rng, (n_o, n_o) + mesh)
    hf = herm(rng, (n_o, n_o) + mesh)
    sig = np.zeros((d.r, n_o, n_o) + mesh, dtype=np.complex128)
    st = {"sig_hf_k": hf, "sig_iw": sig}
    m = type("M", (), {"H_k": h})()
    out = qp.quasiparticle(m, d, st, mu=0.3)
    eye = np.eye(n_o)[:, :, None, None]
    assert rel_err(out["z"], eye * np.ones(mesh)) < 1e-15
    assert rel_err(out["hqp"], h + hf - 0.3 * eye) < 1e-14
    ev = np.linalg.eigvalsh(np.moveaxis(h + hf, (0, 1), (-2, -1))) - 0.3
    assert rel_err(out["bands"], np.moveaxis(ev, -1, 0)) < 1e-14


def test_one_orbital_is_z_times_energy(d):
    rng = np.random.default_rng(7)
    mesh = (4, 2)
    h = rng.standard_normal((1, 1) + mesh) + 0j
    a = np.abs(rng.standard_normal((1, 1) + mesh)) + 0j
    e = -0.8
    sig = one_pole(d, a, e)
    hf = np.zeros_like(h)
    st = {"sig_hf_k": hf, "sig_iw": sig}
    m = type("M", (), {"H_k": h})()
    out = qp.quasiparticle(m, d, st, mu=0.1)
    w0 = np.pi / d.beta
    z = 1.0 / (1.0 + a / (w0 ** 2 + e ** 2))
    want = z * (h - a * e / (w0 ** 2 + e ** 2) - 0.1)
    assert rel_err(out["hqp"], want) < 1e-9
    assert rel_err(out["bands"][0], want[0, 0]) < 1e-9


def test_scalar_self_energy_scales_the_bands(d):
    """Sigma^C = a I / (i w - e): Z = z I commutes with H, so the bands are z (eps_n + s0 - mu)."""
    rng = np.random.default_rng(8)
    n_o, mesh = 3, (3, 2)
    h = herm(rng, (n_o, n_o) + mesh)
    aa, e, mu = 0.6, 1.4, -0.2
    a = aa * np.eye(n_o)[:, :, None, None] * np.ones(mesh)
    sig = one_pole(d, a.astype(np.complex128), e)
    st = {"sig_hf_k": np.zeros_like(h), "sig_iw": sig}
    m = type("M", (), {"H_k": h})()
    out = qp.quasiparticle(m, d, st, mu=mu)
    w0 = np.pi / d.beta
    z = 1.0 / (1.0 + aa / (w0 ** 2 + e ** 2))
    s0 = -aa * e / (w0 ** 2 + e ** 2)
    eps = np.moveaxis(np.linalg.eigvalsh(np.moveaxis(h, (0, 1), (-2, -1))), -1, 0)
    assert rel_err(out["bands"], z * (eps + s0 - mu)) < 1e-8


def test_orbital_rotation_covariance(d):
    rng = np.random.default_rng(9)
    n_o, mesh = 3, (2, 2)
    h = herm(rng, (n_o, n_o) + mesh)
    hf = herm(rng, (n_o, n_o) + mesh)
    a = herm(rng, (n_o, n_o) + mesh)
    a = np.einsum("abxy,cbxy->acxy", a, np.conj(a)) * 0.1  # positive, so Z^{-1} > 1
    sig = one_pole(d, a, 0.9)
    u, _ = np.linalg.qr(rng.standard_normal((n_o, n_o)) + 1j * rng.standard_normal((n_o, n_o)))
    rot = lambda x: np.einsum("ab,bc...,dc->ad...", u, x, np.conj(u))
    m = type("M", (), {"H_k": h})()
    m2 = type("M", (), {"H_k": rot(h)})()
    o1 = qp.quasiparticle(m, d, {"sig_hf_k": hf, "sig_iw": sig}, mu=0.2)
    sig2 = np.stack([rot(s) for s in sig])
    o2 = qp.quasiparticle(m2, d, {"sig_hf_k": rot(hf), "sig_iw": sig2}, mu=0.2)
    assert rel_err(o2["bands"], o1["bands"]) < 1e-12
    assert rel_err(o2["hqp"], rot(o1["hqp"])) < 1e-12
    assert rel_err(o2["z"], rot(o1["z"])) < 1e-12


def test_gw_state_renormalisation_below_one():
    """The GW self-energy has a positive spectral function, so Im Sigma(i pi/beta) <= 0 and 0 < Z <= 1."""
    from paper_2604_22223_amd import workloads as wl
    w = wl.five_orbital(n=4, norb=2, n_target=2.0, U=1.0, J=0.1, Vnn=0.2, beta=10.0, omega_max=20.0,
                        eps=1e-10, scale_mesh=4)
    dd = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    st = gw.gw_iteration(m, dd, gw.initial_state(m, dd))
    out = qp.quasiparticle(m, dd, st, mu=st["mu"])
    ev = np.linalg.eigvalsh(np.moveaxis(out["z"], (0, 1), (-2, -1)))
    assert ev.min() > 0.0 and ev.max() <= 1.0 + 1e-12
    # a renormalised band is narrower than the band it comes from
    assert np.ptp(out["bands"]) < np.ptp(np.linalg.eigvalsh(np.moveaxis(m.H_k + out["sig0"], (0, 1), (-2, -1))))


# ----------------------------------------------------------------------------
# bands along a k path (Fourier interpolation of the mesh values)
# ----------------------------------------------------------------------------

def test_path_on_mesh_points_equals_mesh():
    """At the mesh's own k points the interpolation returns the mesh values: every path output equals the mesh
    output (a 5 x 6 mesh: odd and even sides, the split n/2 shell included)."""
    w = wl.random_model((5, 6), [2, 1], seed=3, beta=10.0, omega_max=20.0, eps=1e-10)
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    st = gw.gw_iteration(m, d, gw.initial_state(m, d))
    ref = qp.quasiparticle(m, d, st, mu=st["mu"])
    k = np.array([[i / 5, j / 6] for i in range(5) for j in range(6)])
    out = qp.quasiparticle_path(m, d, st, k, mu=st["mu"])
    for key in ("sig0", "zinv", "z", "hqp", "bands"):
        r = ref[key]
        assert np.abs(out[key] - r.reshape(r.shape[:-2] + (-1,))).max() < 1e-12, key


@pytest.mark.parametrize("seed", [22223, 5])
def test_path_tight_binding_is_analytic(seed):
    """With no self-energy the path bands are the eigenvalues of H0(k') - mu with H0(k') summed directly over the
    model's bond list (x, y, x + y, x - y and their reverses), at points off the mesh.  The random complex hoppings
    break k -> -k, so a wrong sign of the interpolation phase fails."""
    n = 6
    w = wl.five_orbital(n=n, seed=seed, U=1.0, J=0.1, Vnn=0.2, beta=10.0, omega_max=20.0, eps=1e-8, scale_mesh=n)
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    zero = {"sig_hf_k": np.zeros_like(m.H_k), "sig_iw": np.zeros((d.r,) + m.H_k.shape, dtype=np.complex128)}
    rng = np.random.default_rng(1)
    k = rng.uniform(0.0, 1.0, size=(17, 2))
    mu = 0.37
    out = qp.quasiparticle_path(m, d, zero, k, mu=mu)
    bonds = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]
    for p, f in enumerate(k):
        h = np.zeros((5, 5), dtype=np.complex128)
        for (r1, r2) in bonds:
            h += w["H_R"][:, :, r1 % n, r2 % n] * np.exp(-2j * np.pi * (f[0] * r1 + f[1] * r2))
        ev = np.linalg.eigvalsh(h - mu * np.eye(5))
        assert np.abs(out["bands"][:, p] - ev).max() < 1e-12, p
    assert np.abs(out["z"] - np.eye(5)[:, :, None]).max() < 1e-14


def test_path_graphene_dispersion():
    """Graphene with no self-energy: the bands at any k' are -mu -+ |t| |1 + e^{2 pi i f1} + e^{2 pi i f2}|."""
    w = wl.graphene(n=12, U=3.0, ohno=False, beta=10.0, omega_max=100.0, eps=1e-8)
    d = DLR(w["beta"], w["omega_max"], w["eps"])
    m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
    zero = {"sig_hf_k": np.zeros_like(m.H_k), "sig_iw": np.zeros((d.r,) + m.H_k.shape, dtype=np.complex128)}
    k = np.array([[0.0, 0.0], [1 / 3, 2 / 3], [0.5, 0.0], [0.123, 0.456], [0.7, 0.31]])
    out = qp.quasiparticle_path(m, d, zero, k, mu=0.2)
    gam = np.abs(1.0 + np.exp(2j * np.pi * k[:, 0]) + np.exp(2j * np.pi * k[:, 1]))
    ref = np.stack([-0.2 - 2.7 * gam, -0.2 + 2.7 * gam])
    assert np.abs(out["bands"] - ref).max() < 1e-12
