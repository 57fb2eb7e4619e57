"""qgw_quasiparticle and qgw_quasiparticle_path against the oracle (Z class, SigStc class, Eq. eq-z-factor,
Eq. eq-quasi-particle-Hamiltonian).

Inputs are the oracle's state after one GW iteration on three models (multi-site
random, five orbitals on a ragged 10 x 10 mesh, graphene), passed as data to both
sides.  Sigma(k, 0), Z(k) and H_QP(k) are unique, so they are compared entry by
entry; the bands are compared in ascending order.  The bar is the FP64 parity
bar, 1e-10.
"""
import numpy as np
import pytest

from conftest import rel_err
from oracle import gw, quasiparticle as qp
from oracle.dlr import DLR
from paper_2604_22223_amd import qgw
from paper_2604_22223_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES = {
    "random_2+1_6x6": lambda: wl.random_model((6, 6), [2, 1], seed=3, beta=10.0, omega_max=20.0, eps=1e-10),
    "five_orbital_10x10": lambda: wl.five_orbital(n=10, U=1.0, J=0.1, Vnn=0.2, beta=20.0, omega_max=25.0,
                                                  eps=1e-10, scale_mesh=10),
    "graphene_12": lambda: wl.graphene(n=12, U=3.0, beta=10.0, omega_max=100.0, eps=1e-8),
    "random3d_2+1_4x4x4": lambda: wl.random_model_3d((4, 4, 4), [2, 1], seed=3, beta=10.0, omega_max=20.0,
                                                     eps=1e-10, U=1.0, J=0.1, Vnn=0.2),
}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


# number of mesh axes of the current case (2, or 3 on a cubic mesh); set by the ``case`` fixture
_MESH_DIM = [2]


def flat(x):
    return np.ascontiguousarray(x.reshape(x.shape[:-_MESH_DIM[0]] + (-1,)))


def dev(x):
    torch = _torch()
    return torch.from_numpy(flat(np.asarray(x, dtype=np.complex128))).to("cuda:0")


def host(t):
    return t.cpu().numpy()


class Case:
    def __init__(self, w):
        self.w = w
        self.d = DLR(w["beta"], w["omega_max"], w["eps"])
        self.m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
        self.st = gw.gw_iteration(self.m, self.d, gw.initial_state(self.m, self.d))
        self.dim = len(w["mesh"])
        self.plan = qgw.Plan.from_nodes(w["mesh"][0], w["site_norb"], w["beta"], self.d.nodes(), dim=self.dim)


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print("\n[quasiparticle case] %s" % request.param, flush=True)
    c = Case(CASES[request.param]())
    _MESH_DIM[0] = c.dim
    return c


@pytest.mark.parametrize("mu_mode", ["printed", "fermi_level"])
def test_quasiparticle_matches_oracle(case, mu_mode):
    st, m, d = case.st, case.m, case.d
    mu = 0.0 if mu_mode == "printed" else st["mu"]
    ref = qp.quasiparticle(m, d, st, mu=mu)
    sig0, z, hqp, bands = case.plan.quasiparticle(dev(m.H_k), dev(st["sig_hf_k"]), dev(st["sig_iw"]), mu=mu)
    assert rel_err(host(sig0), flat(ref["sig0"])) < TOL
    assert rel_err(host(z), flat(ref["z"])) < TOL
    assert rel_err(host(hqp), flat(ref["hqp"])) < TOL
    assert rel_err(host(bands), flat(ref["bands"][None])[0]) < TOL


def test_zero_self_energy_gives_z_one(case):
    st, m, d = case.st, case.m, case.d
    zero = np.zeros_like(st["sig_iw"])
    sig0, z, hqp, bands = case.plan.quasiparticle(dev(m.H_k), dev(st["sig_hf_k"]), dev(zero), mu=0.25)
    n_o = m.n_o
    eye = np.broadcast_to(np.eye(n_o)[:, :, None], (n_o, n_o, m.n_k))
    assert rel_err(host(z), eye) < 1e-14
    ev = np.linalg.eigvalsh(np.moveaxis(gw.hermitian_part(m.H_k + st["sig_hf_k"]), (0, 1), (-2, -1))) - 0.25
    assert rel_err(host(bands), np.moveaxis(ev, -1, 0).reshape(n_o, -1)) < 1e-12


def test_rejects_non_positive_z(case):
    """A self-energy whose slope makes Z^{-1} negative is reported, not returned as numbers."""
    st, m, d = case.st, case.m, case.d
    n_o = m.n_o
    # Z^{-1} = 1 + a / (w0^2 + e^2) < 0
    a = -5.0 * np.eye(n_o).reshape((n_o, n_o) + (1,) * case.dim) * np.ones(m.mesh)
    bad = a[None] / (d.iw.reshape((-1,) + (1,) * a.ndim) - 0.01)
    with pytest.raises(qgw.QGWError) as e:
        case.plan.quasiparticle(dev(m.H_k), dev(st["sig_hf_k"]), dev(bad))
    assert e.value.status == 6


def _path_points(dim, n, seed=7):
    """Mesh points (where the interpolant is the mesh value), a line through Gamma and the zone edge (f = 1/2,
    the split n/2 shell), and random off-mesh points."""
    rng = np.random.default_rng(seed)
    mesh = np.array([[1, 2] + [0] * (dim - 2), [n - 1, 0] + [1] * (dim - 2)], dtype=np.float64) / n
    line = np.linspace(0.0, 0.5, 9)[:, None] * np.ones((1, dim))
    return np.concatenate([mesh, line, rng.uniform(-0.5, 1.0, size=(21, dim))])


@pytest.mark.parametrize("mu_mode", ["printed", "fermi_level"])
def test_quasiparticle_path_matches_oracle(case, mu_mode):
    """Bands along a path (Fig. fig-band-dos (a)): the Fourier-interpolated outputs at mesh, zone-edge and random
    off-mesh points against the oracle, entry by entry at the FP64 bar."""
    st, m, d = case.st, case.m, case.d
    mu = 0.0 if mu_mode == "printed" else st["mu"]
    kf = _path_points(case.dim, m.mesh[0])
    ref = qp.quasiparticle_path(m, d, st, kf, mu=mu)
    sig0, z, hqp, bands = case.plan.quasiparticle_path(dev(m.H_k), dev(st["sig_hf_k"]), dev(st["sig_iw"]), kf, mu=mu)
    assert rel_err(host(sig0), ref["sig0"]) < TOL
    assert rel_err(host(z), ref["z"]) < TOL
    assert rel_err(host(hqp), ref["hqp"]) < TOL
    assert rel_err(host(bands), ref["bands"]) < TOL
    # on the mesh points the path call returns the mesh call's values
    mref = qp.quasiparticle(m, d, st, mu=mu)
    for p, f in enumerate(kf[:2]):
        idx = tuple(int(round(x * m.mesh[0])) % m.mesh[0] for x in f)
        assert np.abs(host(bands)[:, p] - mref["bands"][(slice(None),) + idx]).max() < 1e-10


def test_quasiparticle_path_rejects_bad_points(case):
    st, m = case.st, case.m
    args = (dev(m.H_k), dev(st["sig_hf_k"]), dev(st["sig_iw"]))
    kf = np.full((3, case.dim), 0.25)
    kf[1, 0] = np.nan
    with pytest.raises(qgw.QGWError) as e:
        case.plan.quasiparticle_path(*args, kf)
    assert e.value.status == 6
    with pytest.raises(qgw.QGWError) as e:
        case.plan.quasiparticle_path(*args, np.zeros((0, case.dim)))
    assert e.value.status == 1
