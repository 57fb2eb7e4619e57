"""Input generators: shapes and the symmetries of a physical Hamiltonian (not GPU)."""
import numpy as np

from paper_2604_22223_amd import workloads as wl
from oracle import lattice


def _reflect_swap(x):
    return np.conj(lattice.reflect(np.swapaxes(x, 0, 1)))


def test_five_orbital_model():
    w = wl.five_orbital(n=24)
    assert w["H_R"].shape == (5, 5, 24, 24) and w["V_R"].shape == (25, 25, 24, 24)
    # Hermitian H0: H(-R) = H(R)^dagger
    assert np.abs(w["H_R"] - _reflect_swap(w["H_R"])).max() < 1e-15
    # band width over the 24 x 24 mesh is 4 eV
    hk = np.moveaxis(np.fft.fft2(w["H_R"], axes=(-2, -1)), (0, 1), (-2, -1))
    ev = np.linalg.eigvalsh(hk)
    assert abs((ev.max() - ev.min()) - 4.0) < 1e-12
    # interaction symmetric under exchange of the two pairs: V_ab(R) = V_ba(-R)
    assert np.abs(w["V_R"] - lattice.reflect(np.swapaxes(w["V_R"], 0, 1))).max() == 0.0
    v0 = w["V_R"][:, :, 0, 0].real
    assert v0[0, 0] == 4.0 and v0[0, 6] == 4.0 - 2 * 0.7 and v0[1, 5] == 0.7 and v0[1, 1] == 0.7


def test_graphene_model():
    w = wl.graphene(n=12, ohno=True)
    assert np.abs(w["H_R"] - _reflect_swap(w["H_R"])).max() < 1e-15
    assert np.abs(w["V_R"] - lattice.reflect(np.swapaxes(w["V_R"], 0, 1))).max() < 1e-15
    hk = np.moveaxis(np.fft.fft2(w["H_R"], axes=(-2, -1)), (0, 1), (-2, -1))
    ev = np.linalg.eigvalsh(hk)
    assert abs(ev.max() - 3 * 2.7) < 1e-12            # |3t| at Gamma
    assert abs(w["V_R"][0, 0, 0, 0] - 3.0) < 1e-15
    # three A-B bonds at a_cc, each U / sqrt(1 + (U a_cc / 14.397)^2)
    v1 = 3.0 / np.sqrt(1 + (3.0 * 1.42 / 14.397) ** 2)
    assert abs(w["V_R"][0, 1, 0, 0] - v1) < 1e-14


def test_random_model_seeded():
    a = wl.random_model((4, 4), [2, 1], seed=3)
    b = wl.random_model((4, 4), [2, 1], seed=3)
    assert np.array_equal(a["H_R"], b["H_R"]) and np.array_equal(a["V_R"], b["V_R"])
    assert a["V_R"].shape == (5, 5, 4, 4)


def test_cubic_models():
    w = wl.cubic_five_orbital(n=8)
    assert w["H_R"].shape == (5, 5, 8, 8, 8) and w["V_R"].shape == (25, 25, 8, 8, 8)
    assert w["n_target"] == 5.0 and w["beta"] == 100.0 and w["omega_max"] == 25.0
    refl = lambda x: lattice.reflect(np.swapaxes(x, 0, 1), 3)
    assert np.abs(w["H_R"] - np.conj(refl(w["H_R"]))).max() == 0.0
    assert np.abs(w["V_R"] - refl(w["V_R"])).max() == 0.0
    # band width 12 t of the simple cubic lattice
    hk = np.moveaxis(np.fft.fftn(w["H_R"], axes=(-3, -2, -1)), (0, 1), (-2, -1))
    ev = np.linalg.eigvalsh(hk)
    assert abs((ev.max() - ev.min()) - 12.0) < 1e-12
    r = wl.random_model_3d((4, 3, 2), [2, 1], seed=3)
    assert r["H_R"].shape == (3, 3, 4, 3, 2) and r["V_R"].shape == (5, 5, 4, 3, 2)
    assert np.abs(r["H_R"] - np.conj(refl(r["H_R"]))).max() < 1e-15
    assert np.abs(r["V_R"] - refl(r["V_R"])).max() == 0.0


def test_graphene_ohno_36_bare_bubble_instability():
    """The Ohno potential cut off after the fifth shell is nearly flat out to the cut, so V(q) has negative
    eigenvalues (attractive channels).  At U = 3 eV (36 x 36, beta = 40) the bare bubble overcomes them:
    1 - P0(q, i nu) V(q) has a negative eigenvalue at nu = 0, so the first W^C = V (1 - P0 V)^-1 - V has a pole
    on the imaginary axis.  At U = 1 eV it stays positive definite."""
    from oracle import gw
    from oracle.dlr import DLR
    mins = {}
    for U in (3.0, 1.0):
        w = wl.graphene(n=36, U=U, ohno=True, beta=40.0, omega_max=100.0, eps=1e-10)
        vm = np.moveaxis(np.fft.fft2(w["V_R"], axes=(-2, -1)), (0, 1), (-2, -1))
        assert np.linalg.eigvalsh(vm).min() < -0.5 * U                    # attractive channels
        d = DLR(w["beta"], w["omega_max"], w["eps"])
        m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
        P = gw.gw_iteration(m, d, gw.initial_state(m, d), keep=True)["intermediates"]["P_nu_q"]
        pm = np.moveaxis(P, (1, 2), (-2, -1))
        mins[U] = np.linalg.eigvals(np.eye(2) - pm @ vm[None]).real.min()
    assert mins[3.0] < -0.1 and mins[1.0] > 0.3, mins


def test_five_orbital_24_bare_bubble_instability():
    """The five-orbital model at U = 4, J = 0.7, V = 1 eV (beta = 50, the 24 x 24 band structure sampled on 12 x 12
    to keep the oracle quick): 1 - P0 V has eigenvalues with negative real part, the density-wave instability that
    ends its self-consistent loop; at the benchmark's U = 1, J = 0.1, V = 0.2 eV all eigenvalues lie near 1."""
    from oracle import gw
    from oracle.dlr import DLR
    mins = []
    for kw in ({}, {"U": 1.0, "J": 0.1, "Vnn": 0.2}):
        w = wl.five_orbital(n=12, beta=50.0, omega_max=25.0, eps=1e-10, scale_mesh=24, **kw)
        d = DLR(w["beta"], w["omega_max"], w["eps"])
        m = gw.Model(w["mesh"], w["site_norb"], w["H_R"], w["V_R"], w["beta"], w["n_target"])
        P = gw.gw_iteration(m, d, gw.initial_state(m, d), keep=True)["intermediates"]["P_nu_q"]
        pm = np.moveaxis(P, (1, 2), (-2, -1))
        vm = np.moveaxis(m.V_q, (0, 1), (-2, -1))
        mins.append(np.linalg.eigvals(np.eye(m.n_b) - pm @ vm[None]).real.min())
    assert mins[0] < -1.0 and mins[1] > 0.9, mins
