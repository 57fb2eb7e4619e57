"""The two forms of the 25 x 25 Dyson-W kernel (Eq. eq-screened-coulomb), each pinned through
qgw_plan_set_tuning: V P on the matrix cores, or on the VALU.  Both are compared with the oracle's solve
W^C = (I - V P)^{-1} V - V, and the adjoint call (which runs the same kernel twice, once on the
conjugate-transposed system) with the oracle's reverse mode, at the FP64 bar 1e-10; in FP32 both forms stay
within the rounding bar of a partially pivoted solve, a few N_b cond(I - V P) units of single precision.

Inputs are seeded: a Hermitian V(q) per q and a random P(q, i nu) per node, scaled so that I - V P is well
conditioned, on a 4 x 4 mesh (16 q points) with the DLR nodes of beta = 10 / eV, omega_max = 20 eV.
"""
import numpy as np
import pytest

from conftest import rel_err
from oracle import adjoint as ad
from oracle import gw
from oracle.dlr import DLR
from paper_2604_22223_amd import qgw

pytestmark = pytest.mark.gpu

TOL = 1e-10
N = 4
NB = 25


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def dev(x, dt=np.complex128):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def crand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def data():
    d = DLR(10.0, 20.0, 1e-10)
    rng = np.random.default_rng(25)
    nk = N * N
    v = crand(rng, (nk, NB, NB))
    vq = 0.1 * (v + np.conj(np.swapaxes(v, 1, 2)))
    pnu = 0.1 * crand(rng, (d.r, nk, NB, NB))
    wbar = crand(rng, (d.r, nk, NB, NB))
    # oracle layouts: V_q [A, B, n1, n2], P_nu [r, A, B, n1, n2]
    V_o = np.moveaxis(vq.reshape(N, N, NB, NB), (2, 3), (0, 1))
    P_o = np.moveaxis(pnu.reshape(d.r, N, N, NB, NB), (3, 4), (1, 2))
    wc_o = gw.dyson_W(V_o, P_o)
    wc_ref = np.moveaxis(wc_o, (1, 2), (3, 4)).reshape(d.r, nk, NB, NB)
    Wb_o = np.moveaxis(wbar.reshape(d.r, N, N, NB, NB), (3, 4), (1, 2))
    vb_o, pb_o = ad.dyson_W_adj(Wb_o, V_o, P_o)
    vb_ref = np.moveaxis(vb_o, (2, 3), (0, 1)).reshape(nk, NB, NB)
    pb_ref = np.moveaxis(pb_o, (1, 2), (3, 4)).reshape(d.r, nk, NB, NB)
    a = np.eye(NB) - np.broadcast_to(vq[None], pnu.shape) @ pnu
    cond = float(np.linalg.cond(a.reshape(-1, NB, NB)).max())
    return dict(d=d, vq=vq, pnu=pnu, wbar=wbar, wc_ref=wc_ref, vb_ref=vb_ref, pb_ref=pb_ref, cond=cond)


@pytest.mark.parametrize("mfma", [1, 0])
def test_forward_fp64_matches_oracle(data, mfma):
    torch = _torch()
    p = qgw.Plan.from_nodes(N, [5], 10.0, data["d"].nodes())
    p.set_tuning({"dyson_w25_mfma": mfma})
    print("\n[dyson w25] forward FP64, matrix-core V P = %d" % mfma, flush=True)
    out = torch.empty((p.r, p.n_k, NB, NB), dtype=torch.complex128, device="cuda:0")
    p.dyson_W(dev(data["vq"]), dev(data["pnu"]), out)
    p.sync_status()
    assert rel_err(host(out), data["wc_ref"]) < TOL
    p.close()


@pytest.mark.parametrize("mfma", [1, 0])
def test_adjoint_fp64_matches_oracle(data, mfma):
    torch = _torch()
    p = qgw.Plan.from_nodes(N, [5], 10.0, data["d"].nodes())
    p.set_tuning({"dyson_w25_mfma": mfma})
    print("\n[dyson w25] adjoint FP64, matrix-core V P = %d" % mfma, flush=True)
    vq, pnu = dev(data["vq"]), dev(data["pnu"])
    pbar, vbar = torch.empty_like(pnu), torch.empty_like(vq)
    p.dyson_W_bwd(vq, pnu, dev(data["wbar"]), pbar, vbar)
    p.sync_status()
    assert rel_err(host(pbar), data["pb_ref"]) < TOL
    assert rel_err(host(vbar), data["vb_ref"]) < TOL
    p.close()


@pytest.mark.parametrize("mfma", [1, 0])
def test_forward_fp32_within_rounding(data, mfma):
    torch = _torch()
    p = qgw.Plan.from_nodes(N, [5], 10.0, data["d"].nodes(), precision=qgw.F32)
    p.set_tuning({"dyson_w25_mfma": mfma})
    print("\n[dyson w25] forward FP32, matrix-core V P = %d" % mfma, flush=True)
    out = torch.empty((p.r, p.n_k, NB, NB), dtype=torch.complex64, device="cuda:0")
    p.dyson_W(dev(data["vq"], np.complex64), dev(data["pnu"], np.complex64), out)
    p.sync_status()
    tol = 4.0 * NB * data["cond"] * 2.0 ** -24
    ref = data["wc_ref"]
    err = float(np.abs(host(out) - ref).max()) / max(float(np.abs(ref).max()), float(np.abs(data["vq"]).max()))
    assert err < tol, (err, tol)
    p.close()


def test_forms_agree_and_tuning_is_validated(data):
    """The two forms differ only in the order of the V P sums; out-of-range choices are refused."""
    torch = _torch()
    p = qgw.Plan.from_nodes(N, [5], 10.0, data["d"].nodes())
    vq, pnu = dev(data["vq"]), dev(data["pnu"])
    outs = []
    for mfma in (1, 0):
        p.set_tuning({"dyson_w25_mfma": mfma})
        out = torch.empty((p.r, p.n_k, NB, NB), dtype=torch.complex128, device="cuda:0")
        p.dyson_W(vq, pnu, out)
        outs.append(host(out))
    assert rel_err(outs[0], outs[1]) < 1e-12
    for bad in ({"dyson_w25_mfma": 2}, {"orbital_map_rows": 7}, {"mfma_blocks_per_cu": 9}):
        with pytest.raises(qgw.QGWError) as e:
            p.set_tuning(bad)
        assert e.value.status == 1
    with pytest.raises(qgw.QGWError):
        p.set_tuning({}, precision=3)
    p.close()
