"""The C ABI of libqgw on the CPU: the library loads, exports every entry
point that include/qgw.h declares, validates arguments before touching a
device, and its host DLR builder agrees with the oracle's construction.
No GPU compute here."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2604_22223_amd import qgw
from oracle.dlr import DLR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "qgw.h")).read()
    return sorted(set(re.findall(r"^\s*(?:qgw_status|const char \*|int32_t)\s*(qgw_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(qgw.LIB_PATH), "libqgw.so is not built"
    out = subprocess.run(["nm", "-D", "--defined-only", qgw.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (qgw_\w+)", out))
    declared = header_functions()
    assert len(declared) >= 19
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    assert sorted(declared) == sorted(qgw.EXPORTS)
    L = qgw.lib()
    for f in declared:
        assert hasattr(L, f)


def _desc(n=6, site_norb=(2, 1), r=3, precision=0, beta=10.0, tau=(0.1, 0.5, 0.9)):
    so = np.array(site_norb, dtype=np.int32)
    om = np.linspace(-1, 1, r)
    tt = np.array(tau[:r], dtype=np.float64)
    nf = np.arange(r, dtype=np.int64)
    nb = np.arange(r, dtype=np.int64)
    keep = (so, om, tt, nf, nb)
    d = qgw.PlanDesc(n, len(so), so.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), beta, r,
                     om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     tt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     nf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                     nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), precision, 0)
    return d, keep


def _create(d):
    h = ctypes.c_void_p()
    rc = qgw.lib().qgw_plan_create(ctypes.byref(d), ctypes.byref(h))
    if rc == 0:
        qgw.lib().qgw_plan_destroy(h)
    return rc


@pytest.mark.parametrize("kw,code", [
    (dict(n=7), 3),                      # mesh side 7: no compiled transform
    (dict(n=0), 1),
    (dict(site_norb=(3, 3)), 3),         # N_b = 18: no compiled Dyson-W solver
    (dict(site_norb=(9,)), 3),           # more than 8 orbitals
    (dict(precision=5), 1),
    (dict(beta=-1.0), 1),
    (dict(tau=(0.0, 0.5, 0.9)), 1),      # tau/beta must be inside (0, 1)
])
def test_plan_validation_before_device(kw, code):
    d, keep = _desc(**kw)
    assert _create(d) == code
    assert len(qgw.lib().qgw_last_error()) > 0


def test_null_arguments_rejected():
    L = qgw.lib()
    assert L.qgw_plan_create(None, None) == 1
    assert L.qgw_dlr_transform(None, 0, 1, 1.0, 0.0, 0, None, None, None) == 1
    assert L.qgw_dyson_W(None, None, None, None, None) == 1
    assert L.qgw_gw_iteration(None, 1, 0.0, None, None, None, None) == 1
    assert L.qgw_plan_destroy(None) == 0


def test_no_device_reported_on_cpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    d, keep = _desc()
    assert _create(d) == 4                # QGW_ERR_DEVICE


def _kt(t, x):
    t = np.asarray(t)[:, None]
    x = np.asarray(x)[None, :]
    return np.where(x >= 0, np.exp(-t * np.maximum(x, 0)) / (1 + np.exp(-np.maximum(x, 0))),
                    np.exp((1 - t) * np.minimum(x, 0)) / (1 + np.exp(np.minimum(x, 0))))


@pytest.mark.parametrize("beta,wmax,eps", [(10.0, 100.0, 1e-8), (50.0, 25.0, 1e-10), (40.0, 100.0, 1e-10)])
def test_host_dlr_builder(beta, wmax, eps):
    """Same rank as the oracle's construction; the library's nodes interpolate
    off-grid poles from Matsubara values as accurately as the oracle's."""
    nd = qgw.dlr_build(beta * wmax, eps)
    d = DLR(beta, wmax, eps)
    r = len(nd["x"])
    assert r == d.r
    assert np.all(np.diff(nd["x"]) > 0) and np.all((nd["tau_t"] > 0) & (nd["tau_t"] < 1))
    rng = np.random.default_rng(1)
    x0 = rng.uniform(-0.9, 0.9, 10) * beta * wmax
    for nodes in [(nd["x"], nd["tau_t"], nd["n_f"]), (d.omega * beta, d.tau_t, d.n_f)]:
        x, t, nf = nodes
        kt = _kt(t, x)
        kf = 1.0 / (1j * np.pi * (2 * nf[:, None] + 1) - x[None, :])
        kt0 = _kt(t, x0)
        kf0 = 1.0 / (1j * np.pi * (2 * nf[:, None] + 1) - x0[None, :])
        interp = kt @ np.linalg.solve(kf, kf0)
        assert np.abs(interp - kt0).max() < 1e-5


def test_host_dlr_builder_errors():
    with pytest.raises(qgw.QGWError) as e:
        qgw.dlr_build(1000.0, 1e-10, max_rank=10)
    assert e.value.status == 2
    with pytest.raises(qgw.QGWError) as e:
        qgw.dlr_build(-1.0, 1e-10)
    assert e.value.status == 1


def test_uniform_grid_node_choice_and_checks():
    """qgw_mf_nodes_for is host arithmetic; qgw_plan_create_mf rejects unsupported grids before any device call."""
    L = qgw.lib()
    assert L.qgw_mf_nodes_for(50.0, 25.0) == 400
    assert L.qgw_mf_nodes_for(100.0, 25.0) == 800
    assert L.qgw_mf_nodes_for(10.0, 1.0) == 16
    assert L.qgw_mf_nodes_for(-1.0, 1.0) == 0
    # the smallest supported N with (2M - 1) pi / beta >= omega_max
    for beta, wmax in [(7.0, 3.0), (20.0, 25.0), (40.0, 30.0)]:
        n = L.qgw_mf_nodes_for(beta, wmax)
        assert (n - 1) * math.pi / beta >= wmax - 1e-9
    d, keep = _desc()
    h = ctypes.c_void_p()
    assert L.qgw_plan_create_mf(ctypes.byref(d), 100, ctypes.byref(h)) == 3       # no compiled transform
    assert L.qgw_plan_create_mf(ctypes.byref(d), 0, ctypes.byref(h)) == 1
    d32, keep32 = _desc(precision=1)
    assert L.qgw_plan_create_mf(ctypes.byref(d32), 64, ctypes.byref(h)) == 3      # FP64 only


def test_cubic_mesh_checks():
    """A cubic mesh side without a compiled 3-D transform, or a mesh dimension other than 2 and 3, is refused
    before any device call."""
    L = qgw.lib()
    h = ctypes.c_void_p()
    d, keep = _desc(n=7)
    d.dim = 3
    assert L.qgw_plan_create(ctypes.byref(d), ctypes.byref(h)) == 3
    d.n = 16
    assert L.qgw_plan_create(ctypes.byref(d), ctypes.byref(h)) == 3      # 16^3 exceeds the cubic set
    d.n, d.dim = 8, 4
    assert L.qgw_plan_create(ctypes.byref(d), ctypes.byref(h)) == 1
