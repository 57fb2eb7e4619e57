"""Thin ctypes binding of libqgw (argument marshalling only).

Every function mirrors a C entry point of ``include/qgw.h`` with the same
name minus the ``qgw_`` prefix.  Device arrays are torch tensors
(complex128 for FP64 plans, complex64 for FP32 plans) on the plan's device;
the work is queued on torch's current stream.  Nothing here computes: if the
shared library is missing, every call raises.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqgw.so")

QGW_OK = 0
STATUS_NAMES = {0: "QGW_OK", 1: "QGW_ERR_INVALID_ARG", 2: "QGW_ERR_SHAPE", 3: "QGW_ERR_UNSUPPORTED",
                4: "QGW_ERR_DEVICE", 5: "QGW_ERR_NOT_CONVERGED", 6: "QGW_ERR_NONFINITE",
                7: "QGW_ERR_ALLOC", 8: "QGW_ERR_SINGULAR"}
QGW_ERR_INVALID_ARG, QGW_ERR_NONFINITE, QGW_ERR_SINGULAR = 1, 6, 8
F64, F32 = 0, 1
F_IW2TAU, F_IW2TAUR, F_TAU2IW, B_TAU2IW, B_IW2TAU, F_IW2BETA, F_IW2GM = range(7)
LAYOUT_SLAB, LAYOUT_MATRIX = 0, 1
(OP_SIGMA_BWD, OP_DYSON_W_BWD, OP_HARTREE_FOCK_BWD, OP_ENERGY, OP_ENERGY_BWD, OP_HF_DENSITY,
 OP_QUASIPARTICLE) = range(7)
R_TO_K, K_TO_R = -1, +1

#: Every C entry point the header declares.
EXPORTS = ["qgw_dlr_build", "qgw_plan_create", "qgw_plan_destroy", "qgw_plan_get_map", "qgw_plan_sizes",
           "qgw_dlr_transform", "qgw_dlr_transform_pairs", "qgw_lattice_fft", "qgw_bubble", "qgw_dyson_W",
           "qgw_sigma", "qgw_hartree_fock", "qgw_dyson_G", "qgw_state_create", "qgw_state_destroy",
           "qgw_state_init_g0", "qgw_gw_iteration", "qgw_state_copy", "qgw_state_profile", "qgw_state_profile_select",
           "qgw_state_set_precision", "qgw_state_set_search_steps", "qgw_state_info", "qgw_check_finite",
           "qgw_dlr_transform_bwd", "qgw_dlr_transform_pairs_bwd", "qgw_lattice_fft_bwd", "qgw_bubble_bwd",
           "qgw_sigma_bwd", "qgw_dyson_W_bwd", "qgw_hartree_fock_bwd", "qgw_dyson_G_bwd", "qgw_pair_layout",
           "qgw_add", "qgw_energy", "qgw_energy_bwd", "qgw_quasiparticle", "qgw_hf_density", "qgw_state_hf_solve", "qgw_plan_autotune", "qgw_batch_create", "qgw_batch_launch", "qgw_batch_read", "qgw_batch_destroy",
           "qgw_plan_create_mf", "qgw_mf_nodes_for", "qgw_workspace_size", "qgw_sync_status", "qgw_dyson_G_noalloc", "qgw_quasiparticle_path_workspace",
           "qgw_quasiparticle_path", "qgw_plan_set_tuning", "qgw_last_error"]


class QGWError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_sites", ctypes.c_int32),
                ("site_norb", ctypes.POINTER(ctypes.c_int32)), ("beta", ctypes.c_double),
                ("rank", ctypes.c_int32), ("omega", ctypes.POINTER(ctypes.c_double)),
                ("tau_t", ctypes.POINTER(ctypes.c_double)), ("n_f", ctypes.POINTER(ctypes.c_int64)),
                ("n_b", ctypes.POINTER(ctypes.c_int64)), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("dim", ctypes.c_int32)]


_lib = None


def lib():
    """Loads libqgw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libqgw.so is not built: run `python -m paper_2604_22223_amd.build`")
        # torch first: the library's libamdhip64.so.7 dependency then binds to
        # the HIP runtime torch already loaded, so device pointers and streams
        # from torch are valid in the library
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        pd, pi32, pi64 = ctypes.POINTER(dbl), ctypes.POINTER(i32), ctypes.POINTER(i64)
        sig = {
            "qgw_dlr_build": [dbl, dbl, i32, pd, pd, pi64, pi64, pi32],
            "qgw_plan_create": [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)],
            "qgw_plan_create_mf": [ctypes.POINTER(PlanDesc), i32, ctypes.POINTER(vp)],
            "qgw_mf_nodes_for": [dbl, dbl],
            "qgw_plan_destroy": [vp],
            "qgw_plan_get_map": [vp, i32, pd],
            "qgw_plan_sizes": [vp, pi32, pi32, pi32, pi32],
            "qgw_dlr_transform": [vp, i32, i64, dbl, dbl, i32, vp, vp, vp],
            "qgw_dlr_transform_pairs": [vp, i32, i32, i32, vp, vp, vp],
            "qgw_lattice_fft": [vp, i32, i64, vp, vp, vp],
            "qgw_bubble": [vp, vp, vp, i32, vp, vp],
            "qgw_dyson_W": [vp, vp, vp, vp, vp],
            "qgw_sigma": [vp, vp, vp, i32, i32, vp, vp],
            "qgw_hartree_fock": [vp, vp, vp, vp, vp],
            "qgw_dyson_G": [vp, vp, vp, dbl, pd, vp, vp],
            "qgw_dyson_G_noalloc": [vp, vp, vp, dbl, pd, vp, vp],
            "qgw_state_create": [vp, vp, vp, dbl, dbl, ctypes.POINTER(vp)],
            "qgw_state_destroy": [vp],
            "qgw_state_init_g0": [vp, pd, vp],
            "qgw_gw_iteration": [vp, i32, dbl, pi32, pd, pd, vp],
            "qgw_state_copy": [vp, i32, vp, pi64, vp],
            "qgw_state_profile": [vp, i32, pd, pi32],
            "qgw_state_profile_select": [vp, ctypes.c_uint32, i32],
            "qgw_state_set_precision": [vp, i32, dbl],
            "qgw_state_set_search_steps": [vp, i32],
            "qgw_state_info": [vp, pi32, pi32, pi32, pi32],
            "qgw_check_finite": [vp, vp, i64, vp],
            "qgw_dlr_transform_bwd": [vp, i32, i64, dbl, dbl, i32, vp, vp, vp],
            "qgw_dlr_transform_pairs_bwd": [vp, i32, i32, i32, vp, vp, vp],
            "qgw_lattice_fft_bwd": [vp, i32, i64, vp, vp, vp],
            "qgw_bubble_bwd": [vp, vp, vp, vp, vp, vp, vp],
            "qgw_sigma_bwd": [vp, vp, vp, i32, vp, vp, vp, vp, i64, vp],
            "qgw_dyson_W_bwd": [vp, vp, vp, vp, vp, vp, vp, i64, vp],
            "qgw_hartree_fock_bwd": [vp, vp, vp, vp, vp, vp, vp, i64, vp],
            "qgw_dyson_G_bwd": [vp, vp, vp, dbl, dbl, dbl, vp, vp, vp, vp],
            "qgw_pair_layout": [vp, i32, i32, i64, vp, vp, vp],
            "qgw_add": [vp, i64, vp, vp, vp, vp],
            "qgw_plan_autotune": [vp, pi32, vp],
            "qgw_plan_set_tuning": [vp, i32, pi32],
            "qgw_energy": [vp, vp, vp, vp, vp, pd, vp, i64, vp],
            "qgw_energy_bwd": [vp, vp, vp, vp, vp, dbl, vp, vp, vp, vp, vp, i64, vp],
            "qgw_quasiparticle": [vp, vp, vp, vp, dbl, vp, vp, vp, pd, vp, i64, vp],
            "qgw_hf_density": [vp, vp, dbl, pd, vp, vp, i64, vp],
            "qgw_quasiparticle_path_workspace": [vp, i32, pi64],
            "qgw_quasiparticle_path": [vp, vp, vp, vp, dbl, pd, i32, vp, vp, vp, pd, vp, i64, vp],
            "qgw_workspace_size": [vp, i32, pi64],
            "qgw_sync_status": [vp, vp],
            "qgw_state_hf_solve": [vp, dbl, i32, pi32, pd, pd, vp],
            "qgw_batch_create": [i32, ctypes.POINTER(vp), i32, i32, i32, ctypes.POINTER(vp)],
            "qgw_batch_launch": [vp, vp],
            "qgw_batch_read": [vp, pd, pd, pi32, pi32, vp],
            "qgw_batch_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.qgw_last_error.argtypes = []
        L.qgw_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != QGW_OK:
        raise QGWError(status, lib().qgw_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _nbytes(t):
    return 0 if t is None else int(t.numel() * t.element_size())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def dlr_build(lam, eps, max_rank=96):
    """Host FP64 DLR node selection; returns dict(x=beta*omega, tau_t, n_f, n_b)."""
    x = np.zeros(max_rank)
    t = np.zeros(max_rank)
    nf = np.zeros(max_rank, dtype=np.int64)
    nb = np.zeros(max_rank, dtype=np.int64)
    r = ctypes.c_int32(0)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    _check(lib().qgw_dlr_build(float(lam), float(eps), int(max_rank), x.ctypes.data_as(dp),
                               t.ctypes.data_as(dp), nf.ctypes.data_as(ip), nb.ctypes.data_as(ip),
                               ctypes.byref(r)))
    r = r.value
    return {"x": x[:r].copy(), "tau_t": t[:r].copy(), "n_f": nf[:r].copy(), "n_b": nb[:r].copy()}


def mf_nodes_for(beta, omega_max):
    """The smallest supported uniform-grid node count reaching omega_max (qgw_mf_nodes_for); 0 if none."""
    return int(lib().qgw_mf_nodes_for(float(beta), float(omega_max)))


class Plan:
    """A libqgw plan: mesh n x n (or n x n x n with dim=3), sites/orbitals, DLR nodes, precision."""

    def __init__(self, n, site_norb, beta, omega, tau_t, n_f, n_b, precision=F64, device=0, dim=2, mf_nodes=0):
        self._keep = [np.ascontiguousarray(site_norb, dtype=np.int32),
                      np.ascontiguousarray(omega, dtype=np.float64),
                      np.ascontiguousarray(tau_t, dtype=np.float64),
                      np.ascontiguousarray(n_f, dtype=np.int64),
                      np.ascontiguousarray(n_b, dtype=np.int64)]
        so, om, tt, nf, nb = self._keep
        d = PlanDesc(int(n), len(so), so.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(beta),
                     len(om), om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     tt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     nf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                     nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(precision), int(device), int(dim))
        h = ctypes.c_void_p()
        if mf_nodes:
            _check(lib().qgw_plan_create_mf(ctypes.byref(d), int(mf_nodes), ctypes.byref(h)))
        else:
            _check(lib().qgw_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.grid = "mf" if mf_nodes else "dlr"
        r, no, nbp, nk = (ctypes.c_int32() for _ in range(4))
        _check(lib().qgw_plan_sizes(h, ctypes.byref(r), ctypes.byref(no), ctypes.byref(nbp), ctypes.byref(nk)))
        self.r, self.n_o, self.n_b, self.n_k = r.value, no.value, nbp.value, nk.value
        self.n = int(n)
        self.dim = int(dim)
        self.beta = float(beta)
        self.precision = int(precision)
        self.device = int(device)

    @classmethod
    def from_nodes(cls, n, site_norb, beta, nodes, precision=F64, device=0, dim=2):
        """``nodes``: dict with omega (eV), tau_t, n_f, n_b."""
        return cls(n, site_norb, beta, nodes["omega"], nodes["tau_t"], nodes["n_f"], nodes["n_b"],
                   precision, device, dim)

    @classmethod
    def uniform(cls, n, site_norb, beta, n_nodes, device=0, dim=2):
        """Uniform Matsubara-grid plan (qgw_plan_create_mf) with ``n_nodes`` = N frequencies / times."""
        none_d, none_i = np.zeros(1), np.zeros(1, dtype=np.int64)
        return cls(n, site_norb, beta, none_d, none_d, none_i, none_i, F64, device, dim, mf_nodes=n_nodes)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().qgw_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_map(self, which):
        rows = 1 if which == F_IW2BETA else self.r
        out = np.zeros(rows * self.r * 2)
        _check(lib().qgw_plan_get_map(self.handle, int(which), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return (out[0::2] + 1j * out[1::2]).reshape(rows, self.r)

    def workspace_size(self, op):
        """Bytes of scratch call ``op`` (OP_*) needs on this plan (qgw_workspace_size)."""
        b = ctypes.c_int64(0)
        _check(lib().qgw_workspace_size(self.handle, int(op), ctypes.byref(b)))
        return b.value

    def workspace(self, op):
        """A device scratch buffer for call ``op`` from torch's caching allocator (None if none is needed)."""
        import torch
        b = self.workspace_size(op)
        if b == 0:
            return None
        return torch.empty(b, dtype=torch.uint8, device="cuda:%d" % self.device)

    def sync_status(self):
        """Waits for the stream, reads and clears the device status word (raises QGWError if it is set)."""
        _check(lib().qgw_sync_status(self.handle, _stream()))

    # ---- step calls ------------------------------------------------------
    def dlr_transform(self, which, x, out, scale=1.0, hermitian=0):
        ncols = x.numel() // self.r
        s = complex(scale)
        _check(lib().qgw_dlr_transform(self.handle, int(which), int(ncols), s.real, s.imag, int(hermitian),
                                       _ptr(x), _ptr(out), _stream()))
        return out

    def dlr_transform_pairs(self, which, in_layout, out_layout, x, out):
        _check(lib().qgw_dlr_transform_pairs(self.handle, int(which), int(in_layout), int(out_layout),
                                             _ptr(x), _ptr(out), _stream()))
        return out

    def lattice_fft(self, direction, x, out):
        batch = x.numel() // self.n_k
        _check(lib().qgw_lattice_fft(self.handle, int(direction), int(batch), _ptr(x), _ptr(out), _stream()))
        return out

    def bubble(self, g_tau_r, g_reflt_r, out, out_q=True):
        _check(lib().qgw_bubble(self.handle, _ptr(g_tau_r), _ptr(g_reflt_r), int(bool(out_q)), _ptr(out), _stream()))
        return out

    def dyson_W(self, v_q, p_nu, out):
        _check(lib().qgw_dyson_W(self.handle, _ptr(v_q), _ptr(p_nu), _ptr(out), _stream()))
        return out

    def sigma(self, g_tau_r, wc, out, in_q=True, out_k=True):
        _check(lib().qgw_sigma(self.handle, _ptr(g_tau_r), _ptr(wc), int(bool(in_q)), int(bool(out_k)), _ptr(out), _stream()))
        return out

    def hartree_fock(self, v_r, n_r, out):
        _check(lib().qgw_hartree_fock(self.handle, _ptr(v_r), _ptr(n_r), _ptr(out), _stream()))
        return out

    def dyson_G(self, h_k, sig_iw, out, n_target=None, mu=0.0):
        m = ctypes.c_double(float(mu))
        nt = float("nan") if n_target is None else float(n_target)
        _check(lib().qgw_dyson_G(self.handle, _ptr(h_k), _ptr(sig_iw), nt, ctypes.byref(m), _ptr(out), _stream()))
        return m.value

    def dyson_G_noalloc(self, h_k, sig_iw, out, n_target=None, mu=0.0):
        """qgw_dyson_G with the search scratch in the library's static device array (allocates nothing)."""
        m = ctypes.c_double(float(mu))
        nt = float("nan") if n_target is None else float(n_target)
        _check(lib().qgw_dyson_G_noalloc(self.handle, _ptr(h_k), _ptr(sig_iw), nt, ctypes.byref(m), _ptr(out),
                                         _stream()))
        return m.value

    def check_finite(self, x):
        _check(lib().qgw_check_finite(self.handle, _ptr(x), int(x.numel()), _stream()))

    # ---- adjoints (cotangent convention zbar = dL/dRe z + i dL/dIm z) ----
    def dlr_transform_bwd(self, which, ybar, xbar, scale=1.0, hermitian=0):
        ncols = xbar.numel() // self.r
        s = complex(scale)
        _check(lib().qgw_dlr_transform_bwd(self.handle, int(which), int(ncols), s.real, s.imag, int(hermitian),
                                           _ptr(ybar), _ptr(xbar), _stream()))
        return xbar

    def dlr_transform_pairs_bwd(self, which, in_layout, out_layout, ybar, xbar):
        _check(lib().qgw_dlr_transform_pairs_bwd(self.handle, int(which), int(in_layout), int(out_layout),
                                                 _ptr(ybar), _ptr(xbar), _stream()))
        return xbar

    def lattice_fft_bwd(self, direction, ybar, xbar):
        batch = ybar.numel() // self.n_k
        _check(lib().qgw_lattice_fft_bwd(self.handle, int(direction), int(batch), _ptr(ybar), _ptr(xbar), _stream()))
        return xbar

    def bubble_bwd(self, g_tau_r, g_reflt_r, pbar_q, gbar_tau, gbar_reflt):
        _check(lib().qgw_bubble_bwd(self.handle, _ptr(g_tau_r), _ptr(g_reflt_r), _ptr(pbar_q), _ptr(gbar_tau),
                                    _ptr(gbar_reflt), _stream()))
        return gbar_tau, gbar_reflt

    def sigma_bwd(self, g_tau_r, wc_q, sigbar, gbar_tau, wcbar_q, out_k=True, workspace=None):
        ws = self.workspace(OP_SIGMA_BWD) if (workspace is None and out_k) else workspace
        _check(lib().qgw_sigma_bwd(self.handle, _ptr(g_tau_r), _ptr(wc_q), int(bool(out_k)), _ptr(sigbar),
                                   _ptr(gbar_tau), _ptr(wcbar_q), _ptr(ws), _nbytes(ws), _stream()))
        return gbar_tau, wcbar_q

    def dyson_W_bwd(self, v_q, p_nu, wcbar, pbar, vbar, workspace=None):
        ws = self.workspace(OP_DYSON_W_BWD) if workspace is None else workspace
        _check(lib().qgw_dyson_W_bwd(self.handle, _ptr(v_q), _ptr(p_nu), _ptr(wcbar), _ptr(pbar), _ptr(vbar),
                                     _ptr(ws), _nbytes(ws), _stream()))
        return pbar, vbar

    def hartree_fock_bwd(self, v_r, n_r, sbar, nbar=None, vbar=None, workspace=None):
        ws = self.workspace(OP_HARTREE_FOCK_BWD) if workspace is None else workspace
        _check(lib().qgw_hartree_fock_bwd(self.handle, _ptr(v_r), _ptr(n_r), _ptr(sbar), _ptr(nbar), _ptr(vbar),
                                          _ptr(ws), _nbytes(ws), _stream()))
        return nbar, vbar

    def dyson_G_bwd(self, h_k, sig_iw, mu, gbar, sigbar, hbar=None, n_target=None, mubar=0.0):
        nt = float("nan") if n_target is None else float(n_target)
        _check(lib().qgw_dyson_G_bwd(self.handle, _ptr(h_k), _ptr(sig_iw), float(mu), nt, float(mubar), _ptr(gbar),
                                     _ptr(sigbar), _ptr(hbar), _stream()))
        return sigbar, hbar

    TUNE_NAMES = ("fft_slabs_per_block", "bubble_slabs_per_block", "sigma_term_lanes", "mfma_blocks_per_cu",
                  "orbital_map_valu", "orbital_map_rows", "dyson_w25_mfma")

    def autotune(self):
        """Times the candidate launch shapes on this plan and keeps the fastest; returns them."""
        ch = (ctypes.c_int32 * 7)()
        _check(lib().qgw_plan_autotune(self.handle, ch, _stream()))
        return dict(zip(self.TUNE_NAMES, list(ch)))

    def set_tuning(self, choices, precision=0):
        """Sets the launch shapes (a dict as autotune returns; missing knobs at their defaults) for the plan's
        FP64 (precision 0) or, on an FP64 plan, its FP32 kernels (precision 1) (qgw_plan_set_tuning)."""
        dflt = {n: 0 for n in self.TUNE_NAMES}
        dflt["orbital_map_valu"] = -1
        dflt["dyson_w25_mfma"] = -1
        dflt.update(choices)
        ch = (ctypes.c_int32 * 7)(*[int(dflt[n]) for n in self.TUNE_NAMES])
        _check(lib().qgw_plan_set_tuning(self.handle, int(precision), ch))

    def energy(self, h_k, shf_k, sig_iw, g_iw):
        """(E, HF part, correlation part) of the Galitskii-Migdal energy."""
        e = np.zeros(3)
        ws = self.workspace(OP_ENERGY)
        _check(lib().qgw_energy(self.handle, _ptr(h_k), _ptr(shf_k), _ptr(sig_iw), _ptr(g_iw),
                                e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(ws), _nbytes(ws), _stream()))
        return tuple(e.tolist())

    def energy_bwd(self, h_k, shf_k, sig_iw, g_iw, ebar, hbar, shfbar, sigbar, gbar):
        ws = self.workspace(OP_ENERGY_BWD)
        _check(lib().qgw_energy_bwd(self.handle, _ptr(h_k), _ptr(shf_k), _ptr(sig_iw), _ptr(g_iw), float(ebar),
                                    _ptr(hbar), _ptr(shfbar), _ptr(sigbar), _ptr(gbar), _ptr(ws), _nbytes(ws),
                                    _stream()))
        return hbar, shfbar, sigbar, gbar

    def quasiparticle(self, h_k, shf_k, sig_iw, mu=0.0):
        """Static self-energy, Z(k), the quasiparticle Hamiltonian and its bands (qgw_quasiparticle).

        Returns (sig0, z, hqp, bands): three [n_o, n_o, N_k] complex tensors and [n_o, N_k] real bands."""
        import torch
        shape = tuple(h_k.shape)
        sig0 = torch.empty(shape, dtype=torch.complex128, device=h_k.device)
        z = torch.empty_like(sig0)
        hqp = torch.empty_like(sig0)
        bands = torch.empty((shape[0], shape[-1]), dtype=torch.float64, device=h_k.device)
        ws = self.workspace(OP_QUASIPARTICLE)
        _check(lib().qgw_quasiparticle(self.handle, _ptr(h_k), _ptr(shf_k), _ptr(sig_iw), float(mu), _ptr(sig0),
                                       _ptr(z), _ptr(hqp), ctypes.cast(_ptr(bands), ctypes.POINTER(ctypes.c_double)),
                                       _ptr(ws), _nbytes(ws), _stream()))
        return sig0, z, hqp, bands

    def quasiparticle_path(self, h_k, shf_k, sig_iw, kfrac, mu=0.0):
        """The quasiparticle outputs at path points ``kfrac`` ([n_path, dim] fractional coordinates, host data) by
        Fourier interpolation from the mesh (qgw_quasiparticle_path).

        Returns (sig0, z, hqp, bands): three [n_o, n_o, n_path] complex tensors and [n_o, n_path] real bands."""
        import numpy as np
        import torch
        kf = np.ascontiguousarray(np.asarray(kfrac, dtype=np.float64).reshape(-1, self.dim))
        npt = kf.shape[0]
        no = self.n_o
        dev = h_k.device
        sig0 = torch.empty((no, no, npt), dtype=torch.complex128, device=dev)
        z = torch.empty_like(sig0)
        hqp = torch.empty_like(sig0)
        bands = torch.empty((no, npt), dtype=torch.float64, device=dev)
        b = ctypes.c_int64(0)
        _check(lib().qgw_quasiparticle_path_workspace(self.handle, int(npt), ctypes.byref(b)))
        ws = torch.empty(b.value, dtype=torch.uint8, device=dev)
        _check(lib().qgw_quasiparticle_path(
            self.handle, _ptr(h_k), _ptr(shf_k), _ptr(sig_iw), float(mu),
            kf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(npt), _ptr(sig0), _ptr(z), _ptr(hqp),
            ctypes.cast(_ptr(bands), ctypes.POINTER(ctypes.c_double)), _ptr(ws), _nbytes(ws), _stream()))
        return sig0, z, hqp, bands

    def hf_density(self, h_k, n_target=None, mu=0.0, out=None):
        """(mu, n(k)): Fermi-function density of the static Hamiltonian h_k (qgw_hf_density)."""
        import torch
        out = torch.empty_like(h_k) if out is None else out
        m = ctypes.c_double(mu)
        nt = float("nan") if n_target is None else float(n_target)
        ws = self.workspace(OP_HF_DENSITY)
        _check(lib().qgw_hf_density(self.handle, _ptr(h_k), nt, ctypes.byref(m), _ptr(out), _ptr(ws), _nbytes(ws),
                                    _stream()))
        return m.value, out

    def add(self, a, b, out):
        _check(lib().qgw_add(self.handle, int(a.numel()), _ptr(a), _ptr(b), _ptr(out), _stream()))
        return out

    def pair_layout(self, x, out, in_layout, out_layout):
        nn = x.numel() // (self.n_b * self.n_b * self.n_k)
        _check(lib().qgw_pair_layout(self.handle, int(in_layout), int(out_layout), int(nn), _ptr(x), _ptr(out),
                                     _stream()))
        return out


class State:
    """Self-consistent GW state on the device (FP64 plans)."""

    def __init__(self, plan, H0_R, V_R, n_target=None, mixing=1.0):
        self.plan = plan
        self._H0_R, self._V_R = H0_R, V_R
        h = ctypes.c_void_p()
        nt = float("nan") if n_target is None else float(n_target)
        _check(lib().qgw_state_create(plan.handle, _ptr(H0_R), _ptr(V_R), nt, float(mixing), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().qgw_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_g0(self, mu=None):
        """G = G0 (qgw_state_init_g0).  mu: the search's start (with a target filling) or the fixed mu; None starts
        from the state's previous G0, or from the centre of H0's Gershgorin bounds the first time."""
        m = ctypes.c_double(math.nan if mu is None else float(mu))
        _check(lib().qgw_state_init_g0(self.handle, ctypes.byref(m), _stream()))
        return m.value

    def iterate(self, n_iter=1, tol=0.0):
        done = ctypes.c_int32(0)
        ds = ctypes.c_double(math.nan)
        mu = ctypes.c_double(math.nan)
        _check(lib().qgw_gw_iteration(self.handle, int(n_iter), float(tol), ctypes.byref(done), ctypes.byref(ds),
                                      ctypes.byref(mu), _stream()))
        return done.value, ds.value, mu.value

    def hf_solve(self, tol=1e-10, max_iter=200):
        """Hartree-Fock self-consistency (qgw_state_hf_solve): (passes, last max |dSigma_HF|, mu)."""
        done = ctypes.c_int32(0)
        ds = ctypes.c_double(math.nan)
        mu = ctypes.c_double(math.nan)
        _check(lib().qgw_state_hf_solve(self.handle, float(tol), int(max_iter), ctypes.byref(done),
                                        ctypes.byref(ds), ctypes.byref(mu), _stream()))
        return done.value, ds.value, mu.value

    STEP_NAMES = ["a12_density_hf", "a1_dlr_g", "a2_fft_g", "a3a4_bubble", "a5_dlr_p", "a6_dyson_w",
                  "a7_dlr_w", "a8a9a10_sigma", "a11_dlr_sigma", "a14_delta_mix", "a13_dyson_g"]

    def profile(self, mode=2, per_precision=False):
        """mode 1: reset + enable, 0: disable, 2: read.

        Returns (ms per step dict, iterations) summed over both precisions, or
        with per_precision a dict {"f64": (ms dict, iters), "f32": (ms dict, iters)}."""
        ns = len(self.STEP_NAMES)
        ms = np.zeros(2 * ns)
        it = (ctypes.c_int32 * 2)()
        _check(lib().qgw_state_profile(self.handle, int(mode), ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), it))
        rows = {"f64": (dict(zip(self.STEP_NAMES, ms[:ns].tolist())), it[0]),
                "f32": (dict(zip(self.STEP_NAMES, ms[ns:].tolist())), it[1])}
        if per_precision:
            return rows
        return dict(zip(self.STEP_NAMES, (ms[:ns] + ms[ns:]).tolist())), it[0] + it[1]

    def profile_select(self, steps=None, in_line=False):
        """Steps the next profile(1) times (names from STEP_NAMES, None: all) and whether a12 then runs on the
        caller's stream ahead of a1 (qgw_state_profile_select)."""
        names = self.STEP_NAMES if steps is None else list(steps)
        mask = 0
        for n in names:
            mask |= 1 << self.STEP_NAMES.index(n)
        _check(lib().qgw_state_profile_select(self.handle, mask, 1 if in_line else 0))

    def set_search_steps(self, first_round=0):
        """Newton evaluations of mu queued per iteration before the read-back (qgw_state_set_search_steps; 0 adapts)."""
        _check(lib().qgw_state_set_search_steps(self.handle, int(first_round)))

    def set_precision(self, mode, switch_tol=1e-4):
        """mode 0: FP64 throughout; 1: FP32 bulk steps until |dSigma| <= switch_tol, then FP64."""
        _check(lib().qgw_state_set_precision(self.handle, int(mode), float(switch_tol)))

    def info(self):
        """(precision of the last iteration, FP32 iterations, FP64 iterations)."""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qgw_state_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), None))
        return a.value, b.value, c.value

    def mu_evals(self):
        """N_e(mu) evaluations of the last iteration's chemical-potential search."""
        e = ctypes.c_int32()
        _check(lib().qgw_state_info(self.handle, None, None, None, ctypes.byref(e)))
        return e.value

    def array(self, which):
        """Copy of a state array as a torch tensor (0 G, 1 Sigma_C, 2 Sigma_HF, 3 P, 4 W^C, 5 n)."""
        import torch
        p = self.plan
        shapes = {0: (p.r, p.n_o, p.n_o, p.n_k), 1: (p.r, p.n_o, p.n_o, p.n_k), 2: (p.n_o, p.n_o, p.n_k),
                  3: (p.r, p.n_k, p.n_b, p.n_b), 4: (p.r, p.n_k, p.n_b, p.n_b), 5: (p.n_o, p.n_o, p.n_k)}
        out = torch.empty(shapes[which], dtype=torch.complex128, device="cuda:%d" % p.device)
        nbytes = ctypes.c_int64(0)
        _check(lib().qgw_state_copy(self.handle, int(which), _ptr(out), ctypes.byref(nbytes), _stream()))
        assert nbytes.value == out.numel() * 16
        return out


def batch_solve(b64, tol, b32=None, switch_tol=None, max_replays=60):
    """Replays batches until every state's max |Delta Sigma| <= tol after an FP64 replay, or max_replays.

    Host control only: each replay is one of the library's captured graphs.  With ``b32`` (an FP32 batch over the
    same states) the FP32 replays come first, until every state is at ``switch_tol`` or stalled (its |Delta Sigma|
    is not below half its best so far, which also ends the phase for a state that oscillates), the batch form of a
    state's mixed schedule (qgw_state_set_precision mode 1).
    Returns a dict: per state the FP64 replay count at which it first met tol (-1 if never) and the seconds since
    the first replay at that point (nan if never), the FP32 and FP64 replay counts, and the final statuses."""
    import time
    n = len(b64.states)
    at = np.full(n, -1, dtype=np.int64)
    t_at = np.full(n, np.nan)
    n32 = n64 = 0
    best = None
    phase32 = b32 is not None
    statuses = np.zeros(n, dtype=np.int32)
    t0 = time.perf_counter()
    for _ in range(max_replays):
        b = b32 if phase32 else b64
        b.launch()
        ds, _, st = b.read()
        now = time.perf_counter() - t0
        statuses = np.maximum(statuses, st)
        if phase32:
            n32 += 1
            if best is not None and np.all((ds <= switch_tol) | (ds > 0.5 * best)):
                phase32 = False
            best = ds if best is None else np.minimum(best, ds)
            continue
        n64 += 1
        hit = (at < 0) & (ds <= tol)
        at[hit] = n64
        t_at[hit] = now
        if np.all(at >= 0):
            break
    return {"fp64_replays_to_tol": at, "seconds_to_tol": t_at, "fp32_replays": n32, "fp64_replays": n64,
            "status": statuses}


class Batch:
    """Many started states advanced together by one graph launch (qgw_batch_*)."""

    def __init__(self, states, precision=F64, n_iter=1, mu_steps=12):
        self.states = list(states)
        arr = (ctypes.c_void_p * len(self.states))(*[s.handle.value for s in self.states])
        h = ctypes.c_void_p()
        _check(lib().qgw_batch_create(len(self.states), arr, int(precision), int(n_iter), int(mu_steps),
                                      ctypes.byref(h)))
        self.handle = h

    def launch(self):
        _check(lib().qgw_batch_launch(self.handle, _stream()))

    def read(self, with_evals=False):
        """(max |Delta Sigma|, mu, status) per state after the stream has drained; status is the worst search
        status of every replay since the previous read.  with_evals adds the last search's evaluation counts."""
        n = len(self.states)
        ds, mu = np.zeros(n), np.zeros(n)
        st = np.zeros(n, dtype=np.int32)
        ev = np.zeros(n, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int32)
        _check(lib().qgw_batch_read(self.handle, ds.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), st.ctypes.data_as(ip),
                                    ev.ctypes.data_as(ip), _stream()))
        return (ds, mu, st, ev) if with_evals else (ds, mu, st)

    def close(self):
        if self.handle:
            lib().qgw_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

