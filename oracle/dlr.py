"""Discrete Lehmann representation (DLR), plain FP64 NumPy/SciPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): not for the product path.

The paper compresses every imaginary-time / Matsubara axis with the DLR
(method section, the sentence after Eq. eq:bare-green-freq, citing Kaye, Chen
& Parcollet, PRB 105, 235115 (2022)).  This module builds it from that
published construction:

* Lehmann kernel, in physical units with the convention
  X(i w_n) = int_0^beta e^{i w_n tau} X(tau) dtau:

      K(tau, w)      = -exp(-w tau) / (1 + exp(-beta w))       (0 < tau < beta)
      K_F(i w_n, w)  = 1 / (i w_n - w),   w_n = (2n+1) pi / beta
      K_B(i nu_n, w) = tanh(beta w / 2) / (i nu_n - w),  nu_n = 2 n pi / beta

  K_F and K_B are the fermionic and bosonic Matsubara transforms of the same
  K(tau, w); bosonic functions are expanded in the same (fermionic-kernel)
  basis.
* Real frequencies w_l: pivoted QR over the columns of K sampled on fine
  composite-Chebyshev grids (dyadically refined toward tau = 0, beta and
  w = 0), keeping the columns whose pivot exceeds eps * (first pivot).
* Imaginary-time nodes tau_k: pivoted QR over the rows of K(tau_fine, w_l).
* Matsubara nodes n_k (fermionic and bosonic): pivoted QR over the rows of
  K_F / K_B on all |n| <= n_max.
* Composite maps between node values are formed by linear solves with the
  r x r interpolation matrices (never an explicit inverse).

Dimensionless variables are used for the selection: t = tau / beta in [0, 1],
x = beta * w in [-Lambda, Lambda], Lambda = beta * omega_max.
"""
import numpy as np
import scipy.linalg


# ----------------------------------------------------------------------------
# kernel
# ----------------------------------------------------------------------------

def kernel_tau_dimless(t, tc, x):
    """k(t, x) = exp(-t x) / (1 + exp(-x)), t = tau/beta, tc = 1 - t.

    Overflow-safe: for x < 0 the equal form exp(tc x) / (1 + exp(x)) is used,
    with tc supplied by the caller so that points near t = 1 keep full
    relative accuracy.  Broadcasts over (t, tc) against x.
    """
    t = np.asarray(t, dtype=np.float64)
    tc = np.asarray(tc, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    pos = x >= 0
    xp = np.where(pos, x, 0.0)
    xn = np.where(pos, 0.0, x)
    val_pos = np.exp(-t * xp) / (1.0 + np.exp(-xp))
    val_neg = np.exp(tc * xn) / (1.0 + np.exp(xn))
    return np.where(pos, val_pos, val_neg)


def kernel_tau(tau_t, omega, beta, reflect=False):
    """Physical K(tau, w) = -exp(-w tau)/(1+exp(-beta w)) at tau = beta * t.

    ``tau_t`` are dimensionless nodes t in [0, 1]; with ``reflect`` the kernel
    is evaluated at beta - tau, i.e. at t' = 1 - t (the reflected point that
    the bubble needs; the tau nodes are not symmetric about beta / 2).
    """
    t = np.asarray(tau_t, dtype=np.float64)[:, None]
    x = beta * np.asarray(omega, dtype=np.float64)[None, :]
    if reflect:
        return -kernel_tau_dimless(1.0 - t, t, x)
    return -kernel_tau_dimless(t, 1.0 - t, x)


def kernel_tau_beta(omega, beta):
    """K(beta^-, w) = -1 / (1 + exp(beta w)), overflow-safe."""
    x = beta * np.asarray(omega, dtype=np.float64)
    return -kernel_tau_dimless(np.ones_like(x), np.zeros_like(x), x)


def matsubara_f(n, beta):
    """Fermionic Matsubara frequencies w_n = (2n+1) pi / beta."""
    return (2.0 * np.asarray(n, dtype=np.float64) + 1.0) * np.pi / beta


def matsubara_b(n, beta):
    """Bosonic Matsubara frequencies nu_n = 2 n pi / beta."""
    return 2.0 * np.asarray(n, dtype=np.float64) * np.pi / beta


def kernel_iw_f(n, omega, beta):
    """K_F(i w_n, w) = 1 / (i w_n - w) for fermionic nodes n (rows) and w (cols)."""
    wn = matsubara_f(n, beta)[:, None]
    w = np.asarray(omega, dtype=np.float64)[None, :]
    return 1.0 / (1j * wn - w)


def kernel_iw_b(n, omega, beta):
    """K_B(i nu_n, w) = tanh(beta w / 2) / (i nu_n - w); limit -beta/2 at nu = w = 0."""
    nu = matsubara_b(n, beta)[:, None]
    w = np.asarray(omega, dtype=np.float64)[None, :]
    num = np.tanh(0.5 * beta * w) * np.ones_like(nu)
    den = 1j * nu - w
    out = np.empty(np.broadcast(nu, w).shape, dtype=np.complex128)
    zero = (nu == 0) & (w == 0)
    out[~zero] = num[~zero] / den[~zero]
    out[zero] = -0.5 * beta
    return out


def fermi_divided_differences(omega, beta):
    """D[l, l'] = (1/beta) sum_n 1 / ((i w_n - w_l)(i w_n - w_l')) over all fermionic n.

    Partial fractions and sum_n 1/(i w_n - x) e^{i w_n 0+} = beta f(x) give the
    divided difference (f(w_l) - f(w_l')) / (w_l - w_l') of the Fermi function
    f(x) = 1 / (1 + e^{beta x}), and -beta f (1 - f) on the diagonal.
    """
    w = np.asarray(omega, dtype=np.float64)
    f = 0.5 * (1.0 - np.tanh(0.5 * beta * w))
    dw = w[:, None] - w[None, :]
    df = f[:, None] - f[None, :]
    same = dw == 0.0
    out = np.where(same, 0.0, df / np.where(same, 1.0, dw))
    diag = -beta * f * (1.0 - f)
    out[np.arange(len(w)), np.arange(len(w))] = diag
    return out


# ----------------------------------------------------------------------------
# node selection
# ----------------------------------------------------------------------------

def _chebyshev_panels(edges, order):
    """Chebyshev points of the first kind on each panel [edges[i], edges[i+1]]."""
    j = np.arange(order)
    x = np.cos(np.pi * (2 * j + 1) / (2 * order))[::-1]
    pts = [0.5 * (a + b) + 0.5 * (b - a) * x for a, b in zip(edges[:-1], edges[1:])]
    return np.concatenate(pts)


def fine_grids(lam, order=24):
    """Fine composite-Chebyshev grids for the kernel matrix.

    Returns (t, tc, x): dimensionless times t with their complements tc = 1 - t
    (exact for the mirrored half), and real frequencies x in [-lam, lam].
    The x panels are dyadically refined toward 0; the t panels toward 0 and
    (by mirroring) toward 1.
    """
    npan = max(int(np.ceil(np.log2(lam))), 1)
    x_edges = np.concatenate([[0.0], lam * 2.0 ** (-np.arange(npan - 1, -1, -1, dtype=np.float64))])
    x_pos = _chebyshev_panels(x_edges, order)
    x = np.concatenate([-x_pos[::-1], x_pos])
    t_edges = np.concatenate([[0.0], 0.5 * 2.0 ** (-np.arange(npan, -1, -1, dtype=np.float64))])
    th = _chebyshev_panels(t_edges, order)
    t = np.concatenate([th, 1.0 - th[::-1]])
    tc = np.concatenate([1.0 - th, th[::-1]])
    return t, tc, x


def _pivoted_selection(mat, count=None, eps=None):
    """Column indices chosen by QR with column pivoting.

    With ``eps`` the count is the number of pivots |R_ii| > eps * |R_00|.
    """
    _, r_fac, piv = scipy.linalg.qr(mat, mode="economic", pivoting=True)
    if count is None:
        d = np.abs(np.diag(r_fac))
        count = int(np.sum(d > eps * d[0]))
    return piv[:count]


def default_nmax(lam):
    """Largest |n| of the Matsubara candidate set."""
    return max(int(np.ceil(2.0 * lam)), 200)


class DLR:
    """DLR basis for inverse temperature ``beta`` and real-frequency cutoff.

    Attributes (all sorted ascending):
      omega   real frequencies w_l (physical units, eV)
      tau_t   dimensionless imaginary-time nodes t_k = tau_k / beta
      n_f     fermionic Matsubara node integers (w = (2n+1) pi / beta)
      n_b     bosonic Matsubara node integers   (nu = 2 n pi / beta)
    """

    def __init__(self, beta, omega_max=None, eps=1e-10, lam=None, nodes=None):
        self.beta = float(beta)
        if lam is None:
            lam = self.beta * float(omega_max)
        self.lam = float(lam)
        self.eps = float(eps)
        if nodes is not None:
            self.omega = np.asarray(nodes["omega"], dtype=np.float64)
            self.tau_t = np.asarray(nodes["tau_t"], dtype=np.float64)
            self.n_f = np.asarray(nodes["n_f"], dtype=np.int64)
            self.n_b = np.asarray(nodes["n_b"], dtype=np.int64)
        else:
            self._select()
        self.r = len(self.omega)
        self._build_maps()

    # -- node selection ------------------------------------------------------
    def _select(self):
        t, tc, x = fine_grids(self.lam)
        kfine = kernel_tau_dimless(t[:, None], tc[:, None], x[None, :])
        cols = _pivoted_selection(kfine, eps=self.eps)
        x_sel = np.sort(x[cols])
        r = len(x_sel)
        ksel = kernel_tau_dimless(t[:, None], tc[:, None], x_sel[None, :])
        rows = _pivoted_selection(ksel.T, count=r)
        self.tau_t = np.sort(t[rows])
        nmax = default_nmax(self.lam)
        nf_all = np.arange(-nmax, nmax, dtype=np.int64)
        kf = 1.0 / (1j * np.pi * (2.0 * nf_all[:, None] + 1.0) - x_sel[None, :])
        self.n_f = np.sort(nf_all[_pivoted_selection(kf.T, count=r)])
        nb_all = np.arange(-nmax, nmax + 1, dtype=np.int64)
        kb = kernel_iw_b(nb_all, x_sel / self.beta, self.beta)
        self.n_b = np.sort(nb_all[_pivoted_selection(kb.T, count=r)])
        self.omega = x_sel / self.beta

    def nodes(self):
        return {"omega": self.omega.copy(), "tau_t": self.tau_t.copy(),
                "n_f": self.n_f.copy(), "n_b": self.n_b.copy()}

    # -- interpolation matrices and composite maps ---------------------------
    def _build_maps(self):
        b = self.beta
        self.K_tau = kernel_tau(self.tau_t, self.omega, b)               # [k, l]
        self.K_taur = kernel_tau(self.tau_t, self.omega, b, reflect=True)  # at beta - tau_k
        self.K_f = kernel_iw_f(self.n_f, self.omega, b)                  # [m, l]
        self.K_b = kernel_iw_b(self.n_b, self.omega, b)                  # [m, l]
        self.K_beta = kernel_tau_beta(self.omega, b)                     # [l]
        self.iw = 1j * matsubara_f(self.n_f, b)
        self.inu = 1j * matsubara_b(self.n_b, b)
        # map A = K_out @ inv(K_in), formed as solve(K_in^T, K_out^T)^T
        self.F_iw2tau = _right_solve(self.K_tau.astype(np.complex128), self.K_f)
        self.F_iw2taur = _right_solve(self.K_taur.astype(np.complex128), self.K_f)
        self.F_tau2iw = _right_solve(self.K_f, self.K_tau.astype(np.complex128))
        self.B_tau2iw = _right_solve(self.K_b, self.K_tau.astype(np.complex128))
        self.B_iw2tau = _right_solve(self.K_tau.astype(np.complex128), self.K_b)
        self.F_iw2beta = _right_solve(self.K_beta[None, :].astype(np.complex128), self.K_f)[0]
        # Matsubara-sum form: (1/beta) sum_n A(i w_n) B(i w_n) = sum_{m m'} A_m F_gm[m, m'] B_m'
        # over the node values of two fermionic DLR functions (all n, not only the nodes)
        self.D_sum = fermi_divided_differences(self.omega, b)
        kinv_t_d = np.linalg.solve(self.K_f.T, self.D_sum.astype(np.complex128))     # K^{-T} D
        self.F_gm = np.linalg.solve(self.K_f.T, kinv_t_d.T).T                        # K^{-T} D K^{-1}

    # coefficient-level helpers (used by the tests and the energy)
    def coeffs_from_iw_f(self, x_iw):
        """DLR coefficients g_l from values at the fermionic Matsubara nodes (axis 0)."""
        return _solve_axis0(self.K_f, x_iw)

    def coeffs_from_tau(self, x_tau):
        return _solve_axis0(self.K_tau.astype(np.complex128), x_tau)


def _right_solve(k_out, k_in):
    """k_out @ inv(k_in) via a linear solve with k_in^T."""
    return np.linalg.solve(k_in.T, k_out.T).T


def _solve_axis0(mat, x):
    shp = x.shape
    sol = np.linalg.solve(mat, x.reshape(shp[0], -1))
    return sol.reshape(shp)


def apply_map(mat, x):
    """out[m, ...] = sum_t mat[m, t] * x[t, ...] (the DLR node axis is axis 0)."""
    shp = x.shape
    out = mat @ x.reshape(shp[0], -1)
    return out.reshape((mat.shape[0],) + shp[1:])
