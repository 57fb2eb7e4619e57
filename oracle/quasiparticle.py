"""Quasiparticle post-processing of a GW self-energy, plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): not for the product path.

The Z and SigStc class paragraphs take the zero-frequency limit of the
self-energy Sigma(k, i w_n) held in DLR form.  On the Matsubara axis the
frequencies closest to zero are +-pi/beta; nearer to the real axis the DLR
expansion (poles on the real axis, Sigma^C(z) = sum_l c_l / (z - w_l)) no
longer follows the self-energy, whose cut lies there.  So the limit is taken
at +-pi/beta, from the interpolant's values there (equal to the node values
when n = 0 and n = -1 are nodes):

* static self-energy (SigStc class): the mean of Sigma(k, +-i pi/beta),
  Sigma(k, 0) = Sigma_HF(k) + Herm Sigma^C(k, i pi/beta), because
  Sigma(-i w) = Sigma(i w)^H;
* renormalisation (Z class, Eq. eq-z-factor): dSigma/d(i w) at w = 0 as the
  central difference over +-pi/beta,
  Z(k)^{-1} = 1 - (S - S^H) / (2 i pi/beta),  S = Sigma^C(k, i pi/beta),
  which is Hermitian (for one orbital: 1 - Im S / (pi/beta));
* quasiparticle Hamiltonian (Eq. eq-quasi-particle-Hamiltonian):
  H_QP(k) = sqrt(Z(k)) (H0(k) + Sigma(k, 0) - mu) sqrt(Z(k)) with the principal
  square root of the Hermitian positive matrix Z; mu = 0 is the equation as
  printed, a chemical potential puts the bands relative to the Fermi level;
* quasiparticle bands: the eigenvalues of H_QP(k), ascending.

Bands along a path of k points off the mesh (Fig. fig-band-dos (a)) need
H0, Sigma_HF and S at those points.  Reading: Fourier interpolation of the
mesh values, X(k') = sum_R w(R) exp(-i k'.R) X(R) with X(R) the inverse DFT
of the mesh values and each axis's R taken in (-n/2, n/2]; for even n the
n/2 term is split equally between +n/2 and -n/2, which gives the weight
cos(pi f n) for fractional coordinate f.  On mesh points this returns the
mesh values themselves; hoppings shorter than half the mesh come back as
the analytic H0(k').

Arrays carry orbital indices first and the mesh axes last; the
self-energy carries the node axis before them.
"""
import numpy as np

from . import lattice
from .gw import hermitian_part


def _orbital_last(x):
    """[a, b, *mesh] -> [*mesh, a, b]."""
    return np.moveaxis(x, (0, 1), (-2, -1))


def _orbital_first(x):
    return np.moveaxis(x, (-2, -1), (0, 1))


def dlr_value_at(dlr, sig_iw, z):
    """The DLR interpolant sum_l c_l / (z - w_l) of values on the fermionic Matsubara nodes."""
    c = dlr.coeffs_from_iw_f(sig_iw)
    w = 1.0 / (z - dlr.omega)
    return np.tensordot(w, c, axes=(0, 0))


def sigma_first_matsubara(dlr, sig_iw):
    """S = Sigma^C(k, i pi / beta)."""
    return dlr_value_at(dlr, sig_iw, 1j * np.pi / dlr.beta)


def static_self_energy(dlr, sig_hf_k, sig_iw):
    """Sigma(k, 0) = Sigma_HF(k) + (S + S^H) / 2 (SigStc class)."""
    s = sigma_first_matsubara(dlr, sig_iw)
    return hermitian_part(sig_hf_k + s)


def z_inverse(dlr, sig_iw):
    """Z(k)^{-1} = 1 - (S - S^H) / (2 i pi/beta) (Eq. eq-z-factor, central difference over +-pi/beta)."""
    return z_inverse_from_s(sigma_first_matsubara(dlr, sig_iw), dlr.beta)


def z_inverse_from_s(s, beta):
    """Z^{-1} = 1 - (S - S^H) / (2 i pi/beta) from S = Sigma^C(i pi/beta)."""
    w0 = np.pi / beta
    ds = (s - np.conj(np.swapaxes(s, 0, 1))) / (2j * w0)
    n_o = s.shape[0]
    eye = np.eye(n_o).reshape((n_o, n_o) + (1,) * (s.ndim - 2))
    return eye - ds


def matrix_power_hermitian(x, p):
    """x^p for Hermitian positive x [a, b, ...] through its eigen-decomposition."""
    ev, u = np.linalg.eigh(_orbital_last(x))
    if np.any(ev <= 0.0):
        raise ValueError("Z(k)^{-1} is not positive definite")
    out = np.einsum("...ai,...i,...bi->...ab", u, ev ** p, np.conj(u))
    return _orbital_first(out)


def qp_hamiltonian(H_k, sig0_k, zinv_k, mu=0.0):
    """sqrt(Z) (H0 + Sigma(k, 0) - mu) sqrt(Z) (Eq. eq-quasi-particle-Hamiltonian), Hermitian part."""
    sz = _orbital_last(matrix_power_hermitian(zinv_k, -0.5))
    n_o = H_k.shape[0]
    a = _orbital_last(H_k + sig0_k) - mu * np.eye(n_o)
    return hermitian_part(_orbital_first(sz @ a @ sz))


def qp_bands(hqp_k):
    """Eigenvalues of H_QP(k), ascending: [band, *mesh]."""
    ev = np.linalg.eigvalsh(_orbital_last(hqp_k))
    return np.moveaxis(ev, -1, 0)


def quasiparticle(model, dlr, state, mu=0.0):
    """All quasiparticle outputs of a GW state (keys sig0, zinv, z, hqp, bands)."""
    sig0 = static_self_energy(dlr, state["sig_hf_k"], state["sig_iw"])
    zinv = z_inverse(dlr, state["sig_iw"])
    z = matrix_power_hermitian(zinv, -1.0)
    hqp = qp_hamiltonian(model.H_k, sig0, zinv, mu)
    return {"sig0": sig0, "zinv": zinv, "z": z, "hqp": hqp, "bands": qp_bands(hqp)}


def interpolation_phases(mesh, kfrac):
    """w(R) exp(-2 pi i f.R) for every mesh R and path point f (fractional coordinates): [npt, *mesh]."""
    kfrac = np.atleast_2d(np.asarray(kfrac, dtype=np.float64))
    out = np.ones((kfrac.shape[0],) + tuple(mesh), dtype=np.complex128)
    for a, n in enumerate(mesh):
        R = np.arange(n)
        rep = np.where(R < n / 2.0, R, R - n).astype(np.float64)
        f = kfrac[:, a][:, None]
        ph = np.exp(-2j * np.pi * f * rep[None, :])
        if n % 2 == 0:
            ph[:, n // 2] = np.cos(np.pi * f[:, 0] * n)
        shape = [kfrac.shape[0]] + [1] * len(mesh)
        shape[1 + a] = n
        out = out * ph.reshape(shape)
    return out


def fourier_interpolate(x_k, kfrac):
    """X(k') from the mesh values x_k [a, b, *mesh] at the points kfrac [npt, d]: [a, b, npt]."""
    d = len(np.atleast_2d(kfrac)[0])
    mesh = x_k.shape[-d:]
    x_r = lattice.R_from_k(x_k, d)
    ph = interpolation_phases(mesh, kfrac)
    axes = tuple(range(x_k.ndim - d, x_k.ndim))
    return np.tensordot(x_r, ph, axes=(axes, tuple(range(1, d + 1))))


def quasiparticle_path(model, dlr, state, kfrac, mu=0.0):
    """The quasiparticle outputs at path points kfrac [npt, d] (fractional coordinates of the reciprocal basis):
    H0, Sigma_HF and S = Sigma^C(i pi/beta) interpolated from the mesh, then the relations above per point."""
    h = fourier_interpolate(model.H_k, kfrac)
    shf = fourier_interpolate(state["sig_hf_k"], kfrac)
    s = fourier_interpolate(sigma_first_matsubara(dlr, state["sig_iw"]), kfrac)
    sig0 = hermitian_part(shf + s)
    zinv = z_inverse_from_s(s, dlr.beta)
    z = matrix_power_hermitian(zinv, -1.0)
    hqp = qp_hamiltonian(h, sig0, zinv, mu)
    return {"h0": h, "sig0": sig0, "zinv": zinv, "z": z, "hqp": hqp, "bands": qp_bands(hqp)}
