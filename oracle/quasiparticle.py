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

Arrays carry orbital indices first and the mesh axes last; the
self-energy carries the node axis before them.
"""
import numpy as np

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
    s = sigma_first_matsubara(dlr, sig_iw)
    w0 = np.pi / dlr.beta
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
