"""Lattice Fourier transforms, plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): not for the product path.

Eq. eq:fourier-transform-kr defines X(k) = sum_R X(R) exp(-i k.(R + tau_p - tau_q))
and X(R) = (1/N_k) sum_k X(k) exp(+i k.(R + tau_p - tau_q)).  The basis-vector
phase exp(-i k.(tau_p - tau_q)) is a k-dependent diagonal unitary gauge that
cancels in every product of k-space matrices and in every R-space quantity, so
the oracle works in the cell-periodic gauge (phase dropped): the transforms are
plain d-dimensional DFTs over the mesh, with k.R = 2 pi sum_a k_a R_a / n_a.

The mesh axes are the last ``d`` axes of every array (d = 2 for a square or
rectangular mesh, d = 3 for a cubic one).
"""
import numpy as np


def mesh_axes(d):
    return tuple(range(-d, 0))


def k_from_R(x_r, d=2):
    """X(k) = sum_R X(R) exp(-i k.R)  (numpy's forward DFT, unnormalised)."""
    return np.fft.fftn(x_r, axes=mesh_axes(d))


def R_from_k(x_k, d=2):
    """X(R) = (1/N_k) sum_k X(k) exp(+i k.R)  (numpy's inverse DFT)."""
    return np.fft.ifftn(x_k, axes=mesh_axes(d))


def reflect(x_r, d=2):
    """X(-R) on the periodic mesh: index R -> (-R) mod n along every mesh axis."""
    out = x_r
    for ax in mesh_axes(d):
        n = x_r.shape[ax]
        out = np.take(out, (-np.arange(n)) % n, axis=ax)
    return out


def mesh_of(x, lead):
    """The mesh shape of an array with ``lead`` leading (node / orbital / pair) axes."""
    return tuple(x.shape[lead:])


def pair_list(site_norb):
    """Product ('pair') basis of Eq. eq:many-body-hamiltonian.

    For every basis site p with n_p orbitals (global offset o_p), the pairs
    alpha = (p; i, l) with i, l in [0, n_p), ordered site-major then i then l,
    map to global orbital indices (o_p + i, o_p + l).  N_b = sum_p n_p^2.
    """
    out = []
    off = 0
    for n in site_norb:
        for i in range(n):
            for l in range(n):
                out.append((off + i, off + l))
        off += n
    return np.array(out, dtype=np.int64).reshape(-1, 2)
