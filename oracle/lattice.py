"""Lattice Fourier transforms, plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): not for the product path.

Eq. eq:fourier-transform-kr defines X(k) = sum_R X(R) exp(-i k.(R + tau_p - tau_q))
and X(R) = (1/N_k) sum_k X(k) exp(+i k.(R + tau_p - tau_q)).  The basis-vector
phase exp(-i k.(tau_p - tau_q)) is a k-dependent diagonal unitary gauge that
cancels in every product of k-space matrices and in every R-space quantity, so
the oracle works in the cell-periodic gauge (phase dropped): the transforms are
plain 2-D DFTs over the mesh, with k.R = 2 pi (k1 R1 / n1 + k2 R2 / n2).

The mesh axes are the last two axes of every array.
"""
import numpy as np


def k_from_R(x_r):
    """X(k) = sum_R X(R) exp(-i k.R)  (numpy's forward DFT, unnormalised)."""
    return np.fft.fft2(x_r, axes=(-2, -1))


def R_from_k(x_k):
    """X(R) = (1/N_k) sum_k X(k) exp(+i k.R)  (numpy's inverse DFT)."""
    return np.fft.ifft2(x_k, axes=(-2, -1))


def reflect(x_r):
    """X(-R) on the periodic mesh: index R -> (-R) mod n along both mesh axes."""
    n1, n2 = x_r.shape[-2:]
    i1 = (-np.arange(n1)) % n1
    i2 = (-np.arange(n2)) % n2
    return x_r[..., i1, :][..., :, i2]


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
