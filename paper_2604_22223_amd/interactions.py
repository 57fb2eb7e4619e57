"""Interaction tensors of the model inputs (V class of the paper's code overview;
interaction paragraph after Eq. eq:many-body-hamiltonian).

Inputs only, like ``workloads``: these functions build the bare interaction V
that both the HIP path and the test oracle consume; none of the GW method's
arithmetic is here.

Local interactions
------------------
* Slater parametrisation of a shell of angular momentum l with Slater
  integrals F^0, F^2, .., F^2l.  In the complex spherical-harmonic basis
      U_{m1 m2 m3 m4} = sum_k F^k sum_q c^k(m1, m3) c^k(m4, m2),
  with the Gaunt coefficients
      c^k(m, m') = (-1)^m (2l + 1) (l k l; 0 0 0) (l k l; -m, m - m', m'),
  nonzero only for m1 + m2 = m3 + m4.  U_{m1 m2 m3 m4} = <m1 m2|v|m3 m4>:
  electron 1 goes m3 -> m1, electron 2 m4 -> m2.  It is then rotated to real
  (cubic) harmonics, for l = 2 in the order (xy, yz, z^2, xz, x^2 - y^2).
* In the pair basis of the Hamiltonian (c+_i c+_j c_k c_l with the pairs
  (i, l) and (j, k)) the tensor is V_{(il),(jk)} = U_{i j l k}; the Kanamori
  tensor of the same basis has V_(ii),(ii) = U, V_(ii),(jj) = U',
  V_(ij),(ji) = V_(ij),(ij) = J.
* Slater -> Kanamori: U, U' and J are the averages of the Slater tensor's
  intra-orbital, inter-orbital direct and exchange elements over the shell.
  Kanamori -> Slater: F^0 and F^2 (with a fixed ratio F^4 / F^2, F^6 / F^2)
  solve the same two averages for given U and J.  Both follow from the
  linearity of the tensor in the F^k.

Non-local density-density interactions
--------------------------------------
* Ohno form: V(d) = U / sqrt(1 + (U d / e^2)^2), e^2 = 14.397 eV Angstrom;
  between orbitals with different on-site values U_i, U_j it takes their
  mean (U_i + U_j) / 2.
* JTH form: the same function of distance, with one on-site value U_0 shared
  by every orbital of an equivalence class, so all orbital pairs of two
  sites interact alike: V_ij(d) = U_0 / sqrt(1 + (U_0 d / e^2)^2).
"""
import math

import numpy as np

#: Coulomb constant e^2 / (4 pi eps0) in eV * Angstrom.
COULOMB_EV_ANGSTROM = 14.397


# ----------------------------------------------------------------------------
# angular algebra
# ----------------------------------------------------------------------------

def wigner3j(j1, j2, j3, m1, m2, m3):
    """Wigner 3j symbol (j1 j2 j3; m1 m2 m3) for integer arguments (Racah's formula)."""
    if m1 + m2 + m3 != 0:
        return 0.0
    if j3 < abs(j1 - j2) or j3 > j1 + j2 or abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    f = math.factorial
    tri = f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3) / f(j1 + j2 + j3 + 1)
    pre = math.sqrt(tri * f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2) * f(j3 + m3) * f(j3 - m3))
    tmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    tmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = 0.0
    for t in range(tmin, tmax + 1):
        s += (-1) ** t / (f(t) * f(j3 - j2 + t + m1) * f(j3 - j1 + t - m2) * f(j1 + j2 - j3 - t)
                          * f(j1 - t - m1) * f(j2 - t + m2))
    return (-1) ** (j1 - j2 - m3) * pre * s


def gaunt(l, k, m, mp):
    """c^k(l m, l m') = (-1)^m (2l + 1) (l k l; 0 0 0) (l k l; -m, m - m', m')."""
    return (-1) ** m * (2 * l + 1) * wigner3j(l, k, l, 0, 0, 0) * wigner3j(l, k, l, -m, m - mp, mp)


def real_harmonics(l):
    """T[a, m + l]: real harmonic a as sum_m T[a, m] Y_lm (Condon-Shortley phases), rows ordered m = -l .. l:
    for m > 0 the cosine type (Y_{l,-m} + (-1)^m Y_lm) / sqrt(2) sits at +m and the sine type
    i (Y_{l,-m} - (-1)^m Y_lm) / sqrt(2) at -m; for l = 2 that is (xy, yz, z^2, xz, x^2 - y^2)."""
    n = 2 * l + 1
    T = np.zeros((n, n), dtype=np.complex128)
    s = 1.0 / math.sqrt(2.0)
    for m in range(-l, l + 1):
        a = m + l
        if m == 0:
            T[a, l] = 1.0
        elif m > 0:
            T[a, l - m] = s
            T[a, l + m] = s * (-1) ** m
        else:
            mm = -m
            T[a, l - mm] = 1j * s
            T[a, l + mm] = -1j * s * (-1) ** mm
    return T


# ----------------------------------------------------------------------------
# Slater and Kanamori
# ----------------------------------------------------------------------------

def slater_tensor(l, F, basis="real"):
    """U_{abcd} = <ab|v|cd> of a shell of angular momentum l from the Slater integrals F = (F^0, F^2, .., F^2l)
    (missing ones are zero), in the complex (basis="complex") or real harmonic basis."""
    n = 2 * l + 1
    F = list(F) + [0.0] * (l + 1 - len(F))
    U = np.zeros((n, n, n, n), dtype=np.complex128)
    for kk in range(l + 1):
        k = 2 * kk
        if F[kk] == 0.0:
            continue
        c = np.array([[gaunt(l, k, m, mp) for mp in range(-l, l + 1)] for m in range(-l, l + 1)])
        for m1 in range(n):
            for m2 in range(n):
                for m3 in range(n):
                    m4 = m1 + m2 - m3
                    if 0 <= m4 < n:
                        U[m1, m2, m3, m4] += F[kk] * c[m1, m3] * c[m4, m2]
    if basis == "complex":
        return U
    T = real_harmonics(l)
    Ur = np.einsum("ai,bj,ck,dl,ijkl->abcd", T.conj(), T.conj(), T, T, U)
    assert np.abs(Ur.imag).max() < 1e-12 * max(1.0, np.abs(Ur).max())
    return Ur.real.astype(np.complex128)


def pair_tensor(U):
    """V_{(il),(jk)} = U_{i j l k}: the on-site tensor in the pair basis of the Hamiltonian (pairs (i, l) ordered
    i-major)."""
    n = U.shape[0]
    return np.ascontiguousarray(np.transpose(U, (0, 2, 1, 3)).reshape(n * n, n * n))


def kanamori_tensor(norb, U, J, Up=None):
    """The Kanamori form in the same basis: U_{iiii} = U, U_{ijij} = U' (direct), U_{ijji} = U_{iijj} = J, i != j;
    U' = U - 2J unless given."""
    up = U - 2.0 * J if Up is None else Up
    T = np.zeros((norb,) * 4, dtype=np.complex128)
    for i in range(norb):
        for j in range(norb):
            if i == j:
                T[i, i, i, i] = U
            else:
                T[i, j, i, j] = up
                T[i, j, j, i] = J
                T[i, i, j, j] = J
    return T


def kanamori_averages(U):
    """(U, U', J): averages over the shell of U_{aaaa}, U_{abab} and U_{abba} (a != b)."""
    n = U.shape[0]
    off = ~np.eye(n, dtype=bool)
    d = np.einsum("aaaa->a", U).real
    direct = np.einsum("abab->ab", U).real[off]
    exch = np.einsum("abba->ab", U).real[off]
    return float(d.mean()), float(direct.mean()), float(exch.mean())


def kanamori_from_slater(l, F):
    """Kanamori parameters (U, U', J) of the Slater shell: the averages of kanamori_averages."""
    return kanamori_averages(slater_tensor(l, F))


def slater_from_kanamori(l, U, J, ratios=None):
    """Slater integrals (F^0, F^2, .., F^2l) whose shell averages are the Kanamori U and J, with the higher
    integrals at fixed ratios to F^2 (F^4 / F^2 = 0.625 for d, F^4 / F^2 = 0.668 and F^6 / F^2 = 0.494 for f;
    common atomic values).  The averages are linear in the F^k, so F^0 and F^2 solve a 2 x 2 system."""
    if ratios is None:
        ratios = {0: [], 1: [], 2: [0.625], 3: [0.668, 0.494]}[l]
    if l == 0:
        return [float(U)]
    shape = [0.0, 1.0] + list(ratios)
    u0, _, j0 = kanamori_from_slater(l, [1.0])          # F^0 alone: U = F^0, J = 0
    u2, _, j2 = kanamori_from_slater(l, shape)          # F^2 = 1 with the ratios
    a = np.array([[u0, u2], [j0, j2]])
    f0, f2 = np.linalg.solve(a, np.array([U, J]))
    return [float(f0), float(f2)] + [float(f2 * r) for r in ratios]


def racah(F):
    """Racah parameters (A, B, C) of a d shell: F_0 = F^0, F_2 = F^2 / 49, F_4 = F^4 / 441,
    A = F_0 - 49 F_4, B = F_2 - 5 F_4, C = 35 F_4."""
    F = list(F) + [0.0] * (3 - len(F))
    f0, f2, f4 = F[0], F[1] / 49.0, F[2] / 441.0
    return f0 - 49.0 * f4, f2 - 5.0 * f4, 35.0 * f4


# ----------------------------------------------------------------------------
# Ohno and JTH
# ----------------------------------------------------------------------------

def ohno(U, d):
    """U / sqrt(1 + (U d / e^2)^2): the on-site value at d = 0, e^2 / d far away."""
    return U / math.sqrt(1.0 + (U * d / COULOMB_EV_ANGSTROM) ** 2)


def density_potential(kind, mesh, cell, positions, site_norb, onsite, cutoff, equivalent_u=None):
    """Non-local density-density interaction V_(ii),(jj)(R) between orbital i of site p (cell R) and orbital j of
    site q (cell 0), at distance d = |R + tau_p - tau_q| with 0 < d <= cutoff (Angstrom), on the periodic mesh.

    kind "ohno": V_ij = ohno((U_i + U_j) / 2, d), onsite[a] the on-site value of orbital a (numbered site by
    site); kind "jth": V_ij = ohno(equivalent_u, d) for every orbital pair (one shared on-site value).
    cell: lattice vectors as rows (2-D or 3-D, matching the mesh); positions: site positions (Angstrom).
    Returns V_R [N_b, N_b, *mesh] with only the density pairs (ii), (jj) set; the on-site (R = 0, p = q) block
    is left to the local interaction."""
    mesh = tuple(int(x) for x in mesh)
    dim = len(mesh)
    cell = np.asarray(cell, dtype=np.float64)
    assert cell.shape == (dim, dim)
    pos = [np.asarray(x, dtype=np.float64) for x in positions]
    n_o = int(sum(site_norb))
    offs = np.cumsum([0] + [n * n for n in site_norb])
    orb0 = np.cumsum([0] + list(site_norb))
    nb = int(offs[-1])
    V = np.zeros((nb, nb) + mesh, dtype=np.complex128)
    lengths = np.linalg.norm(cell, axis=1)
    reach = [int(math.ceil(cutoff / max(L, 1e-12))) + 2 for L in lengths]
    import itertools
    for p, npp in enumerate(site_norb):
        for q, nq in enumerate(site_norb):
            for R in itertools.product(*[range(-r, r + 1) for r in reach]):
                d = float(np.linalg.norm(np.asarray(R, dtype=np.float64) @ cell + pos[p] - pos[q]))
                if not (1e-9 < d <= cutoff * (1.0 + 1e-12)):
                    continue
                idx = tuple(int(R[a]) % mesh[a] for a in range(dim))
                for i in range(npp):
                    for j in range(nq):
                        if kind == "ohno":
                            u = 0.5 * (onsite[orb0[p] + i] + onsite[orb0[q] + j])
                        elif kind == "jth":
                            u = equivalent_u
                        else:
                            raise ValueError(kind)
                        V[(offs[p] + i * npp + i, offs[q] + j * nq + j) + idx] += ohno(u, d)
    assert n_o == orb0[-1]
    return V
