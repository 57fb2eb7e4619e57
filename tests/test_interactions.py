"""Pins of the interaction generators (Slater, Kanamori, Ohno, JTH; the V class
and the interaction paragraph after Eq. eq:many-body-hamiltonian).  CPU only.

Expected values come from outside the generators: the Racah-parameter table of
the d shell (A + 4B + 3C on every orbital, exchange 3B + C, 4B + C, B + C or C
by orbital pair), the p-shell closed forms, invariance of the Coulomb tensor
of a full shell under a random rotation (its real-harmonic representation
built from the orbitals' polynomials, independently of the Gaunt
coefficients), and the graphene Ohno potential written out in workloads.
"""
import math

import numpy as np
import pytest

from paper_2604_22223_amd import interactions as it
from paper_2604_22223_amd import workloads as wl

D_NAMES = ["xy", "yz", "z2", "xz", "x2y2"]


@pytest.mark.parametrize("F", [[4.0, 7.5, 4.6875], [1.0, 3.0, 2.0], [0.0, 0.0, 5.0]])
def test_d_shell_racah_table(F):
    """Real d orbitals (xy, yz, z^2, xz, x^2 - y^2): U_aaaa = A + 4B + 3C; exchange J_ab = U_abba equals the pair
    hopping U_aabb and is 3B + C within t2g, 4B + C for (z^2, x^2 - y^2) and (xy, z^2), C for (xy, x^2 - y^2),
    B + C for (yz, z^2), (xz, z^2), 3B + C for (yz, x^2 - y^2), (xz, x^2 - y^2); direct U'_ab = U - 2 J_ab."""
    U = it.slater_tensor(2, F)
    A, B, C = it.racah(F)
    J = {("xy", "yz"): 3 * B + C, ("xy", "xz"): 3 * B + C, ("yz", "xz"): 3 * B + C,
         ("z2", "x2y2"): 4 * B + C, ("xy", "z2"): 4 * B + C, ("xy", "x2y2"): C,
         ("yz", "z2"): B + C, ("xz", "z2"): B + C, ("yz", "x2y2"): 3 * B + C, ("xz", "x2y2"): 3 * B + C}
    ix = {n: i for i, n in enumerate(D_NAMES)}
    u = A + 4 * B + 3 * C
    assert np.abs(np.einsum("aaaa->a", U) - u).max() < 1e-12
    for (a, b), jab in J.items():
        i, j = ix[a], ix[b]
        for val in (U[i, j, j, i], U[j, i, i, j], U[i, i, j, j], U[j, j, i, i]):
            assert abs(val - jab) < 1e-12, (a, b, val, jab)
        assert abs(U[i, j, i, j] - (u - 2 * jab)) < 1e-12


def test_p_shell_closed_forms():
    """p shell: U = F0 + 4/25 F2, U' = F0 - 2/25 F2, J = 3/25 F2 for every pair of real p orbitals."""
    F0, F2 = 2.0, 5.0
    U = it.slater_tensor(1, [F0, F2])
    off = ~np.eye(3, dtype=bool)
    assert np.abs(np.einsum("aaaa->a", U) - (F0 + 4 * F2 / 25)).max() < 1e-13
    assert np.abs(np.einsum("abab->ab", U)[off] - (F0 - 2 * F2 / 25)).max() < 1e-13
    assert np.abs(np.einsum("abba->ab", U)[off] - 3 * F2 / 25).max() < 1e-13
    assert np.abs(np.einsum("aabb->ab", U)[off] - 3 * F2 / 25).max() < 1e-13


def test_monopole_only_is_direct_coulomb():
    for l in (1, 2, 3):
        n = 2 * l + 1
        U = it.slater_tensor(l, [1.7])
        ref = 1.7 * np.einsum("ac,bd->abcd", np.eye(n), np.eye(n))
        assert np.abs(U - ref).max() < 1e-13


@pytest.mark.parametrize("l,F", [(2, [4.0, 7.5, 4.6875]), (3, [3.0, 6.0, 4.0, 3.0])])
def test_tensor_symmetries(l, F):
    """<ab|v|cd> = <ba|v|dc> (the two electrons), = <cd|v|ab>* (Hermitian); m1 + m2 = m3 + m4 in the complex
    basis."""
    for basis in ("complex", "real"):
        U = it.slater_tensor(l, F, basis=basis)
        assert np.abs(U - np.transpose(U, (1, 0, 3, 2))).max() < 1e-12
        assert np.abs(U - np.conj(np.transpose(U, (2, 3, 0, 1)))).max() < 1e-12
    Uc = it.slater_tensor(l, F, basis="complex")
    n = 2 * l + 1
    m = np.arange(n)
    bad = (m[:, None, None, None] + m[None, :, None, None]) != (m[None, None, :, None] + m[None, None, None, :])
    assert np.abs(Uc[bad]).max() == 0.0


def _d_polys(x):
    """Real d orbitals as quadratic polynomials with a common normalisation (the real harmonics up to one
    constant): xy, yz, (3z^2 - r^2) / (2 sqrt 3), xz, (x^2 - y^2) / 2."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    r2 = X * X + Y * Y + Z * Z
    return np.stack([X * Y, Y * Z, (3 * Z * Z - r2) / (2 * math.sqrt(3.0)), X * Z, 0.5 * (X * X - Y * Y)], -1)


def test_d_shell_rotation_invariance():
    """The Coulomb tensor of a full d shell is invariant under every rotation O: with D the 5 x 5 representation
    of O on the real d orbitals (from the polynomials, p_a(O^T x) = sum_b D_ab p_b(x)), U = D D U D^T D^T."""
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    O = q * np.sign(np.linalg.det(q))
    pts = rng.standard_normal((40, 3))
    P = _d_polys(pts)
    PO = _d_polys(pts @ O)            # p_a(O^T x) for each sample x (rows of pts are x^T)
    D = np.linalg.lstsq(P, PO, rcond=None)[0].T
    assert np.abs(D @ D.T - np.eye(5)).max() < 1e-12
    U = it.slater_tensor(2, [4.0, 7.5, 4.6875]).real
    Ur = np.einsum("ai,bj,ck,dl,ijkl->abcd", D, D, D, D, U)
    assert np.abs(Ur - U).max() < 1e-12
    # a planted error fails: dropping the F^4 Gaunt term's sign on one element breaks the invariance
    V = U.copy()
    V[0, 1, 1, 0] += 0.05
    V[1, 0, 0, 1] += 0.05
    assert np.abs(np.einsum("ai,bj,ck,dl,ijkl->abcd", D, D, D, D, V) - V).max() > 1e-3


def test_kanamori_slater_round_trip_and_t2g():
    F = [4.0, 7.5, 4.6875]
    U, Up, J = it.kanamori_from_slater(2, F)
    assert abs(Up - (U - 2 * J)) < 1e-12          # pairwise U' = U - 2 J_ab holds for the real d orbitals
    Fb = it.slater_from_kanamori(2, U, J)
    assert np.allclose(Fb, F, rtol=0, atol=1e-12)
    # the Kanamori averages of the slater tensor built from (U, J) are (U, U - 2J, J)
    for (u, j) in ((3.0, 0.5), (1.0, 0.1)):
        Fk = it.slater_from_kanamori(2, u, j)
        uu, up, jj = it.kanamori_from_slater(2, Fk)
        assert abs(uu - u) < 1e-12 and abs(jj - j) < 1e-12 and abs(up - (u - 2 * j)) < 1e-12


def test_pair_tensor_matches_kanamori_block():
    """pair_tensor maps <ij|v|lk> to V_(il),(jk): the Kanamori tensor lands on the Kanamori pair block of the
    model generators; a monopole-only d shell is the Kanamori block with J = 0."""
    for norb, U, J in ((3, 2.0, 0.4), (5, 4.0, 0.7)):
        v = it.pair_tensor(it.kanamori_tensor(norb, U, J))
        assert np.abs(v - wl.kanamori(norb, U, J)).max() == 0.0
    assert np.abs(it.pair_tensor(it.slater_tensor(2, [1.3])) - wl.kanamori(5, 1.3, 0.0)).max() < 1e-13


def test_ohno_reproduces_graphene_and_jth_limits():
    """density_potential("ohno") on the graphene geometry equals the graphene generator's V(R) off site; JTH with
    one orbital per site is Ohno; the Ohno function interpolates U at d = 0 and e^2 / d far away."""
    n, U = 12, 3.0
    w = wl.graphene(n=n, U=U, ohno=True, beta=10.0, omega_max=100.0, eps=1e-8)
    acc = wl.GRAPHENE_ACC
    a = math.sqrt(3.0) * acc
    cell = np.array([[a, 0.0], [0.5 * a, 0.5 * math.sqrt(3.0) * a]])
    pos = [np.zeros(2), (cell[0] + cell[1]) / 3.0]
    cut = 3.0 * acc
    v = it.density_potential("ohno", (n, n), cell, pos, [1, 1], [U, U], cut)
    ref = w["V_R"].copy()
    ref[0, 0, 0, 0] = ref[1, 1, 0, 0] = 0.0
    assert np.abs(v - ref).max() < 1e-14
    vj = it.density_potential("jth", (n, n), cell, pos, [1, 1], None, cut, equivalent_u=U)
    assert np.abs(vj - v).max() == 0.0
    assert abs(it.ohno(U, 0.0) - U) == 0.0
    d = 1e4
    assert abs(it.ohno(U, d) * d / it.COULOMB_EV_ANGSTROM - 1.0) < 1e-6


def test_jth_shares_one_value_across_orbitals():
    """Two sites with two orbitals of different on-site values: Ohno takes each pair's mean, JTH one value for
    all pairs."""
    cell = np.array([[3.0, 0.0], [0.0, 3.0]])
    pos = [np.zeros(2), np.array([1.5, 0.0])]
    onsite = [2.0, 4.0, 3.0, 5.0]
    vo = it.density_potential("ohno", (4, 4), cell, pos, [2, 2], onsite, 1.6)
    vj = it.density_potential("jth", (4, 4), cell, pos, [2, 2], None, 1.6, equivalent_u=3.5)
    # site 0 pairs (00), (11) are 0 and 3; site 1 pairs (00), (11) are 4 and 7; site 0 in cell R meets site 1 of
    # cell 0 at d = 1.5 for R = 0 and R = a1
    for (a, i), (b, j) in (((0, 0), (4, 2)), ((3, 1), (7, 3)), ((0, 0), (7, 3))):
        for R in ((0, 0), (1, 0)):
            assert abs(vo[(a, b) + R] - it.ohno(0.5 * (onsite[i] + onsite[j]), 1.5)) < 1e-15
            assert abs(vj[(a, b) + R] - it.ohno(3.5, 1.5)) < 1e-15
    assert np.count_nonzero(vj) == np.count_nonzero(vo) == 2 * 2 * 4   # site orders x bonds x orbital pairs
