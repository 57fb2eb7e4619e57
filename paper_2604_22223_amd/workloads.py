"""Seeded synthetic lattice models (inputs only).

This module builds the inputs of a GW calculation -- the one-body Hamiltonian
H0(R) and the pair interaction V(R) on a periodic mesh -- for the model
families of the paper (graphene with on-site and Ohno-type interactions,
validation section; the degenerate five-orbital extended Hund-Hubbard model,
benchmark section) and for the seeded variants the benchmark uses.  It holds
none of the method's arithmetic: no transforms, no Dyson solves, no bubble.
Both the HIP path and the test oracle consume its arrays.

Array conventions
-----------------
* ``H_R[a, b, R1, R2]`` is the matrix element of H0 between orbital a in cell
  R = R1 a1 + R2 a2 and orbital b in cell 0 (eV), indices taken mod the mesh;
  on a 3-D mesh ``H_R[a, b, R1, R2, R3]`` with R = R1 a1 + R2 a2 + R3 a3.
* ``V_R[alpha, beta, R1, R2]`` is the interaction between pair alpha = (p; i, l)
  in cell R and pair beta = (q; j, k) in cell 0, i.e. V_{ijkl}^{pq}(R) of the
  paper's Hamiltonian with c+_i c_l at p and c+_j c_k at q.  Pairs are ordered
  site-major, then i, then l.
"""
import math

import numpy as np

#: Coulomb constant e^2 / (4 pi eps0) in eV * Angstrom (Ohno potential scale).
COULOMB_EV_ANGSTROM = 14.397
#: Carbon-carbon distance in graphene (Angstrom); the paper gives no geometry.
GRAPHENE_ACC = 1.42


def pair_count(site_norb):
    return int(sum(n * n for n in site_norb))


def _kanamori_block(norb, U, J):
    """On-site rotationally invariant Kanamori tensor in the pair basis.

    U' = U - 2J; V_(ii),(ii) = U; V_(ii),(jj) = U'; V_(ij),(ji) = J (exchange,
    spin flip); V_(ij),(ij) = J (pair hopping), i != j.
    """
    nb = norb * norb
    v = np.zeros((nb, nb), dtype=np.complex128)
    up = U - 2.0 * J
    for i in range(norb):
        for j in range(norb):
            a_ii = i * norb + i
            a_jj = j * norb + j
            if i == j:
                v[a_ii, a_ii] = U
            else:
                v[a_ii, a_jj] = up
                v[i * norb + j, j * norb + i] = J
                v[i * norb + j, i * norb + j] = J
    return v


def _hopping_bandwidth(hops, norb, n):
    """max_k eps_max - min_k eps_min of H0(k) = sum_R t(R) e^{-ik.R} on an n x n mesh."""
    ks = 2.0 * np.pi * np.arange(n) / n
    lo, hi = np.inf, -np.inf
    for k1 in ks:
        for k2 in ks:
            h = np.zeros((norb, norb), dtype=np.complex128)
            for (r1, r2), t in hops.items():
                h += t * np.exp(-1j * (k1 * r1 + k2 * r2))
            ev = np.linalg.eigvalsh(0.5 * (h + h.conj().T))
            lo = min(lo, ev[0])
            hi = max(hi, ev[-1])
    return hi - lo


def five_orbital(n=24, seed=22223, bandwidth=4.0, U=4.0, J=0.7, Vnn=1.0,
                 beta=50.0, omega_max=25.0, eps=1e-10, n_target=6.0,
                 norb=5, scale_mesh=24, slater_F=None):
    """Extended Hund-Hubbard model on a square lattice, one site, ``norb`` orbitals.

    Hopping: i.i.d. complex Gaussian norb x norb matrices on the bonds
    x, y, x+y, x-y (seeded), t(-R) = t(R)^dagger, no on-site term, scaled so
    that the band width over a ``scale_mesh`` x ``scale_mesh`` mesh equals
    ``bandwidth``.  Interaction: on-site Kanamori (U, J), or with
    ``slater_F`` = (F^0, F^2, F^4) the full Slater tensor of a d shell in the
    real-harmonic basis (norb = 5; U and J are then ignored), plus a
    nearest-neighbour density-density V_(ii),(jj)(+-x, +-y) = Vnn.
    """
    rng = np.random.default_rng(seed)
    hops = {}
    for r in [(1, 0), (0, 1), (1, 1), (1, -1)]:
        t = (rng.standard_normal((norb, norb)) + 1j * rng.standard_normal((norb, norb))) / math.sqrt(2.0)
        hops[r] = t
        hops[(-r[0], -r[1])] = t.conj().T
    scale = bandwidth / _hopping_bandwidth(hops, norb, scale_mesh)
    H_R = np.zeros((norb, norb, n, n), dtype=np.complex128)
    for (r1, r2), t in hops.items():
        H_R[:, :, r1 % n, r2 % n] += scale * t
    nb = norb * norb
    V_R = np.zeros((nb, nb, n, n), dtype=np.complex128)
    if slater_F is None:
        V_R[:, :, 0, 0] = _kanamori_block(norb, U, J)
    else:
        from . import interactions
        assert norb == 5, "the Slater tensor is that of a d shell"
        V_R[:, :, 0, 0] = interactions.pair_tensor(interactions.slater_tensor(2, slater_F))
        U, _, J = interactions.kanamori_from_slater(2, slater_F)
    for (r1, r2) in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        for i in range(norb):
            for j in range(norb):
                V_R[i * norb + i, j * norb + j, r1 % n, r2 % n] += Vnn
    return {"name": "five_orbital_%dx%d" % (n, n), "mesh": (n, n), "site_norb": [norb],
            "H_R": H_R, "V_R": V_R, "beta": float(beta), "omega_max": float(omega_max),
            "eps": float(eps), "n_target": float(n_target), "seed": seed,
            "interaction": {"U": float(U), "J": float(J), "V_nn": float(Vnn)}}


def graphene(n=12, t=-2.7, U=3.0, ohno=False, beta=10.0, omega_max=100.0, eps=1e-8,
             n_target=2.0, shells=5):
    """Graphene honeycomb, sites A and B with one p_z orbital each.

    Geometry: a = sqrt(3) a_cc, a1 = a (1, 0), a2 = a (1/2, sqrt(3)/2),
    tau_A = 0, tau_B = (a1 + a2) / 3.  Nearest-neighbour hopping t on the
    three A-B bonds.  Interaction: on-site U, and with ``ohno`` the Ohno
    potential V(d) = U / sqrt(1 + (U d / 14.397 eV A)^2) between sites at
    distance d up to the ``shells``-th neighbour shell.
    """
    acc = GRAPHENE_ACC
    a = math.sqrt(3.0) * acc
    a1 = np.array([a, 0.0])
    a2 = np.array([0.5 * a, 0.5 * math.sqrt(3.0) * a])
    tau = [np.zeros(2), (a1 + a2) / 3.0]
    H_R = np.zeros((2, 2, n, n), dtype=np.complex128)
    for (r1, r2) in [(0, 0), (-1, 0), (0, -1)]:
        H_R[0, 1, r1 % n, r2 % n] += t
        H_R[1, 0, (-r1) % n, (-r2) % n] += t
    V_R = np.zeros((2, 2, n, n), dtype=np.complex128)
    V_R[0, 0, 0, 0] = U
    V_R[1, 1, 0, 0] = U
    if ohno:
        shell_d = acc * np.array([1.0, math.sqrt(3.0), 2.0, math.sqrt(7.0), 3.0])[:shells]
        dmax = shell_d[-1] * (1.0 + 1e-9)
        reach = int(math.ceil(dmax / a)) + 2
        for p in range(2):
            for q in range(2):
                for r1 in range(-reach, reach + 1):
                    for r2 in range(-reach, reach + 1):
                        d = np.linalg.norm(r1 * a1 + r2 * a2 + tau[p] - tau[q])
                        if 1e-9 < d <= dmax:
                            V_R[p, q, r1 % n, r2 % n] += U / math.sqrt(1.0 + (U * d / COULOMB_EV_ANGSTROM) ** 2)
    name = "graphene_%s_%dx%d" % ("ohno" if ohno else "onsite", n, n)
    return {"name": name, "mesh": (n, n), "site_norb": [1, 1], "H_R": H_R, "V_R": V_R,
            "beta": float(beta), "omega_max": float(omega_max), "eps": float(eps),
            "n_target": float(n_target)}


def local_model(mesh, site_norb, levels, V_local, beta, omega_max, eps, n_target=None):
    """Flat-band (atomic-limit) model: no hopping, on-site levels and interaction (2-D or 3-D mesh)."""
    mesh = tuple(int(x) for x in mesh)
    r0 = (0,) * len(mesh)
    n_o = int(sum(site_norb))
    H_R = np.zeros((n_o, n_o) + mesh, dtype=np.complex128)
    H_R[(slice(None), slice(None)) + r0] = np.diag(np.asarray(levels, dtype=np.float64))
    nb = pair_count(site_norb)
    V_R = np.zeros((nb, nb) + mesh, dtype=np.complex128)
    V_R[(slice(None), slice(None)) + r0] = V_local
    return {"name": "local", "mesh": mesh, "site_norb": list(site_norb), "H_R": H_R,
            "V_R": V_R, "beta": float(beta), "omega_max": float(omega_max), "eps": float(eps),
            "n_target": n_target}


def kanamori(norb, U, J):
    """The on-site Kanamori pair tensor for one site with ``norb`` orbitals."""
    return _kanamori_block(norb, U, J)


def random_model(mesh, site_norb, seed, bandwidth=3.0, U=2.0, J=0.3, Vnn=0.4,
                 beta=10.0, omega_max=20.0, eps=1e-8, n_target=None):
    """Small seeded model with every site coupled, for parity tests.

    Random complex hoppings between all orbitals on the bonds x, y, x+y
    (and their Hermitian partners), random on-site levels, Kanamori on every
    site, and density-density V between every site pair on the x, y bonds.
    """
    rng = np.random.default_rng(seed)
    n1, n2 = mesh
    n_o = int(sum(site_norb))
    hops = {}
    onsite = rng.standard_normal((n_o, n_o)) + 1j * rng.standard_normal((n_o, n_o))
    hops[(0, 0)] = 0.25 * (onsite + onsite.conj().T)
    for r in [(1, 0), (0, 1), (1, 1)]:
        t = (rng.standard_normal((n_o, n_o)) + 1j * rng.standard_normal((n_o, n_o))) / math.sqrt(2.0)
        hops[r] = t
        hops[(-r[0], -r[1])] = t.conj().T
    scale = bandwidth / max(_hopping_bandwidth(hops, n_o, 8), 1e-12)
    H_R = np.zeros((n_o, n_o, n1, n2), dtype=np.complex128)
    for (r1, r2), t in hops.items():
        H_R[:, :, r1 % n1, r2 % n2] += scale * t
    nb = pair_count(site_norb)
    V_R = np.zeros((nb, nb, n1, n2), dtype=np.complex128)
    offs = np.cumsum([0] + [n * n for n in site_norb])
    for p, n in enumerate(site_norb):
        V_R[offs[p]:offs[p + 1], offs[p]:offs[p + 1], 0, 0] = _kanamori_block(n, U, J)
    for p, npp in enumerate(site_norb):
        for q, nq in enumerate(site_norb):
            for (r1, r2) in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
                for i in range(npp):
                    for j in range(nq):
                        V_R[offs[p] + i * npp + i, offs[q] + j * nq + j, r1 % n1, r2 % n2] += Vnn
    if n_target is None:
        n_target = float(n_o)
    return {"name": "random_%s_%dx%d_s%d" % ("-".join(map(str, site_norb)), n1, n2, seed),
            "mesh": (n1, n2), "site_norb": list(site_norb), "H_R": H_R, "V_R": V_R,
            "beta": float(beta), "omega_max": float(omega_max), "eps": float(eps),
            "n_target": float(n_target)}


def _bandwidth_nd(hops, norb, n, d):
    """max_k eps_max - min_k eps_min of H0(k) = sum_R t(R) e^{-ik.R} on an n^d mesh."""
    ks = np.stack(np.meshgrid(*([2.0 * np.pi * np.arange(n) / n] * d), indexing="ij"), axis=-1).reshape(-1, d)
    h = np.zeros((len(ks), norb, norb), dtype=np.complex128)
    for r, t in hops.items():
        h += np.exp(-1j * (ks @ np.asarray(r, dtype=np.float64)))[:, None, None] * t
    ev = np.linalg.eigvalsh(0.5 * (h + np.conj(np.swapaxes(h, -1, -2))))
    return float(ev.max() - ev.min())


def cubic_five_orbital(n=8, t=1.0, U=1.0, J=0.1, Vnn=0.2, beta=100.0, omega_max=25.0, eps=1e-10,
                       n_target=None, norb=5):
    """Degenerate ``norb``-orbital extended Hund-Hubbard model on a simple cubic lattice.

    The benchmark model of the paper's performance section: orbital-diagonal
    nearest-neighbour hopping -t on the six bonds +-x, +-y, +-z (so that
    H0(k) = -2 t (cos k1 + cos k2 + cos k3) I), on-site Kanamori (U, J) and a
    nearest-neighbour density-density V_(ii),(jj) = Vnn on the same bonds,
    on an n x n x n mesh.  The paper states no filling; the default is half
    filling (one electron per spin-orbital pair, n_target = norb).
    """
    if n_target is None:
        n_target = float(norb)
    H_R = np.zeros((norb, norb, n, n, n), dtype=np.complex128)
    nb = norb * norb
    V_R = np.zeros((nb, nb, n, n, n), dtype=np.complex128)
    V_R[:, :, 0, 0, 0] = _kanamori_block(norb, U, J)
    for r in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
        idx = tuple(x % n for x in r)
        for i in range(norb):
            H_R[(i, i) + idx] += -t
            for j in range(norb):
                V_R[(i * norb + i, j * norb + j) + idx] += Vnn
    return {"name": "cubic_five_orbital_%d^3" % n, "mesh": (n, n, n), "site_norb": [norb],
            "H_R": H_R, "V_R": V_R, "beta": float(beta), "omega_max": float(omega_max),
            "eps": float(eps), "n_target": float(n_target)}


def random_model_3d(mesh, site_norb, seed, bandwidth=3.0, U=2.0, J=0.3, Vnn=0.4,
                    beta=10.0, omega_max=20.0, eps=1e-8, n_target=None):
    """``random_model`` on a 3-D mesh: random complex hoppings between all
    orbitals on the bonds x, y, z, x+y, y+z (and their Hermitian partners),
    random on-site levels, Kanamori on every site, density-density V between
    every site pair on the six bonds +-x, +-y, +-z."""
    rng = np.random.default_rng(seed)
    mesh = tuple(int(x) for x in mesh)
    n_o = int(sum(site_norb))
    hops = {}
    onsite = rng.standard_normal((n_o, n_o)) + 1j * rng.standard_normal((n_o, n_o))
    hops[(0, 0, 0)] = 0.25 * (onsite + onsite.conj().T)
    for r in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, 1)]:
        t = (rng.standard_normal((n_o, n_o)) + 1j * rng.standard_normal((n_o, n_o))) / math.sqrt(2.0)
        hops[r] = t
        hops[tuple(-x for x in r)] = t.conj().T
    scale = bandwidth / max(_bandwidth_nd(hops, n_o, 4, 3), 1e-12)
    H_R = np.zeros((n_o, n_o) + mesh, dtype=np.complex128)
    for r, t in hops.items():
        H_R[(slice(None), slice(None)) + tuple(x % m for x, m in zip(r, mesh))] += scale * t
    nb = pair_count(site_norb)
    V_R = np.zeros((nb, nb) + mesh, dtype=np.complex128)
    offs = np.cumsum([0] + [n * n for n in site_norb])
    for p, n in enumerate(site_norb):
        V_R[offs[p]:offs[p + 1], offs[p]:offs[p + 1], 0, 0, 0] = _kanamori_block(n, U, J)
    for p, npp in enumerate(site_norb):
        for q, nq in enumerate(site_norb):
            for r in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
                idx = tuple(x % m for x, m in zip(r, mesh))
                for i in range(npp):
                    for j in range(nq):
                        V_R[(offs[p] + i * npp + i, offs[q] + j * nq + j) + idx] += Vnn
    if n_target is None:
        n_target = float(n_o)
    return {"name": "random3d_%s_%dx%dx%d_s%d" % (("-".join(map(str, site_norb)),) + mesh + (seed,)),
            "mesh": mesh, "site_norb": list(site_norb), "H_R": H_R, "V_R": V_R,
            "beta": float(beta), "omega_max": float(omega_max), "eps": float(eps),
            "n_target": float(n_target)}


def batch_sweep(count=64, seed=22223):
    """Seeded instances of uneven size for the batched runs.

    Instance i draws, from default_rng(seed + i): orbitals n_o in 1..5; mesh
    side in {12, 16, 18, 20, 24, 30, 32, 36, 40, 48}; beta log-uniform in
    [10, 100] /eV; U uniform in [1, 6] eV, J = U x U[0, 0.2] (0 for one
    orbital), V_nn = U x U[0, 0.3]; band width uniform in [2, 6] eV; filling
    per spin-orbital uniform in [0.2, 0.8]; omega_max = 25 eV, eps = 1e-10.
    The hopping of instance i is the five-orbital construction with seed
    seed + i.
    """
    sides = [12, 16, 18, 20, 24, 30, 32, 36, 40, 48]
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        norb = int(rng.integers(1, 6))
        n = int(sides[int(rng.integers(0, len(sides)))])
        beta = float(10.0 ** rng.uniform(1.0, 2.0))
        U = float(rng.uniform(1.0, 6.0))
        J = float(U * rng.uniform(0.0, 0.2)) if norb > 1 else 0.0
        Vnn = float(U * rng.uniform(0.0, 0.3))
        bw = float(rng.uniform(2.0, 6.0))
        fill = float(rng.uniform(0.2, 0.8))
        w = five_orbital(n=n, seed=seed + i, bandwidth=bw, U=U, J=J, Vnn=Vnn, beta=beta, omega_max=25.0,
                         eps=1e-10, n_target=2.0 * norb * fill, norb=norb, scale_mesh=n)
        w["name"] = "sweep_%02d_o%d_%dx%d" % (i, norb, n, n)
        out.append(w)
    return out


# The benchmark workloads, by name.
def workload(name):
    if name == "graphene_g0w0_12":
        return graphene(n=12, U=3.0, ohno=False, beta=10.0, omega_max=100.0, eps=1e-8)
    if name == "graphene_ohno_36":
        return graphene(n=36, U=3.0, ohno=True, beta=40.0, omega_max=100.0, eps=1e-10)
    # the five-orbital workloads carry the interaction of the paper's five-orbital benchmark (U = 1, J = 0.1,
    # V = 0.2 eV), not the model's stronger defaults
    if name == "five_orbital_24":
        return five_orbital(n=24, U=1.0, J=0.1, Vnn=0.2, beta=50.0, omega_max=25.0, eps=1e-10)
    if name == "five_orbital_48":
        return five_orbital(n=48, U=1.0, J=0.1, Vnn=0.2, beta=100.0, omega_max=25.0, eps=1e-10)
    if name == "cubic_five_orbital_8":
        return cubic_five_orbital(n=8, t=1.0, U=1.0, J=0.1, Vnn=0.2, beta=100.0, omega_max=25.0, eps=1e-10)
    raise KeyError(name)
