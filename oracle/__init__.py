"""Plain FP64 CPU oracle for one GW iteration on a tight-binding lattice.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constant generators); the two
meet only through the seeded input generators, which hold none of the method's
arithmetic.

Modules
-------
dlr      discrete Lehmann representation: node selection and composite maps
         (method section, DLR paragraph after the bare Green's function; the
         construction follows Kaye, Chen & Parcollet, PRB 105, 235115 (2022)).
lattice  k <-> R transforms (Eq. eq:fourier-transform-kr) in the cell-periodic
         gauge.
gw       G0, bubble P, screened W, GW self-energy, Hartree/Fock, Dyson G with
         the chemical-potential bisection, the SCF loop (Fig. fig-self (b)).
hf       Hartree-Fock self-consistency (Fig. fig-self (a)): Fermi-function
         density of the static Hamiltonian, chemical potential, the loop.
quasiparticle  static self-energy, renormalisation Z(k) (Eq. eq-z-factor) and
         the quasiparticle Hamiltonian and bands
         (Eq. eq-quasi-particle-Hamiltonian).
mf       the same iteration on uniform Matsubara and imaginary-time grids
         (the conventional representation the performance section compares
         the DLR with).

Every function is written for readability against the paper, not speed.
"""
