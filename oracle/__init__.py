"""CPU oracle for the Lanczos ground-state method on two-species lattice models.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The library
(``paper_1511_00863_amd``) never imports it and shares no code with it.

Everything here is plain, slow and float64, written from the paper:

* ``basis``       -- per-spin occupation-bitstring basis (Sec. 2.1, Eq. 2)
* ``hopping``     -- per-spin hopping matrices by explicit operator application,
                     ELL export (Sec. 2.1, Fig. 2)
* ``hamiltonian`` -- H = H_up x I + I x H_dn + diag(U n_up n_dn) (Eq. 1, 3-5)
* ``fock``        -- brute force in the full Fock space from Jordan-Wigner
                     Kronecker products (tiny lattices)
* ``elements``    -- (H x) at selected basis states from the operator form of
                     Eq. 1, term by term, with no matrix (any sector size)
* ``observables`` -- occupation moments <n_a n_b> of a state (diagonal
                     observables in the occupation basis, Sec. 2.1)
* ``lanczos``     -- the Lanczos iteration in the paper's order (Alg. 1), the
                     lowest eigenvalue of T (Sec. 2.2), the two-pass ground state
* ``mlp``         -- float64 forward/backward/Adam of the start-vector network,
                     with optional bfloat16 rounding of matmul operands

Each function cites the passage it follows.  Readings of passages the paper
leaves open are listed in the module docstrings.  Parity status: every function
is pinned by ``tests/test_oracle_*.py`` against closed forms, brute force,
printed values or library routines of a different algorithm, except the trained
network's output, which is parity unpinned (training is not reproducible across
implementations; it is assessed through the energy it reaches).
"""
