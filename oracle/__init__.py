"""Plain FP64 CPU oracle for the THC-MPO H|psi> method (arXiv 2409.12708).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only ``tests/``, the smoke check
in ``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` use it.
It shares no code with the HIP library (``paper_2409_12708_amd``) and never
imports it; the only module both sides read is ``synth`` (seeded inputs).

Every function follows a passage of the paper, cited by section / equation /
algorithm / appendix, and is written for a reader to check by eye: library
primitives (numpy matmul, ``numpy.linalg.qr``, ``svd``, ``eigh``) are used as
steps, with no blocking or fusion beyond what the paper states.

Modules
-------
fermion      Jordan-Wigner operators and dense Fock-space Hamiltonians (eq. 1).
thc          THC reconstruction (eq. thc), spin-site coefficients, kinetic
             spectral split (App. D).
mps          MPS primitives: layer apply (eq. elementary_MPO + App. C),
             QR/SVD compression (Fig. 3), direct sum, overlap.
hamiltonian  Algorithm 1 (sequential sum) and the pairwise reduction tree
             (Sec. 4.5, Fig. 11) for H = T + V.
lanczos      Global Krylov (Lanczos) step with Gram-Schmidt (Sec. 2.2).
evolution    Krylov time evolution exp(-i delta H~) of a complex state held as
             a pair of real MPS (Sec. 2.2, App. A).
gradient     Energy gradient with respect to the THC factors (Sec. 2.3).
hf           Closed-form Hartree-Fock energy of eq. 1 for a determinant.
blocksparse  Layers, compression, direct sum and the compressed H|psi> for MPS
             stored block-sparse in the abelian quantum numbers (N, 2 S_z)
             (Sec. 4.1).

Parity status: every function is pinned by
a ``-m "not gpu"`` test against a dense definition, a closed form or an
invariant, except the *truncated* H|psi> at bond dimensions where the exact
state cannot be formed densely: "parity unpinned" beyond the untruncated
regime and the compression invariants (Eckart-Young per bond, idempotence,
left-canonical output) that are checked at every size.
"""
