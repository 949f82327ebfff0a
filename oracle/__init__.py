"""FP64 CPU oracle for the local-Hamiltonian path of linear-scaling
Daubechies-wavelet DFT (Mohr et al., arXiv:1401.7441).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference against which the GPU library is checked.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (the HIP library and its Python binding) never does, and the two
share no code: not the filter tables, not the helpers, not the index maps.

Modules
-------
filters      Least-asymmetric Daubechies-16 filters, scaling-function moments,
             magic filter and kinetic filter, derived in mpmath from the
             mathematics (paper Sec. II.B; the operators are defined by
             reference to the standard BigDFT construction, Sec. III.B).
wavelet      1D and 3D synthesis / analysis / magic filter / kinetic operators
             on dense boxes (paper Sec. III.B, Eq. (Phi)).
locreg       Localization regions and segment lists (paper Sec. III,
             the projector L^(alpha) and the enlarged L'^(beta)).
hamiltonian  Localized application of the local Hamiltonian to one support
             function, H|phi> = L' H L |phi> (paper Sec. III.B).
sparse       Sparsity pattern and values of the overlap and Hamiltonian
             matrices S_ab = <phi_a|phi_b>, H_ab = <phi_a|H|phi_b>
             (paper Sec. II.A, below Eq. (band_structure_energy)).
update       The support-function update step with the localized gradient
             (paper Sec. III.A and IV.A), fixed step length.
precond      Kinetic + confinement preconditioning of the gradient (paper
             Sec. IV.A, Eq. (precond)), conjugate-gradient steps.
density      Fine-grid values of the support functions and the density
             rho = sum_ab phi_a K^ab phi_b (paper Sec. II, Eq. (density)).
foe          Density kernel by the Fermi operator expansion (paper Sec. IV.B,
             App. B): Chebyshev recursion on truncated sparse matrices.

Parity status: every function here is pinned by a check that does not reuse
its own formula (closed forms, invariants, brute force); see the tests marked
``not gpu``.  No function is "parity unpinned".
"""
