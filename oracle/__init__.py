"""CPU oracle for the tight-binding Schrodinger-Poisson hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  Every routine is a plain, slow FP64 (complex128 where
the Hamiltonian is complex) implementation of the definition it cites, with
no blocking, fusion or reordering beyond that definition.

Modules
-------
tb       lattice neighbours, Slater-Koster blocks built by rotation, on-site
         blocks (spin-orbit, dangling-bond passivation), Bloch phases,
         scalar CSR Hamiltonian and H.x.
lanczos  Lanczos with full (CGS2) reorthogonalisation, Ritz pairs, explicit
         residuals, Rayleigh-quotient refinement, converged-set selection.
poisson  finite-difference Poisson operator, FP64 conjugate gradients and a
         spectral (FFT x,y / DST z) exact solve.
scf      Fermi-Dirac charge with the Fermi level from neutrality and the
         self-consistent loop with linear mixing.
conv     direct 3-D convolution network (forward, backward, Adam).
"""
