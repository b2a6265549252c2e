"""Plain FP64 CPU oracle for the Chebyshev-filtered subspace iteration of the
real-space finite-difference Kohn-Sham method for extended systems
(Ghosh & Suryanarayana, "SPARC: Accurate and efficient finite-difference
formulation and parallel implementation of DFT: Extended systems").

THIS PACKAGE IS TEST INFRASTRUCTURE. It is the slow, obviously correct
reference that the HIP library is checked against. Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path (the C-ABI library and its Python binding) never does, and shares no code
with it.

Every function follows a passage of the paper (cited in its docstring) in the
paper's order and notation, using numpy in float64 / complex128.  Library
primitives (np.linalg.qr, np.linalg.eigh, np.fft) serve as single steps.

Modules
  fd       finite-difference weights, Bloch-phased shifts, H applied to a block
  cell     synthetic cell: local potential and Kleinman-Bylander projectors
  chefsi   Chebyshev filter (recurrence and direct), Rayleigh-Ritz, Lanczos
  scf      occupations, density, Poisson, Slater exchange, energy, SCF loop
  forces   atomic forces: local component, non-local component with the
           gradient on the orbitals, FD gradient
  bands    band structure at fixed potential (dense H(k)), density of states
  pseudocharge  pseudocharge electrostatics: truncation radius, pseudocharge and
           self energy, overlap correction, local and correction forces
  density_net  3-D convolutional network forward/backward for the initial density

Parity status: every function is pinned by a CPU test against closed forms,
invariants or brute force (tests/test_oracle_*.py), except the effect of the
learned initial density, which is "parity unpinned" (assessed only by the SCF
it seeds).
"""
