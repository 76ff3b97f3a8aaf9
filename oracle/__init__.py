"""CPU oracle for the PQMC field-update sweep -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct float64 (complex128 for U < 0) NumPy
implementation of what the GPU path computes, written from the paper
(Du & He, arXiv:2506.09611) section by section.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does, and it shares no code with the HIP library (the only shared
module is `synth`, the seeded input generator).

Modules
  philox  -- Philox4x64-10 counter-based generator (Salmon et al., SC'11).
  pqmc    -- the walker: propagation, QR stabilisation, local / delayed /
             block force-bias updates, Green's function.
  brute   -- from-scratch configuration weights and Green's functions used
             to pin `pqmc` (definition of W(X), Eq. (9); G, Eq. (12)).
  soc     -- the spin-orbit coupled (Rashba) Hubbard walker: one 2N-dimensional
             complex sector, spin-s^y decoupling, rank-two local and delayed
             updates (Appendix A), with its brute-force weight and G.
  observables -- energy and double occupancy of the standard Hubbard model
             from G (Eq. (1), mixed estimate), for the precision-form error
             statements.
"""
