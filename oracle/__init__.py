"""CPU FP64 oracle for the generalized Basic Scheme on lattice patterns.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only the tests, the smoke check
and the CPU-baseline leg of the benchmark use it.  It shares no code with
the HIP library (``paper_1605_05712_amd``); the only modules both sides use
are the seeded input generators in ``synth``.

Modules
-------
lattice       exact-integer patterns P(M), generating sets G(M^T), Smith
              normal form, determinantal divisors (Sec. 2.1-2.2).
dft           naive pattern DFT F(M) (eq. Fouriermatrix) and a fast route
              through the oracle's own Smith-normal-form ordering (Sec. 2.2).
elasticity    stiffness tensors, the Green operator Gamma^0 (Sec. 3.1),
              Algorithm 1 with the equilibrium residual, C_eff (Def. 3.1).
closed_forms  laminate (Sec. 4.1) and generalized Hashin structure (Sec. 4.2).
accelerated   conjugate gradients on the same Lippmann-Schwinger system (the
              accelerated schemes named in Sec. 1 and Sec. 6).
conductivity  the steady-state heat (conductivity) problem named in Sec. 3:
              scalar Green operator, Basic Scheme and CG, K_eff.

Readings of the paper where it is silent or garbled are listed in the
module docstrings where they are applied.
"""
