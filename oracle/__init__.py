"""CPU oracle for the batched Henry / MLMC hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 NumPy/SciPy code written from the paper's problem statement
(density-driven flow, section 2.1; discretisation, section 2.3; MLMC, section 3).
It exists to check the HIP library: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
path; the two meet only through the seeded inputs in ``henry_inputs``.

Modules:
  kl       analytic Karhunen-Loeve eigenpairs of the exponential covariance
  henry    fields, discrete residual/Jacobian, Newton + sparse direct LU time loop, QoI
  mlmc     multilevel Monte Carlo estimator and optimal sample numbers (section 3)
  adjoint  discrete adjoint of the implicit-Euler/Newton solve (checked against FD)
"""
