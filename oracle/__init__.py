"""FP64 CPU oracle for Kahler-Dirac multigrid on the staggered operator.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the HIP path; only the seeded input generators in ``synth`` serve both.

Pinned parts: D (free spectrum, symmetries, gauge covariance, free FFT solve),
B and B^-1 (the printed 2D block of Sec. 2.1, free unitarity), A (free circle,
gamma_5^{L/R} hermiticity), S (reconstruction against dense LU), P and A_hat
(P^dag P = 1, epsilon P = P sigma_3, P^dag (B^-1 D) P = sigma_3 A_hat^dag sigma_3,
nearest-neighbour sparsity), the MG solve (dense LU, CG-eo, FFT, gauge
covariance).  Parity unpinned: the relaxed near-null vector values (random by
construction; only their low Rayleigh quotient is checked).
"""
