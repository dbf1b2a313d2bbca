"""Plain FP64 CPU oracle for the pseudospectral P_N transport time step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it. It shares no code with the HIP
library (different basis, different transform, different time-stepping
form); the seeded input generators in ``rte_inputs`` are the only thing
both sides read.

Parity status: every function here is pinned by a CPU test against a fact
that does not come from this package (exact quadrature of spherical
harmonics, Gauss-Legendre nodes, closed-form P_1 dispersion, matrix
exponentials, conservation laws, exact spectral derivatives). Physical
accuracy against the true transport equation or the paper's Monte-Carlo
figures is "parity unpinned": the figure data are not available.
"""
from .pn import (  # noqa: F401
    alpha, beta, sh_index, sh_lm, coupling_matrices, real_basis_transform,
    wavenumbers, pml_depth, pml_profile, potentials, operator, rk4_step,
    solve, to_complex_basis, to_real_basis, mode_matrix, rk4_poly,
    hg_phase, hg_legendre_moments, real_coupling, operator_transpose,
    adjoint_gradient, full_moments, euler_step, steady_state, expo_advance,
    source_profile, source_moments, rk4_source_step,
)
