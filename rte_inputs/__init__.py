"""Seeded synthetic inputs for the pseudospectral P_N transport solver.

This module produces data only: optical maps (mu_a, mu_s, g), initial
radiance moments, source moments and detector positions, all as float64
NumPy arrays in the layout both solvers take:

* scalar maps: ``[z][y][x]`` (x fastest), shape ``(n, n, n)``;
* moment fields: ``[a][z][y][x]`` with ``a = l*l + l + m`` in the real
  spherical-harmonic basis, shape ``((N+1)**2, n, n, n)``;
* voxel indices: linear ``(z*n + y)*n + x`` as int64.

It holds none of the method's arithmetic (no transforms of the solution,
no coupling coefficients, no potentials, no boundary layer profile). The
oracle and the GPU path each compute those themselves from these inputs.
"""
from .phantoms import (  # noqa: F401
    Workload,
    collimated_slab_source,
    delta_ic,
    fourier_mode_ic,
    gaussian_ic,
    homogeneous_maps,
    lognormal_maps,
    outer_layer_detectors,
    sphere_maps,
    workload,
    WORKLOADS,
    RequestSpec,
    serving_requests,
)
