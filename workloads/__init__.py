"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds only input generation: grids, potentials, initial data and
the time functions f_r(t), A(t) that define a problem. None of the solver's
arithmetic lives here.
"""
from .synth import (  # noqa: F401
    Problem,
    periodic_grid,
    free_grid,
    periodic_1d_256_problem,
    periodic_2d_512_problem,
    free_2d_256_problem,
    free_3d_32_problem,
    periodic_2d_1024_problem,
    periodic_3d_128_problem,
    sampled_potential_problem,
    sampled_2d_512_problem,
    batch_64_problems,
    periodic_problem_from_seed,
    free_problem_from_seed,
    moving_well_problem,
    gaussian_well_ground_state,
    ionization_1d_problem,
    gaussian_well_ground_state_2d,
    periodic_well_ground_state,
    ionization_2d_problem,
    wavepacket,
    example2_long_time_problem,
)
