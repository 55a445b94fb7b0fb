"""FP64 CPU oracle for the RKL2 conduction super-step (serial by default;
the cell loops can run on several threads with the same result bits).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product path never does.
"""
from .oracle import (  # noqa: F401
    Grid, ghost_shape, build, load, set_threads, threads, mc, stages, coeffs, dt_par, flux_div, face_flux, rkl2_fixed, superstep, subcycle,
    stages_rkl1, rkl1_fixed, superstep_rkl1, aag_gain, aag_stages, aag_taus, aag_fixed, aag_superstep,
)
