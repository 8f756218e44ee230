"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds inputs only: THC factors X and core Z shaped like a
molecular two-electron-integral factorisation, the initial CP factors, and
the orbital energies / Laplace points and weights of the batched workload.  It holds
none of the CP-ALS arithmetic.  Every random number a CP-ALS run consumes
(the initial factors) or the warm-start network's training consumes
(initial weights, minibatch order) is drawn here and handed to both the
oracle and the GPU path as an input.
"""
from .thc import (make_thc, init_factors, init_factors_uniform, make_lt_system,
                  lt_points, lt_quadrature, LT_SYSTEMS, planted_diag_thc, make_df, mlp_init_params, minibatch_order)

__all__ = ["make_thc", "init_factors", "init_factors_uniform", "make_lt_system",
           "lt_points", "lt_quadrature", "LT_SYSTEMS", "make_df", "planted_diag_thc", "mlp_init_params", "minibatch_order"]
