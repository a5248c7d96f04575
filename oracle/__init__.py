"""Plain FP64 CPU oracle of the R3DSP per-frame hot path.

TEST INFRASTRUCTURE ONLY. This package is imported by the test-suite, by the
entry point's smoke check and by the benchmark's CPU-baseline leg, and by
nothing else: the product path (the HIP library and its Python binding)
never imports, calls or links it, and it imports nothing from the product.
It is deliberately slow and literal: each function follows one passage of the
paper (cited in its docstring) and is written so that it can be checked
against that passage by eye.
"""
from .r3d_oracle import (  # noqa: F401
    Model, State, validate, histogram, modified_irf, correlation, cost_from_histogram,
    cost_from_histogram_pirf, cost_from_photons, flat_component, prior_components, log_prior,
    posterior_moments, background_intensity, pi0_next, init_state, step, run,
    gaussian_irf_sigma, filter_loss, filter_loss_grad_fd, argmax_with_margin,
    min_divergence, msl_objective, msl_min_divergence, gauss_cost, gauss_min_divergence,
)
