"""Seeded synthetic single-photon lidar workloads.

This package only draws inputs: photon times of arrival (CSR, int16) or
per-bin photon-count histograms (fp16), the instrument response that produced
them, and the ground-truth depth. It holds none of the reconstruction
method's arithmetic, and both the CPU oracle and the GPU path consume what it
returns.
"""
from .scenes import (  # noqa: F401
    Workload, CsrFrame, gaussian_irf, default_nu, cross_nu,
    csr_frame_from_counts, config1, config2, config3, config4, config5,
    random_csr, tiny_workload,
)
