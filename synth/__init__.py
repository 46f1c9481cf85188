"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module holds no arithmetic of the reconstruction method: it draws the
scenes (ground-truth images), the binary sensing masks and the workload
parameter sets.  Measurements y = Phi(x) are computed by each side with its
own forward operator.
"""
from .scenes import cacti_video, mri_phantom, msfa_cube
from .masks import cacti_masks, mri_line_mask
from .workloads import WORKLOADS, Workload, sigma_schedule, make_instance

__all__ = [
    "cacti_video", "mri_phantom", "msfa_cube", "cacti_masks", "mri_line_mask",
    "WORKLOADS", "Workload", "sigma_schedule", "make_instance",
]
