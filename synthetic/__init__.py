"""Seeded synthetic cohorts shaped like the DARC paper's brain and cardiac workloads.

This package only draws random numbers and evaluates closed-form phantoms; it
holds none of the registration method's arithmetic (no trilinear sampling, no
scaling-and-squaring, no dissimilarity, no gradients).  Both the FP64 oracle
tests and the HIP path read their inputs from here, so the two see
bit-identical FP32 volumes.
"""

from .cohorts import (  # noqa: F401
    WORKLOADS,
    Workload,
    make_cohort,
    smooth_random_field,
    blob_template_params,
    eval_blobs,
    eval_nested_ellipsoids,
)
