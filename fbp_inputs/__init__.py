"""Seeded synthetic inputs for the accelerated FBP library, its tests and its benchmark.

This package only *produces data*: random-ellipse (and ellipsoid-stack) phantoms, their exact
line integrals on the four linogram line classes and on a uniform parallel-beam sinogram,
Poisson-noised variants, and integer test arrays.  It contains none of the reconstruction
arithmetic (no ramp filter, no recursive filter, no Hough transform, no back projection), so
both the CPU oracle and the HIP path can consume its outputs without sharing any code.
"""
from .phantom import (  # noqa: F401
    EllipseSet,
    random_ellipses,
    random_ellipsoids,
    ellipsoid_slices,
    phantom_image,
    linogram_line_params,
    linogram,
    parallel_sinogram,
    poisson_noisy,
    volume_linogram,
    random_int_array,
    support_mask,
)
