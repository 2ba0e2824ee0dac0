"""Accelerated filtered back projection (recursive ramp filter + Fast Hough Transform back
projection) as HIP kernels for AMD MI355X (gfx950), behind the C ABI of include/fhtfbp.h.

The Python layer only marshals arguments to ``libfhtfbp.so``; see ``api``.
"""
from .api import (  # noqa: F401
    FBP_NO_ROW_SCALE, FBP_INPUT_IS_FHT, FBP_ZERO_WINDOW, FBP_NO_SCRATCH, FbpError, Plan,
    fbp_plan, fbp_plan_set_coefficients, fbp_filter, fht_backproject, fht_forward,
    fbp_reconstruct, fbp_reconstruct_noalloc, fbp_fit_ramp_iir, fbp_direct_parallel,
    fbp_direct_filter,
    fbp_direct_backproject, fbp_direct_linogram, fbp_filter_coef_grad, load_library, strerror,
    fbp_reconstruct_many, fbp_graph_create, Graph, fbp_resample_sinogram,
    fbp_reconstruct_sinogram, fbp_reconstruct_sinogram_padded,
)
from .autograd import FBPReconstruct, fbp_reconstruct_autograd  # noqa: F401,E402
