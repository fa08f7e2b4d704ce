"""planefit for MI355X: per-pixel RGBD plane fitting with HIP kernels.

After Papadakis & Willis, "Real-Time Surface Fitting to RGBD Sensor Data":
each pixel's k x k window is fitted with a plane in tan(theta)/disparity
space (Eq. 12), from integral-image window sums (Sec. II-C) and closed-form
camera-only moments.  The library is libplanefit.so (C ABI in
include/planefit.h); this package is its Python binding.
"""
from ._binding import (  # noqa: F401
    EXPORTS, MODES, PRECISIONS, STATUS_ILL_CONDITIONED, STATUS_INVALID, Plan,
    PlanefitArgumentError, PlanefitError, fit_planes, fit_planes_backward,
    batch_band_heights, batch_workspace_bytes, fit_planes_backward_batch, fit_planes_batch,
    fit_planes_differentiable, fit_planes_xyz, fit_rects, get_plan, integral_images, load_library,
    status_string,
)

__all__ = ["fit_planes", "fit_planes_batch", "batch_band_heights", "batch_workspace_bytes", "fit_planes_backward", "fit_planes_backward_batch",
           "fit_planes_differentiable",
           "fit_planes_xyz", "integral_images", "fit_rects", "Plan", "get_plan", "load_library", "status_string",
           "PlanefitError", "PlanefitArgumentError", "MODES", "PRECISIONS",
           "STATUS_INVALID", "STATUS_ILL_CONDITIONED", "EXPORTS"]
