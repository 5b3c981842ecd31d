"""MI355X (gfx950) differentiable Gaussian-splatting hot path of TAMBRIDGE
(arXiv 2405.19614): batched EWA projection, exact (tile, depth) binning,
LDS-staged front-to-back compositing, its recomputing backward, the Huber
re-projection residual and a graph-captured mapping / pose-refinement step,
the SSIM term of the mapping loss, behind the C ABI in include/gs.h.
"""
from .binding import (Camera, Context, GSError, GSRenderFn, Gaussians, JointRefinement, MappingStep,
                      PAPER_FUSION_BRIDGE,
                      PAPER_MAPPING, SSIMLossFn, StepOptions, as_cameras, default_context, render, sh_coeffs,
                      select_viewpoints, split_images, ssim_loss)
from . import _abi

__all__ = ["Camera", "Context", "GSError", "GSRenderFn", "Gaussians", "JointRefinement", "MappingStep",
           "PAPER_FUSION_BRIDGE",
           "PAPER_MAPPING", "SSIMLossFn", "StepOptions", "as_cameras", "default_context", "render", "sh_coeffs",
           "select_viewpoints", "split_images", "ssim_loss", "_abi"]
