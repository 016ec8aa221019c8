"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package produces only *inputs* of the product-convolution method: the box
domain, an adaptively refined leaf tiling, the sample points (corners of the
leaves), the impulse responses of a spatially varying Gaussian blur on local
patches, and random vectors.  It contains none of the method's own arithmetic
(no weighting functions, no extension, no convolution): those live separately
in the oracle and in the HIP library.

The blur operator stands in for the spatially varying blur of the paper's
numerical section (Sec. 5.1): A[y, x] = exp(-sum_i (y_i-x_i)^2 / (2 s_i(x)^2)) / Z(x)
when |y_i - x_i| <= R_i(x) = ceil(4 s_i(x)) for every axis, else 0.
"""

from .fields import cosine_field, cfg0_sigma
from .grids import (uniform_nodes, tensor_leaves, quadtree_leaves,
                    corner_points, tune_quadtree)
from .blur import BlurOperator
from .configs import make_config, make_serving_ops, Workload

__all__ = [
    "cosine_field", "cfg0_sigma", "uniform_nodes", "tensor_leaves",
    "quadtree_leaves", "corner_points", "tune_quadtree", "BlurOperator",
    "make_config", "make_serving_ops", "Workload",
]
