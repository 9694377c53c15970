"""MI355X (gfx950) ISDF: weighted K-means interpolation points, least-squares
interpolation vectors and their adjoint, after arXiv:2208.07731.

The computation lives in libisdf.so (hand-written HIP kernels behind the C ABI
of include/isdf.h); this package is the Python binding.
"""
from .api import (ISDFError, KMeansResult, QRCPResult, cluster_residual, exchange, fit,  # noqa: F401
                  fit_backward, fit_residual, kmeans, poisson, qrcp)
from .autograd import ISDFFit, ISDFLoss  # noqa: F401

__all__ = ["kmeans", "fit", "fit_backward", "fit_residual", "cluster_residual", "poisson", "exchange", "qrcp",
           "ISDFFit", "ISDFLoss", "ISDFError", "KMeansResult", "QRCPResult"]
