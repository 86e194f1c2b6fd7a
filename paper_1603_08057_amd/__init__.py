"""rsfgp: recursive skeletonization factorization of spatial Gaussian-process
covariance matrices on AMD Instinct MI355X, with the log-likelihood and score
equations built on it (Minden, Damle, Ho and Ying, "Fast spatial Gaussian
process maximum likelihood estimation via skeletonization factorizations").

This module is a thin ctypes binding of the C ABI in include/rsfgp.h: it only
marshals arguments.  Every step of the computation runs in the HIP library
(librsfgp.so, built in-tree by paper_1603_08057_amd.build).  PyTorch supplies
device memory and the current stream.  There is no CPU fallback: without the
built library, or without a HIP device, the calls raise.
"""
from ._lib import (  # noqa: F401
    MATERN12, MATERN32, MATERN52, RQ, MATERN32_ANISO, RQ_ANISO, PRECISIONS, RsfError, Factor, BatchedFactor, Options, GradInfo, library_path, load,
    trace_enable, trace_read, trace_busy_ms, trace_kernels, cond_mean, cond_sample,
)
from .autograd import loglik_fn  # noqa: F401
from .mle import fit, FitResult  # noqa: F401
