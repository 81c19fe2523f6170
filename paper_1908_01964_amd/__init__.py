"""MI355X (gfx950) implementation of rank-constrained SCM estimation.

Kubo, Takamune, Kitamura, Saruwatari, "Acceleration of rank-constrained
spatial covariance matrix estimation for blind speech extraction",
APSIPA 2019.  The hot path - FP64 per-frequency setup, per-bin
precomputation, the naive and second-stage accelerated EM iterations, the
Wiener-filter extraction and the adjoint - runs in hand-written HIP kernels
behind the C ABI of include/rcscm.h (librcscm.so); ``rcscm`` is its ctypes
binding and ``autograd`` wraps the adjoint as a torch.autograd.Function.
"""
from .rcscm import (Context, RcscmError, default_params, header_functions, lib,  # noqa: F401
                    to_device, workspace_bytes)

__all__ = ["Context", "RcscmError", "default_params", "header_functions", "lib", "to_device",
           "workspace_bytes"]
