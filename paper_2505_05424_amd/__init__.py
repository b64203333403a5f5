"""MI355X (gfx950) solver for dynamic optimal transport on a staggered grid as
a linear SOCP, by the inexact proximal ALM of arXiv 2505.05424 (Algorithm 2).

The compute path is the HIP library libdotsocp.so (C ABI in
include/dotsocp.h); `binding` is its ctypes wrapper (argument marshalling
only; device buffers are passed as raw pointers, e.g. of torch tensors) and
`serving` the host driver of the serving contexts.
"""
from . import binding  # noqa: F401

__all__ = ["binding"]
