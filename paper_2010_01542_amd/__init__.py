"""MI355X (gfx950) implementation of the vertex-centric (Pregel) superstep.

The compute path is libvc.so (HIP kernels behind the C ABI in include/vc.h);
``vc`` is its ctypes binding.  PyTorch is used for device memory and streams.
"""
from .vc import (CC_HASHMIN, PAGERANK, PPR, SSSP, UNREACHED, Batch, Completion, Graph, Server, Stats, VcError,
                 load)

__all__ = ["Graph", "Batch", "Server", "Completion", "Stats", "VcError", "load", "PAGERANK", "CC_HASHMIN", "SSSP", "PPR", "UNREACHED"]
