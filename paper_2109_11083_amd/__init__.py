"""MI355X-native Lees-Edwards shear-flow MD hot path (arXiv 2109.11083).

The product is the C-ABI library libleshear.so (include/le.h) built from the
HIP sources in csrc/; `binding` marshals its arguments and `sim.Sim` wraps
one simulation with torch-allocated device memory.
"""
from . import binding  # noqa: F401

__all__ = ["binding", "inputs"]
