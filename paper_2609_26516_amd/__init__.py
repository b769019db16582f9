"""MI355X (gfx950) implementation of the hot path of tensor-network simulation
of dynamic circuits: the MPS compression step of a unitary chunk, measurement
probability, collapse and branch retention (top-M or adaptive pruning),
behind the C ABI of include/dcs.h (libdcs.so, built in-tree by ``python -m
paper_2609_26516_amd.build``).

Modules: ``capi`` (ctypes binding, same names as the C functions),
``engine`` (single-path and multi-path drivers over the binding),
``validation`` (the paper's validation studies run on the drivers).
"""
__all__ = ["capi", "engine", "build", "validation"]
