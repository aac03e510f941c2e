"""MI355X (gfx950) implementation of the unified fourth-order BGK lattice
Boltzmann model for the d-dimensional linear hyperbolic equation
(arXiv:2410.13165): C-ABI library liblbm.so plus a ctypes binding.

The binding is imported lazily so that `paper_2410_13165_amd.inputs` and
`paper_2410_13165_amd.build` work without the compiled library.
"""

__all__ = ["Lattice", "Batch", "Field", "LbmError", "load_library", "equilibrium_weights",
           "stability_map"]


def __getattr__(name):
    if name in __all__:
        from . import lbm as _lbm
        return getattr(_lbm, name)
    raise AttributeError(name)
