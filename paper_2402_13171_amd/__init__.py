"""MI355X-native D3Q27 cumulant lattice-Boltzmann solver with actuator-line
rotor coupling (after the waLBerla-wind method, arXiv 2402.13171).

The compute path is a HIP shared library (``liblbm.so``) with a C ABI,
declared in ``include/lbm.h``; :mod:`.lbm` is the thin ctypes binding and
:class:`Lbm` the convenience wrapper that allocates device memory through
PyTorch. Importing this package does not load the library; the first use
does, and fails loudly if it has not been built.
"""
__all__ = ["Lbm", "lib", "roofline"]


def __getattr__(name):
    if name in ("Lbm", "lib"):
        from . import lbm
        return getattr(lbm, name)
    raise AttributeError(name)
