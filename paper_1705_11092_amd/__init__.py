"""D2Q9 cascaded lattice Boltzmann step with the consistent forcing scheme
(Fei & Luo) as hand-written HIP for gfx950 behind a C-ABI library.

Submodules load lazily: ``clbm`` is the ctypes binding of the library,
``inputs`` builds seeded synthetic workloads, ``serve`` is the
continuous-batching solve server.
"""
__all__ = ["clbm", "inputs", "serve"]
