"""hpgmx: mixed-precision GMRES-IR with a geometric-multigrid preconditioner
on a 27-point stencil, as hand-written HIP for gfx950 behind a C ABI.

Importing the package loads nothing native; ``paper_2507_11512_amd.hpgmx``
loads ``libhpgmx.so`` and fails loudly if it has not been built.
"""
__all__ = ["hpgmx", "inputs"]
