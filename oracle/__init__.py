"""CPU oracle for the HPG-MxP hot path -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C (OpenMP) behind ctypes, evaluated on the natural lexicographic
ordering I = i + nx*(j + ny*k).  Only tests/, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package; the product
library never does, and the two share no code.
"""
from .oracle import (  # noqa: F401
    Stats, absrow, build_lib, color, gmres_ir, gs, inject, load, num_threads, prolong_add, set_num_threads,
    restrict_fused, spmv, spmv_rows, vcycle,
    stencil_from_beta, spmv_c, gs_c, vcycle_c, gmres_ir_c, stencil_correlation, transpose_stencil,
)
