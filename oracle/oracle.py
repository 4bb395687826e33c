"""ctypes front end of the C oracle (test infrastructure only).

Every function takes and returns float64 numpy arrays in natural
lexicographic order I = i + nx*(j + ny*k).  ``beta`` is the nonsymmetry
shift of the x-neighbour entries (-1-beta at di = -1, -1+beta at di = +1);
``faces_only`` selects the reading where only the two x face neighbours carry
the shift.  Sweep kinds: 0 forward, 1 backward, 2 symmetric.
"""
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhpgmx_oracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


class _CStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("breakdown", C.c_int), ("rho0", C.c_double),
                ("final_rel_res", C.c_double), ("est_rel_res", C.c_double)]


@dataclass
class Stats:
    iters: int
    restarts: int
    converged: bool
    breakdown: bool
    rho0: float
    final_rel_res: float
    est_rel_res: float


def build_lib():
    from .build import build_oracle
    return build_oracle()


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build_lib()
    lib = C.CDLL(_LIB_PATH)
    i, d = C.c_int, C.c_double
    lib.or_num_threads.argtypes = []
    lib.or_num_threads.restype = i
    lib.or_set_num_threads.argtypes = [i]
    lib.or_coef.argtypes = [d, i, i, i, i]
    lib.or_coef.restype = d
    lib.or_spmv.argtypes = [i, i, i, d, i, _dp, _dp]
    lib.or_spmv_rows.argtypes = [i, i, i, d, i, _dp, _ip, C.c_int64, _dp]
    lib.or_absrow.argtypes = [i, i, i, d, i, _dp, _dp]
    lib.or_color.argtypes = [i, i, i]
    lib.or_color.restype = i
    lib.or_gs.argtypes = [i, i, i, d, i, i, _dp, _dp]
    lib.or_inject.argtypes = [i, i, i, _dp, _dp]
    lib.or_prolong_add.argtypes = [i, i, i, _dp, _dp]
    lib.or_restrict_fused.argtypes = [i, i, i, d, i, _dp, _dp, _dp]
    lib.or_vcycle.argtypes = [i, i, i, d, i, i, i, i, i, i, i, _dp, _dp]
    lib.or_gmres_ir.argtypes = [i, i, i, d, i, i, i, i, i, i, i, i, i, d, _dp, _dp,
                                C.POINTER(_CStats), C.c_void_p, C.c_void_p, C.c_void_p,
                                C.POINTER(C.c_int), C.c_void_p, i]
    lib.or_gmres_ir.restype = i
    lib.or_stencil_from_beta.argtypes = [d, i, _dp]
    lib.or_spmv_c.argtypes = [i, i, i, _dp, _dp, _dp]
    lib.or_gs_c.argtypes = [i, i, i, _dp, i, _dp, _dp]
    lib.or_vcycle_c.argtypes = [i, i, i, _dp, i, i, i, i, i, i, _dp, _dp]
    lib.or_gmres_ir_c.argtypes = [i, i, i, _dp, i, i, i, i, i, i, i, i, d, _dp, _dp,
                                  C.POINTER(_CStats), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_int), C.c_void_p, i]
    lib.or_gmres_ir_c.restype = i
    lib.or_stencil_correlation.argtypes = [i, i, i, _dp, _dp, _dp]
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(dims):
    if isinstance(dims, int):
        return dims, dims, dims
    nx, ny, nz = dims
    return int(nx), int(ny), int(nz)


def spmv(dims, x, beta=0.5, faces_only=False):
    nx, ny, nz = _dims(dims)
    x = _f64(x)
    y = np.empty(nx * ny * nz)
    load().or_spmv(nx, ny, nz, beta, int(faces_only), x, y)
    return y


def spmv_rows(dims, x, rows, beta=0.5, faces_only=False):
    nx, ny, nz = _dims(dims)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.empty(rows.size)
    load().or_spmv_rows(nx, ny, nz, beta, int(faces_only), _f64(x), rows, rows.size, y)
    return y


def absrow(dims, x, beta=0.5, faces_only=False):
    nx, ny, nz = _dims(dims)
    y = np.empty(nx * ny * nz)
    load().or_absrow(nx, ny, nz, beta, int(faces_only), _f64(x), y)
    return y


def num_threads():
    return load().or_num_threads()


def set_num_threads(n):
    """Threads of the oracle's OpenMP loops from now on (in this process)."""
    load().or_set_num_threads(int(n))


def color(i, j, k):
    return load().or_color(int(i), int(j), int(k))


def gs(dims, r, z, sweep=0, beta=0.5, faces_only=False):
    """One Gauss-Seidel sweep; returns the new z (input z is not modified)."""
    nx, ny, nz = _dims(dims)
    z = _f64(z).copy()
    load().or_gs(nx, ny, nz, beta, int(faces_only), int(sweep), _f64(r), z)
    return z


def inject(dims, v):
    nx, ny, nz = _dims(dims)
    out = np.empty((nx // 2) * (ny // 2) * (nz // 2))
    load().or_inject(nx, ny, nz, _f64(v), out)
    return out


def prolong_add(dims, zc, z):
    nx, ny, nz = _dims(dims)
    z = _f64(z).copy()
    load().or_prolong_add(nx, ny, nz, _f64(zc), z)
    return z


def restrict_fused(dims, r, z, beta=0.5, faces_only=False):
    nx, ny, nz = _dims(dims)
    out = np.empty((nx // 2) * (ny // 2) * (nz // 2))
    load().or_restrict_fused(nx, ny, nz, beta, int(faces_only), _f64(r), _f64(z), out)
    return out


def vcycle(dims, r, levels, pre=1, post=1, coarsest=1, sweep=0, beta=0.5,
           faces_only=False, f32=False):
    nx, ny, nz = _dims(dims)
    z = np.empty(nx * ny * nz)
    load().or_vcycle(nx, ny, nz, beta, int(faces_only), int(levels), int(pre), int(post),
                     int(coarsest), int(sweep), int(f32), _f64(r), z)
    return z


def gmres_ir(dims, b, x0=None, levels=4, pre=1, post=1, coarsest=1, sweep=0,
             restart=30, max_iters=10000, tol=1e-9, beta=0.5, faces_only=False,
             f32=False, want_first_cycle=False, hist_len=0):
    """Alg. 3 on the CPU.  Returns (x, Stats[, first-cycle dict])."""
    nx, ny, nz = _dims(dims)
    n = nx * ny * nz
    b = _f64(b)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    st = _CStats()
    m = int(restart)
    Q1 = H1 = y1 = None
    k1 = C.c_int(0)
    if want_first_cycle:
        Q1 = np.zeros((m + 1, n))
        H1 = np.zeros((m, m + 1))
        y1 = np.zeros(m)
    hist = np.zeros(max(hist_len, 0))

    def ptr(a):
        return None if a is None else a.ctypes.data_as(C.c_void_p)

    rc = load().or_gmres_ir(nx, ny, nz, beta, int(faces_only), int(levels), int(pre), int(post),
                            int(coarsest), int(sweep), int(f32), m, int(max_iters), float(tol),
                            b, x, C.byref(st), ptr(Q1), ptr(H1), ptr(y1), C.byref(k1),
                            ptr(hist) if hist_len > 0 else None, int(hist_len))
    if rc != 0:
        raise RuntimeError(f"oracle gmres_ir failed with status {rc}")
    stats = Stats(st.iters, st.restarts, bool(st.converged), bool(st.breakdown), st.rho0,
                  st.final_rel_res, st.est_rel_res)
    out = [x, stats]
    if want_first_cycle:
        k = k1.value
        out.append({"k": k, "Q": Q1[:k + 1].T.copy(), "Hbar": H1[:k, :k + 1].T.copy(),
                    "y": y1[:k].copy()})
    if hist_len > 0:
        out.append(hist[:min(stats.iters, hist_len)].copy())
    return tuple(out)


# ---- general 27-entry stencils (slot s = 9(dk+1) + 3(dj+1) + (di+1)) ----------------------
def stencil_from_beta(beta=0.5, faces_only=False):
    c = np.empty(27)
    load().or_stencil_from_beta(float(beta), int(faces_only), c)
    return c


def spmv_c(dims, coef27, x):
    nx, ny, nz = _dims(dims)
    y = np.empty(nx * ny * nz)
    load().or_spmv_c(nx, ny, nz, _f64(coef27), _f64(x), y)
    return y


def gs_c(dims, coef27, r, z, sweep=0):
    nx, ny, nz = _dims(dims)
    z = _f64(z).copy()
    load().or_gs_c(nx, ny, nz, _f64(coef27), int(sweep), _f64(r), z)
    return z


def vcycle_c(dims, coef27, r, levels, pre=1, post=1, coarsest=1, sweep=0, f32=False):
    nx, ny, nz = _dims(dims)
    z = np.empty(nx * ny * nz)
    load().or_vcycle_c(nx, ny, nz, _f64(coef27), int(levels), int(pre), int(post), int(coarsest),
                       int(sweep), int(f32), _f64(r), z)
    return z


def gmres_ir_c(dims, coef27, b, x0=None, levels=3, pre=1, post=1, coarsest=1, sweep=0,
               restart=30, max_iters=10000, tol=1e-9, f32=False):
    nx, ny, nz = _dims(dims)
    x = np.zeros(nx * ny * nz) if x0 is None else _f64(x0).copy()
    st = _CStats()
    rc = load().or_gmres_ir_c(nx, ny, nz, _f64(coef27), int(levels), int(pre), int(post),
                              int(coarsest), int(sweep), int(f32), int(restart), int(max_iters),
                              float(tol), _f64(b), x, C.byref(st), None, None, None, None, None, 0)
    if rc != 0:
        raise RuntimeError(f"oracle gmres_ir_c failed with status {rc}")
    return x, Stats(st.iters, st.restarts, bool(st.converged), bool(st.breakdown), st.rho0,
                    st.final_rel_res, st.est_rel_res)


def stencil_correlation(dims, lam, x):
    """out[s] = sum_i lam_i x_{i+d_s} over in-grid pairs (the adjoint gradient of the
    stencil entries is -out)."""
    nx, ny, nz = _dims(dims)
    out = np.empty(27)
    load().or_stencil_correlation(nx, ny, nz, _f64(lam), _f64(x), out)
    return out


def transpose_stencil(coef27):
    """The stencil of A^T: entry at offset d is the entry of A at offset -d."""
    return np.ascontiguousarray(np.asarray(coef27, dtype=np.float64)[::-1])
