"""Thin ctypes binding of libhpgmx.so (argument marshalling only).

Every function has the name of the C entry point it wraps (without the
``hpgmx_`` prefix) and takes torch tensors on the GPU; the data pointers and
the current HIP stream are handed to the library as plain pointers.  All
arithmetic runs in the library's HIP kernels.  If the library has not been
built this module raises ImportError: there is no fallback path.
"""
import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhpgmx.so")

F64, F32, F16, BF16, F16_MG, BF16_MG = 0, 1, 2, 3, 4, 5
GS_FORWARD, GS_BACKWARD, GS_SYMMETRIC = 0, 1, 2
COLS_INT32, COLS_OFFSET16 = 0, 1
SOLVE_PROFILE = 1
SOLVE_GRAPH = 2
SOLVE_AUTOTUNE = 4

K_GS, K_GS_ZERO, K_RESTRICT, K_PROLONG, K_SPMV_DOT, K_CGS_DOT, K_CGS_NORM, K_NORMALIZE, \
    K_RESID64, K_CAST, K_TRSM, K_GEMV, K_UPDATE, K_PERMUTE, K_SPMV, K_DOT, K_FINISH = range(17)
K_COUNT = 17
KERNEL_NAMES = ["gs", "gs_zero", "restrict", "prolong", "spmv_dot", "cgs_dot", "cgs_norm",
                "normalize", "resid64", "cast", "trsm", "gemv", "update", "permute", "spmv", "dot", "finish"]

# batched kernel kinds of the tile table
BK_SPMV, BK_GS, BK_GS_ZERO, BK_RESTRICT, BK_RESID64 = range(5)
BK_COUNT = 5
BK_NAMES = ["spmv", "gs", "gs_zero", "restrict", "resid64"]
MAX_BATCH = 8

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "ENONFINITE"}

EXPORTS = ["hpgmx_setup_problem", "hpgmx_setup_problem_stencil", "hpgmx_stencil_grad",
           "hpgmx_workspace_bytes", "hpgmx_bind_workspace",
           "hpgmx_mg_setup", "hpgmx_gmres_ir_solve", "hpgmx_spmv", "hpgmx_smooth",
           "hpgmx_vcycle", "hpgmx_restrict_residual", "hpgmx_prolong_add",
           "hpgmx_rhs_from_x", "hpgmx_profile_get", "hpgmx_stream_copy", "hpgmx_destroy",
           "hpgmx_last_error", "hpgmx_batch_autotune", "hpgmx_batch_set_tuning",
           "hpgmx_batch_get_tuning", "hpgmx_workspace_bytes_batched", "hpgmx_spmv_batched",
           "hpgmx_smooth_batched", "hpgmx_vcycle_batched", "hpgmx_gmres_ir_solve_batched",
           "hpgmx_presmooth_restrict", "hpgmx_presmooth_restrict_batched", "hpgmx_krylov_cycle_get",
           "hpgmx_stencil_grad_noalloc", "hpgmx_set_column_format",
           "hpgmx_set_layout"]


class ProblemDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("beta", C.c_double)]


class StencilDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("coef", C.c_double * 27)]


class MgDesc(C.Structure):
    _fields_ = [("levels", C.c_int), ("pre_sweeps", C.c_int), ("post_sweeps", C.c_int),
                ("coarsest_sweeps", C.c_int), ("sweep", C.c_int)]


class SolveDesc(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iters", C.c_int), ("tol", C.c_double),
                ("inner_dtype", C.c_int), ("res_hist_host", C.POINTER(C.c_double)),
                ("res_hist_len", C.c_int), ("flags", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("breakdown", C.c_int), ("rho0", C.c_double), ("final_rel_res", C.c_double),
                ("est_rel_res", C.c_double), ("solve_ms", C.c_double)]


class BatchTuning(C.Structure):
    _fields_ = [("rhs_per_lane", (C.c_int * 8) * BK_COUNT), ("ms", (C.c_double * 8) * BK_COUNT)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(or python paper_2507_11512_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    H = C.c_void_p
    sig = {
        "hpgmx_setup_problem": [C.POINTER(ProblemDesc), vp, C.POINTER(H)],
        "hpgmx_setup_problem_stencil": [C.POINTER(StencilDesc), vp, C.POINTER(H)],
        "hpgmx_stencil_grad": [H, vp, vp, vp],
        "hpgmx_stencil_grad_noalloc": [H, vp, vp, vp],
        "hpgmx_set_column_format": [H, i],
        "hpgmx_set_layout": [H, i, i, i, C.c_longlong, i],
        "hpgmx_workspace_bytes": [H, C.POINTER(MgDesc), i, C.c_uint, C.POINTER(C.c_size_t)],
        "hpgmx_bind_workspace": [H, vp, C.c_size_t],
        "hpgmx_mg_setup": [H, C.POINTER(MgDesc)],
        "hpgmx_gmres_ir_solve": [H, vp, vp, C.POINTER(SolveDesc), C.POINTER(SolveStats)],
        "hpgmx_spmv": [H, i, i, vp, vp],
        "hpgmx_smooth": [H, i, i, i, vp, vp, i],
        "hpgmx_vcycle": [H, i, vp, vp],
        "hpgmx_restrict_residual": [H, i, i, vp, vp, vp],
        "hpgmx_prolong_add": [H, i, i, vp, vp],
        "hpgmx_rhs_from_x": [H, vp, vp],
        "hpgmx_profile_get": [H, i, i, C.POINTER(d), C.POINTER(C.c_longlong)],
        "hpgmx_stream_copy": [H, vp, vp, C.c_size_t, i, C.POINTER(d)],
        "hpgmx_destroy": [H],
        "hpgmx_batch_autotune": [H, i, i, C.POINTER(BatchTuning)],
        "hpgmx_batch_set_tuning": [H, i, i, C.POINTER(BatchTuning)],
        "hpgmx_batch_get_tuning": [H, i, i, C.POINTER(BatchTuning)],
        "hpgmx_workspace_bytes_batched": [H, C.POINTER(MgDesc), i, i, C.c_uint, C.POINTER(C.c_size_t)],
        "hpgmx_spmv_batched": [H, i, i, i, vp, vp],
        "hpgmx_smooth_batched": [H, i, i, i, i, vp, vp, i],
        "hpgmx_vcycle_batched": [H, i, i, vp, vp],
        "hpgmx_gmres_ir_solve_batched": [H, i, vp, vp, C.POINTER(SolveDesc), C.POINTER(SolveStats)],
        "hpgmx_presmooth_restrict": [H, i, i, i, i, vp, vp, vp],
        "hpgmx_presmooth_restrict_batched": [H, i, i, i, i, i, vp, vp, vp],
        "hpgmx_krylov_cycle_get": [H, i, C.POINTER(i), vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.hpgmx_last_error.argtypes = [H]
    lib.hpgmx_last_error.restype = C.c_char_p
    return lib


lib = _load()


class HpgmxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(h, st):
    if st != 0:
        msg = lib.hpgmx_last_error(h) if h else b""
        raise HpgmxError(st, (msg or b"").decode())


def _ptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    return C.c_void_p(t.data_ptr())


def _vec_dtype(dtype):
    """torch dtype of the multigrid vectors of a precision at the ABI."""
    import torch
    return {F64: torch.float64, F16_MG: torch.float16, BF16_MG: torch.bfloat16}.get(dtype, torch.float32)


@dataclass
class Stats:
    iters: int
    restarts: int
    converged: bool
    breakdown: bool
    rho0: float
    final_rel_res: float
    est_rel_res: float
    solve_ms: float


# ---- one function per C entry point ------------------------------------------------------
def setup_problem(nx, ny, nz, beta=0.5, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    h = C.c_void_p()
    desc = ProblemDesc(int(nx), int(ny), int(nz), float(beta))
    _check(None, lib.hpgmx_setup_problem(C.byref(desc), C.c_void_p(stream.cuda_stream), C.byref(h)))
    return h


def setup_problem_stencil(nx, ny, nz, coef27, stream=None):
    """A general 27-point stencil; coef27[t] multiplies the neighbour at offset
    (di, dj, dk), t = 9(dk+1) + 3(dj+1) + (di+1)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    coef = [float(c) for c in coef27]
    if len(coef) != 27:
        raise ValueError("coef27 must have 27 entries")
    h = C.c_void_p()
    desc = StencilDesc(int(nx), int(ny), int(nz), (C.c_double * 27)(*coef))
    _check(None, lib.hpgmx_setup_problem_stencil(C.byref(desc), C.c_void_p(stream.cuda_stream),
                                                 C.byref(h)))
    return h


def stencil_grad(h, lam, x, out27):
    """out27[t] = sum_i lam_i x_{i + d_t} (device FP64 tensors; out27 has 27 entries)."""
    _check(h, lib.hpgmx_stencil_grad(h, _ptr(lam), _ptr(x), _ptr(out27)))


def stencil_grad_noalloc(h, lam, x, out27):
    """stencil_grad without any device allocation by the library (fixed scratch)."""
    _check(h, lib.hpgmx_stencil_grad_noalloc(h, _ptr(lam), _ptr(x), _ptr(out27)))


def workspace_bytes(h, levels=4, pre=1, post=1, coarsest=1, sweep=GS_FORWARD, restart=30,
                    dtype_mask=(1 << F64) | (1 << F32)):
    mg = MgDesc(levels, pre, post, coarsest, sweep)
    out = C.c_size_t()
    _check(h, lib.hpgmx_workspace_bytes(h, C.byref(mg), int(restart), int(dtype_mask), C.byref(out)))
    return out.value


def bind_workspace(h, tensor):
    _check(h, lib.hpgmx_bind_workspace(h, _ptr(tensor), tensor.numel() * tensor.element_size()))


def set_column_format(h, fmt):
    _check(h, lib.hpgmx_set_column_format(h, int(fmt)))


def set_layout(h, tile_order=-1, ell_chunk_log2=-1, ldq_pad=-1, pair_rows=-1, spmv_in_sweep=-1):
    _check(h, lib.hpgmx_set_layout(h, int(tile_order), int(ell_chunk_log2), int(ldq_pad), int(pair_rows),
                                   int(spmv_in_sweep)))


def mg_setup(h, levels=4, pre=1, post=1, coarsest=1, sweep=GS_FORWARD):
    mg = MgDesc(int(levels), int(pre), int(post), int(coarsest), int(sweep))
    _check(h, lib.hpgmx_mg_setup(h, C.byref(mg)))


def gmres_ir_solve(h, b, x, restart=30, max_iters=10000, tol=1e-9, inner_dtype=F32,
                   hist_len=0, profile=False, graph=False):
    """Solves in place: x holds x0 on entry and the solution on exit."""
    import numpy as np
    hist = np.zeros(max(hist_len, 1))
    desc = SolveDesc(int(restart), int(max_iters), float(tol), int(inner_dtype),
                     hist.ctypes.data_as(C.POINTER(C.c_double)) if hist_len > 0 else None,
                     int(hist_len), (SOLVE_PROFILE if profile else 0) | (SOLVE_GRAPH if graph else 0))
    st = SolveStats()
    _check(h, lib.hpgmx_gmres_ir_solve(h, _ptr(b), _ptr(x), C.byref(desc), C.byref(st)))
    s = Stats(st.iters, st.restarts, bool(st.converged), bool(st.breakdown), st.rho0,
              st.final_rel_res, st.est_rel_res, st.solve_ms)
    if hist_len > 0:
        return s, hist[:min(st.iters, hist_len)].copy()
    return s


def spmv(h, level, dtype, x, y):
    _check(h, lib.hpgmx_spmv(h, int(level), int(dtype), _ptr(x), _ptr(y)))


def smooth(h, level, dtype, sweep, r, z, zero_guess=False):
    _check(h, lib.hpgmx_smooth(h, int(level), int(dtype), int(sweep), _ptr(r), _ptr(z),
                               int(bool(zero_guess))))


def vcycle(h, dtype, r, z):
    _check(h, lib.hpgmx_vcycle(h, int(dtype), _ptr(r), _ptr(z)))


def restrict_residual(h, level, dtype, r, z, r_coarse):
    _check(h, lib.hpgmx_restrict_residual(h, int(level), int(dtype), _ptr(r), _ptr(z),
                                          _ptr(r_coarse)))


def presmooth_restrict(h, level, dtype, sweep, nsweeps, r, z, r_coarse):
    _check(h, lib.hpgmx_presmooth_restrict(h, int(level), int(dtype), int(sweep), int(nsweeps), _ptr(r),
                                           _ptr(z), _ptr(r_coarse)))


def krylov_cycle_get(h, dtype, N, restart):
    """The last cycle of the last single solve with this inner dtype:
    (k, Q (k+1, N) float64 GPU tensor of stored columns, scale (k+1,),
    Hbar (k+1, k), y (k,)) -- numpy arrays except Q."""
    import numpy as np
    import torch
    m = int(restart)
    Q = torch.empty((m + 1, int(N)), dtype=torch.float64, device="cuda")
    scale = np.zeros(m + 1)
    Hb = np.zeros(m * (m + 1))
    y = np.zeros(m)
    k = C.c_int(0)
    _check(h, lib.hpgmx_krylov_cycle_get(h, int(dtype), C.byref(k), _ptr(Q), scale.ctypes.data_as(C.c_void_p),
                                         Hb.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p)))
    k = k.value
    Hbar = Hb[:k * (k + 1)].reshape(k, k + 1).T.copy()
    return k, Q[:k + 1], scale[:k + 1].copy(), Hbar, y[:k].copy()


def prolong_add(h, level, dtype, z_coarse, z):
    _check(h, lib.hpgmx_prolong_add(h, int(level), int(dtype), _ptr(z_coarse), _ptr(z)))


def rhs_from_x(h, x, b):
    _check(h, lib.hpgmx_rhs_from_x(h, _ptr(x), _ptr(b)))


def _tuning_dict(t):
    return {"rhs_per_lane": [[t.rhs_per_lane[k][l] for l in range(8)] for k in range(BK_COUNT)],
            "ms": [[t.ms[k][l] for l in range(8)] for k in range(BK_COUNT)]}


def batch_autotune(h, nrhs, dtype):
    """Times every tile shape of the batched kernels and adopts the fastest;
    returns the table ({"rhs_per_lane": [kind][level], "ms": [kind][level]})."""
    t = BatchTuning()
    _check(h, lib.hpgmx_batch_autotune(h, int(nrhs), int(dtype), C.byref(t)))
    return _tuning_dict(t)


def batch_set_tuning(h, nrhs, dtype, rhs_per_lane):
    """rhs_per_lane: [kind][level] (0 = the library's fixed rule), or an int for all."""
    t = BatchTuning()
    for k in range(BK_COUNT):
        for l in range(8):
            v = rhs_per_lane if isinstance(rhs_per_lane, int) else rhs_per_lane[k][l]
            t.rhs_per_lane[k][l] = int(v)
    _check(h, lib.hpgmx_batch_set_tuning(h, int(nrhs), int(dtype), C.byref(t)))


def batch_get_tuning(h, nrhs, dtype):
    t = BatchTuning()
    _check(h, lib.hpgmx_batch_get_tuning(h, int(nrhs), int(dtype), C.byref(t)))
    return _tuning_dict(t)


def workspace_bytes_batched(h, nrhs, levels=4, pre=1, post=1, coarsest=1, sweep=GS_FORWARD, restart=30,
                            dtype_mask=(1 << F64) | (1 << F32)):
    mg = MgDesc(levels, pre, post, coarsest, sweep)
    out = C.c_size_t()
    _check(h, lib.hpgmx_workspace_bytes_batched(h, C.byref(mg), int(nrhs), int(restart), int(dtype_mask),
                                                C.byref(out)))
    return out.value


def spmv_batched(h, level, dtype, X, Y):
    """Y[j] = A X[j]; X, Y: (nrhs, N_level) GPU tensors."""
    _check(h, lib.hpgmx_spmv_batched(h, int(level), int(dtype), int(X.shape[0]), _ptr(X), _ptr(Y)))


def smooth_batched(h, level, dtype, sweep, R, Z, zero_guess=False):
    _check(h, lib.hpgmx_smooth_batched(h, int(level), int(dtype), int(sweep), int(R.shape[0]), _ptr(R),
                                       _ptr(Z), int(bool(zero_guess))))


def presmooth_restrict_batched(h, level, dtype, sweep, nsweeps, R, Z, R_coarse):
    _check(h, lib.hpgmx_presmooth_restrict_batched(h, int(level), int(dtype), int(sweep), int(nsweeps),
                                                   int(R.shape[0]), _ptr(R), _ptr(Z), _ptr(R_coarse)))


def vcycle_batched(h, dtype, R, Z):
    _check(h, lib.hpgmx_vcycle_batched(h, int(dtype), int(R.shape[0]), _ptr(R), _ptr(Z)))


def gmres_ir_solve_batched(h, B, X, restart=30, max_iters=10000, tol=1e-9, inner_dtype=F32,
                           hist_len=0, profile=False, graph=False, autotune=False):
    """Solves in place for every row of X (nrhs, N); returns a list of Stats
    (and the (nrhs, hist_len) residual histories if hist_len > 0)."""
    import numpy as np
    nrhs = int(B.shape[0])
    hist = np.zeros((nrhs, max(hist_len, 1)))
    flags = (SOLVE_PROFILE if profile else 0) | (SOLVE_GRAPH if graph else 0) | \
        (SOLVE_AUTOTUNE if autotune else 0)
    desc = SolveDesc(int(restart), int(max_iters), float(tol), int(inner_dtype),
                     hist.ctypes.data_as(C.POINTER(C.c_double)) if hist_len > 0 else None,
                     int(hist_len), flags)
    st = (SolveStats * nrhs)()
    _check(h, lib.hpgmx_gmres_ir_solve_batched(h, nrhs, _ptr(B), _ptr(X), C.byref(desc), st))
    out = [Stats(s.iters, s.restarts, bool(s.converged), bool(s.breakdown), s.rho0, s.final_rel_res,
                 s.est_rel_res, s.solve_ms) for s in st]
    if hist_len > 0:
        return out, [hist[j, :min(out[j].iters, hist_len)].copy() for j in range(nrhs)]
    return out


def profile_get(h, kernel, level=0):
    ms, n = C.c_double(), C.c_longlong()
    _check(h, lib.hpgmx_profile_get(h, int(kernel), int(level), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def stream_copy(h, src, dst, nbytes, reps=20):
    ms = C.c_double()
    _check(h, lib.hpgmx_stream_copy(h, _ptr(src), _ptr(dst), int(nbytes), int(reps), C.byref(ms)))
    return ms.value


def destroy(h):
    if h:
        _check(None, lib.hpgmx_destroy(h))


def last_error(h):
    return (lib.hpgmx_last_error(h) or b"").decode()


# ---- convenience object -------------------------------------------------------------------
class Problem:
    """One stencil problem with its multigrid hierarchy on the current GPU.

    >>> P = Problem(128, beta=0.5, levels=4, sweep='forward')
    >>> x, stats = P.solve(b, tol=1e-9, restart=30, precision='mxp')

    `cols` picks the column-index format ("int32" or "offset16"); `layout`,
    for layout studies only, is a dict of set_layout's keyword arguments.
    """

    _SWEEPS = {"forward": GS_FORWARD, "backward": GS_BACKWARD, "symmetric": GS_SYMMETRIC}
    _PREC = {"fp64": F64, "mxp": F32, "fp32": F32, "fp16": F16, "bf16": BF16,
             "fp16-mg": F16_MG, "bf16-mg": BF16_MG}

    def __init__(self, n, beta=0.5, levels=4, sweep="forward", pre=1, post=1, coarsest=1,
                 stream=None, workspace=None, coef=None, cols="int32", layout=None):
        import torch
        self.dims = (n, n, n) if isinstance(n, int) else tuple(n)
        self.N = self.dims[0] * self.dims[1] * self.dims[2]
        self.levels = levels
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if coef is None:
            self.h = setup_problem(*self.dims, beta=beta, stream=self.stream)
        else:
            self.h = setup_problem_stencil(*self.dims, coef, stream=self.stream)
        sw = self._SWEEPS[sweep] if isinstance(sweep, str) else int(sweep)
        try:
            set_column_format(self.h, {"int32": COLS_INT32, "offset16": COLS_OFFSET16}[cols])
            if layout is not None:
                set_layout(self.h, **layout)
            if workspace is not None:
                bind_workspace(self.h, workspace)
                self.workspace = workspace
            mg_setup(self.h, levels, pre, post, coarsest, sw)
        except Exception:
            destroy(self.h)
            self.h = None
            raise

    def level_dims(self, level):
        return tuple(d >> level for d in self.dims)

    def rhs_from_x(self, x):
        import torch
        b = torch.empty_like(x, dtype=torch.float64)
        rhs_from_x(self.h, x, b)
        return b

    def solve(self, b, x0=None, tol=1e-9, restart=30, max_iters=10000, precision="mxp",
              hist_len=0, profile=False, graph=False):
        import torch
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        prec = self._PREC[precision] if isinstance(precision, str) else int(precision)
        with torch.cuda.stream(self.stream):
            out = gmres_ir_solve(self.h, b, x, restart, max_iters, tol, prec, hist_len, profile, graph)
        return (x, *out) if isinstance(out, tuple) else (x, out)

    def solve_batched(self, B, X0=None, tol=1e-9, restart=30, max_iters=10000, precision="mxp",
                      hist_len=0, profile=False, graph=False, autotune=False):
        """B: (nrhs, N) FP64 GPU tensor, nrhs <= 8.  Returns (X, [Stats per rhs])."""
        import torch
        X = torch.zeros_like(B) if X0 is None else X0.clone()
        prec = self._PREC[precision] if isinstance(precision, str) else int(precision)
        with torch.cuda.stream(self.stream):
            out = gmres_ir_solve_batched(self.h, B, X, restart, max_iters, tol, prec, hist_len, profile,
                                         graph, autotune)
        return (X, *out) if isinstance(out, tuple) else (X, out)

    def stencil_grad(self, lam, x):
        """27 FP64 values sum_i lam_i x_{i + d_t} (see hpgmx_stencil_grad)."""
        import torch
        out = torch.empty(27, dtype=torch.float64, device=lam.device)
        with torch.cuda.stream(self.stream):
            stencil_grad(self.h, lam, x, out)
        return out

    def close(self):
        if self.h:
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
