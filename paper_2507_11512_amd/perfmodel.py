"""Flop and byte models for the GMRES-IR / multigrid hot path.

Flops follow the benchmark's rule that operations of every precision count
the same (Sec. 3: the reported rate is a mixed-precision rate), with the
fused residual-restriction counted only at the coarse points (Sec. 3.2).
The same model is used for the FP64 and the mixed-precision solver, so their
ratio is the time ratio times the iteration-count penalty min(1, n_d/n_ir).

Bytes are algorithmic: what each kernel must move once -- every matrix
entry (value + column index for the 26 off-diagonal slots, value for the
diagonal), every vector entry read or written once per launch; the repeated
reads of neighbouring vector entries are not counted.  A column index is
`idx` bytes: 4 for int32 indices (the default format), 2 for the 16-bit
column offsets of HPGMX_COLS_OFFSET16.
"""
from dataclasses import dataclass

SLOTS = 26
IDX = 4   # bytes of a stored int32 column index


def dims_of(n):
    return (n, n, n) if isinstance(n, int) else tuple(int(v) for v in n)


def level_dims(dims, levels):
    out = []
    nx, ny, nz = dims
    for _ in range(levels):
        out.append((nx, ny, nz))
        nx, ny, nz = nx // 2, ny // 2, nz // 2
    return out


def nrows(d):
    return d[0] * d[1] * d[2]


def nnz(d):
    """True nonzeros of the Dirichlet-truncated 27-point operator."""
    return (3 * d[0] - 2) * (3 * d[1] - 2) * (3 * d[2] - 2)


def nnz_coarse_rows(d):
    """Nonzeros of the fine rows at the injection points (2I, 2J, 2K)."""
    f = 1
    for n in d:
        c = n // 2
        f *= 3 * c - 1
    return f


@dataclass
class Config:
    dims: tuple
    levels: int = 4
    pre: int = 1
    post: int = 1
    coarsest: int = 1
    sweep: int = 0          # 0 forward, 1 backward, 2 symmetric
    restart: int = 30


def gs_sweep_flops(d, sweep):
    return (4 if sweep == 2 else 2) * nnz(d)


def vcycle_flops(cfg):
    L = level_dims(cfg.dims, cfg.levels)
    f = 0
    for l, d in enumerate(L):
        if l == cfg.levels - 1:
            f += cfg.coarsest * gs_sweep_flops(d, cfg.sweep)
        else:
            dc = L[l + 1]
            f += (cfg.pre + cfg.post) * gs_sweep_flops(d, cfg.sweep)
            f += 2 * nnz_coarse_rows(d) + nrows(dc)   # fused residual-restriction
            f += nrows(dc)                            # prolongation-correction
    return f


def inner_step_flops(cfg, kb):
    """One inner step with kb basis vectors already present."""
    d = cfg.dims
    N = nrows(d)
    return vcycle_flops(cfg) + 2 * nnz(d) + 8 * kb * N + 2 * N + N


def outer_flops(cfg):
    d = cfg.dims
    return 2 * nnz(d) + 4 * N_(d)


def N_(d):
    return nrows(d)


def end_of_cycle_flops(cfg, kk):
    N = nrows(cfg.dims)
    return 2 * kk * N + N + vcycle_flops(cfg)


def solve_flops(cfg, cycles):
    """cycles: list of inner-step counts per restart cycle.  Counts one outer
    residual per cycle plus the final one."""
    f = 0
    for kk in cycles:
        f += outer_flops(cfg)
        for k in range(kk):
            f += inner_step_flops(cfg, k + 1)
        f += end_of_cycle_flops(cfg, kk)
    f += outer_flops(cfg)
    return f


def fixed_iteration_cycles(iters, restart):
    cycles = []
    left = iters
    while left > 0:
        cycles.append(min(restart, left))
        left -= restart
    return cycles


# ---- bytes --------------------------------------------------------------------------------------
# dtype codes: 0 FP64; 1 FP32; 2 / 3 binary16 / bfloat16 matrices; 4 / 5 the
# whole multigrid hierarchy (matrices and work vectors) in binary16 / bfloat16.
def vb(dtype):
    """Matrix value bytes."""
    return {0: 8, 1: 4, 2: 2, 3: 2, 4: 2, 5: 2}[dtype]


def wb(dtype):
    """Krylov vector bytes (the basis, the SpMV output)."""
    return 8 if dtype == 0 else 4


def mgb(dtype):
    """Multigrid work-vector bytes."""
    return {0: 8, 4: 2, 5: 2}.get(dtype, 4)


def gs_colour_bytes(rows, active_slots, dtype, idx=IDX):
    """One colour launch: matrix slice for `active_slots` slots + diagonal,
    r read, z written, neighbour z counted once per row (none when no slot
    is active: the first colour of a sweep from a zero guess)."""
    v, w = vb(dtype), mgb(dtype)
    return rows * (active_slots * (v + idx) + v + (3 if active_slots else 2) * w)


def spmv_bytes(rows, dtype, idx=IDX):
    """The SpMV of an inner step: x is the V-cycle's output (a multigrid
    vector), y a Krylov vector."""
    v = vb(dtype)
    return rows * (SLOTS * (v + idx) + v + mgb(dtype) + wb(dtype))


def spmv_split_bytes(rows, late_slots, dtype, idx=IDX):
    """SpMV rows whose sum over the slots to earlier colours was written by
    the colour's own smoother launch: the `late_slots` remaining slots, the
    diagonal, x, the partial sum read and y written."""
    v = vb(dtype)
    return rows * (late_slots * (v + idx) + v + mgb(dtype) + 2 * wb(dtype))


def cgs_pass_bytes(rows, kb, dtype):
    """w <- w - Q c fused with a reduction: kb columns and w read, w written."""
    return rows * (kb + 2) * wb(dtype)


def cgs_dot_bytes(rows, kb, dtype):
    """h2 = Q^T (w - Q h1) with w not written: kb columns and w read."""
    return rows * (kb + 1) * wb(dtype)


def restrict_bytes(coarse_rows, dtype, idx=IDX):
    v, w = vb(dtype), mgb(dtype)
    return coarse_rows * (SLOTS * (v + idx) + v + 3 * w)


def restrict_after_sweep_bytes(coarse_rows, dtype, slots=8, K=1, idx=IDX):
    """The fused restriction after a single sweep from zero: `slots` matrix
    slots of each injection row (8 after a forward sweep), z read once and
    r_c written (K vectors)."""
    v, w = vb(dtype), mgb(dtype)
    return coarse_rows * (slots * (v + idx) + 2 * K * w)


def prolong_bytes(coarse_rows, dtype):
    return coarse_rows * 3 * mgb(dtype)


def resid64_bytes(rows, idx=IDX):
    return rows * (SLOTS * (8 + idx) + 8 + 4 * 8)


# ---- bytes of the batched kernels (K interleaved right-hand sides) -------------------------------
# The matrix is read once per launch for all K vectors; vector traffic scales
# with K.  Per right-hand side and row the matrix share is (26 (v + IDX) + v) / K.
def bgs_colour_bytes(rows, active_slots, dtype, K):
    v, w = vb(dtype), wb(dtype)
    return rows * (active_slots * (v + IDX) + v + (3 if active_slots else 2) * K * w)


def bspmv_bytes(rows, dtype, K):
    v, w = vb(dtype), wb(dtype)
    return rows * (SLOTS * (v + IDX) + v + 2 * K * w)


def brestrict_bytes(coarse_rows, dtype, K):
    v, w = vb(dtype), wb(dtype)
    return coarse_rows * (SLOTS * (v + IDX) + v + 3 * K * w)


def bprolong_bytes(coarse_rows, dtype, K):
    return coarse_rows * 3 * K * wb(dtype)


def bresid64_bytes(rows, K):
    """b - A x (b, x read, r written) plus the norm pass over r."""
    return rows * (SLOTS * (8 + IDX) + 8 + 4 * 8 * K)


def bdot_bytes(rows, kb, dtype, K):
    """h1 = Q^T w: kb basis columns and w, each K entries per row."""
    return rows * K * (kb + 1) * wb(dtype)


def zero_guess_active_slots(colour, forward=True):
    """Slots of a colour-c row that couple to colours relaxed earlier."""
    n = 0
    for t in range(27):
        if t == 13:
            continue
        di, dj, dk = t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1
        flip = (di & 1) | ((dj & 1) << 1) | ((dk & 1) << 2)
        cn = colour ^ flip
        if (cn < colour) if forward else (cn > colour):
            n += 1
    return n


def penalty(n_d, n_ir):
    """Iteration-count penalty of the mixed-precision rate (Sec. 3): the rate
    is multiplied by n_d / n_ir when that ratio is below one, and left as is
    otherwise."""
    if not n_d or not n_ir:
        return 1.0
    return min(1.0, n_d / n_ir)
