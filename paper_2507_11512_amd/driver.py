"""The benchmark driver around the solver (Sec. 3, "The HPG-MxP benchmark",
and the validation modes of Sec. 3.3): validation, the timed phases and the
report.

The driver only sequences solves through callables and adds up times; it
holds none of the method's arithmetic.

Validation modes (Sec. 3.3):
  * standard  -- the FP64 solver runs to the tolerance (at most max_iters
                 inner steps) and gives n_d; the mixed-precision solver runs
                 to the same tolerance and gives n_ir.
  * fullscale -- the FP64 solver runs for at most max_iters inner steps or
                 until the tolerance, whichever comes first, and the relative
                 residual tau it reaches is recorded; the mixed-precision
                 solver then runs until it reaches tau and gives n_ir.
The rate of the mixed-precision phase is multiplied by min(1, n_d / n_ir).

Timed phases: fixed-iteration solves from a zero initial guess, either a
given number of them or repeated until a running time is filled (the
benchmark's official duration is 1800 s).
"""
import math
import time
from dataclasses import dataclass, field

from . import perfmodel

MODES = ("standard", "fullscale")

# Motifs of the benchmark's timing report and the kernels that make them up
# (kernel names as in hpgmx.KERNEL_NAMES).
MOTIFS = {
    "GS": ("gs", "gs_zero"),
    "SpMV": ("spmv_dot", "spmv"),   # spmv_dot: the reserved fused id
    "Restr": ("restrict",),
    "Prolong": ("prolong",),
    "Ortho": ("cgs_dot", "cgs_norm", "normalize", "dot", "finish"),
    "Outer": ("resid64", "cast", "update", "permute"),
    "Other": ("trsm", "gemv"),
}


@dataclass
class SolveOutcome:
    iters: int
    converged: bool
    final_rel_res: float
    seconds: float


@dataclass
class Validation:
    mode: str
    tol: float
    max_iters: int
    n_d: int
    n_ir: int
    tau: float                 # relative residual the MxP run had to reach
    fp64: SolveOutcome
    mxp: SolveOutcome
    penalty: float = field(init=False)

    def __post_init__(self):
        self.penalty = perfmodel.penalty(self.n_d, self.n_ir)


def validate(solve, mode="standard", tol=1e-9, max_iters=10000, mxp_iter_cap=None):
    """solve(precision, tol, max_iters) -> SolveOutcome, precision "fp64" or
    "mxp".  The convergence tests of the solver are strict ("<"), so the
    fullscale target is the next double above tau."""
    if mode not in MODES:
        raise ValueError(f"validation mode must be one of {MODES}")
    d = solve("fp64", tol, max_iters)
    if mode == "standard" or d.converged:
        tau = tol
        target = tol
    else:
        tau = d.final_rel_res
        target = math.nextafter(tau, math.inf)
    cap = mxp_iter_cap if mxp_iter_cap is not None else (max_iters if mode == "standard" else 10 * max_iters)
    m = solve("mxp", target, cap)
    return Validation(mode, tol, max_iters, d.iters, m.iters, tau, d, m)


@dataclass
class TimedPhase:
    solves: int
    seconds: float

    @property
    def seconds_per_solve(self):
        return self.seconds / self.solves


def timed_phase(run_once, steps=None, duration=None, clock=time.perf_counter):
    """Runs run_once() (one fixed-iteration solve, returning when it has
    finished) `steps` times, or, if duration is given, until `duration`
    seconds are filled (at least once)."""
    if (steps is None) == (duration is None):
        raise ValueError("give exactly one of steps and duration")
    t0 = clock()
    n = 0
    if steps is not None:
        for _ in range(int(steps)):
            run_once()
            n += 1
    else:
        while True:
            run_once()
            n += 1
            if clock() - t0 >= duration:
                break
    return TimedPhase(n, clock() - t0)


def motif_times(kernel_ms):
    """kernel_ms: {kernel name: ms} (names without level/precision suffixes
    are summed over levels by the caller) -> {motif: ms}."""
    out = {m: 0.0 for m in MOTIFS}
    for name, ms in kernel_ms.items():
        for motif, members in MOTIFS.items():
            if name in members:
                out[motif] += ms
                break
        else:
            raise KeyError(f"kernel {name!r} belongs to no motif")
    return out


def report(problem, validation, phases, flops_per_solve, motifs=None):
    """The benchmark report as text.

    problem: dict of descriptive fields; validation: Validation or None;
    phases: {"mxp": TimedPhase, "double": TimedPhase (optional)};
    motifs: {"mxp": {motif: ms per solve}, ...} (optional)."""
    L = ["HPG-MxP-style benchmark report", ""]
    L.append("Problem:")
    for k, v in problem.items():
        L.append(f"  {k}: {v}")
    pen = 1.0
    if validation is not None:
        v = validation
        pen = v.penalty
        L += ["", f"Validation ({v.mode}):",
              f"  tolerance: {v.tol:.1e}   FP64 iteration limit: {v.max_iters}",
              f"  double: iterations={v.fp64.iters} converged={int(v.fp64.converged)} "
              f"rel_res={v.fp64.final_rel_res:.3e} time={v.fp64.seconds:.3f} s",
              f"  target for mxp: {v.tau:.3e}",
              f"  mxp: iterations={v.mxp.iters} converged={int(v.mxp.converged)} "
              f"rel_res={v.mxp.final_rel_res:.3e} time={v.mxp.seconds:.3f} s",
              f"  n_d / n_ir = {v.n_d} / {v.n_ir}; penalty min(1, n_d/n_ir) = {pen:.4f}"]
    rates = {}
    for name in ("mxp", "double"):
        ph = phases.get(name)
        if ph is None:
            continue
        raw = flops_per_solve / ph.seconds_per_solve / 1e9
        final = raw * pen if name == "mxp" else raw
        rates[name] = final
        L += ["", f"Benchmark phase ({name}):",
              f"  solves: {ph.solves}   time: {ph.seconds:.3f} s   per solve: {ph.seconds_per_solve * 1e3:.2f} ms",
              f"  GFLOP/s raw: {raw:.2f}" + (f"   GFLOP/s final (penalised): {final:.2f}" if name == "mxp" else "")]
        if motifs and name in motifs:
            tot = sum(motifs[name].values())
            L.append("  motif times per solve (ms, % of kernel time):")
            for mo, ms in motifs[name].items():
                L.append(f"    {mo:8s} {ms:10.2f}  {100 * ms / tot if tot else 0:5.1f} %")
    if "mxp" in rates and "double" in rates:
        L += ["", f"Speedup mxp / double (penalised): {rates['mxp'] / rates['double']:.3f}"]
    return "\n".join(L) + "\n"
