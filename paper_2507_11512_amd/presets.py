"""Named workloads of the HPG-MxP hot path.

Each preset fixes the problem (grid, stencil, multigrid hierarchy, column
format), the solver settings (restart, tolerance, inner precisions) and how
the right-hand sides are drawn.  The stencil is the nonsymmetric 27-point
operator of Sec. 3.1 (26 on the diagonal, -1 - beta / -1 + beta on the -x /
+x neighbours, -1 elsewhere, truncated at the Dirichlet boundary) with
beta = 0.5, and every right-hand side is b = A u for a known u, so the
error of a solve is measured against the exact solution.

    tiny          16^3, 3 levels, symmetric GS, FP32 inner / FP64 outer
    mid           128^3, 4 levels, forward GS; the second start x0 ~ U(-1, 1)
    full          320^3, 4 levels, forward GS, int32 column indices (one
                  GPU's share of the paper's weak-scaling runs, Table 1)
    lowprec-fp16  256^3, matrices and multigrid vectors in binary16
    lowprec-bf16  256^3, the same in bfloat16
    batched       192^3, 8 right-hand sides b_j = A u_j, u_j ~ N(0, 1)

Every preset also runs the all-FP64 solver on the same problem, which gives
the iteration count n_d of the validation (Sec. 3.3).

    >>> from paper_2507_11512_amd import presets
    >>> P = presets.problem("mid")          # an hpgmx.Problem on the current GPU
    >>> summary = presets.run("tiny")       # solves and errors, as a dict

`bench.py --preset NAME` times a preset.
"""
from dataclasses import dataclass

from . import inputs


@dataclass(frozen=True)
class Preset:
    name: str
    n: int                       # grid edge; the problem is n^3
    levels: int
    sweep: str = "forward"       # forward | backward | symmetric
    restart: int = 30
    tol: float = 1e-9
    inner: str = "fp32"          # fp32 | fp16 | bf16 | fp16-mg | bf16-mg
    nrhs: int = 1
    cols: str = "int32"
    beta: float = 0.5
    random_start: bool = False   # also solve from x0 ~ U(-1, 1) (inputs.random_x0)
    note: str = ""

    @property
    def precision(self):
        """The Problem.solve precision name of the mixed-precision solver."""
        return "mxp" if self.inner == "fp32" else self.inner

    def bench_defaults(self):
        """Defaults of bench.py's flags for this preset."""
        return {"n": self.n, "levels": self.levels, "sweep": self.sweep, "inner": self.inner,
                "nrhs": self.nrhs, "cols": self.cols, "beta": self.beta, "restart": self.restart}


PRESETS = {p.name: p for p in [
    Preset("tiny", 16, 3, sweep="symmetric",
           note="4096 unknowns; 3-level V-cycle, one symmetric sweep before and after"),
    Preset("mid", 128, 4, random_start=True,
           note="2.1M unknowns; from x0 = 0 and from the seeded x0 ~ U(-1, 1)"),
    Preset("full", 320, 4,
           note="32.8M unknowns, ~885M nonzeros; FP32 ELL values, int32 column indices"),
    Preset("lowprec-fp16", 256, 4, inner="fp16-mg",
           note="16.8M unknowns; matrices and multigrid vectors in binary16, FP32 arithmetic"),
    Preset("lowprec-bf16", 256, 4, inner="bf16-mg",
           note="16.8M unknowns; matrices and multigrid vectors in bfloat16, FP32 arithmetic"),
    Preset("batched", 192, 4, nrhs=8,
           note="7.1M unknowns, 8 right-hand sides b_j = A u_j, u_j ~ N(0, 1) seeded"),
]}


def get(name):
    try:
        return PRESETS[name]
    except KeyError:
        raise KeyError(f"unknown preset {name!r}; known: {', '.join(sorted(PRESETS))}") from None


def problem(name, **overrides):
    """An hpgmx.Problem for the preset (keyword arguments override the
    Problem's own)."""
    from . import hpgmx
    p = get(name)
    kw = dict(beta=p.beta, levels=p.levels, sweep=p.sweep, cols=p.cols)
    kw.update(overrides)
    return hpgmx.Problem(p.n, **kw)


def exact_solutions(name):
    """The known solutions u of the preset's right-hand sides b = A u, as
    float64 numpy arrays (one per right-hand side)."""
    p = get(name)
    dims = (p.n, p.n, p.n)
    if p.nrhs == 1:
        return [inputs.ones(dims)]
    return [inputs.batch_u(dims, j) for j in range(p.nrhs)]


def run(name, max_iters=10000, fp64=True):
    """Solves the preset's problem with the mixed-precision solver (and the
    FP64 solver when fp64 is set) on the current GPU and returns, per solve,
    the iteration count, the final relative residual and the relative error
    against the exact solution."""
    import torch
    p = get(name)
    P = problem(name)
    out = {"preset": p.name, "n": p.n, "nrhs": p.nrhs, "tol": p.tol, "solves": []}
    try:
        us = [torch.from_numpy(u).cuda() for u in exact_solutions(name)]
        bs = [P.rhs_from_x(u) for u in us]
        precs = [("mxp", p.precision)] + ([("fp64", "fp64")] if fp64 else [])
        starts = [("zero", None)]
        if p.random_start:
            starts.append(("random", torch.from_numpy(inputs.random_x0((p.n, p.n, p.n))).cuda()))
        for label, prec in precs:
            for start, x0 in starts:
                if p.nrhs == 1:
                    x, st = P.solve(bs[0], x0=x0, tol=p.tol, restart=p.restart, max_iters=max_iters,
                                    precision=prec, graph=True)
                    xs, sts = [x], [st]
                else:
                    X, sts = P.solve_batched(torch.stack(bs), tol=p.tol, restart=p.restart,
                                             max_iters=max_iters, precision=prec, graph=True)
                    xs = list(X)
                for j, (x, st) in enumerate(zip(xs, sts)):
                    out["solves"].append({
                        "solver": label, "precision": prec, "start": start, "rhs": j,
                        "iters": st.iters, "converged": bool(st.converged),
                        "rel_res": st.final_rel_res,
                        "rel_err": ((x - us[j]).norm() / us[j].norm()).item()})
    finally:
        P.close()
    return out
