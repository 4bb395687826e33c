#!/usr/bin/env python3
"""HPG-MxP-style benchmark of the MI355X GMRES-IR / multigrid hot path.

Workload: one GPU's full share of the paper's runs (Table 1): a 320^3 grid,
nonsymmetric 27-point stencil (beta = 0.5), b = A 1, x0 = 0, GMRES(30),
4-level V-cycle with one forward multicolour Gauss-Seidel sweep before and
after the coarse-grid correction and one on the coarsest grid, tolerance
1e-9, at most 300 inner steps per timed solve.

Phases (Sec. 3 "The HPG-MxP benchmark"):
  1. validation: FP64 GMRES to a 1e-9 relative residual gives n_d, the
     FP32-inner GMRES-IR to the same tolerance gives n_ir;
  2. timed mixed-precision phase: `--steps` solves of 300 inner steps each
     (one step = one solve), after `--warmup` untimed ones;
  3. timed FP64 phase, same shape;
  4. one profiled solve (HIP events around every launch) for per-kernel
     HBM bandwidth, a streaming-copy bandwidth reference, and the CPU oracle
     timed on a bounded sample of the same workload.
`value` = flops(model) / time of the mixed-precision solves x min(1, n_d/n_ir).

With --nrhs k (k = 2..8) the same phases run on k right-hand sides at once
through the batched solver (the batched workload: 192^3, k = 8,
b_j = A u_j with u_j ~ N(0, 1) seeded 11512 + j): the batched kernels'
tile shapes are autotuned first, `value` is the aggregate rate over the k
right-hand sides, and n_d, n_ir are summed over them.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MxP vs FP64 GMRES-MG GFLOP/s at 1e-9 rel. residual; kernel HBM GB/s"
PEAK_HBM_GBPS = 8000.0
FINISH_PARTIALS = 1024  # workgroups of a grid-stride reduction: partial sums per coefficient


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


SWEEP_CODE = {"forward": 0, "backward": 1, "symmetric": 2}


def parse(argv=None):
    from paper_2507_11512_amd import presets
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--preset", choices=sorted(presets.PRESETS), default=None,
                    help="a named workload; sets the defaults of --n, --levels, --sweep, --inner, --nrhs, "
                         "--cols and --beta (flags given explicitly still win)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=320, help="grid edge (the workload is n^3)")
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--sweep", choices=["forward", "backward", "symmetric"], default="forward",
                    help="Gauss-Seidel sweep of the smoother (one pre-, one post-sweep per level)")
    ap.add_argument("--beta", type=float, default=0.5,
                    help="nonsymmetry of the stencil's x-neighbour entries (0: the symmetric member)")
    ap.add_argument("--iters", type=int, default=300, help="inner steps per timed solve")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--cpu-iters", type=int, default=30, help="inner steps of the CPU-oracle sample (30: one restart cycle)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-cpu-extra", action="store_true",
                    help="CPU baseline: only the one-cycle sample (skip the 16^3/128^3 solves and the 1-thread run)")
    ap.add_argument("--no-validation", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the timed FP64 phase")
    ap.add_argument("--no-profile", action="store_true", help="skip the HIP-event kernel profile")
    ap.add_argument("--inner", choices=["fp32", "fp16", "bf16", "fp16-mg", "bf16-mg"], default="fp32",
                    help="inner precision of the mixed-precision solver (fp16/bf16: 16-bit matrices; "
                         "fp16-mg/bf16-mg: matrices and multigrid work vectors in 16 bits)")
    ap.add_argument("--cols", choices=["int32", "offset16"], default="int32",
                    help="storage of the ELL column indices (int32, or 16-bit offsets; single right-hand side only)")
    ap.add_argument("--eager", action="store_true",
                    help="launch every kernel from the host instead of replaying captured inner steps")
    ap.add_argument("--nrhs", type=int, default=1,
                    help="right-hand sides solved at once (>1: the batched solver)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched runs: keep the library's fixed tile rule")
    ap.add_argument("--validation", choices=["standard", "fullscale"], default="standard",
                    help="validation mode (Sec. 3.3); fullscale: MxP must reach the residual the FP64 "
                         "solver reached within --val-max-iters")
    ap.add_argument("--val-max-iters", type=int, default=10000, help="FP64 iteration limit of the validation")
    ap.add_argument("--duration", type=float, default=None,
                    help="fill this many seconds per timed phase with solves instead of running --steps "
                         "(the benchmark's official running time is 1800 s)")
    ap.add_argument("--report", default=None, help="write the benchmark report (text) to this path")
    pre, _ = ap.parse_known_args(argv)
    if pre.preset:
        ap.set_defaults(**presets.PRESETS[pre.preset].bench_defaults())
    return ap.parse_args(argv)


def vcycle_bytes(cfg, B, hp, pm, colour, restrict_after, restrict_full, prolong):
    """Adds the algorithmic bytes of one V-cycle to B[(kernel id, level)].
    colour(rows, slots): one colour launch over `rows` rows reading `slots`
    off-diagonal slots; restrict_after(rc, slots): the restriction after a
    single sweep from zero; restrict_full(rc), prolong(rc): the general
    restriction and the prolongation onto rc coarse rows."""
    L = pm.level_dims(cfg.dims, cfg.levels)
    fwd, sym = cfg.sweep != 1, cfg.sweep == 2
    per_sweep = 15 if sym else 8   # the backward half of a symmetric sweep skips its first colour
    for l, d in enumerate(L):
        cr = pm.nrows(d) // 8      # even dims on every level but possibly the coarsest
        coarsest = l == cfg.levels - 1
        nsw = cfg.coarsest if coarsest else cfg.pre
        if nsw > 0:                # the first sweep starts from zero
            for c in range(8):
                B[(hp.K_GS_ZERO, l)] += colour(cr, pm.zero_guess_active_slots(c, fwd))
            if sym:
                B[(hp.K_GS, l)] += 7 * colour(cr, pm.SLOTS)
        full = max(nsw - 1, 0) + (0 if coarsest else cfg.post)
        B[(hp.K_GS, l)] += full * per_sweep * colour(cr, pm.SLOTS)
        if not coarsest:
            rc = pm.nrows(L[l + 1])
            # one forward (backward) sweep from zero: the restriction reads 8 (18) slots
            B[(hp.K_RESTRICT, l)] += (restrict_after(rc, 8 if fwd else 18) if cfg.pre == 1 and not sym
                                      else restrict_full(rc))
            B[(hp.K_PROLONG, l)] += prolong(rc)


def kernel_bytes_table(cfg, cycles, dtype, hp, pm, idx=4, spmv_in_sweep=2):
    """Algorithmic bytes per (kernel id, level) over one solve with the given
    cycles (idx: bytes of a stored column index).  spmv_in_sweep as the
    library's layout setting: with 1 the last colour launch of each inner
    V-cycle also writes its colour's rows of w = A z and the SpMV covers the
    other 7/8 of the rows; with 2 (the default) the launches at sweep
    positions 2-6 also write partial sums of their rows, and the SpMV reads
    only the remaining slots of those rows."""
    from collections import defaultdict
    B = defaultdict(float)

    def vcyc():
        vcycle_bytes(cfg, B, hp, pm,
                     lambda rows, slots: pm.gs_colour_bytes(rows, slots, dtype, idx),
                     lambda rc, slots: pm.restrict_after_sweep_bytes(rc, dtype, slots, idx=idx),
                     lambda rc: pm.restrict_bytes(rc, dtype, idx),
                     lambda rc: pm.prolong_bytes(rc, dtype))

    N = pm.nrows(cfg.dims)
    w = pm.wb(dtype)
    fused = spmv_in_sweep in (1, 2) and cfg.levels > 1 and cfg.post >= 1
    split = fused and spmv_in_sweep == 2
    last = N // 8 if fused else 0   # rows of the last colour (even grids)
    fwd = cfg.sweep == 0
    # sweep positions 2-6: slots left to the SpMV
    late = [26 - pm.zero_guess_active_slots(c if fwd else 7 - c, fwd) for c in range(2, 7)] if split else []
    mg16 = dtype in (hp.F16_MG, hp.BF16_MG)
    cast_mg = N * (w + pm.mgb(dtype)) if mg16 else 0   # scaled 16-bit copy of the V-cycle input
    for kk in cycles:
        B[(hp.K_RESID64, 0)] += pm.resid64_bytes(N, idx)
        B[(hp.K_CAST, 0)] += N * (8 + w)
        B[(hp.K_FINISH, 0)] += FINISH_PARTIALS * 8                   # the residual's norm
        for k in range(kk):
            B[(hp.K_CAST, 0)] += cast_mg
            vcyc()
            B[(hp.K_GS, 0)] += last * w * (1 + len(late))   # fused rows of w, partial sums
            B[(hp.K_SPMV, 0)] += pm.spmv_bytes(N - last * (1 + len(late)), dtype, idx)
            for ls in late:
                B[(hp.K_SPMV, 0)] += pm.spmv_split_bytes(last, ls, dtype, idx)
            B[(hp.K_DOT, 0)] += pm.bdot_bytes(N, k + 1, dtype, 1)
            B[(hp.K_CGS_DOT, 0)] += pm.cgs_dot_bytes(N, k + 1, dtype)
            B[(hp.K_CGS_NORM, 0)] += pm.cgs_pass_bytes(N, k + 1, dtype)
            B[(hp.K_FINISH, 0)] += FINISH_PARTIALS * 8 * (2 * (k + 1) + 1)  # partial sums read
        B[(hp.K_GEMV, 0)] += N * (kk + 1) * w
        B[(hp.K_CAST, 0)] += cast_mg
        vcyc()
        B[(hp.K_UPDATE, 0)] += N * (16 + pm.mgb(dtype))
    B[(hp.K_RESID64, 0)] += pm.resid64_bytes(N, idx)
    B[(hp.K_PERMUTE, 0)] += 3 * 2 * N * 8
    return B


def kernel_bytes_table_batched(cfg, cycles, dtype, K, hp, pm, spmv_in_sweep=2):
    """As kernel_bytes_table for K right-hand sides in lockstep (the partial
    SpMV sums of spmv_in_sweep = 2 for FP32 and FP64 batches)."""
    from collections import defaultdict
    B = defaultdict(float)

    def vcyc():
        vcycle_bytes(cfg, B, hp, pm,
                     lambda rows, slots: pm.bgs_colour_bytes(rows, slots, dtype, K),
                     lambda rc, slots: pm.restrict_after_sweep_bytes(rc, dtype, slots, K),
                     lambda rc: pm.brestrict_bytes(rc, dtype, K),
                     lambda rc: pm.bprolong_bytes(rc, dtype, K))

    N = pm.nrows(cfg.dims)
    w = pm.wb(dtype)
    split = spmv_in_sweep in (2,) and dtype in (0, 1) and cfg.levels > 1 and cfg.post >= 1
    last = N // 8 if split else 0
    fwd = cfg.sweep == 0
    late = [26 - pm.zero_guess_active_slots(c if fwd else 7 - c, fwd) for c in range(2, 7)] if split else []
    v = pm.vb(dtype)
    for kk in cycles:
        B[(hp.K_RESID64, 0)] += pm.bresid64_bytes(N, K)
        B[(hp.K_CAST, 0)] += N * K * (8 + w)
        for k in range(kk):
            vcyc()
            B[(hp.K_GS, 0)] += last * K * w * (1 + len(late))   # fused rows of w, partial sums
            B[(hp.K_SPMV, 0)] += pm.bspmv_bytes(N - last * (1 + len(late)), dtype, K)
            for ls in late:   # remaining slots, diagonal, x, partial sums read, y written
                B[(hp.K_SPMV, 0)] += last * (ls * (v + pm.IDX) + v + 3 * K * w)
            B[(hp.K_DOT, 0)] += pm.bdot_bytes(N, k + 1, dtype, K)
            B[(hp.K_CGS_DOT, 0)] += K * pm.cgs_dot_bytes(N, k + 1, dtype)
            B[(hp.K_CGS_NORM, 0)] += K * pm.cgs_pass_bytes(N, k + 1, dtype)
        B[(hp.K_GEMV, 0)] += N * K * (kk + 1) * w
        vcyc()
        B[(hp.K_UPDATE, 0)] += N * K * (16 + w)
    B[(hp.K_RESID64, 0)] += pm.bresid64_bytes(N, K)
    B[(hp.K_PERMUTE, 0)] += 3 * 2 * N * K * 8
    return B


def source_sha():
    h = hashlib.sha256()
    for f in ("stencil_kernels.hip", "krylov_kernels.hip", "krylov_batch.hip", "batch_kernels.hip",
              "hpgmx_internal.hpp", "ell_device.hpp", "krylov_device.hpp"):
        with open(os.path.join(ROOT, "paper_2507_11512_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, kernel_name):
    """HBM bytes per launch from committed rocprofv3 counter runs of this
    workload ("320^3", "192^3x8"), if they were taken on the current kernel
    sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("source_sha") != source_sha():
        return None
    k = t.get("workloads", {}).get(workload, {}).get("kernels", {}).get(kernel_name)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the solver runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2507_11512_amd import hpgmx as hp
    from paper_2507_11512_amd import perfmodel as pm

    torch.cuda.set_device(0)
    if args.nrhs > 1:
        return run_batched(args, hp, pm, torch, np)
    graph = not args.eager
    PREC = {"fp64": "fp64", "mxp": args.inner}
    n, L, m = args.n, args.levels, args.restart
    cfg = pm.Config(dims=(n, n, n), levels=L, pre=1, post=1, coarsest=1, sweep=SWEEP_CODE[args.sweep], restart=m)
    N = n ** 3
    log(f"setup {n}^3 levels={L} (device: {torch.cuda.get_device_name(0)})")
    t = time.time()
    P = hp.Problem(n, beta=args.beta, levels=L, sweep=args.sweep, cols=args.cols)
    idx = 2 if args.cols == "offset16" else 4
    b = P.rhs_from_x(torch.ones(N, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    log(f"setup done in {time.time() - t:.2f}s")

    # ---- 1. validation ---------------------------------------------------------------
    from paper_2507_11512_amd import driver
    n_d = n_ir = None
    val = {}
    validation = None
    if not args.no_validation:
        xs = {}

        def solve(prec, tol, max_iters):
            x, st = P.solve(b, tol=tol, restart=m, max_iters=max_iters, precision=PREC[prec], graph=graph)
            err = (x - 1.0).norm().item() / (N ** 0.5)
            xs[prec] = x
            val[prec] = {"iters": st.iters, "restarts": st.restarts, "converged": st.converged,
                         "final_rel_res": st.final_rel_res, "time_to_tol_s": st.solve_ms / 1e3, "tol": tol,
                         "x_err_vs_ones": err}
            log(f"validation {prec}: tol={tol:.3e} iters={st.iters} res={st.final_rel_res:.3e} "
                f"|x-1|/|1|={err:.3e} time={st.solve_ms / 1e3:.3f}s")
            return driver.SolveOutcome(st.iters, st.converged, st.final_rel_res, st.solve_ms / 1e3)
        validation = driver.validate(solve, args.validation, tol=1e-9, max_iters=args.val_max_iters)
        val["mode"] = args.validation
        val["tau"] = validation.tau
        val["mxp"]["x_err_vs_fp64"] = ((xs["mxp"] - xs["fp64"]).norm() / xs["fp64"].norm()).item()
        del xs
        n_d, n_ir = validation.n_d, validation.n_ir
    penalty = pm.penalty(n_d, n_ir)

    # ---- 2./3. timed phases ------------------------------------------------------------------
    cycles = pm.fixed_iteration_cycles(args.iters, m)
    flops = pm.solve_flops(cfg, cycles)
    res = {}
    phases = {}
    for prec in (("mxp",) if args.no_fp64 else ("mxp", "fp64")):
        for _ in range(args.warmup):
            P.solve(b, tol=0.0, restart=m, max_iters=args.iters, precision=PREC[prec], graph=graph)
        torch.cuda.synchronize()

        def once():
            _, st = P.solve(b, tol=0.0, restart=m, max_iters=args.iters, precision=PREC[prec], graph=graph)
            assert st.iters == args.iters
        ph = timed(driver, once, args, torch)
        phases["mxp" if prec == "mxp" else "double"] = ph
        dt = ph.seconds_per_solve
        res[prec] = {"s_per_solve": dt, "gflops_raw": flops / dt / 1e9, "solves": ph.solves}
        log(f"timed {prec}: {ph.solves} solves, {dt * 1e3:.1f} ms/solve ({args.iters} iters) -> "
            f"{flops / dt / 1e9:.1f} GFLOP/s raw")
    value = res["mxp"]["gflops_raw"] * penalty
    fp64_gflops = res["fp64"]["gflops_raw"] if "fp64" in res else None

    # ---- 4a. per-kernel profile (HIP events around each launch) ---------------------------
    kernels = {}
    dominant = None
    inner_code = {"fp32": hp.F32, "fp16": hp.F16, "bf16": hp.BF16, "fp16-mg": hp.F16_MG,
                  "bf16-mg": hp.BF16_MG}[args.inner]
    prof_precs = () if args.no_profile else (("mxp", inner_code),) if args.no_fp64 else (("mxp", inner_code), ("fp64", hp.F64))
    for prec, dt_code in prof_precs:
        _, st = P.solve(b, tol=0.0, restart=m, max_iters=args.iters, precision=PREC[prec], profile=True)
        profile_kernels(hp, P.h, kernel_bytes_table(cfg, cycles, dt_code, hp, pm, idx), prec, kernels)
        log(f"profiled {prec} solve: {st.solve_ms:.1f} ms with events")
    mxp_k = {k: v for k, v in kernels.items() if k.endswith("_mxp")}
    dom_name = max(mxp_k, key=lambda k: mxp_k[k]["total_ms"]) if mxp_k else None
    dominant = mxp_k[dom_name] if mxp_k else None
    for k, v in sorted(mxp_k.items(), key=lambda kv: -kv[1]["total_ms"])[:10]:
        log(f"  {k:24s} {v['total_ms']:9.2f} ms  {v['launches']:6d} launches  {v['GBps']:7.1f} GB/s")

    # ---- 4b. streaming copy reference ---------------------------------------------------------
    nbytes = 1 << 31
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    cms = hp.stream_copy(P.h, src, dst, nbytes, reps=10)
    copy_gbps = 2 * nbytes / (cms / 1e3) / 1e9
    del src, dst
    log(f"stream copy: {copy_gbps:.1f} GB/s (read+write)")

    # ---- 4c. CPU oracle on a bounded sample ------------------------------------------------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, n, N, L, m, cfg, pm, np)

    traffic = load_traffic(f"{n}^3" + ("" if args.cols == "int32" else " offset16"), dom_name) if dominant else None
    if args.report:
        write_report(args.report, driver,
                     {"grid": f"{n} x {n} x {n} ({N} unknowns)",
                      "operator": f"27-point stencil, beta = {args.beta:g}, Dirichlet-truncated",
                      "solver": f"GMRES({m})-IR, {args.inner} inner / fp64 outer; {L}-level V-cycle, "
                                f"{args.sweep} multicolour Gauss-Seidel 1/1/1",
                      "inner steps per timed solve": args.iters,
                      "launch": "eager" if args.eager else "hipGraph per inner step",
                      "device": torch.cuda.get_device_name(0)},
                     validation, phases, flops, kernels, L)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": res["mxp"]["solves"],
        "warmup": args.warmup,
        "ms_per_step": round(res["mxp"]["s_per_solve"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f32 (f16 matrices)", "bf16": "f32 (bf16 matrices)",
                  "fp16-mg": "f32 (f16 matrices and multigrid vectors)",
                  "bf16-mg": "f32 (bf16 matrices and multigrid vectors)"}[args.inner]
                 + "-inner/f64-outer",
        "data": "synthetic: generated 27-point stencil, b = A*1, x0 = 0",
        "config": {"workload": f"hpg-mxp {n}^3 27-pt nonsym beta={args.beta:g}, GMRES({m})-IR ({args.inner} inner), {L}-level "
                               f"V-cycle {args.sweep} multicolour GS 1/1/1, {args.iters} inner steps per solve",
                   "grid": [n, n, n], "unknowns": N, "restart": m, "levels": L, "sweep": args.sweep,
                   "iters_per_solve": args.iters, "column_indices": args.cols,
                   "launch": "eager" if args.eager else "hipGraph per inner step"},
        "fp64_gflops": round(fp64_gflops, 2) if fp64_gflops else None,
        "speedup_vs_fp64": round(value / fp64_gflops, 4) if fp64_gflops else None,
        "raw_speedup_vs_fp64": round(res["mxp"]["gflops_raw"] / fp64_gflops, 4) if fp64_gflops else None,
        "penalty": round(penalty, 4),
        "n_d": n_d, "n_ir": n_ir,
        "validation": val,
        "fp64_ms_per_step": round(res["fp64"]["s_per_solve"] * 1e3, 3) if "fp64" in res else None,
        "flops_per_solve": flops,
        "solve_bytes": solve_rates(cfg, cycles, inner_code, res, penalty, hp, pm, idx),
        "roofline": {"bound": "hbm", "kernel": dom_name,
                     "achieved": dominant["GBps"] if dominant else None, "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": dominant["frac_peak"] if dominant else None,
                     "bytes_per_launch": dominant["bytes_per_launch"] if dominant else None,
                     "avg_us": dominant["avg_us"] if dominant else None,
                     "traffic": traffic, "copy_GBps": round(copy_gbps, 1)},
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    P.close()
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(args, n, N, L, m, cfg, pm, np):
    """The FP64 CPU oracle timed on the host: one restart cycle of the
    workload on every host thread (the reported value), plus full solves of
    the 16^3 and 128^3 configurations to 1e-9 and a one-thread sample."""
    import oracle
    threads = oracle.num_threads()
    bh = oracle.spmv(n, np.ones(N), beta=args.beta)
    t0 = time.perf_counter()
    oracle.gmres_ir(n, bh, levels=L, sweep=cfg.sweep, restart=m, max_iters=args.cpu_iters, tol=0.0, beta=args.beta)
    dt = time.perf_counter() - t0
    cflops = pm.solve_flops(cfg, [args.cpu_iters])
    cpu = {"value": round(cflops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"{n}^3 FP64 oracle, one GMRES({m}) cycle cut at {args.cpu_iters} inner steps "
                     f"(2 outer residuals, {args.cpu_iters} V-cycle+SpMV+CGS2 steps, end-of-cycle "
                     f"V-cycle), {dt:.1f} s wall", "cpu_model": cpu_model()}
    log(f"cpu oracle: {cpu['value']} GFLOP/s on {threads} threads ({dt:.1f}s)")
    runs = []

    def full(nn, levels, sweep, nthreads):
        oracle.set_num_threads(nthreads)
        c = pm.Config(dims=(nn, nn, nn), levels=levels, pre=1, post=1, coarsest=1, sweep=sweep, restart=m)
        b = oracle.spmv(nn, np.ones(nn ** 3), beta=args.beta)
        t = time.perf_counter()
        _, st = oracle.gmres_ir(nn, b, levels=levels, sweep=sweep, restart=m, tol=1e-9, beta=args.beta)
        t = time.perf_counter() - t
        cyc = pm.fixed_iteration_cycles(st.iters, m)
        runs.append({"sample": f"{nn}^3 full FP64 solve to 1e-9 ({'symmetric' if sweep == 2 else 'forward'} GS)",
                     "threads": nthreads, "seconds": round(t, 3), "iters": st.iters,
                     "GFLOP/s": round(pm.solve_flops(c, cyc) / t / 1e9, 3)})
        log(f"cpu oracle: {runs[-1]}")

    if not args.no_cpu_extra:
        full(16, 3, 2, threads)
        full(128, 4, 0, threads)
        oracle.set_num_threads(1)
        c = pm.Config(dims=(128, 128, 128), levels=4, pre=1, post=1, coarsest=1, sweep=0, restart=m)
        b = oracle.spmv(128, np.ones(128 ** 3), beta=args.beta)
        t = time.perf_counter()
        oracle.gmres_ir(128, b, levels=4, sweep=0, restart=m, max_iters=m, tol=0.0, beta=args.beta)
        t = time.perf_counter() - t
        runs.append({"sample": f"128^3 FP64 oracle, one GMRES({m}) cycle", "threads": 1, "seconds": round(t, 3),
                     "GFLOP/s": round(pm.solve_flops(c, [m]) / t / 1e9, 3)})
        log(f"cpu oracle: {runs[-1]}")
        full(16, 3, 2, 1)
        oracle.set_num_threads(threads)
    cpu["more"] = runs
    return cpu


def solve_rates(cfg, cycles, inner_code, res, penalty, hp, pm, idx=4):
    """Algorithmic bytes of a whole fixed-iteration solve and the rate at
    which each solver moved them; equal_efficiency_speedup is what the byte
    model alone predicts (both solvers at the same GB/s), times the
    iteration penalty."""
    out = {}
    for prec, code in (("mxp", inner_code), ("fp64", hp.F64)):
        nbytes = sum(v for (kid, _), v in kernel_bytes_table(cfg, cycles, code, hp, pm, idx).items()
                     if kid != hp.K_FINISH)
        out[prec] = {"bytes": nbytes}
        if prec in res:
            out[prec]["GBps"] = round(nbytes / res[prec]["s_per_solve"] / 1e9, 1)
    out["equal_efficiency_speedup"] = round(out["fp64"]["bytes"] / out["mxp"]["bytes"] * penalty, 4)
    return out


def timed(driver, once, args, torch):
    """One timed phase: --steps solves, or --duration seconds of them."""
    def run():
        once()
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    if args.duration is not None:
        return driver.timed_phase(run, duration=args.duration)
    return driver.timed_phase(run, steps=args.steps)


def write_report(path, driver, problem, validation, phases, flops, kernels, levels):
    """The benchmark report; motif times per solve from the profiled solves."""
    motifs = {}
    for tag, name in (("mxp", "mxp"), ("fp64", "double")):
        per = {}
        for kname, v in kernels.items():
            if not kname.endswith("_" + tag):
                continue
            base = kname.rsplit("_", 2)[0]
            per[base] = per.get(base, 0.0) + v["total_ms"]
        if per:
            motifs[name] = driver.motif_times(per)
    with open(path, "w") as f:
        f.write(driver.report(problem, validation, phases, flops, motifs))
    log(f"report written to {path}")


def profile_kernels(hp, handle, table, prec_tag, kernels):
    for (kid, lvl), nbytes in sorted(table.items()):
        ms, cnt = hp.profile_get(handle, kid, lvl)
        if cnt == 0 or ms <= 0:
            continue
        name = f"{hp.KERNEL_NAMES[kid]}_l{lvl}_{prec_tag}"
        gbps = nbytes / (ms / 1e3) / 1e9
        kernels[name] = {"launches": cnt, "total_ms": round(ms, 4), "avg_us": round(ms / cnt * 1e3, 3),
                         "bytes_per_launch": nbytes / cnt, "GBps": round(gbps, 1),
                         "frac_peak": round(gbps / PEAK_HBM_GBPS, 4)}


def run_batched(args, hp, pm, torch, np):
    """The phases of main() for k right-hand sides in lockstep."""
    k = args.nrhs
    if k > hp.MAX_BATCH:
        raise SystemExit(f"--nrhs must be at most {hp.MAX_BATCH}")
    if args.inner.endswith("-mg"):
        raise SystemExit("batched runs keep FP32 multigrid vectors: --inner fp32, fp16 or bf16")
    if args.cols != "int32":
        raise SystemExit("batched runs read int32 column indices")
    if args.validation != "standard":
        raise SystemExit("batched runs validate in the standard mode only")
    from paper_2507_11512_amd import driver
    graph = not args.eager
    n, L, m = args.n, args.levels, args.restart
    cfg = pm.Config(dims=(n, n, n), levels=L, pre=1, post=1, coarsest=1, sweep=SWEEP_CODE[args.sweep], restart=m)
    N = n ** 3
    from paper_2507_11512_amd import inputs
    log(f"setup {n}^3 levels={L}, {k} right-hand sides (device: {torch.cuda.get_device_name(0)})")
    t = time.time()
    P = hp.Problem(n, beta=args.beta, levels=L, sweep=args.sweep)
    U_ = torch.stack([torch.from_numpy(inputs.batch_u((n, n, n), j)) for j in range(k)]).cuda()
    B = torch.empty_like(U_)
    for j in range(k):
        hp.rhs_from_x(P.h, U_[j], B[j])
    torch.cuda.synchronize()
    log(f"setup done in {time.time() - t:.2f}s")
    inner_code = {"fp32": hp.F32, "fp16": hp.F16, "bf16": hp.BF16, "fp16-mg": hp.F16_MG,
                  "bf16-mg": hp.BF16_MG}[args.inner]
    tuning = {}
    if not args.no_autotune:
        for name, code in ((args.inner, inner_code), ("fp64", hp.F64)):
            tt = hp.batch_autotune(P.h, k, code)
            tuning[name] = {hp.BK_NAMES[b]: tt["rhs_per_lane"][b][:L] for b in range(hp.BK_COUNT)}
            log(f"autotuned tiles ({name}): {tuning[name]}")

    PREC = {"fp64": "fp64", "mxp": args.inner}
    val = {}
    n_d = n_ir = None
    if not args.no_validation:
        xs = {}
        for prec in ("fp64", "mxp"):
            X, sts = P.solve_batched(B, tol=1e-9, restart=m, precision=PREC[prec], graph=graph)
            errs = [((X[j] - U_[j]).norm() / U_[j].norm()).item() for j in range(k)]
            xs[prec] = X
            val[prec] = {"iters": [s.iters for s in sts], "converged": all(s.converged for s in sts),
                         "max_final_rel_res": max(s.final_rel_res for s in sts),
                         "time_to_1e-9_s": sts[0].solve_ms / 1e3, "max_x_err_vs_u": max(errs)}
            log(f"validation {prec}: iters={val[prec]['iters']} max res={val[prec]['max_final_rel_res']:.3e} "
                f"max |x-u|/|u|={max(errs):.3e} time={sts[0].solve_ms / 1e3:.3f}s")
        val["mxp"]["max_x_err_vs_fp64"] = max(
            ((xs["mxp"][j] - xs["fp64"][j]).norm() / xs["fp64"][j].norm()).item() for j in range(k))
        del xs
        n_d, n_ir = sum(val["fp64"]["iters"]), sum(val["mxp"]["iters"])
    penalty = pm.penalty(n_d, n_ir)

    cycles = pm.fixed_iteration_cycles(args.iters, m)
    flops = k * pm.solve_flops(cfg, cycles)
    res = {}
    for prec in (("mxp",) if args.no_fp64 else ("mxp", "fp64")):
        for _ in range(args.warmup):
            P.solve_batched(B, tol=0.0, restart=m, max_iters=args.iters, precision=PREC[prec], graph=graph)
        torch.cuda.synchronize()

        def once():
            _, sts = P.solve_batched(B, tol=0.0, restart=m, max_iters=args.iters, precision=PREC[prec],
                                     graph=graph)
            assert all(s.iters == args.iters for s in sts)
        ph = timed(driver, once, args, torch)
        dt = ph.seconds_per_solve
        res[prec] = {"s_per_solve": dt, "gflops_raw": flops / dt / 1e9, "solves": ph.solves}
        log(f"timed batched {prec}: {dt * 1e3:.1f} ms per {k}-rhs solve ({args.iters} iters) -> "
            f"{flops / dt / 1e9:.1f} GFLOP/s raw")
    value = res["mxp"]["gflops_raw"] * penalty
    fp64_gflops = res["fp64"]["gflops_raw"] if "fp64" in res else None

    kernels = {}
    if not args.no_profile:
        for prec, code in (("mxp", inner_code),) + (() if args.no_fp64 else (("fp64", hp.F64),)):
            _, sts = P.solve_batched(B, tol=0.0, restart=m, max_iters=args.iters, precision=PREC[prec],
                                     profile=True)
            profile_kernels(hp, P.h, kernel_bytes_table_batched(cfg, cycles, code, 8 if k > 4 else (4 if k > 2 else 2),
                                                                hp, pm), prec, kernels)
            log(f"profiled batched {prec} solve: {sts[0].solve_ms:.1f} ms with events")
    mxp_k = {kk_: v for kk_, v in kernels.items() if kk_.endswith("_mxp")}
    dom_name = max(mxp_k, key=lambda q: mxp_k[q]["total_ms"]) if mxp_k else None
    dominant = mxp_k[dom_name] if mxp_k else None
    for name, v in sorted(mxp_k.items(), key=lambda kv: -kv[1]["total_ms"])[:12]:
        log(f"  {name:24s} {v['total_ms']:9.2f} ms  {v['launches']:6d} launches  {v['GBps']:7.1f} GB/s")

    nbytes = 1 << 31
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    cms = hp.stream_copy(P.h, src, dst, nbytes, reps=10)
    copy_gbps = 2 * nbytes / (cms / 1e3) / 1e9
    del src, dst
    log(f"stream copy: {copy_gbps:.1f} GB/s (read+write)")

    cpu = None
    if not args.no_cpu:
        import oracle
        bh = B[0].cpu().numpy()
        t0 = time.perf_counter()
        _, sto = oracle.gmres_ir(n, bh, levels=L, sweep=cfg.sweep, restart=m, max_iters=args.cpu_iters, tol=0.0,
                                 beta=args.beta)
        dt = time.perf_counter() - t0
        cflops = pm.solve_flops(cfg, [args.cpu_iters])
        cpu = {"value": round(cflops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{n}^3 FP64 oracle on right-hand side 0 alone (the oracle solves one at a time), "
                         f"one GMRES({m}) cycle cut at {args.cpu_iters} inner steps, {dt:.1f} s wall"}
        log(f"cpu oracle: {cpu['value']} GFLOP/s on {cpu['cores']} threads ({dt:.1f}s)")

    traffic = load_traffic(f"{n}^3x{k}", dom_name) if dominant else None
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": res["mxp"]["solves"],
        "warmup": args.warmup,
        "ms_per_step": round(res["mxp"]["s_per_solve"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f32 (f16 matrices)", "bf16": "f32 (bf16 matrices)",
                  "fp16-mg": "f32 (f16 matrices and multigrid vectors)",
                  "bf16-mg": "f32 (bf16 matrices and multigrid vectors)"}[args.inner]
                 + "-inner/f64-outer",
        "data": f"synthetic: generated 27-point stencil, b_j = A u_j, u_j ~ N(0,1) seeded 11512+j, x0 = 0",
        "config": {"workload": f"hpg-mxp batched {n}^3 27-pt nonsym beta={args.beta:g}, {k} right-hand sides, "
                               f"GMRES({m})-IR ({args.inner} inner), {L}-level V-cycle {args.sweep} multicolour GS 1/1/1, "
                               f"{args.iters} inner steps per solve",
                   "grid": [n, n, n], "unknowns": N, "nrhs": k, "restart": m, "levels": L,
                   "iters_per_solve": args.iters,
                   "launch": "eager" if args.eager else "hipGraph per inner step",
                   "tiles": tuning or "fixed rule"},
        "fp64_gflops": round(fp64_gflops, 2) if fp64_gflops else None,
        "speedup_vs_fp64": round(value / fp64_gflops, 4) if fp64_gflops else None,
        "raw_speedup_vs_fp64": round(res["mxp"]["gflops_raw"] / fp64_gflops, 4) if fp64_gflops else None,
        "penalty": round(penalty, 4),
        "n_d": n_d, "n_ir": n_ir,
        "validation": val,
        "fp64_ms_per_step": round(res["fp64"]["s_per_solve"] * 1e3, 3) if "fp64" in res else None,
        "flops_per_solve": flops,
        "roofline": {"bound": "hbm", "kernel": dom_name,
                     "achieved": dominant["GBps"] if dominant else None, "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": dominant["frac_peak"] if dominant else None,
                     "bytes_per_launch": dominant["bytes_per_launch"] if dominant else None,
                     "avg_us": dominant["avg_us"] if dominant else None,
                     "traffic": traffic, "copy_GBps": round(copy_gbps, 1)},
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    P.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
