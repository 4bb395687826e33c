"""Named workloads end to end on the GPU, and the launch structure of every
sweep kind against the byte model that prices it."""
import numpy as np
import pytest

import bench
import oracle
from paper_2507_11512_amd import inputs
from paper_2507_11512_amd import perfmodel as pm
from paper_2507_11512_amd import presets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2507_11512_amd import hpgmx
    return hpgmx


def test_preset_tiny(hp):
    """16^3, 3 levels, symmetric GS: both solvers reach 1e-9 with x within
    1e-8 of the exact all-ones solution, in the oracle's step counts."""
    out = presets.run("tiny")
    p = presets.get("tiny")
    b = oracle.spmv(16, inputs.ones(16))
    _, s64 = oracle.gmres_ir(16, b, levels=p.levels, sweep=2, restart=30, tol=1e-9)
    _, s32 = oracle.gmres_ir(16, b, levels=p.levels, sweep=2, restart=30, tol=1e-9, f32=True)
    print("[preset tiny] " + "; ".join(f"{s['solver']} {s['iters']} res {s['rel_res']:.2e} err {s['rel_err']:.2e}"
                                       for s in out["solves"]) + f" | oracle {s64.iters} / {s32.iters}", flush=True)
    for s in out["solves"]:
        assert s["converged"] and s["rel_res"] <= 1e-9 and s["rel_err"] <= 1e-8
        ref = s64 if s["solver"] == "fp64" else s32
        assert abs(s["iters"] - ref.iters) <= 2


def test_preset_mid(hp):
    """128^3 from x0 = 0 and from the seeded x0 ~ U(-1, 1)."""
    out = presets.run("mid")
    print("[preset mid] " + "; ".join(f"{s['solver']}/{s['start']} {s['iters']} res {s['rel_res']:.2e} "
                                      f"err {s['rel_err']:.2e}" for s in out["solves"]), flush=True)
    assert len(out["solves"]) == 4
    for s in out["solves"]:
        assert s["converged"] and s["rel_res"] <= 1e-9 and s["rel_err"] <= 1e-8
    it = {(s["solver"], s["start"]): s["iters"] for s in out["solves"]}
    assert it[("mxp", "zero")] <= it[("fp64", "zero")] + 6


@pytest.mark.parametrize("paired", [False, True])
@pytest.mark.parametrize("sweep", ["forward", "backward", "symmetric"])
def test_launch_counts_match_byte_model(hp, sweep, paired):
    """Colour launches, restrictions and prolongations per level over one
    restart cycle equal what the byte model prices (30 inner V-cycles and
    the one at the end of the cycle); with paired launches a sweep from the
    zero guess takes 4 launches instead of 8 (the bytes are the same)."""
    import torch
    from collections import defaultdict
    d = (32, 32, 32)
    code = bench.SWEEP_CODE[sweep]
    P = hp.Problem(d, beta=0.5, levels=3, sweep=sweep, layout={"pair_rows": (1 << 40) if paired else 0})
    try:
        b = P.rhs_from_x(torch.ones(32 ** 3, dtype=torch.float64, device="cuda"))
        x, st = P.solve(b, tol=0.0, restart=30, max_iters=30, precision="mxp", profile=True)
        assert st.iters == 30
        B = defaultdict(float)
        bench.vcycle_bytes(pm.Config(dims=d, levels=3, sweep=code), B, hp, pm,
                           lambda rows, slots: 1, lambda rc, slots: 1, lambda rc: 1, lambda rc: 1)
        for l in range(3):
            for kid in (hp.K_GS, hp.K_GS_ZERO, hp.K_RESTRICT, hp.K_PROLONG):
                _, n = hp.profile_get(P.h, kid, l)
                want = 31 * B.get((kid, l), 0) // (2 if paired and kid == hp.K_GS_ZERO else 1)
                assert n == want, (sweep, l, hp.KERNEL_NAMES[kid], n)
    finally:
        P.close()
