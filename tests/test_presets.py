"""The named workloads and the bench's flag defaults they set (CPU), and the
launch structure the byte model assumes for each Gauss-Seidel sweep kind."""
from collections import defaultdict

import pytest

import bench
from paper_2507_11512_amd import perfmodel as pm
from paper_2507_11512_amd import presets


def test_five_workloads():
    P = presets.PRESETS
    assert (P["tiny"].n, P["tiny"].levels, P["tiny"].sweep) == (16, 3, "symmetric")
    assert (P["mid"].n, P["mid"].levels, P["mid"].random_start) == (128, 4, True)
    assert (P["full"].n, P["full"].levels, P["full"].cols) == (320, 4, "int32")
    assert (P["lowprec-fp16"].n, P["lowprec-fp16"].inner) == (256, "fp16-mg")
    assert (P["lowprec-bf16"].n, P["lowprec-bf16"].inner) == (256, "bf16-mg")
    assert (P["batched"].n, P["batched"].nrhs) == (192, 8)
    for p in P.values():
        assert p.restart == 30 and p.tol == 1e-9 and p.beta == 0.5
        assert p.levels >= 3 and p.n % (1 << (p.levels - 1)) == 0
    with pytest.raises(KeyError):
        presets.get("nope")


def test_exact_solutions_are_the_seeded_inputs():
    assert len(presets.exact_solutions("tiny")) == 1
    assert (presets.exact_solutions("tiny")[0] == 1).all()


def test_bench_preset_defaults():
    a = bench.parse(["--preset", "tiny"])
    assert (a.n, a.levels, a.sweep, a.inner, a.nrhs) == (16, 3, "symmetric", "fp32", 1)
    a = bench.parse(["--preset", "batched", "--n", "64"])
    assert (a.n, a.nrhs) == (64, 8)     # an explicit flag wins
    a = bench.parse(["--preset", "lowprec-bf16"])
    assert (a.n, a.inner) == (256, "bf16-mg")
    a = bench.parse([])
    assert (a.n, a.levels, a.sweep, a.inner, a.nrhs, a.cols) == (320, 4, "forward", "fp32", 1, "int32")


class _K:
    """Kernel ids as the byte tables use them."""
    K_GS, K_GS_ZERO, K_RESTRICT, K_PROLONG = "gs", "gs_zero", "restrict", "prolong"


def launch_counts(cfg):
    """Launches per (kernel, level) of one V-cycle, by counting through the
    byte model's own structure."""
    B = defaultdict(float)
    bench.vcycle_bytes(cfg, B, _K, pm, lambda rows, slots: 1, lambda rc, slots: 1000 + slots,
                       lambda rc: 1, lambda rc: 1)
    return dict(B)


def test_launch_structure_per_sweep_kind():
    d = (32, 32, 32)
    f = launch_counts(pm.Config(dims=d, levels=3, sweep=0))
    assert f[("gs_zero", 0)] == 8 and f[("gs", 0)] == 8          # zero-guess pre, full post
    assert f[("gs_zero", 2)] == 8 and ("gs", 2) not in f or f[("gs", 2)] == 0
    assert f[("restrict", 0)] == 1008                            # shortcut after a forward sweep
    b = launch_counts(pm.Config(dims=d, levels=3, sweep=1))
    assert b[("restrict", 1)] == 1018                            # 18 slots after a backward sweep
    s = launch_counts(pm.Config(dims=d, levels=3, sweep=2))
    # symmetric: forward half from zero (8), its backward half (7), post sweep 8 + 7
    assert s[("gs_zero", 0)] == 8 and s[("gs", 0)] == 7 + 15
    assert s[("gs_zero", 2)] == 8 and s[("gs", 2)] == 7
    assert s[("restrict", 0)] == 1 and s[("prolong", 0)] == 1    # the general restriction
    two = launch_counts(pm.Config(dims=d, levels=3, pre=2, post=0, sweep=0))
    assert two[("gs", 0)] == 8 and two[("restrict", 0)] == 1


def test_forward_tables_unchanged():
    """The per-kernel byte table of the forward-sweep workload, against the
    level-by-level formulas written out."""
    class H:
        K_GS, K_GS_ZERO, K_RESTRICT, K_PROLONG = 0, 1, 2, 3
        K_SPMV, K_DOT, K_CGS_DOT, K_CGS_NORM, K_RESID64, K_CAST = 4, 5, 6, 7, 8, 9
        K_FINISH, K_GEMV, K_UPDATE, K_PERMUTE = 10, 11, 12, 13
        F16_MG, BF16_MG = 4, 5
    cfg = pm.Config(dims=(64, 64, 64), levels=3, sweep=0)
    T = bench.kernel_bytes_table(cfg, [5], 1, H, pm, spmv_in_sweep=0)
    V = 6  # V-cycles: 5 inner steps + the end of the cycle
    for l, d in enumerate(pm.level_dims(cfg.dims, 3)):
        cr = pm.nrows(d) // 8
        zero = sum(pm.gs_colour_bytes(cr, pm.zero_guess_active_slots(c), 1) for c in range(8))
        assert T[(H.K_GS_ZERO, l)] == pytest.approx(V * zero)
        full = 8 * pm.gs_colour_bytes(cr, 26, 1) if l < 2 else 0
        assert T.get((H.K_GS, l), 0) == pytest.approx(V * full)


def test_fused_spmv_rows_in_the_tables():
    """The last colour's rows of w move from the SpMV to the last colour
    launch: the SpMV loses their row bytes, the GS launch gains the write of
    w, once per inner step."""
    class H:
        K_GS, K_GS_ZERO, K_RESTRICT, K_PROLONG = 0, 1, 2, 3
        K_SPMV, K_DOT, K_CGS_DOT, K_CGS_NORM, K_RESID64, K_CAST = 4, 5, 6, 7, 8, 9
        K_FINISH, K_GEMV, K_UPDATE, K_PERMUTE = 10, 11, 12, 13
        F16_MG, BF16_MG = 4, 5
    cfg = pm.Config(dims=(64, 64, 64), levels=3, sweep=0)
    sep = bench.kernel_bytes_table(cfg, [5], 1, H, pm, spmv_in_sweep=0)
    last = bench.kernel_bytes_table(cfg, [5], 1, H, pm, spmv_in_sweep=1)
    B = 64 ** 3 // 8
    assert last[(H.K_GS, 0)] - sep[(H.K_GS, 0)] == 5 * B * 4
    assert sep[(H.K_SPMV, 0)] - last[(H.K_SPMV, 0)] == 5 * pm.spmv_bytes(B, 1)
    # with partial sums: colours 2 ... 6 leave 20, 18, 8, 6 and 2 slots to the SpMV
    split = bench.kernel_bytes_table(cfg, [5], 1, H, pm)
    assert split[(H.K_GS, 0)] - sep[(H.K_GS, 0)] == 5 * 6 * B * 4
    row = lambda ls: ls * 8 + 4 + 4 + 2 * 4
    assert sep[(H.K_SPMV, 0)] - split[(H.K_SPMV, 0)] == 5 * (6 * pm.spmv_bytes(B, 1) -
                                                             B * sum(map(row, (20, 18, 8, 6, 2))))
    one = pm.Config(dims=(64, 64, 64), levels=1, sweep=0)   # no post-sweep on level 0: nothing fused
    assert bench.kernel_bytes_table(one, [5], 1, H, pm) == bench.kernel_bytes_table(one, [5], 1, H, pm,
                                                                                  spmv_in_sweep=0)
