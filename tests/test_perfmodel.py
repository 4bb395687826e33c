"""Checks of the benchmark accounting (flop/byte models and the penalty)."""
import json
import os

from paper_2507_11512_amd import perfmodel as pm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_validation.json")


def test_penalty_reproduces_the_printed_ratio():
    g = json.load(open(GOLDEN))
    one = g["one_node"]
    assert round(pm.penalty(one["n_d"], one["n_ir"]), 3) == one["standard_ratio_printed"]
    for row in g["table2_fullscale"]:
        # a ratio above one gives no bonus, below one it is the factor itself
        n_ir = 1000
        n_d = round(row["ratio"] * n_ir)
        assert pm.penalty(n_d, n_ir) == min(1.0, n_d / n_ir)
        assert pm.penalty(n_d, n_ir) <= 1.0


def test_nnz_counts():
    assert pm.nnz((320, 320, 320)) == 879217912
    assert pm.nnz((128, 128, 128)) == 55742968
    assert pm.nnz((16, 16, 16)) == 97336
    # rows at the injection points: interior rows have 27 entries, rows on
    # the low faces fewer (the high faces hold no injection points)
    assert pm.nnz_coarse_rows((4, 4, 4)) == 5 ** 3


def test_zero_guess_slots_average_half():
    fwd = [pm.zero_guess_active_slots(c, True) for c in range(8)]
    bwd = [pm.zero_guess_active_slots(c, False) for c in range(8)]
    assert fwd[0] == 0 and fwd[7] == 26 and sum(fwd) == 8 * 13
    assert [a + b for a, b in zip(fwd, bwd)] == [26] * 8


def test_fixed_iteration_cycles_and_flops():
    assert pm.fixed_iteration_cycles(300, 30) == [30] * 10
    assert pm.fixed_iteration_cycles(31, 30) == [30, 1]
    cfg = pm.Config(dims=(320, 320, 320))
    f = pm.solve_flops(cfg, [30] * 10)
    # about 10.5 GFLOP per inner step at 320^3 (SpMV, two GS sweeps per
    # level, CGS2 of 8 k N flops)
    assert 2.9e12 < f < 3.3e12


def test_batched_bytes_reduce_to_single_at_k1():
    for dt in (0, 1):
        assert pm.bspmv_bytes(1000, dt, 1) == pm.spmv_bytes(1000, dt)
        assert pm.bgs_colour_bytes(1000, 13, dt, 1) == pm.gs_colour_bytes(1000, 13, dt)
        assert pm.brestrict_bytes(1000, dt, 1) == pm.restrict_bytes(1000, dt)
        assert pm.bprolong_bytes(1000, dt, 1) == pm.prolong_bytes(1000, dt)
    assert pm.bresid64_bytes(1000, 1) == pm.resid64_bytes(1000)
    # FP32, k = 8: the matrix (216 B/row) is shared, 8 vectors of 4 B in and out
    assert pm.bspmv_bytes(1, 1, 8) == 26 * 8 + 4 + 2 * 8 * 4


def test_single_vector_row_bytes():
    # FP32 SpMV: 26 (4 + 4) + 4 + 4 + 4; GS pass: 26 (4 + 4) + 4 + 3 * 4
    assert pm.spmv_bytes(1, 1) == 220 and pm.gs_colour_bytes(1, 26, 1) == 224
    # with 16-bit column offsets: 26 (4 + 2) + 12 and 26 (4 + 2) + 16
    assert pm.spmv_bytes(1, 1, idx=2) == 168 and pm.gs_colour_bytes(1, 26, 1, idx=2) == 172
    # FP64: 26 (8 + 4) + 8 + 2 * 8 and 26 (8 + 4) + 8 + 3 * 8
    assert pm.spmv_bytes(1, 0) == 336 and pm.gs_colour_bytes(1, 26, 0) == 344
    # the first colour of a sweep from zero reads no neighbour: diagonal, r, z
    assert pm.gs_colour_bytes(1, 0, 1) == 12 and pm.gs_colour_bytes(1, 2, 1) == 2 * 8 + 16
    assert pm.bgs_colour_bytes(1, 0, 1, 8) == 4 + 2 * 8 * 4
