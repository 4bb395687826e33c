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
