"""The benchmark driver (validation modes, timed phases, report) on the CPU,
with the oracle as the solver (Sec. 3 and Sec. 3.3).

On 16^3 (b = A 1, 3 levels, forward sweeps) the FP64 oracle reaches 1e-9 in
about 15 inner steps.  The fullscale mode is exercised by capping the FP64
run below that, which is what happens at large scale in the paper (the FP64
solver hits its iteration limit first): the mixed-precision run must then
reach the residual the capped FP64 run stopped at."""
import pytest

import oracle
from paper_2507_11512_amd import driver, inputs, perfmodel

D = (16, 16, 16)


@pytest.fixture(scope="module")
def solve():
    b = oracle.spmv(D, inputs.ones(D))

    def run(precision, tol, max_iters):
        x, st = oracle.gmres_ir(D, b, levels=3, sweep=0, restart=30, tol=tol, max_iters=max_iters,
                                f32=(precision == "mxp"))
        return driver.SolveOutcome(st.iters, st.converged, st.final_rel_res, 0.0)
    return run


def test_standard_mode_counts_are_the_solvers(solve):
    v = driver.validate(solve, "standard", tol=1e-9, max_iters=10000)
    _, sd = oracle.gmres_ir(D, oracle.spmv(D, inputs.ones(D)), levels=3, sweep=0, tol=1e-9)
    assert v.n_d == sd.iters and v.fp64.converged and v.mxp.converged
    assert v.tau == 1e-9 and v.mxp.final_rel_res < 1e-9
    assert v.penalty == perfmodel.penalty(v.n_d, v.n_ir)


def test_fullscale_mode_targets_the_capped_fp64_residual(solve):
    cap = 6
    v = driver.validate(solve, "fullscale", tol=1e-9, max_iters=cap)
    assert v.n_d == cap and not v.fp64.converged
    assert v.tau == v.fp64.final_rel_res and v.tau > 1e-9
    # the mixed-precision run goes on until it reaches tau, not 1e-9
    assert v.mxp.converged and v.mxp.final_rel_res <= v.tau
    assert v.mxp.final_rel_res > 1e-9
    # when the FP64 run converges, fullscale and standard agree
    v2 = driver.validate(solve, "fullscale", tol=1e-9, max_iters=10000)
    v3 = driver.validate(solve, "standard", tol=1e-9, max_iters=10000)
    assert (v2.n_d, v2.n_ir, v2.tau) == (v3.n_d, v3.n_ir, v3.tau)


def test_fullscale_penalty_is_capped_at_one():
    def fake(precision, tol, max_iters):
        if precision == "fp64":
            return driver.SolveOutcome(max_iters, False, 3e-6, 0.0)
        return driver.SolveOutcome(80 if tol > 3e-6 else 0, True, 2.9e-6, 0.0)
    v = driver.validate(fake, "fullscale", tol=1e-9, max_iters=100)
    assert v.tau == 3e-6 and v.n_d == 100 and v.n_ir == 80 and v.penalty == 1.0
    with pytest.raises(ValueError):
        driver.validate(fake, "bogus")


def test_timed_phase_steps_and_duration():
    t = [0.0]

    def clock():
        return t[0]

    def once():
        t[0] += 0.25
    ph = driver.timed_phase(once, steps=3, clock=clock)
    assert ph.solves == 3 and ph.seconds == pytest.approx(0.75)
    t[0] = 0.0
    ph = driver.timed_phase(once, duration=1.0, clock=clock)
    assert ph.solves == 4 and ph.seconds >= 1.0
    t[0] = 0.0
    ph = driver.timed_phase(once, duration=0.0, clock=clock)
    assert ph.solves == 1
    with pytest.raises(ValueError):
        driver.timed_phase(once)


def test_motifs_cover_every_kernel_once():
    from paper_2507_11512_amd import hpgmx
    names = hpgmx.KERNEL_NAMES
    members = [k for ks in driver.MOTIFS.values() for k in ks]
    assert sorted(members) == sorted(names)
    m = driver.motif_times({n: 1.0 for n in names})
    assert sum(m.values()) == len(names)
    with pytest.raises(KeyError):
        driver.motif_times({"mystery": 1.0})


def test_report_contains_the_phases(solve):
    v = driver.validate(solve, "fullscale", tol=1e-9, max_iters=6)
    phases = {"mxp": driver.TimedPhase(3, 3.0), "double": driver.TimedPhase(3, 6.0)}
    txt = driver.report({"grid": "16x16x16"}, v, phases, flops_per_solve=2e9,
                        motifs={"mxp": {"GS": 2.0, "SpMV": 1.0}})
    assert "Validation (fullscale)" in txt and f"{v.tau:.3e}" in txt
    assert "GFLOP/s raw: 2.00" in txt and "GFLOP/s raw: 1.00" in txt
    assert f"penalty min(1, n_d/n_ir) = {v.penalty:.4f}" in txt
    assert "Speedup mxp / double" in txt and "GS" in txt
