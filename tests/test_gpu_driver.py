"""The benchmark driver's validation modes (Sec. 3.3) through the HIP solver
on the GPU, against the same modes run with the CPU oracle as the solver.

fullscale: the FP64 solver is capped below the step count it needs for 1e-9
(as happens at scale in the paper), the residual tau it reached becomes the
mixed-precision target, and the mixed-precision run stops at the first
residual below tau.  The GPU's n_d and tau must be the oracle's (FP64 runs
follow the same steps: tau to the FP64 level), and n_ir must be within the
reduction-order slack of the oracle's binary32-storage run to the same tau."""
import numpy as np
import pytest

import oracle
from paper_2507_11512_amd import driver, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2507_11512_amd import hpgmx
    return hpgmx


@pytest.mark.parametrize("dims,levels,cap", [((16, 16, 16), 3, 6), ((32, 32, 32), 4, 10)])
def test_fullscale_validation_on_the_gpu(hp, dims, levels, cap):
    import torch
    P = hp.Problem(dims, beta=0.5, levels=levels, sweep="forward")
    b = oracle.spmv(dims, inputs.ones(dims))
    bt = torch.from_numpy(b).cuda()
    try:
        def gpu(precision, tol, max_iters):
            x, st = P.solve(bt, tol=tol, restart=30, max_iters=max_iters, precision=precision)
            res = np.linalg.norm(b - oracle.spmv(dims, x.cpu().numpy())) / np.linalg.norm(b)
            assert abs(res - st.final_rel_res) <= 1e-6 * res
            return driver.SolveOutcome(st.iters, st.converged, st.final_rel_res, st.solve_ms / 1e3)

        def cpu(precision, tol, max_iters):
            x, st = oracle.gmres_ir(dims, b, levels=levels, sweep=0, restart=30, tol=tol, max_iters=max_iters,
                                    f32=(precision == "mxp"))
            return driver.SolveOutcome(st.iters, st.converged, st.final_rel_res, 0.0)

        v = driver.validate(gpu, "fullscale", tol=1e-9, max_iters=cap)
        w = driver.validate(cpu, "fullscale", tol=1e-9, max_iters=cap)
        print(f"[fullscale {dims}] gpu n_d={v.n_d} tau={v.tau:.6e} n_ir={v.n_ir} | "
              f"oracle n_d={w.n_d} tau={w.tau:.6e} n_ir={w.n_ir}", flush=True)
        assert v.n_d == w.n_d == cap and not v.fp64.converged
        assert abs(v.tau - w.tau) <= 1e-9 * w.tau and v.tau > 1e-9
        assert v.mxp.converged and v.mxp.final_rel_res <= v.tau
        assert abs(v.n_ir - w.n_ir) <= 2
        # standard mode on the same problem
        s = driver.validate(gpu, "standard", tol=1e-9, max_iters=10000)
        assert s.fp64.converged and s.mxp.converged and s.tau == 1e-9
        assert s.penalty == min(1.0, s.n_d / s.n_ir)
    finally:
        P.close()
