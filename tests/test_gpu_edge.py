"""Edge cases of the GPU path against the oracle: odd grid dimensions (the 8
colour blocks then differ in size and in their x extents), the largest
restart length (63, the 64-column basis buckets of the single and the batched
Krylov passes), one-level hierarchies and the finite termination of GMRES on
a grid smaller than the restart length.  Tolerances as in
tests/test_gpu_parity.py."""
import numpy as np
import pytest

import oracle
from paper_2507_11512_amd import inputs

pytestmark = pytest.mark.gpu

U = {0: 2.0 ** -53, 1: 2.0 ** -24}


def gamma(n, u):
    return n * u / (1.0 - n * u)


@pytest.fixture(scope="module")
def hp():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2507_11512_amd import hpgmx
    return hpgmx


def dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64 if dtype == 0 else torch.float32)


def host(t):
    return t.double().cpu().numpy()


def rnd(a, dtype):
    return a if dtype == 0 else a.astype(np.float32).astype(np.float64)


ODD = [((7, 5, 9), 1), ((14, 10, 6), 2), ((13, 3, 4), 1)]


@pytest.mark.parametrize("dims,levels", ODD)
@pytest.mark.parametrize("dtype", [0, 1])
def test_odd_grids_kernels(hp, dims, levels, dtype):
    P = hp.Problem(dims, beta=0.5, levels=levels, sweep="forward")
    print(f"[odd] dims={dims} levels={levels} dtype={dtype}", flush=True)
    x = rnd(inputs.uniform(dims, 51), dtype)
    y = dev(np.zeros(x.size), dtype)
    hp.spmv(P.h, 0, dtype, dev(x, dtype), y)
    tol = 2 * gamma(28, U[dtype]) * oracle.absrow(dims, x) + 1e-300
    assert np.all(np.abs(host(y) - oracle.spmv(dims, x)) <= tol)
    for sweep in (0, 1, 2):
        r = rnd(inputs.uniform(dims, 52), dtype)
        z0 = rnd(inputs.uniform(dims, 53), dtype)
        zt = dev(z0, dtype)
        hp.smooth(P.h, 0, dtype, sweep, dev(r, dtype), zt)
        ref = oracle.gs(dims, r, z0, sweep)
        zmax = np.maximum(np.abs(z0), np.abs(ref))
        S = (np.abs(r) + oracle.absrow(dims, zmax) - 26.0 * zmax) / 26.0
        assert np.max(np.abs(host(zt) - ref)) <= 2 * (16 if sweep == 2 else 8) * gamma(28, U[dtype]) * S.max()
    r = rnd(inputs.uniform(dims, 54), dtype)
    z = dev(np.zeros(r.size), dtype)
    hp.vcycle(P.h, dtype, dev(r, dtype), z)
    ref = oracle.vcycle(dims, r, levels, 1, 1, 1, 0)
    assert np.linalg.norm(host(z) - ref) / np.linalg.norm(ref) <= (1e-12 if dtype == 0 else 1e-4)
    P.close()


@pytest.mark.parametrize("dims,levels", ODD)
@pytest.mark.parametrize("precision", ["fp64", "mxp"])
def test_odd_grids_solve_single_and_batched(hp, dims, levels, precision):
    P = hp.Problem(dims, beta=0.5, levels=levels, sweep="forward")
    U_ = np.stack([inputs.batch_u(dims, j) for j in range(5)])
    B = np.stack([oracle.spmv(dims, u) for u in U_])
    X, stats = P.solve_batched(dev(B, 0), tol=1e-11, precision=precision)
    Xh = host(X)
    for j in range(5):
        xo, sto = oracle.gmres_ir(dims, B[j], levels=levels, sweep=0, tol=1e-11)
        xs, sts = P.solve(dev(B[j], 0), tol=1e-11, precision=precision)
        for name, xg, st in (("batched", Xh[j], stats[j]), ("single", host(xs), sts)):
            res = np.linalg.norm(B[j] - oracle.spmv(dims, xg)) / np.linalg.norm(B[j])
            dx = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
            assert st.converged and res <= 1e-9 and dx <= 1e-8, (name, j, res, dx)
        if precision == "fp64":
            assert abs(stats[j].iters - sto.iters) <= 2 and abs(sts.iters - sto.iters) <= 2
    P.close()


def test_longest_restart_single_and_batched(hp):
    """63 inner steps in one cycle (the 64-column buckets): FP64 single and
    batched solves stopped by max_iters match the oracle's 63-step iterate."""
    dims = (16, 16, 16)
    P = hp.Problem(dims, beta=0.5, levels=3, sweep="forward")
    U_ = np.stack([inputs.batch_u(dims, j) for j in range(8)])
    B = np.stack([oracle.spmv(dims, u) for u in U_])
    X, stats = P.solve_batched(dev(B, 0), tol=0.0, restart=63, max_iters=63, precision="fp64")
    Xh = host(X)
    for j in (0, 7):
        xo, sto = oracle.gmres_ir(dims, B[j], levels=3, sweep=0, restart=63, max_iters=63, tol=0.0)
        xs, sts = P.solve(dev(B[j], 0), tol=0.0, restart=63, max_iters=63, precision="fp64")
        assert sto.iters == sts.iters == stats[j].iters == 63
        for xg in (Xh[j], host(xs)):
            assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)
    # the mixed-precision path through the same buckets converges
    X, stats = P.solve_batched(dev(B, 0), tol=1e-9, restart=63, precision="mxp")
    for j in range(8):
        res = np.linalg.norm(B[j] - oracle.spmv(dims, host(X)[j])) / np.linalg.norm(B[j])
        assert stats[j].converged and res <= 1e-9
    P.close()


@pytest.mark.parametrize("precision", ["fp64", "mxp"])
def test_finite_termination_on_a_tiny_grid(hp, precision):
    """N = 8 unknowns, restart 10: FP64 GMRES ends within N steps up to
    rounding (one cycle); the FP32-inner solver needs a refinement cycle or
    two more.  Both reach the dense solution."""
    dims = (2, 2, 2)
    P = hp.Problem(dims, beta=0.5, levels=1, sweep="forward")
    b = oracle.spmv(dims, inputs.uniform(dims, 55))
    x, st = P.solve(dev(b, 0), tol=1e-13, restart=10, precision=precision)
    A = np.stack([oracle.spmv(dims, e) for e in np.eye(8)], axis=1)
    xd = np.linalg.solve(A, b)
    assert st.converged and st.iters <= (10 if precision == "fp64" else 30)
    assert np.linalg.norm(host(x) - xd) <= 1e-11 * np.linalg.norm(xd)
    P.close()
