"""Batched right-hand sides on the GPU: every batched entry point against the
oracle, right-hand side by right-hand side, and against the single-vector
entry points.

Tolerances are those of tests/test_gpu_parity.py (derived there from the
arithmetic).  In addition, per (row, right-hand side) the batched kernels do
the arithmetic of the single-vector kernels in the same order, and the tile
shape R only changes which lane does it, so
  * the batched SpMV, sweep and V-cycle of right-hand side j equal the
    single-vector results on that vector bit for bit, for every R;
  * a batched solve gives every right-hand side the steps of its own solve:
    same iteration count (up to the reduction-order slack of the single
    solve against the oracle) and a solution within the solve bar.
Inputs follow the batched recipe: u_j ~ N(0, 1) from default_rng(11512 + j),
b_j = A u_j (formed by the oracle).
"""
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


_problems = {}


def problem(hp, dims, levels, sweep="forward"):
    key = (tuple(dims), levels, sweep)
    if key not in _problems:
        print(f"[setup] dims={dims} levels={levels} sweep={sweep}", flush=True)
        _problems[key] = hp.Problem(dims, beta=0.5, levels=levels, sweep=sweep)
    return _problems[key]


def dev(a, dtype):
    import torch
    t = torch.float64 if dtype == 0 else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)


def host(t):
    return t.double().cpu().numpy()


def rnd(a, dtype):
    return a if dtype == 0 else a.astype(np.float32).astype(np.float64)


def ldims(dims, level):
    return tuple(int(d) >> level for d in dims)


def widths(nrhs):
    K = 2 if nrhs <= 2 else 4 if nrhs <= 4 else 8
    return [R for R in (1, 2, 4, 8) if R <= K]


def force_tiles(hp, P, nrhs, dtype, R):
    hp.batch_set_tuning(P.h, nrhs, dtype, R)


def _gs_tol(d, r, z_in, z_ref, dtype, passes):
    zmax = np.maximum(np.abs(z_in), np.abs(z_ref))
    S = (np.abs(r) + oracle.absrow(d, zmax) - 26.0 * zmax) / 26.0
    return 2 * passes * gamma(28, U[dtype]) * S.max()


GRIDS = [((16, 16, 16), 3), ((24, 20, 16), 3), ((12, 12, 12), 2)]


@pytest.mark.parametrize("dims,levels", GRIDS)
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_spmv_batched_every_level_and_tile(hp, dims, levels, dtype, nrhs):
    P = problem(hp, dims, levels)
    for lvl in range(levels):
        d = ldims(dims, lvl)
        X = np.stack([rnd(inputs.uniform(d, 1000 + 10 * lvl + j), dtype) for j in range(nrhs)])
        single = []
        for j in range(nrhs):
            y = dev(np.zeros(X.shape[1]), dtype)
            hp.spmv(P.h, lvl, dtype, dev(X[j], dtype), y)
            single.append(host(y))
        for R in widths(nrhs):
            force_tiles(hp, P, nrhs, dtype, R)
            Y = dev(np.zeros(X.shape), dtype)
            hp.spmv_batched(P.h, lvl, dtype, dev(X, dtype), Y)
            got = host(Y)
            for j in range(nrhs):
                ref = oracle.spmv(d, X[j])
                tol = 2 * gamma(28, U[dtype]) * oracle.absrow(d, X[j]) + 1e-300
                assert np.all(np.abs(got[j] - ref) <= tol), (lvl, R, j)
                assert np.array_equal(got[j], single[j]), (lvl, R, j)
    force_tiles(hp, P, nrhs, dtype, 0)


@pytest.mark.parametrize("dims,levels", GRIDS[:2])
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("sweep", [0, 1, 2])
@pytest.mark.parametrize("zero", [False, True])
def test_smooth_batched(hp, dims, levels, dtype, sweep, zero):
    nrhs = 5
    P = problem(hp, dims, levels)
    for lvl in range(levels):
        d = ldims(dims, lvl)
        Rh = np.stack([rnd(inputs.uniform(d, 2000 + 10 * lvl + j), dtype) for j in range(nrhs)])
        Z0 = np.zeros(Rh.shape) if zero else \
            np.stack([rnd(inputs.uniform(d, 3000 + 10 * lvl + j), dtype) for j in range(nrhs)])
        for R in (1, 8):
            force_tiles(hp, P, nrhs, dtype, R)
            Z = dev(Z0 if not zero else np.full(Rh.shape, 7.0), dtype)  # ignored when zero
            hp.smooth_batched(P.h, lvl, dtype, sweep, dev(Rh, dtype), Z, zero_guess=zero)
            got = host(Z)
            for j in range(nrhs):
                ref = oracle.gs(d, Rh[j], Z0[j], sweep)
                tol = _gs_tol(d, Rh[j], Z0[j], ref, dtype, 16 if sweep == 2 else 8)
                assert np.max(np.abs(got[j] - ref)) <= tol, (lvl, R, j)
                z1 = dev(Z0[j], dtype)
                hp.smooth(P.h, lvl, dtype, sweep, dev(Rh[j], dtype), z1, zero_guess=zero)
                assert np.array_equal(got[j], host(z1)), (lvl, R, j)
    force_tiles(hp, P, nrhs, dtype, 0)


@pytest.mark.parametrize("dims,levels,sweep", [((16, 16, 16), 3, "symmetric"),
                                               ((24, 20, 16), 3, "forward"),
                                               ((24, 20, 16), 3, "backward"),
                                               ((32, 32, 32), 4, "forward"),
                                               ((8, 8, 8), 1, "forward")])
@pytest.mark.parametrize("dtype", [0, 1])
def test_vcycle_batched(hp, dims, levels, sweep, dtype):
    nrhs = 4
    P = problem(hp, dims, levels, sweep)
    Rh = np.stack([rnd(inputs.uniform(dims, 4000 + j), dtype) for j in range(nrhs)])
    sw = {"forward": 0, "backward": 1, "symmetric": 2}[sweep]
    for R in widths(nrhs):
        force_tiles(hp, P, nrhs, dtype, R)
        Z = dev(np.zeros(Rh.shape), dtype)
        hp.vcycle_batched(P.h, dtype, dev(Rh, dtype), Z)
        got = host(Z)
        for j in range(nrhs):
            ref = oracle.vcycle(dims, Rh[j], levels, 1, 1, 1, sw)
            err = np.linalg.norm(got[j] - ref) / np.linalg.norm(ref)
            assert err <= (1e-12 if dtype == 0 else 1e-4), (R, j, err)
            z1 = dev(np.zeros(Rh.shape[1]), dtype)
            hp.vcycle(P.h, dtype, dev(Rh[j], dtype), z1)
            assert np.array_equal(got[j], host(z1)), (R, j)
    force_tiles(hp, P, nrhs, dtype, 0)


@pytest.mark.parametrize("dtype", [0, 1, 3])
@pytest.mark.parametrize("sweep", [0, 1])
def test_presmooth_restrict_batched(hp, dtype, sweep):
    """The batched pre-smoother and restriction of the V-cycle: per right-hand
    side bit-identical to the single-vector export for every tile shape, and
    within the single export's bounds against the oracle."""
    dims, levels, nrhs = (24, 20, 16), 3, 5
    P = problem(hp, dims, levels)
    for lvl in range(levels - 1):
        d = tuple(v >> lvl for v in dims)
        dc = tuple(v >> (lvl + 1) for v in dims)
        N, Nc = int(np.prod(d)), int(np.prod(dc))
        Rh = np.stack([inputs.uniform(d, 1400 + 10 * lvl + j) for j in range(nrhs)])
        if dtype != 0:
            Rh = Rh.astype(np.float32).astype(np.float64)
        for R in (1, 2, 4, 8):
            force_tiles(hp, P, nrhs, dtype, R)
            Z = dev(np.zeros((nrhs, N)), dtype)
            RC = dev(np.zeros((nrhs, Nc)), dtype)
            hp.presmooth_restrict_batched(P.h, lvl, dtype, sweep, 1, dev(Rh, dtype), Z, RC)
            Zg, RCg = host(Z), host(RC)
            for j in range(nrhs):
                z1 = dev(np.zeros(N), dtype)
                rc1 = dev(np.zeros(Nc), dtype)
                hp.presmooth_restrict(P.h, lvl, dtype, sweep, 1, dev(Rh[j], dtype), z1, rc1)
                assert np.array_equal(Zg[j], host(z1)) and np.array_equal(RCg[j], host(rc1)), (lvl, R, j)
            j = nrhs - 1
            ref = oracle.restrict_fused(d, Rh[j], Zg[j])
            scale = oracle.inject(d, np.abs(Rh[j]) + oracle.absrow(d, Zg[j]))
            assert np.all(np.abs(RCg[j] - ref) <= 3 * gamma(28, U[0 if dtype == 0 else 1]) * scale + 1e-300)
    force_tiles(hp, P, nrhs, dtype, 0)


def _batch_rhs(dims, nrhs):
    U_ = np.stack([inputs.batch_u(dims, j) for j in range(nrhs)])
    B = np.stack([oracle.spmv(dims, U_[j]) for j in range(nrhs)])
    return U_, B


@pytest.mark.parametrize("dims,levels,sweep,nrhs", [((16, 16, 16), 3, "symmetric", 8),
                                                    ((24, 20, 16), 3, "forward", 3),
                                                    ((32, 32, 32), 4, "forward", 8)])
@pytest.mark.parametrize("precision", ["fp64", "mxp"])
def test_solve_batched_matches_oracle(hp, dims, levels, sweep, nrhs, precision):
    """At tol 1e-9: the residual bar and the iteration counts.  A residual
    of 1e-9 does not bound ||x - x_oracle|| / ||x_oracle|| by 1e-8 for a
    random right-hand side (the error per unit residual grows with the grid),
    so the x parity pair is solved to 1e-11, where both reach FP64 accuracy."""
    P = problem(hp, dims, levels, sweep)
    sw = {"forward": 0, "symmetric": 2}[sweep]
    U_, B = _batch_rhs(dims, nrhs)
    X, stats = P.solve_batched(dev(B, 0), tol=1e-9, precision=precision)
    X11, stats11 = P.solve_batched(dev(B, 0), tol=1e-11, precision=precision)
    Xh, X11h = host(X), host(X11)
    for j in range(nrhs):
        st = stats[j]
        xo, sto = oracle.gmres_ir(dims, B[j], levels=levels, sweep=sw, tol=1e-9)
        xo11, _ = oracle.gmres_ir(dims, B[j], levels=levels, sweep=sw, tol=1e-11)
        res = np.linalg.norm(B[j] - oracle.spmv(dims, Xh[j])) / np.linalg.norm(B[j])
        dx9 = np.linalg.norm(Xh[j] - xo) / np.linalg.norm(xo)
        dx = np.linalg.norm(X11h[j] - xo11) / np.linalg.norm(xo11)
        xs, sts = P.solve(dev(B[j], 0), tol=1e-9, precision=precision)
        print(f"[batch {precision} {dims} j={j}] iters={st.iters} single={sts.iters} oracle={sto.iters} "
              f"res={res:.2e} dx(1e-9)={dx9:.2e} dx(1e-11)={dx:.2e}", flush=True)
        assert st.converged and st.final_rel_res <= 1e-9 and res <= 1e-9
        assert stats11[j].converged and dx <= 1e-8
        assert abs(st.iters - sts.iters) <= 2
        if precision == "fp64":
            assert abs(st.iters - sto.iters) <= 2


@pytest.mark.parametrize("precision", ["fp64", "mxp"])
def test_solve_batched_freezes_each_rhs(hp, precision):
    """Right-hand sides that converge at different steps, run out of
    iterations, or are zero: each follows its own solve exactly."""
    import torch
    dims = (16, 16, 16)
    P = problem(hp, dims, 3)
    _, B = _batch_rhs(dims, 4)
    B[1] = 0.0                                   # b = 0: x = 0, no step
    B[2] = oracle.spmv(dims, inputs.ones(dims))  # smooth: converges earlier
    B[3] *= 1e-3                                 # same direction, other scale
    x0 = np.stack([inputs.random_x0(dims)] * 4)
    for max_iters, restart in ((10000, 30), (7, 5), (0, 30)):
        X, stats = P.solve_batched(dev(B, 0), dev(x0, 0), tol=1e-9, restart=restart, max_iters=max_iters,
                                   precision=precision)
        Xh = host(X)
        for j in range(4):
            xs, sts = P.solve(dev(B[j], 0), dev(x0[j], 0), tol=1e-9, restart=restart, max_iters=max_iters,
                              precision=precision)
            st = stats[j]
            print(f"[freeze {precision} max={max_iters} m={restart} j={j}] iters={st.iters}/{sts.iters} "
                  f"restarts={st.restarts}/{sts.restarts} conv={st.converged}/{sts.converged}", flush=True)
            assert st.converged == sts.converged
            if precision == "fp64":
                assert st.iters == sts.iters and st.restarts == sts.restarts
            else:  # FP32 rounding of a differently ordered sum may move the last step
                assert abs(st.iters - sts.iters) <= 1 and abs(st.restarts - sts.restarts) <= 1
            if j == 1:
                assert st.converged and st.iters == 0 and np.all(Xh[j] == 0.0)
                continue
            xsh = host(xs)
            tol = 1e-10 if precision == "fp64" else 1e-6
            assert np.linalg.norm(Xh[j] - xsh) <= tol * np.linalg.norm(xsh), j
    with pytest.raises(hp.HpgmxError) as e:
        bad = dev(B, 0)
        bad[2, 5] = float("nan")
        P.solve_batched(bad)
    assert e.value.status == -5
    X, stats = P.solve_batched(dev(B[:3], 0), precision=precision)  # still usable
    assert all(s.converged for s in stats)
    assert torch.isfinite(X).all()


def test_solve_batched_tiles_do_not_change_results(hp):
    import torch
    dims = (24, 20, 16)
    nrhs = 8
    P = problem(hp, dims, 3)
    _, B = _batch_rhs(dims, nrhs)
    ref = None
    for R in widths(nrhs):
        force_tiles(hp, P, nrhs, 1, R)
        X, stats = P.solve_batched(dev(B, 0), precision="mxp")
        assert all(s.converged for s in stats)
        if ref is None:
            ref = (X, [s.iters for s in stats])
        else:
            assert [s.iters for s in stats] == ref[1]
            assert torch.equal(X, ref[0]), R
    force_tiles(hp, P, nrhs, 1, 0)


@pytest.mark.parametrize("sweep", ["forward", "backward", "symmetric"])
@pytest.mark.parametrize("precision", ["mxp", "fp64"])
def test_batched_spmv_in_last_sweep(hp, sweep, precision):
    """The batched solver shares its SpMV with the last sweep as the single
    one does: the partial sums left by the sweep (spmv_in_sweep 2) give the
    iterates of the same split sums formed by the SpMV alone (3) bit for
    bit, and each right-hand side converges as with one SpMV over all rows
    (0), in the same number of steps up to rounding."""
    import torch
    dims = (32, 32, 32)
    nrhs = 8
    U_, B = _batch_rhs(dims, nrhs)
    out = {}
    for mode in (0, 2, 3):
        P = hp.Problem(dims, beta=0.5, levels=3, sweep=sweep, layout={"spmv_in_sweep": mode})
        X, stats = P.solve_batched(dev(B, 0), precision=precision)
        P.close()
        out[mode] = (X, [s.iters for s in stats], [s.converged for s in stats])
    assert out[2][1] == out[3][1] and torch.equal(out[2][0], out[3][0])
    assert all(out[0][2]) and all(out[2][2])
    assert all(abs(a - b) <= 2 for a, b in zip(out[0][1], out[2][1])), (out[0][1], out[2][1])
    for j in range(nrhs):   # the FP64 residual of the shared-SpMV solve, recomputed by the oracle
        x = host(out[2][0][j])
        assert np.linalg.norm(B[j] - oracle.spmv(dims, x)) <= 1e-9 * np.linalg.norm(B[j]), j


def test_batched_rows_match_single_solver(hp):
    """With the SpMV shared with the last sweep in both, a right-hand side
    of a batch takes the single solver's SpMV arithmetic: same steps, and
    x equal to the FP32 reduction-order level."""
    dims = (32, 32, 32)
    U_, B = _batch_rhs(dims, 4)
    P = problem(hp, dims, 3)
    X, stats = P.solve_batched(dev(B, 0), precision="mxp")
    for j in range(4):
        x, st = P.solve(dev(B[j], 0), precision="mxp")
        assert abs(st.iters - stats[j].iters) <= 1
        assert np.linalg.norm(host(X[j]) - host(x)) <= 1e-6 * np.linalg.norm(host(x))


@pytest.mark.parametrize("dims,levels,sweep", [((32, 32, 32), 3, "forward"), ((24, 20, 16), 3, "forward"),
                                               ((24, 20, 16), 3, "backward"), ((12, 10, 9), 1, "forward")])
def test_solve_batched_tile_orders_bit_identical(hp, dims, levels, sweep):
    """Every tile order of the batched launches (the plane order of the
    full-grid SpMV and the plane-pair order of the SpMV over the colour pair
    (0, 1) or (6, 7) included; an odd extent falls back to the
    XCD-contiguous order) gives the same iterates bit for bit."""
    import torch
    nrhs = 8
    _, B = _batch_rhs(dims, nrhs)
    ref = None
    for order in (-1, 0, 1, 3):
        P = hp.Problem(dims, beta=0.5, levels=levels, sweep=sweep, layout={"tile_order": order})
        X, stats = P.solve_batched(dev(B, 0), precision="mxp")
        P.close()
        assert all(s.converged for s in stats)
        if ref is None:
            ref = (X, [s.iters for s in stats])
        else:
            assert [s.iters for s in stats] == ref[1] and torch.equal(X, ref[0]), order


@pytest.mark.parametrize("dtype", [0, 1])
def test_autotune_table(hp, dtype):
    dims = (32, 32, 32)
    P = problem(hp, dims, 4)
    for nrhs in (2, 4, 8):
        K = 2 if nrhs == 2 else nrhs
        t = hp.batch_autotune(P.h, nrhs, dtype)
        print(f"[autotune K={K} dtype={dtype}] {t['rhs_per_lane']}", flush=True)
        for k in range(hp.BK_COUNT):
            for lvl in range(4):
                R = t["rhs_per_lane"][k][lvl]
                applies = not (k == hp.BK_RESTRICT and lvl == 3) and not (k == hp.BK_RESID64 and lvl > 0)
                if applies:
                    assert R in (1, 2, 4, 8) and K % R == 0 and t["ms"][k][lvl] > 0.0, (k, lvl)
                else:
                    assert R == 0
        assert hp.batch_get_tuning(P.h, nrhs, dtype)["rhs_per_lane"] == t["rhs_per_lane"]
    _, B = _batch_rhs(dims, 8)
    X, stats = P.solve_batched(dev(B, 0), precision="fp64" if dtype == 0 else "mxp")
    assert all(s.converged for s in stats)


def test_batched_argument_errors(hp):
    import torch
    dims = (16, 16, 16)
    P = problem(hp, dims, 3)
    v = torch.zeros((3, P.N), dtype=torch.float32, device="cuda")
    with pytest.raises(hp.HpgmxError) as e:
        hp.spmv_batched(P.h, 0, 7, v, v.clone())           # no such dtype
    assert e.value.status == -1
    with pytest.raises(hp.HpgmxError) as e:
        hp.batch_set_tuning(P.h, 3, 1, 8)                  # K = 4: R = 8 does not divide
    assert e.value.status == -1
    with pytest.raises(hp.HpgmxError) as e:
        hp.batch_set_tuning(P.h, 3, 1, 3)
    assert e.value.status == -1
    w = torch.zeros((9, P.N), dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HpgmxError) as e:
        hp.gmres_ir_solve_batched(P.h, w, w.clone())        # nrhs > 8
    assert e.value.status == -1
    b = torch.zeros((2, P.N), dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HpgmxError) as e:
        hp.gmres_ir_solve_batched(P.h, b, b.clone(), inner_dtype=5)
    assert e.value.status == -1
    X, stats = P.solve_batched(b)                           # usable; b = 0 gives x = 0
    assert all(s.converged and s.iters == 0 for s in stats) and bool((X == 0).all())


@pytest.mark.parametrize("precision", ["mxp", "fp64"])
def test_batched_graph_replay_matches_eager(hp, precision):
    import torch
    dims = (32, 32, 32)
    P = problem(hp, dims, 4)
    _, B = _batch_rhs(dims, 8)
    Bd = dev(B, 0)
    X_e, st_e = P.solve_batched(Bd, restart=10, precision=precision)
    y = torch.zeros((8, P.N), dtype=torch.float32, device="cuda")
    for rep in range(3):
        X_g, st_g = P.solve_batched(Bd, restart=10, precision=precision, graph=True)
        assert [s.iters for s in st_g] == [s.iters for s in st_e]
        assert torch.equal(X_g, X_e), rep
        hp.spmv_batched(P.h, 0, 1, X_g.float(), y)          # eager work between replays
        torch.cuda.synchronize()


def test_batched_bound_workspace(hp):
    import torch
    dims = (32, 32, 32)
    h = hp.setup_problem(*dims, beta=0.5)
    mask = (1 << 0) | (1 << 1)
    nbytes = hp.workspace_bytes(h, levels=4, restart=30, dtype_mask=mask) + \
        hp.workspace_bytes_batched(h, 8, levels=4, restart=30, dtype_mask=mask)
    ws = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device="cuda")
    off = (-ws.data_ptr()) % 256
    hp.bind_workspace(h, ws.view(torch.uint8)[off:off + nbytes])
    hp.mg_setup(h, 4)
    _, B = _batch_rhs(dims, 8)
    Bd = dev(B, 0)
    X = torch.zeros_like(Bd)
    stats = hp.gmres_ir_solve_batched(h, Bd, X, inner_dtype=1)
    X2 = torch.zeros_like(Bd)
    stats2 = hp.gmres_ir_solve_batched(h, Bd, X2, inner_dtype=0)
    hp.batch_autotune(h, 8, 1)
    ref = problem(hp, dims, 4)
    Xr, str_ = ref.solve_batched(Bd, precision="mxp")
    hp.destroy(h)
    assert all(s.converged for s in stats) and all(s.converged for s in stats2)
    assert [s.iters for s in stats] == [s.iters for s in str_]
    assert torch.equal(X, Xr)


@pytest.mark.parametrize("dtype16,name", [(2, "fp16"), (3, "bf16")])
def test_batched_16bit_matrices_equal_fp32(hp, dtype16, name):
    """With beta = 0.5 every stencil entry (26, -1, -1.5, -0.5) is exact in
    FP16 and BF16, and the 16-bit values are widened exactly before the FP32
    arithmetic: batched SpMV, V-cycle and solve equal the FP32-matrix ones bit
    for bit, for every tile shape."""
    import torch
    dims = (24, 20, 16)
    nrhs = 6
    P = problem(hp, dims, 3)
    X = np.stack([rnd(inputs.uniform(dims, 5000 + j), 1) for j in range(nrhs)])
    for R in widths(nrhs):
        force_tiles(hp, P, nrhs, 1, R)
        force_tiles(hp, P, nrhs, dtype16, R)
        Y32, Y16 = dev(np.zeros(X.shape), 1), dev(np.zeros(X.shape), 1)
        hp.spmv_batched(P.h, 0, 1, dev(X, 1), Y32)
        hp.spmv_batched(P.h, 0, dtype16, dev(X, 1), Y16)
        assert torch.equal(Y32, Y16), R
        Z32, Z16 = dev(np.zeros(X.shape), 1), dev(np.zeros(X.shape), 1)
        hp.vcycle_batched(P.h, 1, dev(X, 1), Z32)
        hp.vcycle_batched(P.h, dtype16, dev(X, 1), Z16)
        assert torch.equal(Z32, Z16), R
    # Batched solves with 16-bit matrices take one SpMV over all rows; the
    # FP32 solve is compared in that mode (not sharing the SpMV with the sweep)
    _, B = _batch_rhs(dims, nrhs)
    Q = hp.Problem(dims, beta=0.5, levels=3, sweep="forward", layout={"spmv_in_sweep": 0})
    X32, s32 = Q.solve_batched(dev(B, 0), precision="mxp")
    X16, s16 = Q.solve_batched(dev(B, 0), precision=name)
    X16p, s16p = P.solve_batched(dev(B, 0), precision=name)
    Q.close()
    assert [s.iters for s in s16] == [s.iters for s in s32] and all(s.converged for s in s16)
    assert torch.equal(X16, X32) and torch.equal(X16p, X16)
    force_tiles(hp, P, nrhs, 1, 0)
    force_tiles(hp, P, nrhs, dtype16, 0)
