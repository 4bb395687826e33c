"""General stencils and the adjoint gradient on the GPU.

The differentiable solve x = A(theta)^{-1} b returns dL/db = lam and
dL/dtheta_t = -sum_i lam_i x_{i+d_t} with A^T lam = dL/dx.  Checked on a 12^3
grid (three levels: 12, 6, 3) against
  * the oracle's general-stencil SpMV, solve and stencil correlation;
  * a dense FP64 reference (numpy solves of the assembled matrix);
  * central finite differences of L through the GPU solver itself.
Inputs follow the batched/adjoint recipe: u ~ N(0,1) seeded 11512, b = A u,
g ~ N(0,1) seeded 11612.
"""
import numpy as np
import pytest

import oracle
from paper_2507_11512_amd import inputs
from tests import refimpl

pytestmark = pytest.mark.gpu

D = (12, 12, 12)
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.fail("no GPU visible")
    return T


@pytest.fixture(scope="module")
def hp(torch):
    from paper_2507_11512_amd import hpgmx
    return hpgmx


def theta0():
    return oracle.stencil_from_beta(0.5)


def perturbed_theta(seed):
    """A nonsymmetric, diagonally dominant stencil off the beta family."""
    rng = np.random.default_rng(seed)
    c = theta0() + rng.uniform(-0.05, 0.05, 27)
    c[13] = 26.0 + 2.0
    return c


def dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("which", ["beta", "random"])
def test_general_stencil_spmv_and_solve(hp, torch, which):
    c = theta0() if which == "beta" else perturbed_theta(3)
    P = hp.Problem(D, levels=3, coef=c)
    x = inputs.uniform(D, 5)
    y = torch.zeros(x.size, dtype=torch.float64, device="cuda")
    hp.spmv(P.h, 0, 0, dev(x, torch), y)
    ref = oracle.spmv_c(D, c, x)
    scale = np.abs(refimpl.stencil_matrix(D, c)) @ np.abs(x)
    assert np.all(np.abs(y.cpu().numpy() - ref) <= 56 * U64 * scale)
    b = inputs.batch_u(D, 0)
    for prec in ("fp64", "mxp"):
        xg, st = P.solve(dev(b, torch), tol=1e-11, precision=prec)
        xo, sto = oracle.gmres_ir_c(D, c, b, levels=3, tol=1e-11)
        assert st.converged and sto.converged
        dx = np.linalg.norm(xg.cpu().numpy() - xo) / np.linalg.norm(xo)
        assert dx <= 1e-8, (prec, dx)
    P.close()


def test_stencil_grad_matches_oracle(hp, torch):
    c = perturbed_theta(4)
    P = hp.Problem(D, levels=3, coef=c)
    lam, x = inputs.normal(D, 7), inputs.normal(D, 8)
    got = P.stencil_grad(dev(lam, torch), dev(x, torch)).cpu().numpy()
    ref = oracle.stencil_correlation(D, lam, x)
    scale = oracle.stencil_correlation(D, np.abs(lam), np.abs(x))
    assert np.all(np.abs(got - ref) <= 2 * D[0] ** 3 * U64 * scale)
    P.close()


@pytest.mark.parametrize("precision", ["fp64", "mxp"])
def test_autograd_gradients(hp, torch, precision):
    from paper_2507_11512_amd.autograd import StencilSolver
    th = perturbed_theta(9)
    A = refimpl.stencil_matrix(D, th).toarray()
    u = inputs.batch_u(D, 0)
    b = A @ u
    g = inputs.adjoint_seed(D)
    solver = StencilSolver(D, levels=3, tol=1e-12, precision=precision)
    bt = dev(b, torch).requires_grad_(True)
    tt = dev(th, torch).requires_grad_(True)
    x = solver(bt, tt)
    L = (dev(g, torch) * x).sum()
    L.backward()
    # dense FP64 reference
    xs = np.linalg.solve(A, b)
    ls = np.linalg.solve(A.T, g)
    grad_theta_ref = np.array([-(ls @ (refimpl.shift_matrix(D, s % 3 - 1, (s // 3) % 3 - 1, s // 9 - 1) @ xs))
                               for s in range(27)])
    gb = bt.grad.cpu().numpy()
    gt = tt.grad.cpu().numpy()
    assert np.linalg.norm(x.detach().cpu().numpy() - xs) <= 1e-9 * np.linalg.norm(xs)
    assert np.linalg.norm(gb - ls) <= 1e-9 * np.linalg.norm(ls)
    assert np.allclose(gt, grad_theta_ref, rtol=1e-7, atol=1e-9 * np.abs(grad_theta_ref).max())
    # central differences through the GPU solver
    eps = 1e-4
    for s in (0, 3, 12, 13, 14, 25):
        tp, tm = th.copy(), th.copy()
        tp[s] += eps
        tm[s] -= eps
        Lp = float((dev(g, torch) * solver(dev(b, torch), dev(tp, torch))).sum())
        Lm = float((dev(g, torch) * solver(dev(b, torch), dev(tm, torch))).sum())
        fd = (Lp - Lm) / (2 * eps)
        assert np.isclose(gt[s], fd, rtol=1e-5, atol=1e-7 * np.abs(gt).max()), (s, gt[s], fd)
    solver.close()


def test_adjoint_of_beta_family_is_negated_beta(hp, torch):
    """A^T for the beta family is the beta family at -beta: the adjoint solve
    through the reversed stencil matches the oracle's -beta solve."""
    P = hp.Problem(D, levels=3, coef=theta0()[::-1].copy())
    g = inputs.adjoint_seed(D)
    lam, st = P.solve(dev(g, torch), tol=1e-11, precision="fp64")
    lo, _ = oracle.gmres_ir(D, g, levels=3, beta=-0.5, tol=1e-11)
    assert np.linalg.norm(lam.cpu().numpy() - lo) <= 1e-8 * np.linalg.norm(lo)
    P.close()


@pytest.mark.parametrize("precision", ["fp64", "mxp"])
def test_autograd_batched_gradients(hp, torch, precision):
    """k = 3 right-hand sides through the batched solver: the gradients equal
    the sums of the per-right-hand-side dense FP64 gradients and the central
    differences of L = sum_j g_j . x_j."""
    from paper_2507_11512_amd.autograd import StencilSolver
    k = 3
    th = perturbed_theta(21)
    A = refimpl.stencil_matrix(D, th).toarray()
    Ub = np.stack([inputs.batch_u(D, j) for j in range(k)])
    Bh = Ub @ A.T                        # rows b_j = A u_j
    G = np.stack([inputs.normal(D, 11612 + j) for j in range(k)])
    solver = StencilSolver(D, levels=3, tol=1e-12, precision=precision)
    bt = dev(Bh, torch).requires_grad_(True)
    tt = dev(th, torch).requires_grad_(True)
    X = solver(bt, tt)
    assert X.shape == (k, D[0] ** 3)
    L = (dev(G, torch) * X).sum()
    L.backward()
    Xs = np.linalg.solve(A, Bh.T).T
    Ls = np.linalg.solve(A.T, G.T).T
    shifts = [refimpl.shift_matrix(D, s % 3 - 1, (s // 3) % 3 - 1, s // 9 - 1) for s in range(27)]
    grad_theta_ref = np.array([-sum(Ls[j] @ (shifts[s] @ Xs[j]) for j in range(k)) for s in range(27)])
    assert np.linalg.norm(X.detach().cpu().numpy() - Xs) <= 1e-9 * np.linalg.norm(Xs)
    assert np.linalg.norm(bt.grad.cpu().numpy() - Ls) <= 1e-9 * np.linalg.norm(Ls)
    gt = tt.grad.cpu().numpy()
    assert np.allclose(gt, grad_theta_ref, rtol=1e-7, atol=1e-9 * np.abs(grad_theta_ref).max())
    eps = 1e-4
    for s in (1, 13, 22):
        tp, tm = th.copy(), th.copy()
        tp[s] += eps
        tm[s] -= eps
        Lp = float((dev(G, torch) * solver(dev(Bh, torch), dev(tp, torch))).sum())
        Lm = float((dev(G, torch) * solver(dev(Bh, torch), dev(tm, torch))).sum())
        fd = (Lp - Lm) / (2 * eps)
        assert np.isclose(gt[s], fd, rtol=1e-5, atol=1e-7 * np.abs(gt).max()), (s, gt[s], fd)
    solver.close()
