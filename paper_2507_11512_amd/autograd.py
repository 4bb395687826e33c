"""Differentiable solve of the stencil system through the adjoint.

x = A(theta)^{-1} b with A the 27-point stencil operator whose 27 entries are
theta.  The backward pass solves the adjoint system A^T lam = dL/dx with the
same mixed-precision GMRES-IR / multigrid solver (A^T is the stencil with
theta reversed) and returns

    dL/db     = lam,
    dL/dtheta = -sum_i lam_i x_{i + d_t}   (t = 0..26, in-grid pairs only).

b may also be a batch of k <= 8 right-hand sides, shape (k, N): then both
solves run through the batched solver (each right-hand side keeps its own
Krylov process) and dL/dtheta sums the correlations of the k pairs
(lam_j, x_j).

Both solves and the gradient reduction run in the HIP library; this module
only wires them into torch.autograd.
"""
from collections import OrderedDict

import torch

from . import hpgmx


def _key(theta):
    return tuple(float(v) for v in theta.detach().cpu().tolist())


class StencilSolver:
    """Keeps the forward and the adjoint problem (each a full multigrid
    hierarchy on the device) for the `max_cached` stencils used most
    recently; older pairs are closed, so a loop that updates theta holds a
    bounded amount of device memory.  A backward pass whose stencil was
    evicted sets its pair up again."""

    def __init__(self, dims, levels=3, sweep="forward", restart=30, tol=1e-10,
                 precision="mxp", max_iters=10000, max_cached=2):
        self.dims = (dims, dims, dims) if isinstance(dims, int) else tuple(dims)
        self.levels, self.sweep = levels, sweep
        self.restart, self.tol, self.precision, self.max_iters = restart, tol, precision, max_iters
        if max_cached < 1:
            raise ValueError("max_cached must be at least 1")
        self.max_cached = int(max_cached)
        self._cache = OrderedDict()
        self.last_stats = None

    def problems(self, theta):
        k = _key(theta)
        if k in self._cache:
            self._cache.move_to_end(k)
            return self._cache[k]
        while len(self._cache) >= self.max_cached:
            _, (fwd, adj) = self._cache.popitem(last=False)
            fwd.close()
            adj.close()
        coef = list(k)
        fwd = hpgmx.Problem(self.dims, levels=self.levels, sweep=self.sweep, coef=coef)
        try:
            adj = hpgmx.Problem(self.dims, levels=self.levels, sweep=self.sweep, coef=coef[::-1])
        except Exception:
            fwd.close()
            raise
        self._cache[k] = (fwd, adj)
        return fwd, adj

    def solve(self, problem, rhs):
        rhs = rhs.contiguous()
        if rhs.dim() == 2:
            x, sts = problem.solve_batched(rhs, tol=self.tol, restart=self.restart,
                                           max_iters=self.max_iters, precision=self.precision)
        else:
            x, st = problem.solve(rhs, tol=self.tol, restart=self.restart,
                                  max_iters=self.max_iters, precision=self.precision)
            sts = [st]
        self.last_stats = sts if rhs.dim() == 2 else sts[0]
        for st in sts:
            if not st.converged:
                raise RuntimeError(f"stencil solve did not converge (rel. residual {st.final_rel_res:.3e})")
        return x

    def __call__(self, b, theta):
        return StencilSolve.apply(b, theta, self)

    def close(self):
        for fwd, adj in self._cache.values():
            fwd.close()
            adj.close()
        self._cache.clear()


class StencilSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, theta, solver):
        fwd, adj = solver.problems(theta)
        x = solver.solve(fwd, b.to(torch.float64))
        ctx.save_for_backward(x, theta)
        ctx.solver = solver
        return x

    @staticmethod
    def backward(ctx, g):
        x, theta = ctx.saved_tensors
        solver = ctx.solver
        fwd, adj = solver.problems(theta)
        lam = solver.solve(adj, g.to(torch.float64).contiguous())
        if lam.dim() == 2:
            grad_theta = -sum(fwd.stencil_grad(lam[j], x[j]) for j in range(lam.shape[0]))
        else:
            grad_theta = -fwd.stencil_grad(lam, x)
        return lam, grad_theta.to(theta.dtype), None
