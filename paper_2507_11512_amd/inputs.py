"""Seeded synthetic inputs shared by the tests, the oracle runs and the bench.

This module holds none of the solver's arithmetic: it only draws the
synthetic vectors that the workloads are defined with, in natural
lexicographic order I = i + nx*(j + ny*k), as float64 numpy arrays.  Products
such as b = A u are formed by whichever side consumes them (the oracle on the
CPU, the library on the GPU).

Workload recipes (the paper's matrix is itself generated, so no dataset is
involved):
  * x_true = 1 for every right-hand side b = A 1 (exact solution all ones);
  * the second start of the 128^3 case: x0 ~ U(-1, 1), numpy default_rng(2507);
  * batched right-hand sides: u_j ~ N(0, 1), default_rng(11512 + j);
  * adjoint seed: g ~ N(0, 1), default_rng(11512 + 100).
"""
import numpy as np

SEED_X0 = 2507
SEED_BATCH = 11512


def n_of(dims):
    if isinstance(dims, int):
        return dims ** 3
    nx, ny, nz = dims
    return int(nx) * int(ny) * int(nz)


def ones(dims):
    return np.ones(n_of(dims))


def random_x0(dims, seed=SEED_X0):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n_of(dims))


def normal(dims, seed):
    return np.random.default_rng(seed).standard_normal(n_of(dims))


def batch_u(dims, j):
    return normal(dims, SEED_BATCH + j)


def adjoint_seed(dims):
    return normal(dims, SEED_BATCH + 100)


def uniform(dims, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n_of(dims))
