"""The allocation-free entry point hpgmx_stencil_grad_noalloc, called through
the C ABI, against hpgmx_stencil_grad on the same inputs: two calls in a row
on one GPU, the second on a smaller grid (the shared scratch then still
holds the first call's partial sums beyond the ones the second reads).  The
two entry points add the same FP64 products in different orders, so they
agree within the FP64 summation bound 2 N u sum |lam_i| |x_j|; the oracle's
correlation is checked the same way."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2507_11512_amd import inputs

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def hp():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2507_11512_amd import hpgmx
    return hpgmx


def _call(hp, fn, h, lam, x, out):
    f = getattr(hp.lib, fn)
    st = f(h, C.c_void_p(lam.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()))
    assert st == 0, (fn, st, hp.last_error(h))


def test_noalloc_gradient_matches_the_allocating_entry_point(hp):
    import torch
    for n, (dims, seed) in enumerate([((48, 40, 36), 1700), ((16, 12, 8), 1710)]):
        print(f"[noalloc] call {n}: dims={dims}", flush=True)
        P = hp.Problem(dims, beta=0.5, levels=2, sweep="forward")
        try:
            lam = inputs.uniform(dims, seed)
            x = inputs.uniform(dims, seed + 1)
            lt = torch.from_numpy(lam).cuda()
            xt = torch.from_numpy(x).cuda()
            a = torch.full((27,), float("nan"), dtype=torch.float64, device="cuda")
            b = torch.full((27,), float("nan"), dtype=torch.float64, device="cuda")
            _call(hp, "hpgmx_stencil_grad_noalloc", P.h, lt, xt, a)   # before anything else ran
            torch.cuda.synchronize()
            _call(hp, "hpgmx_stencil_grad", P.h, lt, xt, b)
            torch.cuda.synchronize()
            ga, gb = a.cpu().numpy(), b.cpu().numpy()
            N = lam.size
            scale = oracle.stencil_correlation(dims, np.abs(lam), np.abs(x))
            ref = oracle.stencil_correlation(dims, lam, x)
            assert np.all(np.isfinite(ga))
            assert np.all(np.abs(ga - gb) <= 2 * N * U64 * scale + 1e-300), np.max(np.abs(ga - gb) / scale)
            assert np.all(np.abs(ga - ref) <= 2 * N * U64 * scale + 1e-300)
        finally:
            P.close()
