"""Host-side check of the adjoint solver's problem cache: a loop that keeps
changing the stencil holds at most `max_cached` (forward, adjoint) problem
pairs, closing each evicted pair once (no GPU: the problem class is replaced
by a stand-in that records its lifetime)."""
import pytest
import torch

from paper_2507_11512_amd import autograd


class FakeProblem:
    live = 0
    closed = 0

    def __init__(self, dims, levels=3, sweep="forward", coef=None):
        self.coef = list(coef)
        self.open = True
        FakeProblem.live += 1

    def close(self):
        assert self.open, "closed twice"
        self.open = False
        FakeProblem.live -= 1
        FakeProblem.closed += 1


@pytest.mark.parametrize("cap", [1, 2, 3])
def test_cache_stays_bounded_across_theta_updates(monkeypatch, cap):
    FakeProblem.live = FakeProblem.closed = 0
    monkeypatch.setattr(autograd.hpgmx, "Problem", FakeProblem)
    s = autograd.StencilSolver((8, 8, 8), max_cached=cap)
    thetas = [torch.full((27,), -1.0 - 0.01 * i, dtype=torch.float64) for i in range(7)]
    for th in thetas:
        th[13] = 26.0
        fwd, adj = s.problems(th)
        assert fwd.coef == adj.coef[::-1]
        assert len(s._cache) <= cap and FakeProblem.live == 2 * len(s._cache)
    assert FakeProblem.closed == 2 * (len(thetas) - cap)
    # the most recent stencil is still cached: asking again creates nothing
    before = FakeProblem.live + FakeProblem.closed
    s.problems(thetas[-1])
    assert FakeProblem.live + FakeProblem.closed == before
    s.close()
    assert FakeProblem.live == 0


def test_cache_size_must_be_positive():
    with pytest.raises(ValueError):
        autograd.StencilSolver(8, max_cached=0)
