"""The persistent batch schedule's host-side parts, on the CPU: the radix
decompositions it can tune over, and a multi-threaded simulation of its
queue protocol (pass-ordered items, per-(solve, pass) and per-level
completion counts, deferred releases, bounded waits) with planted mistakes
that the simulation must catch."""

import numpy as np
import pytest

import paper_1211_5244_amd as P
from paper_1211_5244_amd import _lib

LENGTHS = [4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]


@pytest.mark.parametrize("L", LENGTHS)
def test_radix_choices_factor_the_length(L):
    seen = set()
    for sel in range(3):
        rad = P.poisson_queue_radices(L, sel)
        assert int(np.prod(rad)) == L, (L, sel, rad)
        assert set(rad) <= {2, 3, 4, 8}
        assert rad.count(3) == (1 if L % 3 == 0 else 0)
        seen.add(rad)
    # choice 1 uses no radix 8; choice 2 is choice 0 reversed
    assert 8 not in P.poisson_queue_radices(L, 1)
    assert P.poisson_queue_radices(L, 2) == tuple(reversed(P.poisson_queue_radices(L, 0)))


def test_radix_choice_errors():
    with pytest.raises(P.PoissonError) as e:
        P.poisson_queue_radices(64, 3)
    assert e.value.code == _lib.POISSON_E_ARG
    with pytest.raises(P.PoissonError) as e:
        P.poisson_queue_radices(20, 0)
    assert e.value.code == _lib.POISSON_E_UNSUPPORTED


def _segments(rng, nsolve, hi):
    return [[int(x) for x in rng.integers(1, hi + 1, size=nsolve)] for _ in range(5)]


@pytest.mark.parametrize("workers", [1, 2, 8, 64])
def test_simulated_queue_protocol_holds(workers):
    """Random segment sizes: every item runs once, none passes its wait
    before its dependency's work is done, the counters end at zero."""
    rng = np.random.default_rng(100 + workers)
    for trial in range(4):
        segs = _segments(rng, int(rng.integers(1, 12)), 40)
        waits, releases, violations, timeouts = P.poisson_queue_simulate(segs, workers, seed=trial)
        items = sum(map(sum, segs))
        assert violations == 0 and timeouts == 0
        assert 1 <= releases <= items
        if workers == 1:
            # one worker releases each level once (lists of at most 32 items)
            assert releases <= sum(-(-sum(lv) // 32) for lv in segs)


def test_simulated_many_solves():
    """The composition of the 512-solve batch at one item per segment and at
    a few items per segment."""
    rng = np.random.default_rng(7)
    segs = [[1] * 512 for _ in range(5)]
    P.poisson_queue_simulate(segs, 32, seed=3)
    segs = _segments(rng, 512, 6)
    P.poisson_queue_simulate(segs, 64, seed=4)


def test_simulation_catches_late_release():
    """Releasing held lower-level items only after a wait deadlocks a lone
    worker on its own items: the bounded wait must report it."""
    with pytest.raises(P.PoissonError) as e:
        P.poisson_queue_simulate([[3, 1, 2]] * 5, 1, fault=1)
    assert e.value.code == _lib.POISSON_E_STATE
    assert "ran out" in str(e.value)


def test_simulation_catches_early_completion():
    """Counting an item complete before its work lets a dependent start too
    early: the dependency check must report it."""
    with pytest.raises(P.PoissonError) as e:
        P.poisson_queue_simulate([[1, 1]] * 5, 4, fault=2)
    assert e.value.code == _lib.POISSON_E_STATE
    assert "dependency" in str(e.value)


def test_simulation_argument_checks():
    with pytest.raises(P.PoissonError):
        P.poisson_queue_simulate([[0, 1]] * 5, 2)
    with pytest.raises(P.PoissonError):
        P.poisson_queue_simulate([[1]] * 5, 0)
    with pytest.raises(P.PoissonError):
        P.poisson_queue_simulate([[1]] * 5, 1, fault=3)
