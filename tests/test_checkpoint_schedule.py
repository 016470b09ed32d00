"""The binomial (revolve) checkpoint schedule of the adjoint driver, on a
stand-in simulation that records which state every adjoint step receives:
each step t = T-1 ... 0 gets exactly f(t), no more than the allowed number
of snapshots is held, and the recomputation matches the binomial bound."""
from math import comb

import pytest

from paper_2504_03819_amd.autograd import reverse_binomial


class _Recorder:
    """Holds only a time index; states are tuples (t,)."""

    def __init__(self):
        self.t = 0
        self.seen = []

    def set_state(self, st, t):
        assert st == (t,)
        self.t = t

    def step(self, n):
        assert n >= 1
        self.t += n

    def get_state(self):
        class _S(tuple):
            def clone(self):
                return self
        return _S((self.t,))

    def adjoint_step(self, st):
        # None: the adjoint step takes the simulation's current state
        self.seen.append(self.t if st is None else st[0])


def _bound(t, s):
    """Forward steps a binomial reversal may recompute: T (T-1)/2 without
    snapshots, otherwise at most r T with r the least number of sweeps that
    covers t steps, C(s + r, s) >= t."""
    if s == 0:
        return t * (t - 1) // 2
    r = 0
    while comb(s + r, s) < t:
        r += 1
    return r * t


@pytest.mark.parametrize("T,s", [(1, 0), (2, 0), (7, 0), (9, 1), (9, 2), (40, 3), (200, 5), (500, 8), (64, 64)])
def test_binomial_schedule_visits_every_state_in_reverse(T, s):
    sim = _Recorder()
    stats = reverse_binomial(sim, sim.get_state(), 0, T, s)
    assert sim.seen == list(range(T - 1, -1, -1))
    assert stats["max_held"] <= s
    assert stats["recompute_steps"] <= _bound(T, s)


def test_binomial_schedule_is_quadratic_without_snapshots():
    sim = _Recorder()
    stats = reverse_binomial(sim, sim.get_state(), 0, 10, 0)
    assert stats["recompute_steps"] == 10 * 9 // 2
