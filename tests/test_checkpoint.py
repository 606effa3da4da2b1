"""Host logic of the checkpoint schedules (CPU only).

The binomial schedule is pinned against a brute-force recursion over every
split (the minimum number of forward steps), and both schedules are replayed
on a fake lattice whose state is its step index, so that every reverse step
is checked to receive exactly f_n, in the order n = N-1 .. 0.
"""
import pytest

from paper_1703_04594_amd import checkpoint as ck


def test_binomial_closed_form_and_schedule_are_optimal():
    memo = {}
    for s in range(0, 6):
        for l in range(1, 100):
            dp = ck.min_forward_steps(l, s, memo)
            assert ck.binomial_forward_steps(l, s) == dp, (l, s)
            sch = ck.binomial_schedule(l, s + 1)
            assert sch.forward_steps() == dp, (l, s)
            assert sch.slots_needed <= s + 2   # s + 1 snapshots + one working copy


def test_binomial_repetition_count_matches_beta():
    # beta(c, r) = C(c + r, c) steps are reversible with c checkpoints and r repetitions
    for c in range(1, 6):
        for r in range(1, 6):
            l = ck.beta(c, r)
            assert ck.repetitions(l, c - 1) == r
            assert ck.repetitions(l + 1, c - 1) == r + 1


class FakeState:
    def __init__(self):
        self.n = None

    def copy_(self, other):
        self.n = other.n


class FakeLattice:
    """State = the step index it holds."""

    def __init__(self):
        self.n = 0
        self.expect = None
        self.steps = 0
        self.pending = 0       # reverse steps whose d/dtau term is not yet taken
        self.takes = 0

    def new_state(self):
        return FakeState()

    def get_state(self, out):
        out.n = self.n
        return out

    def set_state(self, s):
        self.n = s.n

    def step(self, k):
        self.n += k
        self.steps += k

    def step_state(self, src, dst):
        assert src is not dst
        dst.n = src.n + 1
        self.steps += 1

    def adjoint_step(self, s, dacc):
        assert s.n == self.expect, (s.n, self.expect)
        assert dacc is None        # the executor defers the d/dtau terms
        self.expect -= 1
        self.pending += 1

    def take_dtau(self, dacc):
        assert self.pending > 0
        self.pending = 0
        self.takes += 1


@pytest.mark.parametrize("N", [1, 2, 7, 50, 257])
@pytest.mark.parametrize("kind", ["sqrt", "binomial2", "binomial5"])
@pytest.mark.parametrize("chain", [False, True])
def test_schedules_feed_every_state_in_reverse_order(N, kind, chain):
    sch = ck.sqrt_schedule(N) if kind == "sqrt" else ck.binomial_schedule(N, int(kind[-1]))
    fwd, bwd = sch.split_at_first_adjoint()
    lat = FakeLattice()
    ex = ck.Executor(lat, None, chain=chain)
    ex.run(fwd)
    ex.materialize()
    assert lat.n == N - 1          # the forward prefix ends holding f_{N-1}
    lat.step(1)                    # the rollout's last step, to f_N
    lat.expect = N - 1
    ex.run(bwd)
    assert lat.expect == -1        # all N reverse steps, each with its own f_n
    assert lat.pending == 0 and lat.takes == 1   # their d/dtau terms taken once, at the end
    assert ex.adjoint_steps == N
    assert ex.forward_steps == sch.forward_steps()
    assert lat.steps == sch.forward_steps() + 1


def test_chaining_removes_most_state_copies():
    """Replayed segments run slot to slot: the 10,000-step binomial schedule
    with 100 slots copies states in or out of the lattice only for the first
    sweep and for multi-step advances."""
    sch = ck.binomial_schedule(10000, 100)
    copies = {}
    for chain in (False, True):
        fwd, bwd = sch.split_at_first_adjoint()
        lat = FakeLattice()
        ex = ck.Executor(lat, None, chain=chain)
        ex.run(fwd)
        ex.materialize()
        lat.step(1)
        lat.expect = 10000 - 1
        ex.run(bwd)
        assert lat.expect == -1
        copies[chain] = ex.state_copies
    assert copies[False] >= 10000
    assert copies[True] < copies[False] / 5


def test_sqrt_schedule_memory_and_cost():
    N = 2000
    sch = ck.sqrt_schedule(N)
    k = 45
    assert sch.slots_needed <= N // k + 1 + k
    # one forward sweep plus one replay of every segment except its first state
    assert sch.forward_steps() <= 2 * N


def test_large_binomial_schedule_is_cheap_to_build():
    sch = ck.binomial_schedule(10000, 93)
    assert sch.forward_steps() == ck.binomial_forward_steps(10000, 92)
    assert sch.forward_steps() < 2.6 * 10000
