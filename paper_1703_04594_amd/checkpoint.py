"""Checkpoint schedules for reversing N time steps with a bounded number of
stored states, as action lists executed against a Lattice.

A reversal needs the forward state f_n at every step n = N-1 .. 0, in that
order, while memory holds only a few states.  Both schedules here are
published methods:

* sqrt(T): store every k-th state (k = ceil(sqrt(N))) during the forward
  sweep; reverse segment by segment, replaying each segment once and keeping
  its k states.  About one extra forward sweep, ~2 sqrt(N) stored states.
* binomial: Griewank's recursive checkpointing (Griewank 1992; Griewank and
  Walther, ACM TOMS 26(1), 2000).  With the segment's first state stored and
  s free snapshot slots, a segment of l steps is split at j: advance j steps
  and store, reverse the right part with s - 1 free slots, then the left part
  with s.  With c = s + 1 checkpoints counting the stored start,
  beta(c, r) = C(c + r, c) is the longest segment reversible with every step
  advanced at most r times, and for the least such r the minimal forward-step
  count is T(l, s) = r l - beta(c + 1, r - 1).  T is convex and piecewise
  linear in l, so the split cost j + T(l - j, s - 1) + T(j, s) is convex in
  j and its minimiser is found by bisection on the forward difference.  A CPU
  test checks the closed form and the schedule's step count against a
  brute-force recursion over all splits.

Actions (tuples):
  ("advance", n0, n1)   the lattice holds f_n0; step it to f_n1
  ("store", n, slot)    copy the lattice state f_n into slot
  ("restore", n, slot)  load f_n from slot into the lattice
  ("free", slot)        release slot
  ("adjoint", n, slot)  reverse step n using f_n held in slot
The forward pass of a rollout executes the prefix up to the first "adjoint"
(it ends holding f_{N-1} at the latest); the backward pass executes the rest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field


def beta(s: int, r: int) -> int:
    return math.comb(s + r, s)


def repetitions(l: int, s: int) -> int:
    """Least r with beta(s + 1, r) >= l, for s free slots besides the start."""
    r = 0
    while beta(s + 1, r) < l:
        r += 1
    return r


def binomial_split(l: int, s: int) -> int:
    """Distance of the first checkpoint for l >= 2 steps and s >= 1 free
    slots: the least minimiser of j + T(l - j, s - 1) + T(j, s)."""
    def cost(j):
        return j + binomial_forward_steps(l - j, s - 1) + binomial_forward_steps(j, s)
    lo, hi = 1, l - 1           # minimiser in [lo, hi]
    while lo < hi:
        mid = (lo + hi) // 2
        if cost(mid + 1) - cost(mid) >= 0:
            hi = mid
        else:
            lo = mid + 1
    return lo


@dataclass
class Schedule:
    actions: list = field(default_factory=list)
    slots_needed: int = 0

    def forward_steps(self) -> int:
        return sum(a[2] - a[1] for a in self.actions if a[0] == "advance")

    def split_at_first_adjoint(self):
        for i, a in enumerate(self.actions):
            if a[0] == "adjoint":
                return self.actions[:i], self.actions[i:]
        return self.actions, []


class _SlotPool:
    def __init__(self):
        self.free: list[int] = []
        self.n = 0
        self.in_use = 0
        self.peak = 0

    def get(self) -> int:
        s = self.free.pop() if self.free else self._new()
        self.in_use += 1
        self.peak = max(self.peak, self.in_use)
        return s

    def _new(self) -> int:
        self.n += 1
        return self.n - 1

    def put(self, s: int):
        self.free.append(s)
        self.in_use -= 1


def sqrt_schedule(N: int, k: int | None = None) -> Schedule:
    if N < 1:
        raise ValueError("N >= 1")
    k = k or max(1, math.isqrt(N - 1) + 1)
    sch = Schedule()
    A = sch.actions
    pool = _SlotPool()
    marks = {}
    # forward sweep: store f_0, f_k, f_2k, ...
    pos = 0
    for a in range(0, N, k):
        if a > pos:
            A.append(("advance", pos, a))
            pos = a
        marks[a] = pool.get()
        A.append(("store", a, marks[a]))
    # reverse segments, last first
    starts = sorted(marks, reverse=True)
    for a in starts:
        b = min(a + k, N)
        seg = {a: marks[a]}
        if pos != a:
            A.append(("restore", a, marks[a]))
            pos = a
        for n in range(a + 1, b):
            A.append(("advance", n - 1, n))
            seg[n] = pool.get()
            A.append(("store", n, seg[n]))
            pos = n
        for n in range(b - 1, a - 1, -1):
            A.append(("adjoint", n, seg[n]))
            if n != a:
                A.append(("free", seg[n]))
                pool.put(seg[n])
        A.append(("free", marks[a]))
        pool.put(marks[a])
        pos = None
    sch.slots_needed = pool.peak
    return sch


def binomial_schedule(N: int, slots: int) -> Schedule:
    """Reverse N steps with at most `slots` stored states (including f_0)."""
    if N < 1 or slots < 1:
        raise ValueError("N >= 1 and slots >= 1")
    sch = Schedule()
    A = sch.actions
    pool = _SlotPool()
    state = {"pos": 0}

    def goto(n0: int, slot: int, n1: int):
        if state["pos"] != n0:
            A.append(("restore", n0, slot))
        if n1 > n0:
            A.append(("advance", n0, n1))
        state["pos"] = n1

    def rev(a: int, b: int, slot_a: int, s: int):
        # f_a is in slot_a; s more slots may be used; lambda holds lambda_b
        l = b - a
        if l == 1:
            A.append(("adjoint", a, slot_a))
            return
        if s == 0:
            tmp = pool.get()
            for n in range(b - 1, a - 1, -1):
                if n == a:
                    A.append(("adjoint", a, slot_a))
                else:
                    goto(a, slot_a, n)
                    A.append(("store", n, tmp))
                    A.append(("adjoint", n, tmp))
            A.append(("free", tmp))
            pool.put(tmp)
            state["pos"] = None
            return
        j = binomial_split(l, s)
        m = a + j
        goto(a, slot_a, m)
        sm = pool.get()
        A.append(("store", m, sm))
        rev(m, b, sm, s - 1)
        A.append(("free", sm))
        pool.put(sm)
        state["pos"] = None
        rev(a, m, slot_a, s)

    s0 = pool.get()
    A.append(("store", 0, s0))
    rev(0, N, s0, slots - 1)
    A.append(("free", s0))
    pool.put(s0)
    sch.slots_needed = pool.peak
    return sch


def min_forward_steps(l: int, s: int, memo=None) -> int:
    """Brute-force minimum forward steps to reverse l steps with f_a stored
    and s free slots (the recursion behind binomial checkpointing)."""
    if memo is None:
        memo = {}
    if l == 1:
        return 0
    if s == 0:
        return l * (l - 1) // 2
    key = (l, s)
    if key not in memo:
        memo[key] = min(j + min_forward_steps(l - j, s - 1, memo) + min_forward_steps(j, s, memo)
                        for j in range(1, l))
    return memo[key]


def binomial_forward_steps(l: int, s: int) -> int:
    """Closed form: r l - beta(s + 2, r - 1), r = repetitions(l, s)."""
    if l == 1:
        return 0
    r = repetitions(l, s)
    return r * l - beta(s + 2, r - 1)


class Executor:
    """Runs schedule actions against a Lattice (with adjoint buffers).

    The current forward state lives either in the lattice or in a slot.  A
    restore only moves that marker; an advance by one step followed by a
    store of the result is run as one step from the current slot straight
    into the target slot (Lattice.step_state), so a replayed segment goes
    from snapshot to snapshot without copying states in or out of the
    lattice.  Results are bitwise those of the plain sequence (set_state,
    step, get_state).  Reverse steps keep their d/dtau terms in the lattice
    (no reduction per step); run() adds them to dtau_acc before it returns."""

    LATTICE = -1

    def __init__(self, lat, dtau_acc, chain: bool = True):
        self.lat = lat
        self.dtau = dtau_acc
        self.chain = chain
        self.pending_dtau = False
        self.slots: dict[int, object] = {}
        self.where = Executor.LATTICE
        self.forward_steps = 0
        self.adjoint_steps = 0
        self.peak_slots = 0
        self.state_copies = 0

    def _slot(self, i):
        if i not in self.slots:
            self.slots[i] = self.lat.new_state()
            self.peak_slots = max(self.peak_slots, len(self.slots))
        return self.slots[i]

    def materialize(self):
        """Make the lattice hold the current forward state."""
        if self.where != Executor.LATTICE:
            self.lat.set_state(self.slots[self.where])
            self.state_copies += 1
            self.where = Executor.LATTICE

    def run(self, actions):
        i = 0
        while i < len(actions):
            act = actions[i]
            op = act[0]
            if op == "advance":
                a, b = act[1], act[2]
                nxt = actions[i + 1] if i + 1 < len(actions) else None
                if (self.chain and self.where != Executor.LATTICE and b - a == 1 and nxt is not None
                        and nxt[0] == "store" and nxt[1] == b and nxt[2] != self.where):
                    self.lat.step_state(self.slots[self.where], self._slot(nxt[2]))
                    self.where = nxt[2]
                    self.forward_steps += 1
                    i += 2
                    continue
                self.materialize()
                self.lat.step(b - a)
                self.forward_steps += b - a
            elif op == "store":
                if self.where == Executor.LATTICE:
                    self.lat.get_state(self._slot(act[2]))
                    self.state_copies += 1
                elif self.where != act[2]:
                    self._slot(act[2]).copy_(self.slots[self.where])
                    self.state_copies += 1
            elif op == "restore":
                if self.chain:
                    self.where = act[2]
                else:
                    self.lat.set_state(self.slots[act[2]])
                    self.state_copies += 1
                    self.where = Executor.LATTICE
            elif op == "adjoint":
                # d/dtau terms kept in the lattice, added to self.dtau at the end
                self.lat.adjoint_step(self.slots[act[2]], None)
                self.adjoint_steps += 1
                self.pending_dtau = True
            elif op == "free":
                pass   # slots are kept allocated and reused by index
            else:
                raise ValueError(op)
            i += 1
        if self.pending_dtau:
            self.lat.take_dtau(self.dtau)
            self.pending_dtau = False
