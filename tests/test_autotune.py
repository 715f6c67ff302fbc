"""Host-side checks of the schedule autotuner: candidates, round-robin timing
after a warm-up, restoring the run, and the pick (a stand-in stepper and a
stand-in torch whose events read a fake clock; no device)."""
import os
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2302_09005_amd import autotune  # noqa: E402


class _Buf:
    """A tensor stand-in: a value that clone/copy_ carry."""

    device = "cuda:0"

    def __init__(self, v):
        self.v = v

    def clone(self):
        return _Buf(self.v)

    def copy_(self, other):
        self.v = other.v


class _Stepper:
    """Each step costs a schedule-dependent time on the fake clock, slower
    while the clock is 'cold' (its first ``cold_steps`` steps)."""

    def __init__(self, clock, cost, cold_steps=0):
        self.clock, self.cost, self.cold = clock, cost, cold_steps
        self.a, self.b = _Buf(0), _Buf(0)
        self.patches, self.per_patch = _Buf(0), _Buf(0)
        self.schedule, self.workgroups = "persistent", 0
        self.plan = types.SimpleNamespace(n_units=10000)
        self.log = []
        self.capturing = None

    def step(self):
        if self.capturing is not None:  # graph capture: record, launch nothing
            self.capturing.append((self.schedule, self.workgroups))
            self.a, self.b = self.b, self.a
            return
        self.run((self.schedule, self.workgroups))

    def run(self, cand):
        c = self.cost[cand]
        if self.cold > 0:
            c *= 1.3
            self.cold -= 1
        self.clock[0] += c
        self.log.append(cand)
        self.a.v += 1
        self.patches.v += 1
        self.a, self.b = self.b, self.a


def _fake_torch(monkeypatch, clock, stepper):
    class Event:
        def __init__(self, enable_timing=False):
            self.t = None

        def record(self):
            self.t = clock[0]

        def elapsed_time(self, other):
            return (other.t - self.t) * 1e3  # ms, the clock counts seconds

    class Graph:
        """Replays the steps recorded while it was being captured."""

        def __init__(self):
            self.steps = []

        def replay(self):
            for c in self.steps:
                stepper[0].run(c)

    class Capture:
        def __init__(self, graph, stream=None):
            self.graph = graph

        def __enter__(self):
            stepper[0].capturing = self.graph.steps

        def __exit__(self, *exc):
            stepper[0].capturing = None

    class Ctx:
        def __init__(self, *a, **k):
            pass

        def __enter__(self):
            return self

        def __exit__(self, *exc):
            return False

    stream = types.SimpleNamespace(wait_stream=lambda other: None)
    cuda = types.SimpleNamespace(
        Event=Event, synchronize=lambda: None, CUDAGraph=Graph, graph=Capture,
        Stream=lambda: stream, stream=Ctx, current_stream=lambda: stream,
        get_device_properties=lambda dev: types.SimpleNamespace(multi_processor_count=256))
    monkeypatch.setitem(sys.modules, "torch", types.SimpleNamespace(cuda=cuda))
    wall = iter(range(10 ** 6))
    monkeypatch.setattr(autotune, "_warm", _counting_warm(autotune._warm))
    import time
    monkeypatch.setattr(time, "perf_counter", lambda: float(next(wall)) * 0.01)


def _counting_warm(fn):
    def w(stepper, seconds):
        stepper.warm_steps = len(stepper.log)
        fn(stepper, seconds)
        stepper.warm_steps = len(stepper.log) - stepper.warm_steps
    return w


def test_candidates():
    assert autotune.candidates(100, 256) == [("per_size", 0), ("persistent", 0)]
    got = autotune.candidates(5000, 256, patchwise=True)
    assert got == [("per_size", 0), ("persistent", 0), ("persistent", 512),
                   ("persistent", 1024), ("persistent", 2048), ("patchwise", 0)]


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("fastest", [("per_size", 0), ("persistent", 0), ("persistent", 1024)])
def test_tune_picks_the_fastest_and_restores_the_run(monkeypatch, fastest, graph):
    clock, holder = [0.0], [None]
    _fake_torch(monkeypatch, clock, holder)
    cands = autotune.candidates(5000, 256, patchwise=True)
    cost = {c: 300e-6 for c in cands}
    cost[("patchwise", 0)] = 0.25
    cost[fastest] = 280e-6
    # the first candidate would win if it alone were timed while the others
    # ran cold: the warm-up must absorb the cold steps
    st = holder[0] = _Stepper(clock, cost, cold_steps=8)
    best, table = autotune.tune(st, steps=3, warmup=1, patchwise=True, graph=graph)
    assert best == fastest
    assert st.warm_steps >= 8
    assert (st.schedule, st.workgroups) == fastest
    # restored: state, descriptors and the buffer order as before tuning
    assert st.a.v == 0 and st.b.v == 0 and st.patches.v == 0
    assert [(s, w) for s, w, _ in table] == cands
    by = {(s, w): u for s, w, u in table}
    assert by[fastest] == pytest.approx(280.0)


@pytest.mark.parametrize("graph", [True, False])
def test_tune_is_round_robin_and_times_patchwise_once(monkeypatch, graph):
    clock, holder = [0.0], [None]
    _fake_torch(monkeypatch, clock, holder)
    cands = autotune.candidates(5000, 256, patchwise=True)
    cost = {c: 300e-6 for c in cands}
    st = holder[0] = _Stepper(clock, cost)
    autotune.tune(st, steps=2, warmup=1, patchwise=True, rounds=3, graph=graph)
    timed = st.log[st.warm_steps:]
    # per round and candidate: an untimed warm-up (one graph replay, or one
    # eager step) and the timed steps; patch-wise once, one eager step
    per_round = [c for c in cands if c[0] != "patchwise"]
    k = 2 + 2 if graph else 1 + 2
    assert timed[:k] == [per_round[0]] * k and timed[k:2 * k] == [per_round[1]] * k
    assert timed.count(("patchwise", 0)) == 1
    for c in per_round:
        assert timed.count(c) == 3 * k
    # nothing ran while a graph was being captured
    assert st.log[:st.warm_steps] == [("persistent", 0)] * st.warm_steps
