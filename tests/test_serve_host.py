"""Host logic of the serving loop (admission by free slots and footprint,
continuous batching in ticks, completion bookkeeping, latency statistics),
driven on the CPU with stand-ins for the device lattice and batch."""
import math

import pytest

from paper_1201_5029_amd import serve


class FakeLattice:
    made = []

    def __init__(self, recipe):
        self.recipe = recipe
        self.steps = 0
        self.closed = False
        self.inits = 1
        FakeLattice.made.append(self)

    def reset(self, recipe):
        assert not self.closed
        self.recipe = recipe
        self.steps = 0
        self.inits += 1
        return self

    def background(self):
        return 0.01 * self.steps, 1.0 + 0.001 * self.steps, -1.0

    def tile(self):
        return (16, 2, 16, 8, 2)

    def set_history(self, cap):
        self.cap = cap

    def history(self):
        return ([], [], [], [])

    def get_fields(self):
        return None, None

    def close(self):
        self.closed = True


class FakeBatch:
    log = []

    def __init__(self):
        self.members = []
        self.tuned = 0

    def add(self, lat):
        self.members.append(lat)

    def remove(self, lat):
        self.members.remove(lat)

    def autotune(self, reps=3):
        self.tuned += 1
        return 0.1

    def step(self, k, dt, order):
        FakeBatch.log.append((k, len(self.members)))
        for m in self.members:
            m.steps += k

    def synchronize(self):
        pass

    def close(self):
        pass


class Clock:
    """Simulated time: each batched step of a tick costs 1 ms per member."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


@pytest.fixture
def fake(monkeypatch):
    clock = Clock()
    FakeBatch.log = []

    class TimedBatch(FakeBatch):
        def step(self, k, dt, order):
            super().step(k, dt, order)
            clock.t += 1e-3 * k * len(self.members)

    monkeypatch.setattr(serve, "Batch", TimedBatch)
    monkeypatch.setattr(serve, "from_recipe", FakeLattice)
    monkeypatch.setattr(serve, "reset_from_recipe", lambda lat, r: lat.reset(r))
    FakeLattice.made = []
    monkeypatch.setattr(serve, "footprint_bytes", lambda **kw: 100 * kw["n"])
    monkeypatch.setattr(serve, "transient_bytes", lambda **kw: 10 * kw["n"])
    serve._TUNED.clear()
    return clock


def _req(i, n, t, steps):
    r = dict(n=n, nfields=2, L=10.0, precision="f32", potential="chaotic2", steps=steps)
    return serve.Request(i, r, t)


def test_admission_slots_and_ticks(fake):
    reqs = [_req(i, 32, 0.0, 30) for i in range(5)]
    res, st = serve.serve(reqs, 0.005, 4, max_slots=2, tick_steps=20, hbm_budget=10 ** 9,
                          clock=fake, sleep=fake.sleep)
    assert st["runs"] == 5 and st["peak_resident"] == 2
    # a tick never runs past the nearest completion: 20 then 10 steps
    assert FakeBatch.log[:2] == [(20, 2), (10, 2)]
    assert all(r["steps"] == 30 for r in res)
    assert all(r["completed"] >= r["admitted"] >= r["arrival"] for r in res)
    assert [r["id"] for r in res] == list(range(5))
    assert st["field_site_updates"] == 5 * 32 ** 3 * 2 * 30


def test_admission_by_footprint_defers(fake):
    reqs = [_req(i, 64, 0.0, 10) for i in range(4)]
    budget = 2 * 100 * 64 + 10 * 64          # two footprints and one call's scratch
    res, st = serve.serve(reqs, 0.005, 4, max_slots=8, tick_steps=10, hbm_budget=budget,
                          clock=fake, sleep=fake.sleep)
    assert st["peak_resident"] == 2 and st["deferred_for_memory"] >= 1 and st["runs"] == 4
    with pytest.raises(ValueError):
        serve.serve([_req(9, 64, 0.0, 10)], 0.005, 4, hbm_budget=100, clock=fake,
                    sleep=fake.sleep)


def test_admission_keeps_the_largest_scratch_free(fake):
    """A resident run whose calls need more scratch than the newcomer's
    keeps that scratch free: the newcomer waits although its own footprint
    and scratch would fit."""
    big, small = _req(0, 128, 0.0, 30), _req(1, 16, 0.0, 10)
    budget = 100 * 128 + 100 * 16 + 10 * 128 - 1
    assert 100 * 128 + 100 * 16 + 10 * 16 <= budget   # the newcomer's own needs fit
    res, st = serve.serve([big, small], 0.005, 4, max_slots=4, tick_steps=10,
                          hbm_budget=budget, clock=fake, sleep=fake.sleep)
    assert st["deferred_for_memory"] >= 1 and st["peak_resident"] == 1
    budget += 1                              # room for the larger scratch: both resident
    res, st = serve.serve([_req(0, 128, 0.0, 30), _req(1, 16, 0.0, 10)], 0.005, 4,
                          max_slots=4, tick_steps=10, hbm_budget=budget, clock=fake,
                          sleep=fake.sleep)
    assert st["peak_resident"] == 2


def test_history_counts_in_the_footprint(fake):
    reqs = [_req(i, 32, 0.0, 100) for i in range(2)]
    budget = 2 * 100 * 32 + 10 * 32          # fits two runs without their records
    res, st = serve.serve(reqs, 0.005, 4, max_slots=4, tick_steps=50, hbm_budget=budget,
                          history=True, clock=fake, sleep=fake.sleep)
    assert st["peak_resident"] == 1 and st["runs"] == 2


def test_retired_handles_serve_later_requests(fake):
    """With two slots, five requests of one configuration need only two
    handles: retired ones are re-initialised for the next request; every
    handle is released by the end; the makespan ends at the last completion."""
    reqs = [_req(i, 32, 0.0, 20) for i in range(5)]
    res, st = serve.serve(reqs, 0.005, 4, max_slots=2, tick_steps=20, hbm_budget=10 ** 9,
                          clock=fake, sleep=fake.sleep)
    assert st["runs"] == 5 and st["reused"] == 3 and len(FakeLattice.made) == 2
    assert sum(m.inits for m in FakeLattice.made) == 5
    assert all(m.closed for m in FakeLattice.made)
    assert all(r["efolds"] == pytest.approx(math.log(1.0 + 0.001 * 20)) for r in res)
    assert st["makespan_s"] == max(r["completed"] for r in res) <= st["wall_s"]


def test_kept_handles_are_released_for_memory(fake):
    """A kept handle of another configuration is released when a new
    request needs its memory; one of the same configuration is reused."""
    big, small = _req(0, 128, 0.0, 10), _req(1, 16, 0.0, 10)
    budget = 100 * 128 + 10 * 128                  # one big run, or one small one
    res, st = serve.serve([big, small], 0.005, 4, max_slots=4, tick_steps=10,
                          hbm_budget=budget, clock=fake, sleep=fake.sleep)
    assert st["runs"] == 2 and st["reused"] == 0 and st["peak_resident"] == 1
    first = FakeLattice.made[0]
    assert first.recipe["n"] == 128 and first.closed
    # same configuration again: the kept handle serves it
    FakeLattice.made = []
    res, st = serve.serve([_req(0, 16, 0.0, 10), _req(1, 16, 0.05, 10)], 0.005, 4,
                          max_slots=4, tick_steps=10, hbm_budget=budget, clock=fake,
                          sleep=fake.sleep)
    assert st["reused"] == 1 and len(FakeLattice.made) == 1


def test_late_arrivals_join_and_latency(fake):
    reqs = [_req(0, 32, 0.0, 40), _req(1, 32, 0.015, 20)]
    res, st = serve.serve(reqs, 0.005, 4, max_slots=4, tick_steps=10, hbm_budget=10 ** 9,
                          clock=fake, sleep=fake.sleep)
    r0, r1 = res
    # run 1 arrives while run 0 is stepping and joins at a later tick
    assert r1["admitted"] >= 0.015 and r1["admitted"] < r0["completed"]
    assert max(n for _, n in FakeBatch.log) == 2
    assert r1["latency"] == pytest.approx(r1["completed"] - 0.015)
    assert st["p99_s"] >= st["p50_s"] > 0
    assert r0["efolds"] == pytest.approx(math.log(1.0 + 0.001 * 40))


def test_tuning_once_per_run_kind(fake):
    serve.serve([_req(0, 32, 0.0, 10)], 0.005, 4, hbm_budget=10 ** 9, clock=fake,
                sleep=fake.sleep)
    assert len(serve._TUNED) == 1
    before = set(serve._TUNED)
    serve.serve([_req(1, 32, 0.0, 10)], 0.005, 4, hbm_budget=10 ** 9, clock=fake,
                sleep=fake.sleep)
    assert serve._TUNED == before


def test_a_caller_pool_keeps_handles_between_calls(fake):
    """A HandlePool passed by the caller supplies and keeps the handles: a
    second call with the same configurations creates none (every request
    re-initialises a kept handle, and one kept from a run with a record
    drops it when the new run keeps none), and nothing is released until
    the pool is closed."""
    pool = serve.HandlePool()
    res, st = serve.serve([_req(i, 32, 0.0, 20) for i in range(3)], 0.005, 4, max_slots=4,
                          tick_steps=20, hbm_budget=10 ** 9, history=True, pool=pool,
                          clock=fake, sleep=fake.sleep)
    assert st["reused"] == 0 and len(FakeLattice.made) == 3 and len(pool) == 3
    assert not any(m.closed for m in FakeLattice.made)
    assert all(m.cap == 20 for m in FakeLattice.made)
    assert pool.bytes == 3 * (100 * 32 + 32 * 20)
    res, st = serve.serve([_req(i, 32, 0.0, 20) for i in range(3)], 0.005, 4, max_slots=4,
                          tick_steps=20, hbm_budget=10 ** 9, pool=pool, clock=fake,
                          sleep=fake.sleep)
    assert st["reused"] == 3 and st["runs"] == 3 and len(FakeLattice.made) == 3
    assert all(m.inits == 2 and m.cap == 0 for m in FakeLattice.made)
    assert len(pool) == 3 and pool.bytes == 3 * 100 * 32
    assert not any(m.closed for m in FakeLattice.made)
    pool.close()
    assert all(m.closed for m in FakeLattice.made) and len(pool) == 0 and pool.bytes == 0
