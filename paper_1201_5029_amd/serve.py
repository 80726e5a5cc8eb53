"""Serving loop: continuous batching of lattice runs on one GPU.

Requests (a workload recipe, a step count and an arrival time) are admitted
while a slot is free and their device footprint fits the memory budget; an
admitted run's state stays resident on the device, joins the shared batch at
the next tick and leaves it when its steps are done.  Every tick advances all
resident runs by the same number of steps with one captured batch step (one
fused pass per stage over every run's tiles), so work of runs that arrived at
different times overlaps on the device.  A run's result is bit-identical to
evolving it alone (same tile shape), because a batch step and an evolve call
apply the same per-tile arithmetic and the pending-drift bookkeeping makes
evolve(a) + evolve(b) equal to evolve(a + b).

The ensemble use is the separate-universe (Delta N) scan over initial
homogeneous values that the paper names (Sec. 2.4 and Sec. 4): each result
carries N = ln a at the end of its run.
"""
import math
import time
from collections import deque

import numpy as np

from .symlat import (Batch, device_memory, footprint_bytes, from_recipe, reset_from_recipe,
                     transient_bytes)


# Run kinds the batch tuner has seen in this process; the library gives
# later lattices of these kinds their tuned shapes when they join a batch.
_TUNED = set()


def _config(recipe):
    """What a lattice handle is made for: a retired run's handle serves a
    later request with the same configuration (re-initialised in place)."""
    return (recipe["n"], recipe["nfields"], recipe["L"], recipe.get("precision", "f64"),
            recipe.get("expand", True), recipe.get("mpl", 1.0), recipe.get("a0", 1.0),
            str(recipe.get("stencil")))


def _kind(recipe):
    return (recipe["n"], recipe["nfields"], recipe.get("precision", "f64"), recipe["potential"],
            str(recipe.get("stencil")))


class Request:
    def __init__(self, rid, recipe, arrival, steps=None):
        self.id = rid
        self.recipe = recipe
        self.arrival = float(arrival)
        self.steps = int(steps if steps is not None else recipe["steps"])
        cfg = dict(n=recipe["n"], nfields=recipe["nfields"], L=recipe["L"],
                   precision=recipe.get("precision", "f64"))
        self.footprint = footprint_bytes(**cfg)
        self.transient = transient_bytes(**cfg)


class HandlePool:
    """Lattice handles of retired runs, kept for later requests with the
    same configuration (re-initialised in place, no device allocation).
    serve() makes one for the call and releases it at the end; a caller
    that passes its own keeps the handles between calls, as a server does
    between bursts of requests, and releases them with close()."""

    def __init__(self):
        self.kept = {}   # configuration -> [(lattice, bytes)]
        self.bytes = 0   # device bytes the kept handles hold

    def __len__(self):
        return sum(len(v) for v in self.kept.values())

    def spare_bytes(self, config):
        """Bytes of the handle take(config) would return, or None."""
        v = self.kept.get(config)
        return v[-1][1] if v else None

    def take(self, config):
        lat, b = self.kept[config].pop()
        self.bytes -= b
        return lat

    def put(self, config, lat, nbytes):
        self.kept.setdefault(config, []).append((lat, nbytes))
        self.bytes += nbytes

    def release_largest(self):
        """Release one kept handle of the configuration whose handles are
        largest (to make room for a request of another configuration)."""
        key = max((k for k in self.kept if self.kept[k]), key=lambda k: self.kept[k][-1][1])
        lat, b = self.kept[key].pop()
        lat.close()
        self.bytes -= b

    def close(self):
        for v in self.kept.values():
            for lat, _ in v:
                lat.close()
        self.kept = {}
        self.bytes = 0


def _resident_bytes(req, history):
    """Device bytes a served run holds while resident (with its per-step
    background record when history is on: 4 doubles per step)."""
    return req.footprint + (32 * req.steps if history else 0)


def serve(requests, dt, order, max_slots=64, tick_steps=25, hbm_budget=None,
          keep_fields=False, tune=True, history=False, pool=None, clock=time.perf_counter,
          sleep=time.sleep):
    """Run the request loop to completion.  Returns (results, stats).

    history: record (eta, a, p_a, rho) at the end of every step of each run
    on the device and return it with the result (for the uniform-density
    Delta N; rho is the density the library derives from the constraint).

    tune: before the first tick, let the batch autotuner pick the pass
    shapes of the runs admitted first unless their kinds were tuned before
    in this process (a run is never retiled once it has stepped; later runs
    of a tuned size start with the tuned shape).

    Handles of retired runs are kept and re-initialised for later requests
    with the same configuration (no device allocation or release on that
    path); kept handles count against the memory budget and are released
    when an admission needs their memory.  pool: a HandlePool that supplies
    and keeps the handles beyond this call (released by its owner); without
    one, the call's own pool is released at the end.

    results: one dict per request with id, n, arrival, admitted, completed,
    latency (s, completion - arrival), eta, a, p_a, efolds = ln a, the pass
    shape it ran with (tile) and the final fields when keep_fields.  stats:
    p50/p99 latency, makespan (loop start to the last completion), wall_s
    (the whole call, releases included), field site-updates, aggregate
    field-site-updates/s over the makespan, admissions deferred for memory,
    peak resident runs, handles reused."""
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    waiting = deque()
    active = {}  # id -> [request, lattice, steps_done, admitted_at]
    results = []
    own_pool = pool is None
    if own_pool:
        pool = HandlePool()
    if hbm_budget is None:
        free, _ = device_memory()
        hbm_budget = int(0.9 * (free + pool.bytes))   # kept handles are counted below
    used = 0        # resident runs
    deferred = 0
    peak = 0
    reused = 0
    last_done = 0.0
    batch = Batch()
    tuned = not tune
    t0 = clock()
    try:
        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission: arrival order, a free slot, and the footprints of the
            # resident runs plus the largest scratch one call of any of them
            # allocates (initial state, read-out) must fit
            while waiting and len(active) < max_slots:
                req = waiting[0]
                need = _resident_bytes(req, history)
                if need + req.transient > hbm_budget:
                    raise ValueError("request %r needs %d bytes, more than the budget %d"
                                     % (req.id, need + req.transient, hbm_budget))
                reserve = max([req.transient] + [a[0].transient for a in active.values()])
                cfg = _config(req.recipe)
                spare = pool.spare_bytes(cfg)
                if spare is not None:
                    if used + pool.bytes - spare + need + reserve > hbm_budget:
                        deferred += 1
                        break
                    lat = pool.take(cfg)
                    reset_from_recipe(lat, req.recipe)
                    if not history:
                        lat.set_history(0)   # a kept handle may still hold a record
                    reused += 1
                else:
                    # release kept handles of other configurations while short of memory
                    while used + pool.bytes + need + reserve > hbm_budget and pool.bytes > 0:
                        pool.release_largest()
                    if used + pool.bytes + need + reserve > hbm_budget:
                        deferred += 1
                        break
                    lat = from_recipe(req.recipe)
                waiting.popleft()
                if history:
                    lat.set_history(req.steps)
                batch.add(lat)
                used += need
                active[req.id] = [req, lat, 0, clock() - t0]
            peak = max(peak, len(active))
            if not active:
                if pending:
                    sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            if not tuned:
                kinds = {_kind(a[0].recipe) for a in active.values()}
                if not kinds <= _TUNED:
                    batch.autotune(reps=3)
                    _TUNED.update(kinds)
                tuned = True
            k = min(tick_steps, min(a[0].steps - a[2] for a in active.values()))
            batch.step(k, dt, order)
            batch.synchronize()
            done_at = clock() - t0
            for rid in list(active):
                entry = active[rid]
                entry[2] += k
                req, lat = entry[0], entry[1]
                if entry[2] >= req.steps:
                    eta, a, p_a = lat.background()
                    res = dict(id=rid, n=req.recipe["n"], arrival=req.arrival,
                               admitted=entry[3], completed=done_at,
                               latency=done_at - req.arrival, eta=eta, a=a, p_a=p_a,
                               efolds=math.log(a), steps=req.steps, tile=lat.tile())
                    if keep_fields:
                        res["phi"], res["pi"] = lat.get_fields()
                    if history:
                        res["history"] = lat.history()
                    results.append(res)
                    last_done = done_at
                    batch.remove(lat)
                    b = _resident_bytes(req, history)
                    pool.put(_config(req.recipe), lat, b)
                    used -= b
                    del active[rid]
    finally:
        for entry in active.values():
            entry[1].close()
        if own_pool:
            pool.close()
        batch.close()
    wall = clock() - t0
    makespan = last_done if results else wall
    lat_s = np.array([r["latency"] for r in results]) if results else np.zeros(1)
    sups = sum(r["n"] ** 3 * req_nf(requests, r["id"]) * r["steps"] for r in results)
    stats = dict(p50_s=float(np.percentile(lat_s, 50)), p99_s=float(np.percentile(lat_s, 99)),
                 makespan_s=makespan, wall_s=wall, field_site_updates=sups,
                 field_site_updates_per_s=sups / makespan if makespan > 0 else float("nan"),
                 deferred_for_memory=deferred, peak_resident=peak, runs=len(results),
                 reused=reused)
    return sorted(results, key=lambda r: r["id"]), stats


def delta_n(phi0, efolds):
    """Separate-universe statistics of a scan over initial homogeneous values
    (the Delta N use of Sec. 2.4): the e-fold count N of each run against
    its initial field phi0 is fitted by least squares with
    N = N0 + N1 d + N2 d^2 / 2, d = phi0 - mean(phi0).  Returns N0, N1, N2,
    the spread sigma_N of N over the scan and the local non-Gaussianity
    f_NL = (5/6) N2 / N1^2 of the Delta N expansion."""
    phi0 = np.asarray(phi0, dtype=np.float64)
    N = np.asarray(efolds, dtype=np.float64)
    if phi0.shape != N.shape or phi0.size < 3:
        raise ValueError("need matching phi0 and N arrays with at least 3 runs")
    d = phi0 - phi0.mean()
    A = np.stack([np.ones_like(d), d, 0.5 * d * d], axis=1)
    (N0, N1, N2), *_ = np.linalg.lstsq(A, N, rcond=None)
    return dict(N0=float(N0), N1=float(N1), N2=float(N2), sigma_N=float(np.std(N)),
                f_NL=float(5.0 / 6.0 * N2 / (N1 * N1)) if N1 != 0 else float("nan"),
                runs=int(N.size))


def uniform_density_efolds(a, rho, rho_ref):
    """ln a where rho first falls to rho_ref, interpolating ln a linearly in
    ln rho between the two recorded steps around the crossing (exact for a
    power law rho ~ a^-p); NaN if rho stays above rho_ref, ln a[0] if it
    starts below."""
    a = np.asarray(a, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    below = np.nonzero(rho <= rho_ref)[0]
    if below.size == 0:
        return float("nan")
    k = int(below[0])
    if k == 0:
        return float(math.log(a[0]))
    x0, x1 = math.log(rho[k - 1]), math.log(rho[k])
    y0, y1 = math.log(a[k - 1]), math.log(a[k])
    t = (math.log(rho_ref) - x0) / (x1 - x0)
    return float(y0 + t * (y1 - y0))


def req_nf(requests, rid):
    for r in requests:
        if r.id == rid:
            return r.recipe["nfields"]
    return 0
