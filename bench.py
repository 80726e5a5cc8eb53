#!/usr/bin/env python3
"""Throughput of the symplectic FRW lattice step on one MI355X.

Default workload: two-field chaotic preheating on a 256^3 lattice, 6th-order
composition (7 fused stage passes per step), dt = 0.0025, FP64 fields,
self-consistent expansion, vacuum initial fluctuations built on the device.
Prints one JSON line:

  value       field-site-updates/s = n^3 * N_f * steps / wall time of the
              timed steps (inputs resident in HBM, both sides synchronised)
  roofline    dominant kernel (fused stage pass): algorithmic bytes per
              launch (4 * b * N_f * n^3: read phi, pi; write phi, pi) over its
              mean launch time from HIP events on the lattice's stream
  cpu_baseline the FP64 oracle timed for one step of the same workload on
              one host core
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--n", type=int, default=256)
    p.add_argument("--order", type=int, default=6)
    p.add_argument("--precision", default="f64", choices=["f64", "f32"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp32", action="store_true", help="skip the FP32-storage line")
    p.add_argument("--no-serve", action="store_true", help="skip the served ensemble")
    p.add_argument("--no-512", action="store_true", help="skip the 512^3 FP32 line")
    p.add_argument("--no-batched", action="store_true", help="skip the batched ensemble line")
    p.add_argument("--no-configs", action="store_true",
                   help="skip the 4th-order 256^3, 128^3 preheating and 128^3 oscillon lines")
    p.add_argument("--no-27", action="store_true", help="skip the 27-point stencil line")
    p.add_argument("--no-linear", action="store_true", help="skip the linearized-integrator line")
    p.add_argument("--serve-runs", type=int, default=96)
    p.add_argument("--serve-steps", type=int, default=500)
    p.add_argument("--tile", default=None,
                   help="tx,vx,tz,pf pass shape instead of the autotuner's choice")
    p.add_argument("--only", default=None,
                   help="comma-separated lines to run beside the main line, for profiler "
                        "runs: fp32, qball512, configs, batched, stencil27, linear, serve "
                        "(the others are skipped, as with their --no- switches)")
    p.add_argument("--shapes", default=None,
                   help="JSON object (or a file holding one) of pass shapes per line instead "
                        "of the tuners' choices: keys main, fp32, qball512, stencil27, "
                        "preheat256_order4, preheat128, oscillon128 ('tx,vx,tz,pf') and "
                        "batched (list of [n, tx, vx, tz, pf]); a run prints the shapes it "
                        "used under 'shapes'")
    return p.parse_args()


SHAPES = {}


def load_shapes(arg):
    """Pass shapes given on the command line (a JSON object or a file)."""
    if not arg:
        return {}
    text = open(arg).read() if os.path.exists(arg) else arg
    return json.loads(text)


def tile_str(t):
    """'tx,vx,tz,pf' of a tile() tuple (tx, vx, ty, tz, pf)."""
    return "%d,%d,%d,%d" % (t[0], t[1], t[3], t[4])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    m = hashlib.sha1()
    for f in ("kernels_step.hip", "device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1201_5029_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_traffic(workload, precision, shape):
    """Calibrated FETCH_SIZE + WRITE_SIZE bytes per pass recorded under
    profiles/ for this workload, precision and pass shape ('tx,vx,tz,pf',
    or 'n:tx,vx,tz,pf;...' for a batch), or None when no record matches or
    the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "pass_kernel_traffic.txt")
    if not os.path.exists(path):
        return None
    h = kernel_source_hash()
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == workload and f[1] == precision and f[2] == shape and f[3] == h:
            return int(f[4])
    return None


def traffic_fields(workload, precision, shape, algorithmic):
    """'traffic' (bytes per pass, or None) and its ratio to the algorithmic
    bytes, for a bench line."""
    t = measured_traffic(workload, precision, shape)
    return {"traffic": t, "traffic_ratio": None if t is None else t / algorithmic}


def _rel_l2(a, b):
    import numpy as np
    return max(float(np.linalg.norm(x - y) / np.linalg.norm(y)) for x, y in zip(a, b))


def _fluct_rel_l2(a, b):
    """rel-L2 of the fluctuation part (each array's mean removed)."""
    import numpy as np
    out = 0.0
    for x, y in zip(a, b):
        dy = y - y.mean()
        ny = np.linalg.norm(dy)
        if ny > 0:
            out = max(out, float(np.linalg.norm((x - x.mean()) - dy) / ny))
    return out


def measure(sl, recipe, steps, warmup, tile=None, fields=None, diag=None):
    """Autotune (or fix) the pass shape, time `steps` steps after a warm-up,
    then time the fused passes with HIP events over a second region of the
    same length.  With a dict `fields`, the final (phi, pi) are stored in it
    as FP64 host arrays; with a dict `diag`, the wall time of creating the
    lattice with its initial state and the median wall times of an energies
    call (the observables pass and its read-back) and of a spectra call are
    stored in it."""
    t_init = time.perf_counter()
    lat = sl.from_recipe(recipe)
    lat.synchronize()
    init_s = time.perf_counter() - t_init
    order, dt = recipe["order"], recipe["dt"]
    if tile:
        tx, vx, tz, pf = (int(x) for x in tile.split(","))
        lat.set_tile(tx, vx, tz, pf)
        log("pass shape fixed to", lat.tile())
    else:
        shape, best = lat.autotune(reps=5)
        log("autotuned pass shape (tx, vx, tz, pf) =", shape, "best stage %.4f ms" % best)
    # at least 33 steps, so that the captured 32-step chunk of the evolve
    # graph is built before the timed region
    lat.evolve(max(warmup, 33), dt, order)
    lat.synchronize()
    t0 = time.perf_counter()
    lat.evolve(steps, dt, order)
    lat.synchronize()
    wall = time.perf_counter() - t0
    # kernel-level timing of the fused pass over a second timed region
    lat.set_kernel_timing(True)
    lat.evolve(steps, dt, order)
    passes, pass_ms = lat.kernel_timing()
    lat.set_kernel_timing(False)
    e = lat.energies()
    if diag is not None:
        ts = []
        for _ in range(5):
            t = time.perf_counter()
            lat.energies()
            ts.append(time.perf_counter() - t)
        diag["init_s"] = init_s
        diag["energies_s"] = sorted(ts)[len(ts) // 2]
        # spectra of one field (DFT on the device, binned; Sec. 2.4): median
        # of three calls
        nbins = int(math.ceil(math.sqrt(3) * recipe["n"] / 2)) + 2   # up to the corner mode
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            lat.spectra(0, nbins)
            ts.append(time.perf_counter() - t)
        diag["spectra_s"] = sorted(ts)[1]
    tile = lat.tile()
    if fields is not None:
        fields["phi"], fields["pi"] = lat.get_fields()
    lat.close()
    return wall, passes, pass_ms, e, tile


def measure_served(sl, nruns, steps):
    """Delta-N ensemble served by the request loop (FP32 storage, 4th order):
    capacity from a burst (all requests at t = 0), then Poisson arrivals at
    0.8x that capacity; beside it the plain FP64 single-run path (each run
    alone, one after the other) on the same GPU."""
    import numpy as np
    import synth
    from paper_1201_5029_amd import serve
    recipes = synth.delta_n_scan(nruns=nruns, steps=steps)
    dt, order = recipes[0]["dt"], recipes[0]["order"]

    def reqs(arrivals):
        return [serve.Request(j, r, t) for j, (r, t) in enumerate(zip(recipes, arrivals))]

    # untimed warm-up, as a server does once at start: a short run of the
    # request mix (10 steps each) tunes the batch's pass shapes on that mix
    # and leaves one handle per slot in the server's pool
    pool = serve.HandlePool()
    warm = [serve.Request(j, r, 0.0, steps=10) for j, r in enumerate(recipes)]
    serve.serve(warm, dt, order, max_slots=nruns, tick_steps=10, pool=pool)
    burst_res, burst = serve.serve(reqs([0.0] * nruns), dt, order, max_slots=nruns, tick_steps=25,
                                   history=True, pool=pool)
    # uniform-density Delta N: ln a where rho = 3 m_pl^2 H^2 first falls to
    # the latest density every run reaches (the largest final density)
    rho = [res["history"][3] for res in burst_res]    # recorded on the device
    rho_ref = max(r[-1] for r in rho)
    n_ud = [serve.uniform_density_efolds(res["history"][1], rho[j], rho_ref)
            for j, res in enumerate(burst_res)]
    capacity = nruns / burst["makespan_s"]
    arrivals = synth.poisson_arrivals(nruns, 0.8 * capacity)
    pois_res, pois = serve.serve(reqs(arrivals), dt, order, max_slots=nruns, tick_steps=25,
                                 pool=pool)
    pool.close()
    # FP64 single-run path, one run after the other; error of the served
    # FP32 results against it (the FP64 path is the one pinned to the oracle)
    t0 = time.perf_counter()
    errs, sups = [], 0
    for j, r in enumerate(recipes):
        lat = sl.from_recipe(dict(r, precision="f64"))
        lat.evolve(steps, dt, order)
        _, a, _ = lat.background()
        errs.append(abs(np.log(a) - burst_res[j]["efolds"]) / np.log(a))
        sups += r["n"] ** 3 * r["nfields"] * steps
        lat.close()
    t64 = time.perf_counter() - t0
    return {
        "workload": "%d preheat runs, n in {32, 64, 96}, FP32 fields, order 4, %d steps" % (nruns, steps),
        "warm_up": "an untimed 10-step run of the request mix tunes the batch shapes and leaves "
                   "one handle per slot in the server's pool; every request re-initialises one",
        "burst": {"makespan_s": burst["makespan_s"], "value": burst["field_site_updates_per_s"],
                  "p50_s": burst["p50_s"], "p99_s": burst["p99_s"], "reused": burst["reused"]},
        "poisson": {"rate_per_s": 0.8 * capacity, "rate_vs_burst_capacity": 0.8,
                    "makespan_s": pois["makespan_s"],
                    "value": pois["field_site_updates_per_s"], "p50_s": pois["p50_s"],
                    "p99_s": pois["p99_s"], "peak_resident": pois["peak_resident"]},
        "fp64_single_runs": {"wall_s": t64, "value": sups / t64},
        "efolds_rel_err_fp32_vs_fp64_max": float(max(errs)),
        "delta_n": serve.delta_n([r["phi0"][0] for r in recipes],
                                 [res["efolds"] for res in burst_res]),
        "delta_n_uniform_density": serve.delta_n(
            [r["phi0"][0] for r, nu in zip(recipes, n_ud) if nu == nu],
            [nu for nu in n_ud if nu == nu]),
        "unit": "field-site-updates/s",
    }


def measure_batched(sl, nruns=96, steps=100):
    """The Delta-N ensemble (96 runs, n in {32, 64, 96}, FP32, 4th order)
    as one batch: pass shapes from the batch autotuner, then `steps` steps
    of the captured batch.  The batched pass time is the tuner's HIP-event
    timing of the pass alone."""
    import synth
    recipes = synth.delta_n_scan(nruns=nruns, steps=steps)
    dt, order = recipes[0]["dt"], recipes[0]["order"]
    lats = [sl.from_recipe(r) for r in recipes]
    fixed = {int(s[0]): s[1:] for s in SHAPES.get("batched", [])}
    for r, lat in zip(recipes, lats):
        if r["n"] in fixed:
            lat.set_tile(*fixed[r["n"]])
    b = sl.Batch()
    for lat in lats:
        b.add(lat)
    if fixed:
        pass_ms = b.time_pass(reps=5)
    else:
        pass_ms = b.autotune(reps=5)
    grid = b.grid()
    shapes = sorted(set((r["n"],) + tuple(lat.tile()) for r, lat in zip(recipes, lats)))
    b.step(10, dt, order)          # captures the batch's chunk graph before the timed region
    b.synchronize()
    t0 = time.perf_counter()
    b.step(steps, dt, order)
    b.synchronize()
    wall = time.perf_counter() - t0
    # error of one member of each size against the same run alone in FP64
    # (the FP64 path is the one pinned to the oracle)
    import numpy as np
    err, seen = {}, set()
    for j, r in enumerate(recipes):
        if r["n"] in seen:
            continue
        seen.add(r["n"])
        ref = sl.from_recipe(dict(r, precision="f64"))
        ref.evolve(10 + steps, dt, order)
        f64, p64 = ref.get_fields()
        f32, p32 = lats[j].get_fields()
        ref.close()
        err[str(r["n"])] = {"phi_rel_l2": _rel_l2(f32, f64), "pi_rel_l2": _rel_l2(p32, p64),
                            "fluct_rel_l2": max(_fluct_rel_l2(f32, f64), _fluct_rel_l2(p32, p64))}
    sites = sum(r["n"] ** 3 for r in recipes)
    stages = len(sl.composition_weights(order))
    bytes_pass = 4 * 4 * 2 * sites
    b.close()
    for lat in lats:
        lat.close()
    return {"workload": "%d preheat runs, n in {32, 64, 96}, FP32 fields, order 4, one batch"
                        % nruns,
            "value": sites * 2 * steps / wall, "unit": "field-site-updates/s",
            "ms_per_step": wall / steps * 1e3,
            "effective_GBs": bytes_pass * stages * steps / wall / 1e9,
            "pass_ms": pass_ms, "pass_achieved_GBs": bytes_pass / (pass_ms * 1e-3) / 1e9,
            "pass_frac": bytes_pass / (pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "bytes_per_pass": bytes_pass, "shapes_n_tx_vx_ty_tz_pf": shapes,
            **traffic_fields("deltaN96_order4", "f32",
                             ";".join("%d:%d,%d,%d,%d" % (q[0], q[1], q[2], q[4], q[5])
                                      for q in shapes), bytes_pass),
            "error_vs_fp64": dict(err, steps=10 + steps,
                                  against="one member of each size advanced alone in FP64"),
            "workgroups": {"launched": grid[1],
                           "form": "persistent" if grid[0] > 0 else "one per tile"}}


def measure_stencil27(sl, steps=50, warmup=5):
    """The 256^3 preheating workload (FP64, 6th order) with the isotropic
    27-point member of the stencil family: same algorithmic bytes per pass
    as the 7-point pass."""
    import synth
    r = dict(synth.preheat(n=256, order=6, dt=0.0025, precision="f64"), stencil="27")
    wall, passes, pass_ms, e, tile = measure(sl, r, steps, warmup, SHAPES.get("stencil27"))
    n3 = 256 ** 3
    avg = pass_ms / passes / 1e3
    return {"workload": "preheat two-field chaotic, 256^3, order 6, FP64, 27-point stencil "
                        "(-128, 14, 3, 1)/30",
            "value": n3 * 2 * steps / wall, "ms_per_step": wall / steps * 1e3,
            "pass_ms": avg * 1e3, "achieved_GBs": 4 * 8 * 2 * n3 / avg / 1e9,
            "frac": 4 * 8 * 2 * n3 / avg / 1e9 / HBM_PEAK_GBS, "tile": list(tile),
            **traffic_fields("preheat256_order6_st27", "f64", tile_str(tile), 4 * 8 * 2 * n3),
            "friedmann_residual": e["friedmann_residual"]}


FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CUs x 128 FP64 flops/clock x 2.4 GHz


def measure_linear(sl, n=256, steps=400, order=6, warmup=20):
    """Linearized integrator on the 256^3 preheating state: growth
    functions per k_eff^2 class, then every Fourier mode advanced.  The
    growth kernel is FP64 ALU work: per class column and stage
    2 (N_f^2 + 3 N_f) flops (two drifts, the k_eff^2 term and the Hessian
    product as fused multiply-adds)."""
    import synth
    r = synth.preheat(n=n, order=order, dt=0.0025, precision="f64")
    lat = sl.from_recipe(r)
    phi, pi = lat.get_fields()
    lat.close()
    nf = r["nfields"]
    lin = sl.Linear(n, nf, r["L"], mpl=r["mpl"])
    lin.set_potential(r["potential"], r["params"])
    lin.set_fields(phi, pi)
    del phi, pi
    lin.evolve(warmup, r["dt"], order)
    lin.synchronize()
    t0 = time.perf_counter()
    lin.evolve(steps, r["dt"], order)
    lin.synchronize()
    wall = time.perf_counter() - t0
    lin.set_kernel_timing(True)
    lin.evolve(steps, r["dt"], order)
    launches, g_ms, t_ms, a_ms = lin.kernel_timing()
    lin.set_kernel_timing(False)
    ncls = lin.classes()
    stages = len(sl.composition_weights(order)) * steps
    flops = ncls * 2 * nf * stages * 2 * (nf * nf + 3 * nf)
    achieved = flops / (g_ms * 1e-3) / 1e12
    lin.close()
    return {"workload": "linearized preheat two-field chaotic, %d^3, order %d, dt 0.0025, FP64"
                        % (n, order),
            "value": n ** 3 * nf * steps / wall, "unit": "field-site-updates/s",
            "ms_per_step": wall / steps * 1e3, "classes": ncls,
            "growth": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                       "launches": launches, "ms": g_ms, "flops": flops},
            "background_table_ms": t_ms,
            "apply_ms": a_ms,
            "apply_GBs": n ** 3 * 2 * 2 * nf * 16 / (a_ms * 1e-3) / 1e9 if a_ms > 0 else None}


# The paper's own runs of the 256^3 chaotic preheating model (4th order,
# FP64; seconds per step on the hardware it names), as field-site-updates/s.
PAPER_256_ORDER4 = {"Tesla C2050": 2 * 256 ** 3 / 0.132, "GTX 470": 2 * 256 ** 3 / 0.152}


def footprint_copy(sl, state, avg_pass_s):
    """For a lattice whose state fits the 256 MB MALL: the rate of a plain
    copy of the same footprint (state/2 bytes read and written, repeated, so
    it stays MALL-resident) -- the ceiling the pass is measured against."""
    if state > 256e6:
        return {}
    gbs = sl.symlat.hbm_copy_bench(state // 2, 50)
    return {"copy_same_footprint_GBs": gbs, "frac_of_footprint_copy": state / avg_pass_s / 1e9 / gbs}


def measure_config(sl, recipe, steps, key, workload, warmup=10):
    """One more workload on the single-lattice path: field-site-updates/s
    and the pass's HBM roofline (for lattices that fit the 256 MB MALL the
    bandwidth is effective, not HBM-only)."""
    wall, passes, pass_ms, e, tile = measure(sl, recipe, steps, warmup, SHAPES.get(key))
    n3 = recipe["n"] ** 3
    nf = recipe["nfields"]
    b = 8 if recipe["precision"] == "f64" else 4
    avg = pass_ms / passes / 1e3
    state = 4 * b * nf * n3
    return {"workload": recipe["workload"], "n": recipe["n"], "order": recipe["order"],
            "dtype": recipe["precision"], "value": n3 * nf * steps / wall,
            "ms_per_step": wall / steps * 1e3, "pass_ms": avg * 1e3,
            "achieved_GBs": state / avg / 1e9, "frac": state / avg / 1e9 / HBM_PEAK_GBS,
            "state_fits_mall": state <= 256e6, "tile": list(tile),
            **traffic_fields(workload, recipe["precision"], tile_str(tile), state),
            **footprint_copy(sl, state, avg),
            "friedmann_residual": e["friedmann_residual"]}


def collect_shapes(out, main_tile):
    """The pass shapes this run used, in the form --shapes takes."""
    sh = {"main": tile_str(main_tile)}
    for key, line in (("fp32", "fp32_storage"), ("qball512", "qball512_fp32"),
                      ("stencil27", "stencil27_fp64"), ("preheat256_order4", "preheat256_fp64_order4"),
                      ("preheat128", "preheat128_fp64_order6"),
                      ("oscillon128", "oscillon128_fp32_order4")):
        if line in out and "tile" in out[line]:
            sh[key] = tile_str(out[line]["tile"])
    if "batched_c4" in out:
        sh["batched"] = [[s[0], s[1], s[2], s[4], s[5]]
                         for s in out["batched_c4"]["shapes_n_tx_vx_ty_tz_pf"]]
    return sh


def fp64_error(sl, recipe, tile, steps=100):
    """An FP32-storage line against the same recipe in FP64 storage on the
    GPU (the path the tests pin to the oracle), `steps` steps from the same
    device initial state: rel-L2 of the full fields and of their
    fluctuation parts."""
    lat = sl.from_recipe(recipe)
    lat.set_tile(*[int(x) for x in tile_str(tile).split(",")])
    lat.evolve(steps, recipe["dt"], recipe["order"])
    f, q = lat.get_fields()
    lat.close()
    ref = sl.from_recipe(dict(recipe, precision="f64"))
    ref.evolve(steps, recipe["dt"], recipe["order"])
    f64, p64 = ref.get_fields()
    ref.close()
    return {"phi_rel_l2": _rel_l2(f, f64), "pi_rel_l2": _rel_l2(q, p64),
            "fluct_rel_l2": max(_fluct_rel_l2(f, f64), _fluct_rel_l2(q, p64)),
            "steps": steps, "against": "the FP64 run of the same workload on the GPU"}


def measure_qball512(sl, steps=20, warmup=3):
    """Q-ball configuration at 512^3 (FP32 fields, 6th order): the headline
    roofline point whose working set (4.3 GB) is far beyond the 256 MB MALL."""
    import synth
    r = synth.qball(n=512, precision="f32")
    f32 = {}
    wall, passes, pass_ms, e, tile = measure(sl, r, steps, warmup, SHAPES.get("qball512"),
                                             fields=f32)
    n3 = 512 ** 3
    avg = pass_ms / passes / 1e3
    # the same run in FP64 storage on the GPU (the path pinned to the oracle)
    total = max(warmup, 33) + 2 * steps
    ref = sl.from_recipe(dict(r, precision="f64"))
    ref.evolve(total, r["dt"], r["order"])
    f64, p64 = ref.get_fields()
    ref.close()
    err = {"phi_rel_l2": _rel_l2(f32["phi"], f64), "pi_rel_l2": _rel_l2(f32["pi"], p64),
           "fluct_rel_l2": max(_fluct_rel_l2(f32["phi"], f64), _fluct_rel_l2(f32["pi"], p64)),
           "steps": total, "against": "the FP64 run of the same workload on the GPU"}
    del f32, f64, p64
    return {"workload": "Q-ball log potential, 512^3, two fields, order 6, dt 0.005, FP32 fields",
            "error_vs_fp64": err,
            "value": n3 * 2 * steps / wall, "ms_per_step": wall / steps * 1e3,
            "pass_ms": avg * 1e3, "achieved_GBs": 4 * 4 * 2 * n3 / avg / 1e9,
            "frac": 4 * 4 * 2 * n3 / avg / 1e9 / HBM_PEAK_GBS, "tile": list(tile),
            **traffic_fields("qball512_order6", "f32", tile_str(tile), 4 * 4 * 2 * n3),
            "friedmann_residual": e["friedmann_residual"]}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "affinity_cpus": affinity}


def cpu_baseline(recipe):
    """FP64 oracle, one composed step of the same workload, one core."""
    import numpy as np  # noqa: F401
    import oracle
    pot = oracle.Potential(recipe["potential"], recipe["params"])
    o = oracle.Lattice(recipe["n"], recipe["L"], pot, mpl=recipe["mpl"])
    o.init_fluctuations(recipe["phi0"], recipe["pi0"], recipe["fluct"], recipe["amplitude"],
                        recipe["seed"])
    t0 = time.perf_counter()
    o.step(recipe["dt"], recipe["order"])
    t = time.perf_counter() - t0
    n3 = recipe["n"] ** 3
    return {"value": n3 * recipe["nfields"] / t, "unit": "field-site-updates/s", "cores": 1,
            "kind": "oracle", "host": host_cpu(),
            "sample": "1 step (%d stage passes) of the %d^3 %s workload, numpy FP64, %.1f s"
                      % (len(oracle.composition_weights(recipe["order"])), recipe["n"],
                         recipe["workload"], t)}


def _oracle_runs(job):
    """Worker of the ensemble comparator: the oracle on one ensemble run,
    `steps` composed steps timed after its initial state is built."""
    recipe, steps = job
    import oracle
    pot = oracle.Potential(recipe["potential"], recipe["params"])
    o = oracle.Lattice(recipe["n"], recipe["L"], pot, mpl=recipe["mpl"])
    o.init_fluctuations(recipe["phi0"], recipe["pi0"], recipe["fluct"], recipe["amplitude"],
                        recipe["seed"])
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step(recipe["dt"], recipe["order"])
    return recipe["n"] ** 3 * recipe["nfields"] * steps, time.perf_counter() - t0


def cpu_ensemble_baseline(steps=16):
    """CPU comparator of the served ensemble: P = (usable host CPUs, at most
    16) oracle processes, each advancing one run of the Delta-N scan (the
    scan's first P runs, FP64) `steps` steps at once; aggregate
    field-site-updates/s = total work / longest worker time.  Forked before
    this process touches the GPU."""
    import multiprocessing as mp
    import synth
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    procs = max(1, min(16, ncpu))
    runs = synth.delta_n_scan()[:procs]
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_runs, [(r, steps) for r in runs])
    work = sum(w for w, _ in res)
    longest = max(t for _, t in res)
    return {"value": work / longest, "unit": "field-site-updates/s", "cores": procs,
            "kind": "oracle", "sample": "%d processes, one Delta-N scan run each (n in %s), "
            "%d steps of order 4, numpy FP64, longest worker %.2f s"
            % (procs, sorted({r["n"] for r in runs}), steps, longest)}


def cpu_parity_config():
    """The oracle on the 32^3 parity configuration in full (200 steps of
    order 4), one core."""
    import synth
    r = synth.preheat(n=32)
    work, t = _oracle_runs((r, 200))
    return {"value": work / t, "unit": "field-site-updates/s", "cores": 1, "seconds": t,
            "sample": "32^3 preheat, 200 steps of order 4, numpy FP64"}


def main():
    args = parse()
    SHAPES.update(load_shapes(args.shapes))
    if args.only is not None:
        keep = set(x for x in args.only.split(",") if x)
        args.no_fp32 = "fp32" not in keep
        args.no_512 = "qball512" not in keep
        args.no_configs = "configs" not in keep
        args.no_batched = "batched" not in keep
        args.no_27 = "stencil27" not in keep
        args.no_linear = "linear" not in keep
        args.no_serve = "serve" not in keep
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the method's multi-GPU forms are not built "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    cpu_pre = {}
    if not args.no_cpu_baseline:
        # host-only legs first: the worker processes are forked before any GPU use
        log("cpu baselines (oracle: ensemble processes, parity configuration) ...")
        cpu_pre["ensemble"] = cpu_ensemble_baseline()
        cpu_pre["parity_32"] = cpu_parity_config()
    import paper_1201_5029_amd as sl
    import synth

    recipe = synth.preheat(n=args.n, order=args.order, dt=0.0025, steps=args.steps,
                           precision=args.precision)
    log("workload", recipe["workload"], args.n, "order", args.order, args.precision)
    f64_fields = {}
    diag = {}
    wall, passes, pass_ms, e, tile = measure(sl, recipe, args.steps, args.warmup,
                                             args.tile or SHAPES.get("main"),
                                             fields=f64_fields if args.precision == "f64" else None,
                                             diag=diag)
    nf = recipe["nfields"]
    n3 = args.n ** 3
    b = 8 if args.precision == "f64" else 4
    stages = len(sl.composition_weights(args.order))
    value = n3 * nf * args.steps / wall
    avg_pass_s = pass_ms / passes / 1e3
    bytes_per_pass = 4 * b * nf * n3
    achieved = bytes_per_pass / avg_pass_s / 1e9
    log("wall %.4f s, %.4f ms/step, pass %.4f ms (%d passes)" %
        (wall, wall / args.steps * 1e3, avg_pass_s * 1e3, passes))
    out = {
        "metric": "lattice site-updates/s per field",
        "value": value,
        "unit": "field-site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "preheat two-field chaotic, %d^3, order %d (%d stages), dt 0.0025, "
                               "%s fields, FP64 reductions and background" %
                               (args.n, args.order, stages, args.precision.upper()),
                   "n": args.n, "nfields": nf, "order": args.order, "stages": stages,
                   "tile": list(tile)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("preheat%d_order%d" % (args.n, args.order),
                                                 args.precision, tile_str(tile)),
                     "kernel": "pass_kernel", "avg_launch_ms": avg_pass_s * 1e3,
                     "bytes_per_launch": bytes_per_pass},
        "friedmann_residual": e["friedmann_residual"],
        "stage_updates_per_s": value * stages,
        # off the step path: the initial state (vacuum modes, DFTs, constraint)
        # and the observables pass (reads phi and pi once: 2 b N_f n^3 bytes)
        "diagnostics": {"init_ms": diag["init_s"] * 1e3,
                        "energies_ms": diag["energies_s"] * 1e3,
                        "energies_read_GBs": 2 * b * nf * n3 / diag["energies_s"] / 1e9,
                        "spectra_ms_one_field": diag["spectra_s"] * 1e3},
    }
    copy_gbs = sl.symlat.hbm_copy_bench(1 << 31, 10)
    out["roofline"]["copy_GBs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = achieved / copy_gbs
    if not args.no_fp32 and args.precision == "f64":
        r32 = dict(recipe, precision="f32")
        f32_fields = {}
        w32, p32, ms32, e32, tile32 = measure(sl, r32, args.steps, args.warmup, SHAPES.get("fp32"),
                                              fields=f32_fields)
        err = {"phi_rel_l2": _rel_l2(f32_fields["phi"], f64_fields["phi"]),
               "pi_rel_l2": _rel_l2(f32_fields["pi"], f64_fields["pi"]),
               "fluct_rel_l2": max(_fluct_rel_l2(f32_fields["phi"], f64_fields["phi"]),
                                   _fluct_rel_l2(f32_fields["pi"], f64_fields["pi"])),
               "steps": 2 * args.steps + max(args.warmup, 33),
               "against": "the FP64 run of the same workload on the GPU (pinned to the oracle)"}
        del f32_fields, f64_fields
        out["fp32_storage"] = {"error_vs_fp64": err,
            "value": n3 * nf * args.steps / w32, "ms_per_step": w32 / args.steps * 1e3,
            "pass_ms": ms32 / p32, "achieved_GBs": 4 * 4 * nf * n3 / (ms32 / p32 / 1e3) / 1e9,
            "frac": 4 * 4 * nf * n3 / (ms32 / p32 / 1e3) / 1e9 / HBM_PEAK_GBS,
            **traffic_fields("preheat%d_order%d" % (args.n, args.order), "f32", tile_str(tile32),
                             4 * 4 * nf * n3),
            "friedmann_residual": e32["friedmann_residual"], "tile": list(tile32)}
    if not args.no_512 and args.precision == "f64" and args.n == 256:
        log("512^3 FP32 Q-ball ...")
        out["qball512_fp32"] = measure_qball512(sl)
    if not args.no_configs and args.precision == "f64" and args.n == 256:
        log("other configurations ...")
        o4 = measure_config(sl, synth.preheat(n=256, order=4, dt=0.0025, precision="f64"), 100,
                            "preheat256_order4", "preheat256_order4")
        o4["paper_context"] = {k: {"value": v, "ratio": o4["value"] / v}
                               for k, v in PAPER_256_ORDER4.items()}
        out["preheat256_fp64_order4"] = o4
        out["preheat128_fp64_order6"] = measure_config(
            sl, synth.preheat(n=128, order=6, dt=0.0025, precision="f64"), 200, "preheat128",
            "preheat128_order6")
        osc = synth.oscillon(n=128)
        out["oscillon128_fp32_order4"] = measure_config(sl, osc, 200, "oscillon128",
                                                        "oscillon128_order4")
        out["oscillon128_fp32_order4"]["error_vs_fp64"] = fp64_error(
            sl, osc, out["oscillon128_fp32_order4"]["tile"])
    if not args.no_batched and args.precision == "f64" and args.n == 256:
        log("batched ensemble ...")
        out["batched_c4"] = measure_batched(sl)
    if not args.no_27 and args.precision == "f64" and args.n == 256:
        log("27-point stencil ...")
        out["stencil27_fp64"] = measure_stencil27(sl)
    if not args.no_linear and args.precision == "f64" and args.n == 256:
        log("linearized integrator ...")
        out["linear_fp64"] = measure_linear(sl)
    if not args.no_serve:
        log("served ensemble ...")
        out["served"] = measure_served(sl, args.serve_runs, args.serve_steps)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 1 step) ...")
        out["cpu_baseline"] = cpu_baseline(recipe)
        out["cpu_baseline"]["parity_32"] = cpu_pre["parity_32"]
        if "served" in out:
            out["served"]["cpu_ensemble_baseline"] = cpu_pre["ensemble"]
    out["shapes"] = collect_shapes(out, tile)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
