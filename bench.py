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
    p.add_argument("--serve-runs", type=int, default=96)
    p.add_argument("--serve-steps", type=int, default=500)
    p.add_argument("--tile", default=None,
                   help="tx,vx,tz,pf pass shape instead of the autotuner's choice")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    m = hashlib.sha1()
    for f in ("kernels_step.hip", "device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1201_5029_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_traffic(workload, precision, tile):
    """Calibrated FETCH_SIZE + WRITE_SIZE bytes per pass recorded under
    profiles/ for this workload, precision and pass shape, or None when no
    record matches or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "pass_kernel_traffic.txt")
    if not os.path.exists(path):
        return None
    h = kernel_source_hash()
    tx, vx, _, tz, pf = tile
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if (f[0] == workload and f[1] == precision and [int(x) for x in f[2:6]] == [tx, vx, tz, pf]
                and f[6] == h):
            return int(f[7])
    return None


def measure(sl, recipe, steps, warmup, tile=None):
    lat = sl.from_recipe(recipe)
    order, dt = recipe["order"], recipe["dt"]
    if tile:
        tx, vx, tz, pf = (int(x) for x in tile.split(","))
        lat.set_tile(tx, vx, tz, pf)
        log("pass shape fixed to", lat.tile())
    else:
        shape, best = lat.autotune(reps=5)
        log("autotuned pass shape (tx, vx, tz, pf) =", shape, "best pass %.4f ms" % best)
    lat.evolve(warmup, dt, order)
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
    tile = lat.tile()
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

    burst_res, burst = serve.serve(reqs([0.0] * nruns), dt, order, max_slots=nruns, tick_steps=25)
    capacity = nruns / burst["makespan_s"]
    arrivals = synth.poisson_arrivals(nruns, 0.8 * capacity)
    pois_res, pois = serve.serve(reqs(arrivals), dt, order, max_slots=nruns, tick_steps=25)
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
        "burst": {"makespan_s": burst["makespan_s"], "value": burst["field_site_updates_per_s"],
                  "p50_s": burst["p50_s"], "p99_s": burst["p99_s"]},
        "poisson": {"rate_per_s": 0.8 * capacity, "makespan_s": pois["makespan_s"],
                    "value": pois["field_site_updates_per_s"], "p50_s": pois["p50_s"],
                    "p99_s": pois["p99_s"], "peak_resident": pois["peak_resident"]},
        "fp64_single_runs": {"wall_s": t64, "value": sups / t64},
        "efolds_rel_err_fp32_vs_fp64_max": float(max(errs)),
        "unit": "field-site-updates/s",
    }


def measure_qball512(sl, steps=20, warmup=3):
    """Q-ball configuration at 512^3 (FP32 fields, 6th order): the headline
    roofline point whose working set (4.3 GB) is far beyond the 256 MB MALL."""
    import synth
    r = synth.qball(n=512, precision="f32")
    wall, passes, pass_ms, e, tile = measure(sl, r, steps, warmup)
    n3 = 512 ** 3
    avg = pass_ms / passes / 1e3
    return {"workload": "Q-ball log potential, 512^3, two fields, order 6, dt 0.005, FP32 fields",
            "value": n3 * 2 * steps / wall, "ms_per_step": wall / steps * 1e3,
            "pass_ms": avg * 1e3, "achieved_GBs": 4 * 4 * 2 * n3 / avg / 1e9,
            "frac": 4 * 4 * 2 * n3 / avg / 1e9 / HBM_PEAK_GBS, "tile": list(tile),
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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the method's multi-GPU forms are not built "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import paper_1201_5029_amd as sl
    import synth

    recipe = synth.preheat(n=args.n, order=args.order, dt=0.0025, steps=args.steps,
                           precision=args.precision)
    log("workload", recipe["workload"], args.n, "order", args.order, args.precision)
    wall, passes, pass_ms, e, tile = measure(sl, recipe, args.steps, args.warmup, args.tile)
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
                                                 args.precision, tile),
                     "kernel": "pass_kernel", "avg_launch_ms": avg_pass_s * 1e3,
                     "bytes_per_launch": bytes_per_pass},
        "friedmann_residual": e["friedmann_residual"],
        "stage_updates_per_s": value * stages,
    }
    copy_gbs = sl.symlat.hbm_copy_bench(1 << 31, 10)
    out["roofline"]["copy_GBs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = achieved / copy_gbs
    if not args.no_fp32 and args.precision == "f64":
        r32 = dict(recipe, precision="f32")
        w32, p32, ms32, e32, tile32 = measure(sl, r32, args.steps, args.warmup)
        out["fp32_storage"] = {
            "value": n3 * nf * args.steps / w32, "ms_per_step": w32 / args.steps * 1e3,
            "pass_ms": ms32 / p32, "achieved_GBs": 4 * 4 * nf * n3 / (ms32 / p32 / 1e3) / 1e9,
            "friedmann_residual": e32["friedmann_residual"], "tile": list(tile32)}
    if not args.no_512 and args.precision == "f64" and args.n == 256:
        log("512^3 FP32 Q-ball ...")
        out["qball512_fp32"] = measure_qball512(sl)
    if not args.no_serve:
        log("served ensemble ...")
        out["served"] = measure_served(sl, args.serve_runs, args.serve_steps)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 1 step) ...")
        out["cpu_baseline"] = cpu_baseline(recipe)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
