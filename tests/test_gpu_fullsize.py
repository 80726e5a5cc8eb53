"""Parity at the benchmark's full size and launch configuration: the 256^3
two-field preheating lattice, 6th order, dt = 0.0025, in the tile shape the
benchmark times (the autotuner's choice, found the same way), one composed
step (7 fused passes) against the oracle run on the full lattice; plus
properties that hold at any size."""
import math

import numpy as np
import pytest

import oracle
import paper_1201_5029_amd as sl
import synth
from gpu_util import fluct_rel_l2, max_rel, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _forget_tuned_shapes():
    """Shapes tuned here stay out of later tests' lattices."""
    yield
    sl.symlat.autotune_forget()


@pytest.fixture(scope="module")
def start256():
    c = synth.preheat(n=256, order=6, dt=0.0025)
    phi, pi = synth.gaussian_state(256, 2, 2560, phi_base=c["phi0"], phi_amp=1e-4, pi_amp=1e-4)
    return c, phi, pi


def test_fullsize_fp64_one_step(start256):
    c, phi, pi = start256
    g = sl.Lattice(256, 2, c["L"], precision="f64", mpl=c["mpl"])
    g.set_potential(c["potential"], c["params"])
    g.set_fields(phi, pi, 1.0)
    g.autotune(reps=2)                       # the shape the benchmark times
    say("256^3 bench tile", g.tile())
    g.evolve(1, c["dt"], 6)
    gphi, gpi = g.get_fields()
    _, a, pa = g.background()
    g.close()
    o = oracle.Lattice(256, c["L"], oracle.Potential(c["potential"], c["params"]), mpl=c["mpl"])
    o.phi[...] = phi
    o.pi[...] = pi
    del phi, pi
    o.solve_constraint()
    o.step(c["dt"], 6)
    ef, ep = max_rel(gphi, o.phi), max_rel(gpi, o.pi)
    say("256^3 one step errors", ef, ep, abs(a - o.a) / o.a, abs(pa - o.p_a) / abs(o.p_a))
    assert max(ef, ep) <= 1e-10
    assert abs(a - o.a) <= 1e-12 * o.a and abs(pa - o.p_a) <= 1e-10 * abs(o.p_a)


def test_fullsize_fp32_vs_fp64_and_residual():
    """Bench-size FP32 storage against the FP64 library run (same device
    initial state) and the Friedmann residual after 100 steps."""
    c = synth.preheat(n=256, order=6, dt=0.0025)
    g64 = sl.from_recipe(c)
    g32 = sl.from_recipe(dict(c, precision="f32"))
    for g in (g64, g32):
        g.autotune(reps=2)                   # the shapes the benchmark times
    say("256^3 tiles", g64.tile(), g32.tile())
    g64.evolve(100, c["dt"], 6)
    g32.evolve(100, c["dt"], 6)
    r64 = g64.energies()["friedmann_residual"]
    r32 = g32.energies()["friedmann_residual"]
    f64, p64 = g64.get_fields()
    f32, p32 = g32.get_fields()
    fl = max(fluct_rel_l2(f32, f64), fluct_rel_l2(p32, p64))
    say("256^3 100 steps: residual f64", r64, "f32", r32, "rel-L2", rel_l2(f32, f64), rel_l2(p32, p64),
        "fluctuations", fl)
    assert r64 < 1e-9 and r32 < 1e-3
    assert rel_l2(f32, f64) < 1e-4 and rel_l2(p32, p64) < 1e-4 and fl < 1e-4


def test_oscillon128_fp32_vs_oracle():
    """Oscillon configuration at its full size (128^3, FP32 fields, 4th order,
    white initial fluctuations built on the device) against the oracle's own
    initial state and evolution, 20 steps."""
    c = synth.oscillon(n=128, precision="f32")
    g = sl.from_recipe(c)
    g.autotune(reps=2)                       # the shape the benchmark times
    g.evolve(20, c["dt"], c["order"])
    gphi, gpi = g.get_fields()
    resid = g.energies()["friedmann_residual"]
    o = oracle.Lattice(128, c["L"], oracle.Potential(c["potential"], c["params"]), mpl=c["mpl"])
    o.init_fluctuations(c["phi0"], c["pi0"], c["fluct"], c["amplitude"], c["seed"])
    o.evolve(20, c["dt"], c["order"])
    e1, e2 = rel_l2(gphi, o.phi), rel_l2(gpi, o.pi)
    # the fluctuation part alone (amplitude 1e-4 around 0.8)
    e3, e4 = fluct_rel_l2(gphi, o.phi), fluct_rel_l2(gpi, o.pi)
    say("oscillon 128^3 fp32 rel-L2", e1, e2, "fluctuations", e3, e4, "residual", resid)
    assert max(e1, e2) <= 1e-4 and resid <= 1e-3 and max(e3, e4) <= 1e-4


def test_qball512_fp32():
    """Q-ball configuration at its full size (512^3, FP32 fields, 6th order):
    FP32 against the FP64 library path (which is pinned to the oracle), the
    Friedmann residual, and the same model at 32^3 with the same dx and dt
    against the oracle."""
    c = synth.qball(n=512, precision="f32")
    g32 = sl.from_recipe(c)
    g32.autotune(reps=2)                     # the shape the benchmark times
    g32.evolve(20, c["dt"], c["order"])
    r32 = g32.energies()["friedmann_residual"]
    f32, p32 = g32.get_fields()
    g32.close()
    g64 = sl.from_recipe(dict(c, precision="f64"))
    g64.evolve(20, c["dt"], c["order"])
    f64, p64 = g64.get_fields()
    g64.close()
    e1, e2 = rel_l2(f32, f64), rel_l2(p32, p64)
    e3, e4 = fluct_rel_l2(f32, f64), fluct_rel_l2(p32, p64)
    say("qball 512^3 fp32 vs fp64", e1, e2, "fluctuations", e3, e4, "residual", r32)
    assert max(e1, e2) <= 1e-4 and r32 <= 1e-3 and max(e3, e4) <= 1e-4
    del f32, p32, f64, p64
    # same dx and dt on a 32^3 lattice, FP64 against the oracle
    small = dict(c, n=32, L=c["L"] * 32 / 512, precision="f64")
    g = sl.from_recipe(small)
    g.evolve(20, c["dt"], c["order"])
    o = oracle.Lattice(32, small["L"], oracle.Potential(c["potential"], c["params"]), mpl=c["mpl"])
    o.init_fluctuations(c["phi0"], c["pi0"], c["fluct"], c["amplitude"], c["seed"])
    o.evolve(20, c["dt"], c["order"])
    gphi, gpi = g.get_fields()
    ef, ep = max_rel(gphi, o.phi), max_rel(gpi, o.pi)
    say("qball 32^3 same dx fp64 vs oracle", ef, ep)
    assert max(ef, ep) <= 1e-10


def test_largest_side_fp32_white():
    """n = 1024, the largest side the library accepts (two FP32 fields,
    4 x 8.6 GB): pass shapes within the grid bounds, two 4th-order steps,
    the Friedmann residual and the background against the homogeneous
    expectation (a grows, p_a stays negative)."""
    n = 1024
    lat = sl.Lattice(n, 2, 40.0, precision="f32", mpl=synth.PREHEAT_MPL)
    lat.set_potential("chaotic2", (1.0, 100.0))
    lat.init_fluctuations([1.0, 0.0], [0.0, 0.0], "white", 1e-6, 20120130)
    tx, vx, ty, tz, pf = lat.tile()
    blocks = math.ceil(n / (tx * vx)) * math.ceil(n / ty) * math.ceil(n / tz)
    say("n=1024 tile", lat.tile(), "blocks", blocks)
    assert blocks <= 65536
    eta0, a0, pa0 = lat.background()
    lat.evolve(2, 0.005, 4)
    e = lat.energies()
    say("n=1024 residual", e["friedmann_residual"], "a", e["a"])
    assert e["friedmann_residual"] < 1e-3
    assert e["a"] > a0 and e["p_a"] < 0 and e["eta"] == pytest.approx(0.01)
    lat.close()


def test_deltan96_batch_fullsize_sampled():
    """The Delta-N ensemble at its full size (96 runs, n in {32, 64, 96},
    FP32, 4th order) as one batch in the shapes the batch tuner picks, as
    the benchmark runs it, 100 steps: sampled members equal the same runs
    advanced alone with the recorded shape, bit for bit; one member of each
    size is within the FP32 gate of the oracle run from the oracle's own
    initial state (rel-L2 per array, Friedmann residual); the background of
    every member grows."""
    steps = 100
    recipes = synth.delta_n_scan(nruns=96, steps=steps)
    lats = [sl.from_recipe(r) for r in recipes]
    b = sl.Batch()
    for lat in lats:
        b.add(lat)
    b.autotune(reps=2)
    a0 = [lat.background()[1] for lat in lats]
    b.step(steps, recipes[0]["dt"], recipes[0]["order"])
    b.synchronize()
    assert all(lat.background()[1] > a for lat, a in zip(lats, a0))
    checked = set()
    for j in (0, 17, 41, 64, 80, 95):          # every size is among them
        r = recipes[j]
        if r["n"] not in checked:
            checked.add(r["n"])
            o = oracle.Lattice(r["n"], r["L"], oracle.Potential(r["potential"], r["params"]),
                               mpl=r["mpl"])
            o.init_fluctuations(r["phi0"], r["pi0"], r["fluct"], r["amplitude"], r["seed"])
            o.evolve(steps, r["dt"], r["order"])
            gphi, gpi = lats[j].get_fields()
            e1, e2 = rel_l2(gphi, o.phi), rel_l2(gpi, o.pi)
            fl = max(fluct_rel_l2(gphi, o.phi), fluct_rel_l2(gpi, o.pi))
            resid = lats[j].energies()["friedmann_residual"]
            ea = abs(lats[j].background()[1] - o.a) / o.a
            say("delta-N member", j, r["n"], "vs oracle: rel-L2", e1, e2, "fluctuations", fl,
                "residual", resid, "a", ea)
            assert max(e1, e2) <= 1e-4 and fl <= 1e-4 and resid <= 1e-3 and ea <= 1e-6, j
            del o, gphi, gpi
        alone = sl.from_recipe(r)
        tx, vx, _, tz, pf = lats[j].tile()
        alone.set_tile(tx, vx, tz, pf)
        alone.evolve(steps, r["dt"], r["order"])
        fa, pa = alone.get_fields()
        fb, pb = lats[j].get_fields()
        say("delta-N member", j, r["n"], lats[j].tile())
        assert np.array_equal(fa, fb) and np.array_equal(pa, pb), j
        assert alone.background() == lats[j].background()
        alone.close()
    b.close()
    for lat in lats:
        lat.close()
