"""The batched form and the preheating configuration at its own dx and dt
against the FP64 oracle (not only against the library's solo path).

* Members of a batch of uneven FP64 lattices in mixed tile shapes (whole-row
  tiles, ragged x and z tiles, both z-march pipelines), stepped 100 steps
  with the batched pass and its captured graph, each within the FP64 gate of
  the oracle run of the same lattice.
* The two-field preheating model of Sec. 3.1 with the dx and dt of its
  256^3 and 128^3 runs (L = 10, dt = 0.0025, 6th order) on a 32^3 lattice,
  100 steps, from the device's own vacuum state against the oracle's, in
  the pass shapes the 256^3 benchmark tunes to (FP64 and FP32 storage).
* 128^3 FP64 at 6th order in its tuned shape, five steps against the oracle
  on the full lattice.
"""
import numpy as np
import pytest

import oracle
import paper_1201_5029_amd as sl
import synth
from gpu_util import fluct_rel_l2, gpu_lattice, max_rel, oracle_lattice, rel_l2, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_L2 = 1e-4
FP32_RESID = 1e-3


@pytest.fixture(autouse=True)
def _forget_tuned_shapes():
    yield
    sl.symlat.autotune_forget()


# (n, tx, vx, tz, pf): whole-row tiles, ragged x tiles, ragged z chunks
BATCH_SHAPES = {
    1: [(16, 8, 2, 4, 1), (20, 10, 2, 5, 1), (24, 8, 2, 7, 1), (32, 16, 2, 32, 1)],
    2: [(16, 8, 2, 16, 2), (20, 16, 2, 6, 2), (24, 12, 2, 8, 2), (32, 8, 2, 5, 2)],
}


@pytest.mark.parametrize("pf", [1, 2])
def test_batch_fp64_members_vs_oracle(pf):
    c = synth.preheat(n=16)
    gs, os_ = [], []
    for j, (n, tx, vx, tz, pf_) in enumerate(BATCH_SHAPES[pf]):
        base = [1.0 + (j - 2) * 1e-5, 0.0]
        phi, pi = synth.gaussian_state(n, 2, 3100 + j, phi_base=base, phi_amp=1e-4, pi_amp=1e-4)
        g = gpu_lattice(n, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"],
                        tile=(tx, vx, tz, pf_))
        gs.append(g)
        os_.append(oracle_lattice(n, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"]))
    b = sl.Batch()
    for g in gs:
        b.add(g)
    b.step(37, c["dt"], 4)          # graph chunks of 8 steps plus an eager tail
    b.step(63, c["dt"], 4)
    b.synchronize()
    for o in os_:
        o.evolve(100, c["dt"], 4)
    for j, (g, o) in enumerate(zip(gs, os_)):
        phi, pi = g.get_fields()
        _, a, pa = g.background()
        ef, ep = max_rel(phi, o.phi), max_rel(pi, o.pi)
        ea, epa = abs(a - o.a) / o.a, abs(pa - o.p_a) / abs(o.p_a)
        say("batched member", j, "n", o.n, "tile", g.tile(), "errors", ef, ep, ea, epa)
        assert max(ef, ep, ea, epa) <= FP64_TOL, (j, o.n)
    b.close()


def _preheat_same_dx(n_full, precision, n=32):
    c = synth.preheat(n=n, order=6, dt=0.0025, precision=precision, L=10.0 * n / n_full)
    return c


def _oracle_from_recipe(c, steps):
    o = oracle.Lattice(c["n"], c["L"], oracle.Potential(c["potential"], c["params"]), mpl=c["mpl"])
    o.init_fluctuations(c["phi0"], c["pi0"], c["fluct"], c["amplitude"], c["seed"])
    o.evolve(steps, c["dt"], c["order"])
    return o


@pytest.mark.parametrize("n_full", [256, 128])
def test_preheat_same_dx_fp64(n_full):
    """FP64 in the 256^3 benchmark's tile family (64 lanes, 2 sites per
    lane, one plane of prefetch), several z-chunks."""
    c = _preheat_same_dx(n_full, "f64")
    g = sl.from_recipe(c)
    g.set_tile(64, 2, 8, 1)
    g.evolve(100, c["dt"], 6)
    o = _oracle_from_recipe(c, 100)
    phi, pi = g.get_fields()
    _, a, pa = g.background()
    ef, ep = max_rel(phi, o.phi), max_rel(pi, o.pi)
    ea, epa = abs(a - o.a) / o.a, abs(pa - o.p_a) / abs(o.p_a)
    say("preheat 32^3 at the dx of %d^3, fp64" % n_full, ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL


@pytest.mark.parametrize("n_full", [256, 128])
def test_preheat_same_dx_fp32(n_full):
    """FP32 storage in the benchmark's FP32 tile family (64 lanes, 4 sites
    per lane, two planes of prefetch)."""
    c = _preheat_same_dx(n_full, "f32")
    g = sl.from_recipe(c)
    g.set_tile(64, 4, 8, 2)
    g.evolve(100, c["dt"], 6)
    resid = g.energies()["friedmann_residual"]
    o = _oracle_from_recipe(c, 100)
    phi, pi = g.get_fields()
    e1, e2 = rel_l2(phi, o.phi), rel_l2(pi, o.pi)
    fl = max(fluct_rel_l2(phi, o.phi), fluct_rel_l2(pi, o.pi))
    _, a, _ = g.background()
    say("preheat 32^3 at the dx of %d^3, fp32 rel-L2" % n_full, e1, e2, "fluctuations", fl,
        "residual", resid, "a", abs(a - o.a) / o.a)
    assert max(e1, e2) <= FP32_L2 and fl <= FP32_L2 and resid <= FP32_RESID
    assert abs(a - o.a) <= 1e-6 * o.a


def test_preheat128_fp64_tuned_shape_vs_oracle():
    """128^3 at 6th order in the shape the tuner picks for it (64 lanes,
    2 sites per lane, 16-plane chunks, two planes of prefetch), five steps
    from the device vacuum state against the oracle's on the full lattice."""
    c = synth.preheat(n=128, order=6, dt=0.0025)
    g = sl.from_recipe(c)
    g.set_tile(64, 2, 16, 2)
    g.evolve(5, c["dt"], 6)
    phi, pi = g.get_fields()
    _, a, pa = g.background()
    g.close()
    o = _oracle_from_recipe(c, 5)
    ef, ep = max_rel(phi, o.phi), max_rel(pi, o.pi)
    ea, epa = abs(a - o.a) / o.a, abs(pa - o.p_a) / abs(o.p_a)
    say("preheat 128^3 fp64 5 steps", ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL
