"""Parity at the benchmark's full size and launch configuration: the 256^3
two-field preheating lattice, 6th order, dt = 0.0025, in the tile shape the
benchmark uses, one composed step (7 fused passes) against the oracle run on
the full lattice; plus properties that hold at any size."""
import numpy as np
import pytest

import oracle
import paper_1201_5029_amd as sl
import synth
from gpu_util import max_rel, rel_l2, say

pytestmark = pytest.mark.gpu


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
    g64.evolve(100, c["dt"], 6)
    g32.evolve(100, c["dt"], 6)
    r64 = g64.energies()["friedmann_residual"]
    r32 = g32.energies()["friedmann_residual"]
    f64, p64 = g64.get_fields()
    f32, p32 = g32.get_fields()
    say("256^3 100 steps: residual f64", r64, "f32", r32, "rel-L2", rel_l2(f32, f64), rel_l2(p32, p64))
    assert r64 < 1e-9 and r32 < 1e-3
    assert rel_l2(f32, f64) < 1e-4 and rel_l2(p32, p64) < 1e-4
