"""GPU parity of the 27-point pass (any member of the cubic stencil family
of eq. (2.7)) against the FP64 oracle with the same weights: fields after
100 steps, ragged tiles, FP32 storage, observables, vacuum initial state,
the stability bound and the batched form."""
import math

import numpy as np
import pytest

import oracle
import paper_1201_5029_amd as sl
import synth
from gpu_util import compare_state, gpu_lattice, max_rel, oracle_lattice, rel_l2, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_L2_TOL = 1e-4

MEMBERS = {"27": oracle.STENCIL_27, "19": oracle.STENCIL_19,
           # not isotropic: exercises every weight with unrelated values
           "skew": (-(6 * 0.4 + 12 * 0.1 + 8 * 0.05), 0.4, 0.1, 0.05)}


def _state(n, seed=303, amp=1e-3):
    c = synth.preheat(n=n)
    phi, pi = synth.gaussian_state(n, 2, seed, phi_base=c["phi0"], phi_amp=amp, pi_amp=amp)
    return c, phi, pi


def _pair(c, phi, pi, st, precision="f64", tile=None):
    kw = dict(mpl=c["mpl"], a0=c["a0"], stencil=st)
    o = oracle_lattice(phi.shape[1], c["L"], c["potential"], c["params"], phi, pi, **kw)
    g = gpu_lattice(phi.shape[1], c["L"], c["potential"], c["params"], phi, pi,
                    precision=precision, tile=tile, **kw)
    return o, g


@pytest.mark.parametrize("name", sorted(MEMBERS))
def test_stencil_member_fp64_100_steps(name):
    st = MEMBERS[name]
    c, phi, pi = _state(24)
    o, g = _pair(c, phi, pi, st)
    say("stencil", name, "tile", g.tile(), "p_a", o.p_a, g.background()[2])
    assert g.stencil() == pytest.approx(st, abs=0)
    assert g.background()[2] == pytest.approx(o.p_a, rel=1e-12)
    g.evolve(100, c["dt"], 4)
    o.evolve(100, c["dt"], 4)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("stencil", name, "errors", ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL


@pytest.mark.parametrize("n,tile", [(20, (16, 1, 3, 1)), (33, (32, 1, 7, 1)),
                                    (36, (64, 1, 5, 1)), (18, (16, 1, 18, 1)),
                                    (20, (16, 2, 3, 1)), (36, (32, 2, 5, 1)),
                                    (34, (64, 2, 7, 1)), (32, (16, 2, 32, 1))])
def test_stencil27_ragged_tiles(n, tile):
    c, phi, pi = _state(n, seed=304)
    o, g = _pair(c, phi, pi, oracle.STENCIL_27, tile=tile)
    say("27-point ragged", n, g.tile())
    g.evolve(30, c["dt"], 6)
    o.evolve(30, c["dt"], 6)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("27-point ragged errors", ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL


def test_stencil27_fp32_storage():
    c, phi, pi = _state(32, seed=305, amp=1e-4)
    o, g = _pair(c, phi, pi, oracle.STENCIL_27, precision="f32")
    g.evolve(100, c["dt"], 4)
    o.evolve(100, c["dt"], 4)
    gphi, gpi = g.get_fields()
    e = g.energies()
    say("27-point fp32 rel-L2", rel_l2(gphi, o.phi), rel_l2(gpi, o.pi),
        "residual", e["friedmann_residual"])
    assert rel_l2(gphi, o.phi) <= FP32_L2_TOL and rel_l2(gpi, o.pi) <= FP32_L2_TOL
    assert e["friedmann_residual"] <= 1e-3


def test_stencil27_energies_and_split_invariance():
    c, phi, pi = _state(16, seed=306)
    o, g = _pair(c, phi, pi, oracle.STENCIL_27)
    g.evolve(7, c["dt"], 4)
    g.evolve(13, c["dt"], 4)
    o.evolve(20, c["dt"], 4)
    eg, eo = g.energies(), o.energies()
    say("27-point energies", eg["rho"], eo["rho"], eg["grad"][:2], eo["grad"])
    for key in ("rho", "pressure", "pot", "h_total"):
        assert eg[key] == pytest.approx(eo[key], rel=1e-10, abs=1e-10 * abs(eo["rho"]))
    for i in range(2):
        assert eg["grad"][i] == pytest.approx(eo["grad"][i], rel=1e-10)
    # evolve(7) + evolve(13) equals evolve(20) bit for bit
    h = gpu_lattice(16, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"],
                    stencil=oracle.STENCIL_27)
    h.evolve(20, c["dt"], 4)
    assert all(np.array_equal(x, y) for x, y in zip(g.get_fields(), h.get_fields()))


def test_stencil27_vacuum_init_matches_oracle():
    c = dict(synth.preheat(n=16), stencil=oracle.STENCIL_27)
    g = sl.from_recipe(c)
    o = oracle.Lattice(16, c["L"], oracle.Potential(c["potential"], c["params"]),
                       mpl=c["mpl"], stencil=oracle.STENCIL_27)
    o.init_fluctuations(c["phi0"], c["pi0"], "vacuum", c["amplitude"], c["seed"])
    phi, _ = g.get_fields()
    base = np.array(c["phi0"])[:, None, None, None]
    err = max_rel(phi - base, o.phi - base)
    say("27-point vacuum init error", err)
    assert err <= 1e-11
    assert g.background()[2] == pytest.approx(o.p_a, rel=1e-10)


def test_stencil_validation_and_stability_bound():
    g = sl.Lattice(16, 2, 10.0)
    g.set_potential("chaotic2", synth.preheat(n=16)["params"])
    with pytest.raises(sl.SymlatError):
        g.set_stencil((-6.0, 1.0, 0.1, 0.0))          # does not annihilate constants
    with pytest.raises(sl.SymlatError):
        g.set_stencil((-8.0, 1.0, 0.1, 0.05))        # not normalised
    with pytest.raises(sl.SymlatError):
        g.set_stencil((math.nan, 1.0, 0.0, 0.0))
    g.set_stencil("27")
    assert g.tile()[4] == 1                            # pf = 1
    with pytest.raises(sl.SymlatError):
        g.set_tile(64, 4, 0, 1)                        # the 27-point pass has vx <= 2
    with pytest.raises(sl.SymlatError):
        g.set_tile(64, 2, 0, 2)                        # and pf = 1
    g.init_fluctuations([1.0, 0.0], [0.0, 0.0], "none")
    # omega_max = sqrt(k_max^2/dx^2 + max m^2): the 27-point zone maximum is
    # at k = (pi, pi, pi), 64/15, below the 7-point 12
    dx = 10.0 / 16
    m2 = synth.PREHEAT_G * 1.0
    lim = sl.stability_limit(4)
    k27 = oracle.stencil_max_keff2(oracle.STENCIL_27)
    dt_ok = 0.999 * lim / math.sqrt(k27 / dx ** 2 + m2)
    dt_bad = 1.001 * lim / math.sqrt(k27 / dx ** 2 + m2)
    g.evolve(1, dt_ok, 4)
    with pytest.raises(sl.SymlatError):
        g.evolve(1, dt_bad, 4)


def test_stencil27_batched_equals_alone():
    recipes = [dict(synth.preheat(n=n, order=4, dt=0.005, precision="f32", seed=20120300 + j),
                    stencil="27") for j, n in enumerate([32, 64, 48])]
    alone = [sl.from_recipe(r) for r in recipes]
    mixed = [sl.from_recipe(r) for r in recipes]
    b = sl.Batch()
    for m in mixed:
        b.add(m)
    plain = sl.from_recipe(synth.preheat(n=32, precision="f32"))
    with pytest.raises(sl.SymlatError):
        b.add(plain)                       # 7-point member in a 27-point batch
    with pytest.raises(sl.SymlatError):
        mixed[0].set_stencil("7")          # kind change inside a batch
    for rep in range(3):
        b.step(10, 0.005, 4)
        for a in alone:
            a.evolve(10, 0.005, 4)
        b.synchronize()
        for a, m in zip(alone, mixed):
            fa, pa = a.get_fields()
            fm, pm = m.get_fields()
            assert np.array_equal(fa, fm) and np.array_equal(pa, pm) and a.background() == m.background()
