"""GPU parity of the HIP path against the FP64 oracle.

Gates: FP64 max relative field error <= 1e-10 after 100 steps (per array,
normalised by the array's max |value|); FP32 storage relative L2 <= 1e-4
after 100 steps in the linear regime with a Friedmann residual <= 1e-3.
Inputs are seeded synthetic states (synth) or each side's own initial-state
generator from the same seed."""
import math

import numpy as np
import pytest

import oracle
import paper_1201_5029_amd as sl
import synth
from gpu_util import compare_state, fluct_rel_l2, gpu_lattice, max_rel, oracle_lattice, rel_l2, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_L2_TOL = 1e-4
FP32_RESID_TOL = 1e-3


def _preheat_state(n, seed=101, amp=1e-4):
    c = synth.preheat(n=n)
    phi, pi = synth.gaussian_state(n, 2, seed, phi_base=c["phi0"], phi_amp=amp, pi_amp=amp)
    return c, phi, pi


def _pair(c, phi, pi, precision="f64", tile=None, **kw):
    args = dict(mpl=c["mpl"], a0=c["a0"])
    args.update(kw)
    o = oracle_lattice(phi.shape[1], c["L"], c["potential"], c["params"], phi, pi, **args)
    g = gpu_lattice(phi.shape[1], c["L"], c["potential"], c["params"], phi, pi,
                    precision=precision, tile=tile, **args)
    return o, g


# ---------------------------------------------------------------------------
# The preheating workload at 32^3 (4th order, dt = 0.005)
# ---------------------------------------------------------------------------

def test_preheat32_fp64_100_steps():
    c, phi, pi = _preheat_state(32)
    o, g = _pair(c, phi, pi)
    say("preheat32 fp64: constraint p_a", o.p_a, g.background()[2])
    assert g.background()[2] == pytest.approx(o.p_a, rel=1e-12)
    g.evolve(100, c["dt"], 4)
    o.evolve(100, c["dt"], 4)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("preheat32 fp64 errors", ef, ep, ea, epa)
    assert max(ef, ep) <= FP64_TOL
    assert ea <= FP64_TOL and epa <= FP64_TOL


def test_preheat32_end_to_end_fp64():
    """Library initial state (device SplitMix64 + DFT) and 100 steps versus
    the oracle's own initial state and 100 steps, same seed."""
    c = synth.preheat(n=32)
    g = sl.from_recipe(c)
    pot = oracle.Potential(c["potential"], c["params"])
    o = oracle.Lattice(32, c["L"], pot, mpl=c["mpl"])
    o.init_fluctuations(c["phi0"], c["pi0"], "vacuum", c["amplitude"], c["seed"])
    phi0, pi0 = g.get_fields()
    say("init error", max_rel(phi0 - np.array(c["phi0"])[:, None, None, None],
                              o.phi - np.array(c["phi0"])[:, None, None, None]))
    assert max_rel(phi0, o.phi) <= 1e-12
    # the fluctuation itself (not only the homogeneous value) agrees
    assert max_rel(phi0 - np.array(c["phi0"])[:, None, None, None],
                   o.phi - np.array(c["phi0"])[:, None, None, None]) <= 1e-11
    g.evolve(100, c["dt"], 4)
    o.evolve(100, c["dt"], 4)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("end-to-end errors", ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL
    e_g, e_o = g.energies(), o.energies()
    assert e_g["friedmann_residual"] < 1e-8
    assert e_g["rho"] == pytest.approx(e_o["rho"], rel=1e-10)


def test_preheat32_fp32_storage():
    c, phi, pi = _preheat_state(32)
    o, g = _pair(c, phi, pi, precision="f32")
    g.evolve(100, c["dt"], 4)
    o.evolve(100, c["dt"], 4)
    gphi, gpi = g.get_fields()
    e1, e2 = rel_l2(gphi, o.phi), rel_l2(gpi, o.pi)
    f1, f2 = fluct_rel_l2(gphi, o.phi), fluct_rel_l2(gpi, o.pi)
    resid = g.energies()["friedmann_residual"]
    _, a, pa = g.background()
    say("preheat32 fp32 rel-L2", e1, e2, "fluctuations", f1, f2, "residual", resid, "a", a, o.a)
    assert max(e1, e2) <= FP32_L2_TOL
    assert max(f1, f2) <= FP32_L2_TOL
    assert resid <= FP32_RESID_TOL
    assert a == pytest.approx(o.a, rel=1e-6)


def test_preheat32_end_to_end_fp32():
    c = synth.preheat(n=32, precision="f32")
    g = sl.from_recipe(c)
    pot = oracle.Potential(c["potential"], c["params"])
    o = oracle.Lattice(32, c["L"], pot, mpl=c["mpl"])
    o.init_fluctuations(c["phi0"], c["pi0"], "vacuum", c["amplitude"], c["seed"])
    g.evolve(100, c["dt"], 4)
    o.evolve(100, c["dt"], 4)
    gphi, gpi = g.get_fields()
    e1, e2 = rel_l2(gphi, o.phi), rel_l2(gpi, o.pi)
    f1, f2 = fluct_rel_l2(gphi, o.phi), fluct_rel_l2(gpi, o.pi)
    resid = g.energies()["friedmann_residual"]
    say("end-to-end fp32", e1, e2, "fluctuations", f1, f2, resid)
    assert max(e1, e2) <= FP32_L2_TOL and resid <= FP32_RESID_TOL
    assert max(f1, f2) <= FP32_L2_TOL


@pytest.mark.parametrize("order,steps", [(2, 30), (6, 20), (8, 10)])
def test_orders_fp64(order, steps):
    c, phi, pi = _preheat_state(16, seed=7)
    o, g = _pair(c, phi, pi)
    g.evolve(steps, c["dt"], order)
    o.evolve(steps, c["dt"], order)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("order", order, ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL


# ---------------------------------------------------------------------------
# Potential families, field counts, background terms
# ---------------------------------------------------------------------------

CASES = [
    ("oscillon", (1.0, 1.0, 0.2), [0.8], 24, 64.0 * 24 / 128, 335.41),
    ("qball", (1.0, -0.1, 1.0), [math.sqrt(2) * 1e-2, 0.0], 20, 100.0 * 20 / 512, 1.0),
    ("free", (1.0, 2.0, 0.5), [0.3, -0.2, 0.1], 16, 5.0, 0.9),
    ("free", tuple(0.5 + 0.25 * i for i in range(8)), [0.1 * (i + 1) for i in range(8)], 12, 4.0, 1.1),
]


@pytest.mark.parametrize("kind,params,base,n,L,mpl", CASES, ids=["oscillon", "qball", "free3", "free8"])
def test_potentials_fp64(kind, params, base, n, L, mpl):
    nf = len(base)
    phi, pi = synth.gaussian_state(n, nf, 33, phi_base=base, phi_amp=1e-3, pi_amp=1e-3)
    if kind == "qball":
        pi[1] += 0.5 * base[0]
    o = oracle_lattice(n, L, kind, params, phi, pi, mpl=mpl)
    g = gpu_lattice(n, L, kind, params, phi, pi, mpl=mpl)
    g.evolve(40, 0.01, 4)
    o.evolve(40, 0.01, 4)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say(kind, nf, ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL


def test_static_background_and_rad_matter_terms():
    c, phi, pi = _preheat_state(16, seed=3)
    o, g = _pair(c, phi, pi, expand=False, a0=1.3)
    g.evolve(30, 0.004, 4)
    o.evolve(30, 0.004, 4)
    ef, ep, _, _, st = compare_state(g, o)
    assert max(ef, ep) <= FP64_TOL and st[3] == 1.3
    o, g = _pair(c, phi, pi, rho_rad0=0.2, rho_mat0=0.1, a0=1.1)
    g.evolve(30, 0.004, 4)
    o.evolve(30, 0.004, 4)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("rad/matter", ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL


# ---------------------------------------------------------------------------
# Tiling edge cases: ragged x/y/z tiles, the smallest lattice, tile overrides
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,tile", [(4, None), (20, None), (36, None), (70, None),
                                    (36, (16, 1, 5)), (36, (64, 1, 7)), (33, (32, 1, 1)),
                                    (36, (32, 2, 5)), (20, (16, 2, 3)), (70, (64, 2, 9))])
def test_ragged_tiles(n, tile):
    c, phi, pi = _preheat_state(n, seed=n)
    o, g = _pair(c, phi, pi, tile=tile)
    say("tile", n, tile, g.tile())
    g.evolve(6, c["dt"], 4)
    o.evolve(6, c["dt"], 4)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("ragged", n, tile, ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL


@pytest.mark.parametrize("n,tile", [(36, (32, 2, 5)), (38, (16, 1, 4)), (64, None)])
def test_ragged_tiles_fp32(n, tile):
    c, phi, pi = _preheat_state(n, seed=n + 1)
    o, g = _pair(c, phi, pi, precision="f32", tile=tile)
    g.evolve(20, c["dt"], 4)
    o.evolve(20, c["dt"], 4)
    gphi, gpi = g.get_fields()
    e1, e2 = rel_l2(gphi, o.phi), rel_l2(gpi, o.pi)
    say("ragged fp32", n, tile, g.tile(), e1, e2)
    assert max(e1, e2) <= FP32_L2_TOL


def test_tile_shapes_agree_bitwise_on_fields():
    """The field update at a site does not depend on the tile shape."""
    c, phi, pi = _preheat_state(40, seed=5)
    outs = []
    for tile in [(16, 1, 3), (32, 2, 40), (64, 1, 8), (16, 2, 7), (64, 2, 0)]:
        g = gpu_lattice(40, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"],
                        expand=False, tile=tile)
        g.evolve(3, c["dt"], 4)
        outs.append(g.get_fields())
    for f, p in outs[1:]:
        assert np.array_equal(f, outs[0][0]) and np.array_equal(p, outs[0][1])


# ---------------------------------------------------------------------------
# Structure: reversibility, split invariance, determinism
# ---------------------------------------------------------------------------

def test_reversibility_gpu():
    c, phi, pi = _preheat_state(24, seed=9)
    g = gpu_lattice(24, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"])
    _, a0, pa0 = g.background()
    g.evolve(40, c["dt"], 4)
    g.evolve(40, -c["dt"], 4)
    f, p = g.get_fields()
    eta, a, pa = g.background()
    assert max_rel(f, phi) <= 1e-12 and max_rel(p, pi) <= 1e-10
    assert a == pytest.approx(a0, rel=1e-13) and pa == pytest.approx(pa0, rel=1e-12)
    assert abs(eta) < 1e-15


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_split_call_invariance_bitwise(precision):
    c, phi, pi = _preheat_state(24, seed=11)
    g1 = gpu_lattice(24, c["L"], c["potential"], c["params"], phi, pi, precision=precision, mpl=c["mpl"])
    g2 = gpu_lattice(24, c["L"], c["potential"], c["params"], phi, pi, precision=precision, mpl=c["mpl"])
    g1.evolve(50, c["dt"], 4)
    g1.evolve(37, c["dt"], 4)
    g1.evolve(13, c["dt"], 4)
    g2.evolve(100, c["dt"], 4)
    f1, p1 = g1.get_fields()
    f2, p2 = g2.get_fields()
    assert np.array_equal(f1, f2) and np.array_equal(p1, p2)
    assert g1.background() == g2.background()


def test_run_to_run_bitwise():
    c, phi, pi = _preheat_state(32, seed=12)
    res = []
    for _ in range(2):
        g = gpu_lattice(32, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"])
        g.evolve(20, c["dt"], 6)
        res.append((g.get_fields(), g.background(), g.energies()["rho"]))
    assert np.array_equal(res[0][0][0], res[1][0][0]) and res[0][1] == res[1][1]
    assert res[0][2] == res[1][2]


# ---------------------------------------------------------------------------
# Observables, spectrum, initial states
# ---------------------------------------------------------------------------

def test_energies_match_oracle():
    c, phi, pi = _preheat_state(20, seed=13, amp=1e-2)
    o, g = _pair(c, phi, pi, rho_rad0=0.05, rho_mat0=0.02)
    g.evolve(7, c["dt"], 4)          # leaves a pending drift: observers apply it
    o.evolve(7, c["dt"], 4)
    eg, eo = g.energies(), o.energies()
    for k in ("rho", "pressure", "pot", "hubble", "a", "p_a", "eta", "w_eos"):
        assert eg[k] == pytest.approx(eo[k], rel=1e-10, abs=1e-300), k
    for k in ("kin", "grad", "mean", "var"):
        np.testing.assert_allclose(eg[k], eo[k], rtol=1e-9, atol=1e-300)
    assert eg["friedmann_residual"] == pytest.approx(eo["friedmann_residual"], rel=1e-3, abs=1e-12)
    scale = abs(eo["p_a"]) ** 2 / (12 * o.VL * o.mpl ** 2)
    assert abs(eg["h_total"] - eo["h_total"]) <= 1e-10 * scale


@pytest.mark.parametrize("n", [16, 15, 128])
def test_spectrum_matches_oracle(n):
    c, phi, pi = _preheat_state(n, seed=14, amp=1e-2)
    o, g = _pair(c, phi, pi)
    g.evolve(3, c["dt"], 4)
    o.evolve(3, c["dt"], 4)
    nb = int(math.ceil(math.sqrt(3) * n / 2)) + 2
    for field in range(2):
        k, P, cnt = g.spectrum(field, nb)
        ko, Po, co = oracle.spectrum(o.phi[field], c["L"], nb)
        assert np.array_equal(cnt, co)
        np.testing.assert_allclose(k, ko, rtol=1e-12)
        np.testing.assert_allclose(P, Po, rtol=1e-8, atol=1e-12 * Po.max())


@pytest.mark.parametrize("n", [24, 15, 32, 64])
def test_vacuum_init_matches_oracle(n):
    """Powers of two take the radix-2 transform, other sizes the direct
    one: both against the oracle's initial state."""
    c = synth.preheat(n=n)
    c["amplitude"] = 1e-3
    g = sl.from_recipe(c)
    pot = oracle.Potential(c["potential"], c["params"])
    o = oracle.Lattice(n, c["L"], pot, mpl=c["mpl"])
    o.init_fluctuations(c["phi0"], c["pi0"], "vacuum", c["amplitude"], c["seed"])
    phi, pi = g.get_fields()
    base = np.array(c["phi0"])[:, None, None, None]
    assert max_rel(phi - base, o.phi - base) <= 1e-11
    assert np.all(pi == 0)
    assert g.background()[2] == pytest.approx(o.p_a, rel=1e-12)


def test_white_init_matches_oracle():
    c = synth.oscillon(n=20, precision="f64")
    g = sl.from_recipe(c)
    pot = oracle.Potential(c["potential"], c["params"])
    o = oracle.Lattice(20, c["L"], pot, mpl=c["mpl"])
    o.init_fluctuations(c["phi0"], c["pi0"], "white", c["amplitude"], c["seed"])
    phi, _ = g.get_fields()
    assert max_rel(phi - 0.8, o.phi - 0.8) <= 1e-12
    assert g.background()[2] == pytest.approx(o.p_a, rel=1e-12)


# ---------------------------------------------------------------------------
# Error paths forced from the host
# ---------------------------------------------------------------------------

def test_error_paths():
    g = sl.Lattice(8, 2, 10.0)
    with pytest.raises(sl.SymlatError) as e:
        g.evolve(1, 0.01, 4)
    assert e.value.status == 4  # SL_E_STATE: no potential
    with pytest.raises(sl.SymlatError):
        g.set_potential("oscillon", (1.0, 1.0, 0.2))   # wrong field count
    g.set_potential("chaotic2", (1.0, 10.0))
    phi, pi = synth.gaussian_state(8, 2, 1, phi_base=[1.0, 0.0])
    g.set_fields(phi, pi, 1.0)
    with pytest.raises(sl.SymlatError) as e:
        g.evolve(1, 10.0, 4)
    assert e.value.status == 6  # SL_E_UNSTABLE
    with pytest.raises(sl.SymlatError) as e:
        g.evolve(1, 0.01, 5)
    assert e.value.status == 1
    bad = phi.copy()
    bad[1, 3, 2, 1] = np.nan
    g.set_fields(bad, pi, 1.0, p_a=-1.0)   # explicit p_a: no constraint solve
    g.evolve(1, 0.001, 4)
    with pytest.raises(sl.SymlatError) as e:
        g.synchronize()
    assert e.value.status == 5  # SL_E_NONFINITE


def test_autotune_keeps_state_and_parity():
    """The autotuner's timing passes leave the state untouched, and the
    tuned shape keeps FP64 parity with the oracle."""
    c, phi, pi = _preheat_state(48, seed=48)
    o, g = _pair(c, phi, pi)
    f0, p0 = g.get_fields()
    b0 = g.background()
    shape, ms = g.autotune(reps=2)
    say("autotuned", shape, ms, g.tile())
    f1, p1 = g.get_fields()
    assert np.array_equal(f0, f1) and np.array_equal(p0, p1) and g.background() == b0
    g.evolve(20, c["dt"], 4)
    o.evolve(20, c["dt"], 4)
    ef, ep, ea, epa, _ = compare_state(g, o)
    assert max(ef, ep, ea, epa) <= FP64_TOL
    # lattices created later with the same key start with the tuned shape
    g2 = gpu_lattice(48, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"])
    assert g2.tile() == g.tile()
    sl.symlat.autotune_forget()


def test_autotune_mid_run_keeps_state_bitwise():
    """Tuning after some steps (a drift pending, history recording) leaves
    the state, the pending drift and the record as they were: the tuned run
    continues bit for bit like a twin given the same shape by hand."""
    c, phi, pi = _preheat_state(32, seed=49)
    g = gpu_lattice(32, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"])
    h = gpu_lattice(32, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"])
    for lat in (g, h):
        lat.set_history(64)
        lat.evolve(7, c["dt"], 4)
    before = g.get_fields(), g.background()
    g.autotune(reps=1)
    tx, vx, _, tz, pf = g.tile()
    h.set_tile(tx, vx, tz, pf)
    after = g.get_fields(), g.background()
    assert all(np.array_equal(x, y) for x, y in zip(before[0], after[0])) and before[1] == after[1]
    for lat in (g, h):
        lat.evolve(10, c["dt"], 4)
    fg, pg = g.get_fields()
    fh, ph = h.get_fields()
    assert np.array_equal(fg, fh) and np.array_equal(pg, ph) and g.background() == h.background()
    assert all(np.array_equal(x, y) for x, y in zip(g.history(), h.history()))
    assert len(g.history()[0]) == 17
    sl.symlat.autotune_forget()


def test_zero_steps_and_empty_batches_are_no_ops():
    c, phi, pi = _preheat_state(16, seed=50)
    g = gpu_lattice(16, c["L"], c["potential"], c["params"], phi, pi, mpl=c["mpl"])
    g.evolve(3, c["dt"], 4)                  # a drift pending
    f0, p0 = g.get_fields()
    b0 = g.background()
    g.evolve(0, c["dt"], 4)
    with pytest.raises(sl.SymlatError):
        g.evolve(0, 1e9, 4)                  # arguments are checked for zero steps too
    f1, p1 = g.get_fields()
    assert np.array_equal(f0, f1) and np.array_equal(p0, p1) and g.background() == b0
    b = sl.Batch()
    b.step(5, c["dt"], 4)                    # no members
    b.add(g)
    b.step(0, c["dt"], 4)
    b.synchronize()
    assert g.background() == b0
    lin = sl.Linear(16, 2, c["L"], mpl=c["mpl"])
    lin.set_potential(c["potential"], c["params"])
    lin.set_fields(phi, pi)
    lf0 = lin.get_fields()
    lin.evolve(0, c["dt"], 4)
    lf1 = lin.get_fields()
    assert all(np.array_equal(x, y) for x, y in zip(lf0, lf1))
