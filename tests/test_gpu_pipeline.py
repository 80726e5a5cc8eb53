"""Pass modes that change how the fused pass moves data but not what it
computes.  The depth-3 pipeline (pass mode 7: the loads of the own column
run three planes ahead, two register sets used in turn, non-temporal
stores) against depth 2 (mode 6), and the 27-point pass with non-temporal
stores (mode 5) against its cached stores (mode 1).  The arithmetic and its
order are the same, so from one synthetic state the two must give bitwise
equal fields, momenta, background, history and energies -- over chunk
lengths 1, 2, 3, odd and even, ragged tiles with idle lanes, both storage
precisions, the potential families, two and four sites per lane, chained
and unchained passes.  Depth 3 also meets the FP64 oracle gate directly."""
import math

import numpy as np
import pytest

import synth
from gpu_util import compare_state, gpu_lattice, max_rel, oracle_lattice, say

pytestmark = pytest.mark.gpu

MODELS = {
    "chaotic2": ((1.0, 9312.25), (1.0, 0.0), 1.0335292),
    "oscillon": ((1.0, 1.0, 0.2), (0.8,), 335.41),
    "qball": ((1.0, -0.1, 1.0), (math.sqrt(2) * 1e-2, 0.0), 1.0),
}

# (family, precision, n, (tx, vx, tz), chaining mode)
CASES = [
    ("chaotic2", "f64", 40, (16, 2, 7), 1),     # ragged x, y and z; odd chunks
    ("chaotic2", "f64", 24, (16, 2, 1), 1),     # one plane per chunk
    ("chaotic2", "f64", 24, (16, 2, 2), 0),     # two planes per chunk
    ("chaotic2", "f32", 36, (16, 4, 3), 1),     # three planes, four sites per lane
    ("chaotic2", "f64", 64, (32, 2, 64), 1),    # whole z-columns
    ("chaotic2", "f32", 64, (16, 4, 16), 0),    # even chunks, unchained
    ("qball", "f32", 32, (32, 2, 8), 1),
    ("qball", "f64", 30, (16, 2, 4), 0),        # 15 of 16 lanes per row active
    ("oscillon", "f64", 26, (8, 2, 5), 1),      # one field, ragged
    ("oscillon", "f32", 24, (8, 4, 6), 1),      # 8 of 32 rows idle
]


# 27-point family: (family, precision, n, stencil, (tx, vx, tz), chaining mode)
CASES27 = [
    ("chaotic2", "f64", 28, "27", (16, 2, 6), 1),
    ("oscillon", "f32", 26, "19", (8, 2, 5), 0),      # ragged: idle lanes store into the sink
    ("chaotic2", "f32", 32, "27", (32, 2, 8), 1),
    ("qball", "f64", 24, "27", (16, 2, 4), 1),
]


def _pair(kind, prec, n, tile, mode, ref_pf, pf, seed, stencil=None):
    params, base, mpl = MODELS[kind]
    nf = len(base)
    scale = max(abs(b) for b in base)
    phi, pi = synth.gaussian_state(n, nf, seed, phi_base=list(base),
                                   phi_amp=1e-3 * scale, pi_amp=1e-3 * scale)
    lats = []
    for p in (ref_pf, pf):
        g = gpu_lattice(n, 0.5 * n, kind, params, phi, pi, precision=prec, mpl=mpl,
                        tile=tuple(tile) + (p,), stencil=stencil)
        g.set_chaining(mode)
        g.set_history(64)
        lats.append(g)
    return lats


@pytest.mark.parametrize("case", range(len(CASES)))
def test_depth3_equals_depth2(case):
    kind, prec, n, tile, mode = CASES[case]
    g0, g1 = _pair(kind, prec, n, tile, mode, 6, 7, 4400 + case)
    say("depth-3 case", case, kind, prec, "n", n, "tile", g1.tile(), "chaining", mode)
    assert g1.tile()[-1] == 7
    _same_runs(kind, prec, g0, g1)


@pytest.mark.parametrize("case", range(len(CASES27)))
def test_27_point_nontemporal_equals_cached(case):
    kind, prec, n, stencil, tile, mode = CASES27[case]
    g0, g1 = _pair(kind, prec, n, tile, mode, 1, 5, 4460 + case, stencil=stencil)
    say("27-point case", case, kind, prec, "n", n, "stencil", stencil, "tile", g1.tile(),
        "chaining", mode)
    assert g1.tile()[-1] == 5
    _same_runs(kind, prec, g0, g1)


def _same_runs(kind, prec, g0, g1):
    lats = [g0, g1]
    for g in lats:
        g.evolve(37, 0.005, 4)      # one captured chunk of 32 steps, 5 eager
        g.evolve(3, 0.005, 6)
        g.evolve(1, 0.005, 2)
    f0, p0 = g0.get_fields()
    f1, p1 = g1.get_fields()
    say("  max rel difference", max_rel(f1, f0), max_rel(p1, p0))
    if kind == "qball":
        # the compiler contracts the log potential's products into fused
        # multiply-adds differently in the two kernels: rounding-level
        # differences only
        tol, tol_a, tol_pa = (1e-12, 1e-14, 1e-12) if prec == "f64" else (1e-6, 1e-12, 1e-9)
        (_, a0, pa0), (_, a1, pa1) = g0.background(), g1.background()
        say("  background", abs(a1 - a0) / abs(a0), abs(pa1 - pa0) / abs(pa0))
        assert max_rel(f1, f0) <= tol and max_rel(p1, p0) <= tol
        assert abs(a1 - a0) <= tol_a * abs(a0) and abs(pa1 - pa0) <= tol_pa * abs(pa0)
        g0.close()
        g1.close()
        return
    assert np.array_equal(f0, f1) and np.array_equal(p0, p1)
    assert g0.background() == g1.background()
    h0, h1 = g0.history(), g1.history()
    assert len(h0[0]) == 41
    for a, b in zip(h0, h1):
        assert np.array_equal(a, b)
    e0, e1 = g0.energies(), g1.energies()
    for k in e0:
        assert e0[k] == e1[k] or (e0[k] != e0[k] and e1[k] != e1[k]), k
    g0.close()
    g1.close()


def test_depth3_fp64_vs_oracle():
    params, base, mpl = MODELS["chaotic2"]
    n = 24
    phi, pi = synth.gaussian_state(n, 2, 4450, phi_base=list(base), phi_amp=1e-3, pi_amp=1e-3)
    g = gpu_lattice(n, 0.5 * n, "chaotic2", params, phi, pi, mpl=mpl, tile=(16, 2, 5, 7))
    o = oracle_lattice(n, 0.5 * n, "chaotic2", params, phi, pi, mpl=mpl)
    g.evolve(40, 0.005, 6)
    o.evolve(40, 0.005, 6)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("depth 3, 24^3 order 6, 40 steps, errors", ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= 1e-10
    g.close()


def test_depth3_needs_nontemporal_stores():
    params, base, mpl = MODELS["chaotic2"]
    phi, pi = synth.gaussian_state(16, 2, 4451, phi_base=list(base))
    g = gpu_lattice(16, 8.0, "chaotic2", params, phi, pi, mpl=mpl)
    for pf in (3, 8, 0):
        with pytest.raises(Exception):
            g.set_tile(16, 2, 4, pf)
    with pytest.raises(Exception):
        g.set_tile(16, 1, 4, 7)     # non-temporal stores need two or four sites per lane
    g.set_tile(16, 2, 4, 7)
    g.close()
