"""Stage chaining: the scalar update that closes a stage folded into the
next fused pass (every workgroup reduces the previous pass's per-tile sums)
against the separate one-workgroup stage finalize.  From one synthetic
state, the two modes must give bitwise equal fields, momenta, background,
history and energies -- over the potential families, both storage
precisions, ragged tiles with idle lanes, the pass modes, the 27-point
stencil, the largest chained tile count (1024) and one past it, and calls
that mix captured chunks of 32 steps with eager tails.  The chained path
also meets the FP64 oracle gate directly."""
import math

import numpy as np
import pytest

import synth
from gpu_util import compare_state, gpu_lattice, oracle_lattice, say

pytestmark = pytest.mark.gpu

MODELS = {
    "chaotic2": ((1.0, 9312.25), (1.0, 0.0), 1.0335292),
    "oscillon": ((1.0, 1.0, 0.2), (0.8,), 335.41),
    "qball": ((1.0, -0.1, 1.0), (math.sqrt(2) * 1e-2, 0.0), 1.0),
    "free": ((0.9, 1.6, 2.5), (0.1, 0.2, 0.3), 1.0),
}

# (family, precision, n, stencil, (tx, vx, tz, pf))
CASES = [
    ("chaotic2", "f64", 40, None, (16, 2, 7, 2)),    # ragged x, y and z tiles
    ("chaotic2", "f32", 36, None, (16, 4, 5, 6)),    # non-temporal, depth 2
    ("oscillon", "f32", 24, None, (8, 1, 3, 1)),     # 8 of 32 rows idle
    ("qball", "f32", 32, None, (32, 2, 8, 5)),       # non-temporal, depth 1
    ("qball", "f64", 30, None, (48, 1, 4, 2)),       # 30 of 48 lanes per row active
    ("free", "f64", 20, None, (16, 1, 4, 1)),        # three fields
    ("chaotic2", "f64", 28, "27", (16, 2, 6, 1)),    # 27-point pass
    ("oscillon", "f64", 26, "19", (8, 2, 0, 1)),     # 19-point, occupancy chunk
    ("chaotic2", "f64", 64, None, (8, 1, 1, 1)),     # exactly 1024 tiles
    ("chaotic2", "f64", 72, None, (8, 1, 1, 1)),     # 1944 tiles: never chained
]


def _pair(kind, prec, n, stencil, tile, seed):
    params, base, mpl = MODELS[kind]
    nf = len(base)
    scale = max(abs(b) for b in base)
    phi, pi = synth.gaussian_state(n, nf, seed, phi_base=list(base),
                                   phi_amp=1e-3 * scale, pi_amp=1e-3 * scale)
    out = []
    for mode in (0, 1):
        g = gpu_lattice(n, 0.5 * n, kind, params, phi, pi, precision=prec, mpl=mpl,
                        tile=tile, stencil=stencil)
        g.set_chaining(mode)
        g.set_history(64)
        out.append(g)
    return out, (phi, pi, params, mpl)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_chained_equals_finalize(case):
    kind, prec, n, stencil, tile = CASES[case]
    (g0, g1), _ = _pair(kind, prec, n, stencil, tile, 4200 + case)
    say("chain case", case, kind, prec, "n", n, "stencil", stencil or "7", "tile", g1.tile())
    for g in (g0, g1):
        g.evolve(37, 0.005, 4)      # one captured chunk of 32 steps, 5 eager
        g.evolve(3, 0.005, 6)
        g.evolve(1, 0.005, 2)
    f0, p0 = g0.get_fields()
    f1, p1 = g1.get_fields()
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


def test_chained_fp64_vs_oracle():
    params, base, mpl = MODELS["chaotic2"]
    n = 24
    phi, pi = synth.gaussian_state(n, 2, 4300, phi_base=list(base), phi_amp=1e-3, pi_amp=1e-3)
    g = gpu_lattice(n, 0.5 * n, "chaotic2", params, phi, pi, mpl=mpl, tile=(16, 2, 5, 6))
    g.set_chaining(1)
    o = oracle_lattice(n, 0.5 * n, "chaotic2", params, phi, pi, mpl=mpl)
    g.evolve(40, 0.005, 6)
    o.evolve(40, 0.005, 6)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("chained 24^3 order 6, 40 steps, errors", ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= 1e-10
    g.close()


def test_chaining_mode_checked():
    params, base, mpl = MODELS["free"]
    phi, pi = synth.gaussian_state(8, 3, 4301, phi_base=list(base))
    g = gpu_lattice(8, 4.0, "free", params, phi, pi, mpl=mpl)
    with pytest.raises(Exception):
        g.set_chaining(2)
    g.set_chaining(-1)
    g.close()
