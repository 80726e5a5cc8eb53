"""The autotuner on a lattice in mid-run: it times real stages with frozen
coefficients, chained or not as sl_evolve would run them, and must leave
the state exactly as it found it -- fields, background with its pending
drift, the history record and the observables -- whatever shape it picks;
the run then continues as an untuned twin does, up to the rounding of the
FP64 lattice sums (whose order follows the tile shape)."""
import numpy as np
import pytest

import paper_1201_5029_amd as sl
import synth
from gpu_util import max_rel, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _forget_tuned_shapes():
    sl.symlat.autotune_forget()
    yield
    sl.symlat.autotune_forget()


def _start(c, mode):
    g = sl.from_recipe(c)
    g.set_chaining(mode)
    g.set_history(64)
    g.evolve(7, c["dt"], c["order"])     # ends with a drift pending
    return g


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", [0, -1])
def test_autotune_keeps_state(prec, mode):
    c = synth.preheat(n=24, precision=prec)
    g = _start(c, mode)
    f0, p0 = g.get_fields()
    b0, h0, e0 = g.background(), g.history(), g.energies()
    shape, best = g.autotune(reps=1)
    say("tuned", prec, "chaining", mode, shape, "best stage ms", best)
    f1, p1 = g.get_fields()
    assert np.array_equal(f0, f1) and np.array_equal(p0, p1)
    assert g.background() == b0
    for a, b in zip(h0, g.history()):
        assert np.array_equal(a, b)
    e1 = g.energies()
    for k in e0:
        assert e0[k] == e1[k], k

    twin = _start(c, mode)
    for lat in (g, twin):
        lat.evolve(10, c["dt"], c["order"])
    (fa, pa), (fb, pb) = g.get_fields(), twin.get_fields()
    _, a_g, pa_g = g.background()
    _, a_t, pa_t = twin.background()
    if prec == "f64":
        err = max(max_rel(fa, fb), max_rel(pa, pb))
        assert err <= 1e-12
    else:
        err = max(rel_l2(fa, fb), rel_l2(pa, pb))
        assert err <= 1e-6
    assert abs(a_g - a_t) <= 1e-13 * abs(a_t) and abs(pa_g - pa_t) <= 1e-11 * abs(pa_t)
    assert len(g.history()[0]) == len(twin.history()[0]) == 17
    say("  after 10 more steps, tuned vs untuned", err)
    g.close()
    twin.close()
