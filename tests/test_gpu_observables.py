"""The observables pass at sizes that span several tiles with ragged edges
(x tiles of 64 lanes, y tiles of 4 rows, z-chunks), with one to three
fields and FP64 or FP32 storage: the constraint solve for p_a and the
energies of the synchronised state (with a pending drift where the state
was stepped) against the oracle's, computed from the same field values."""
import numpy as np
import pytest

import synth
from gpu_util import gpu_lattice, oracle_lattice, say

pytestmark = pytest.mark.gpu

# potential: (parameters, homogeneous fields, m_pl)
MODELS = {
    "chaotic2": ((1.0, 9312.25), (1.0, 0.0), 1.0335292),
    "oscillon": ((1.0, 1.0, 0.2), (0.8,), 335.41),
    "free": ((0.9, 1.6, 2.5), (0.1, 0.2, 0.3), 1.0),
}

# (n, potential, storage, steps before the read-out)
CASES = [(4, "chaotic2", "f64", 2), (5, "oscillon", "f64", 2), (67, "chaotic2", "f64", 2),
         (96, "free", "f64", 1), (130, "oscillon", "f64", 1), (67, "chaotic2", "f32", 0),
         (33, "free", "f32", 0)]


@pytest.mark.parametrize("n,kind,precision,steps", CASES)
def test_observables_across_tiles(n, kind, precision, steps):
    params, base, mpl = MODELS[kind]
    nf = len(base)
    L = 0.5 * n
    scale = max(abs(b) for b in base)
    phi, pi = synth.gaussian_state(n, nf, 7000 + n, phi_base=list(base),
                                   phi_amp=1e-2 * scale, pi_amp=1e-2 * scale)
    g = gpu_lattice(n, L, kind, params, phi, pi, precision=precision, mpl=mpl)
    if precision == "f32":      # the oracle sees the values the library stores
        phi, pi = g.get_fields()
    o = oracle_lattice(n, L, kind, params, phi, pi, mpl=mpl)
    assert g.background()[2] == pytest.approx(o.p_a, rel=1e-10)
    if steps:                   # leaves a drift pending: the observers apply it
        g.evolve(steps, 0.005, 4)
        o.evolve(steps, 0.005, 4)
    eg, eo = g.energies(), o.energies()
    say("n", n, kind, precision, "rho", eg["rho"], eo["rho"], "grad", eg["grad"][:nf],
        eo["grad"][:nf])
    for k in ("rho", "pressure", "pot", "hubble", "a", "p_a", "w_eos"):
        assert eg[k] == pytest.approx(eo[k], rel=1e-10, abs=1e-300), k
    for k in ("kin", "grad", "mean", "var"):
        np.testing.assert_allclose(eg[k][:nf], eo[k][:nf], rtol=1e-9, atol=1e-300, err_msg=k)
    g.close()
