"""GPU parity of the field, energy-density and number-density spectra
(sl_spectra) against the oracle's mode_spectra on the same state."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import gpu_lattice, oracle_lattice, say

pytestmark = pytest.mark.gpu


def _pair(n, kind, params, base, pibase, amp, L, mpl=1.0, precision="f64", stencil=None,
          seed=61):
    nf = len(base)
    phi, pi = synth.gaussian_state(n, nf, seed, phi_base=base, phi_amp=amp, pi_base=pibase,
                                   pi_amp=amp)
    o = oracle_lattice(n, L, kind, params, phi, pi, mpl=mpl, stencil=stencil)
    g = gpu_lattice(n, L, kind, params, phi, pi, precision=precision, mpl=mpl, stencil=stencil)
    return o, g


def _check(o, g, field, nb, rtol):
    k, pf, pe, pn, cnt, m2 = g.spectra(field, nb)
    ko, pfo, peo, pno, co, m2o = oracle.mode_spectra(o, field, nb)
    say("spectra field", field, "m2", m2, m2o, "pe[1:4]", pe[1:4], peo[1:4])
    assert np.array_equal(cnt, co)
    np.testing.assert_allclose(k, ko, rtol=1e-12)
    assert m2 == pytest.approx(m2o, rel=rtol)
    for got, ref in ((pf, pfo), (pe, peo), (pn, pno)):
        np.testing.assert_allclose(got, ref, rtol=rtol, atol=rtol * 1e-3 * np.abs(ref).max())


@pytest.mark.parametrize("n", [16, 15])
def test_spectra_preheat_fp64(n):
    c = synth.preheat(n=n)
    o, g = _pair(n, c["potential"], c["params"], c["phi0"], [0.0, 0.0], 1e-2, c["L"], mpl=c["mpl"])
    g.evolve(3, c["dt"], 4)           # leaves a pending drift: both spectra use phi_sync
    o.evolve(3, c["dt"], 4)
    nb = int(math.ceil(math.sqrt(3) * n / 2)) + 2
    for field in range(2):
        _check(o, g, field, nb, 1e-9)


@pytest.mark.parametrize("kind,params,base,pibase,mpl", [
    ("oscillon", (1.0, 1.0, 0.2), [0.8], [0.0], 335.41),
    ("qball", (1.0, -0.1, 1.0), [math.sqrt(2) * 1e-2, 0.0], [0.0, 0.5 * math.sqrt(2) * 1e-2], 1.0),
])
def test_spectra_other_potentials_27_point(kind, params, base, pibase, mpl):
    o, g = _pair(12, kind, params, base, pibase, 1e-3 * max(abs(b) for b in base), 6.0, mpl=mpl,
                 stencil=oracle.STENCIL_27)
    g.evolve(5, 0.01, 4)
    o.evolve(5, 0.01, 4)
    for field in range(len(base)):
        _check(o, g, field, 14, 1e-9)


def test_spectra_fp32_storage():
    c = synth.preheat(n=16)
    o, g = _pair(16, c["potential"], c["params"], c["phi0"], [0.0, 0.0], 1e-2, c["L"],
                 mpl=c["mpl"], precision="f32")
    # the FP32 lattice holds the state rounded to FP32: compare against the
    # oracle on that same rounded state
    phi, pi = g.get_fields()
    o.phi[...] = phi
    o.pi[...] = pi
    _check(o, g, 0, 16, 1e-9)


def test_spectra_bin_count_edges_and_errors():
    """One bin (it would hold only the excluded zero mode, so it is empty;
    modes beyond the last bin are dropped, as in the oracle), the largest bin
    count, and refused arguments: field out of range, nbins outside
    [1, 2048], no initial state."""
    import paper_1201_5029_amd as sl
    c = synth.preheat(n=10)
    o, g = _pair(10, c["potential"], c["params"], c["phi0"], [0.0, 0.0], 1e-2, c["L"],
                 mpl=c["mpl"])
    _check(o, g, 0, 1, 1e-9)
    _check(o, g, 1, 2048, 1e-9)
    for field, nb in [(2, 8), (-1, 8), (0, 0), (0, 2049)]:
        with pytest.raises(sl.SymlatError) as e:
            g.spectra(field, nb)
        assert e.value.status == 1
    bare = sl.Lattice(8, 2, 10.0)
    with pytest.raises(sl.SymlatError) as e:
        bare.spectra(0, 4)
    assert e.value.status == 4
