"""The allocation-free spectrum entry point (sl_spectrum_noalloc, for
callers that cannot allocate device memory) against sl_spectrum on the same
lattices: two calls in a row, the second on a smaller lattice, so the
second reads scratch the first left behind; then its size limit."""
import numpy as np
import pytest

import paper_1201_5029_amd as sl
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu


def _lattice(n, precision, seed):
    c = synth.preheat(n=n, precision=precision, seed=seed)
    c["amplitude"] = 1e-3
    return sl.from_recipe(c)


def _same_spectrum(lat, field, nbins):
    k0, p0, c0 = lat.spectrum(field, nbins)
    k1, p1, c1 = lat.spectrum_noalloc(field, nbins)
    assert np.array_equal(c0, c1)
    # bin sums use LDS atomics, so their order (and last bits) vary per call
    np.testing.assert_allclose(k1, k0, rtol=1e-12)
    np.testing.assert_allclose(p1, p0, rtol=1e-9, atol=1e-12 * p0.max())
    return p1


def test_noalloc_spectrum_equals_spectrum_two_calls():
    big = _lattice(96, "f32", 20120301)      # the largest side it accepts with 84 bins
    small = _lattice(32, "f64", 20120302)
    big.evolve(3, 0.005, 4)
    small.evolve(5, 0.005, 4)
    p_big = _same_spectrum(big, 1, 84)
    p_small = _same_spectrum(small, 0, 30)
    say("noalloc spectra", p_big[:3], p_small[:3])
    # the first lattice again, after the smaller call
    _same_spectrum(big, 0, 84)
    big.close()
    small.close()


def test_noalloc_spectrum_limit():
    lat = _lattice(96, "f32", 20120303)
    with pytest.raises(sl.SymlatError) as e:
        lat.spectrum_noalloc(0, 900)          # 96^3 with 900 bins exceeds the array
    assert e.value.status == 1 and "scratch" in str(e.value)
    lat.close()
    lat = _lattice(104, "f32", 20120304)     # 2 n^3 complex FP64 alone exceed 32 MiB
    with pytest.raises(sl.SymlatError):
        lat.spectrum_noalloc(0, 10)
    lat.close()
