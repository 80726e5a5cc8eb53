"""CPU checks of the C ABI: the library loads, exports every symbol that
include/symlat.h declares, and its host logic (composition tables,
stability limits, argument validation, footprint) agrees with the oracle
and the header.  No device work is issued."""
import ctypes
import os
import re

import pytest

import oracle
import paper_1201_5029_amd as sl
from paper_1201_5029_amd import symlat as binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "symlat.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sl_[a-z0-9_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = sl.load()
    for name in _declared():
        assert hasattr(lib, name), name
    # and the dynamic symbol table has C (unmangled) names
    out = os.popen("nm -D --defined-only %s" % binding.LIB_PATH).read()
    for name in _declared():
        assert re.search(r"\bT %s\b" % name, out), name


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_composition_weights_match_oracle(order):
    w = sl.composition_weights(order)
    ref = oracle.composition_weights(order)
    assert len(w) == len(ref)
    for a, b in zip(w, ref):
        assert a == pytest.approx(b, rel=2e-15, abs=2e-15)


def test_unknown_order_rejected():
    with pytest.raises(sl.SymlatError):
        sl.composition_weights(5)
    assert sl.stability_limit(3) == -1.0


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_stability_limits_match_oracle_scan(order):
    lim = sl.stability_limit(order)
    scan = oracle.stability_limit(order)
    # the library's table is rounded down to 1e-4 of the oracle's scan
    assert 0 <= scan - lim < 2e-4


@pytest.mark.parametrize("bad", [
    dict(n=3), dict(n=2000), dict(nfields=0), dict(nfields=9), dict(L=0.0),
    dict(L=float("nan")), dict(mpl=-1.0), dict(a0=0.0), dict(rho_rad0=-1.0),
])
def test_invalid_configs_rejected_before_device_work(bad):
    cfg = dict(n=16, nfields=2, L=10.0)
    cfg.update(bad)
    with pytest.raises(sl.SymlatError) as e:
        sl.Lattice(**cfg)
    assert e.value.status == binding.SL_E_INVALID
    assert sl.footprint_bytes(**cfg) == 0


def test_footprint_counts_both_ping_pong_copies():
    f64 = sl.footprint_bytes(n=64, nfields=2, L=10.0, precision="f64")
    f32 = sl.footprint_bytes(n=64, nfields=2, L=10.0, precision="f32")
    state = 64 ** 3 * 2
    assert f64 >= 4 * state * 8 and f64 - 4 * state * 8 < 8 << 20
    assert f32 >= 4 * state * 4 and f64 - f32 == 4 * state * 4


def test_transient_bytes_cover_every_scratch_buffer():
    """The scratch figure covers the transform buffers (two complex n^3
    arrays), the FP64 staging of both arrays of every field and the
    spectra's extra complex copy; it is 0 for an invalid configuration."""
    for n, nf in [(16, 1), (64, 2), (32, 8)]:
        t = sl.transient_bytes(n=n, nfields=nf, L=10.0)
        assert t >= 3 * n ** 3 * 16 and t >= 2 * nf * n ** 3 * 8
        assert t - max(3 * n ** 3 * 16, 2 * nf * n ** 3 * 8) < 64 << 20
    assert sl.transient_bytes(n=3, nfields=2, L=10.0) == 0
    assert sl.transient_bytes(n=64, nfields=2, L=10.0, precision="f32") == \
        sl.transient_bytes(n=64, nfields=2, L=10.0)


def test_null_handles_are_rejected():
    lib = sl.load()
    assert lib.sl_lattice_destroy(None) == binding.SL_OK
    assert lib.sl_evolve(None, 1, 0.1, 4) == binding.SL_E_INVALID
    assert lib.sl_synchronize(None) == binding.SL_E_INVALID
    assert lib.sl_set_potential(None, 0, None, 0) == binding.SL_E_INVALID
    assert lib.sl_get_fields(None, None, None) == binding.SL_E_INVALID
    assert b"NULL" in lib.sl_last_error()
    out = ctypes.c_void_p()
    assert lib.sl_lattice_create(None, None, ctypes.byref(out)) == binding.SL_E_INVALID
    assert lib.sl_batch_set_grid(None, 0) == binding.SL_E_INVALID
    assert lib.sl_batch_get_grid(None, None, None) == binding.SL_E_INVALID
    assert lib.sl_set_tile(None, 8, 1, 0, 1) == binding.SL_E_INVALID


def test_vectors_of_the_wrong_length_are_refused_before_the_call():
    """The library reads exactly nfields (or nparams, or 4) doubles: the
    binding refuses other lengths instead of padding or truncating."""
    with pytest.raises(ValueError):
        binding._dvec([1.0], 2)
    with pytest.raises(ValueError):
        binding._dvec([1.0, 2.0, 3.0], 2)
    assert list(binding._dvec([1.0, 2.0], 2)) == [1.0, 2.0]
