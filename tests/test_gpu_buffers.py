"""A lattice on the caller's field arrays (sl_lattice_create_with_buffers):
the arrays come from the same HIP runtime the library uses; the results
equal those of a lattice that owns its arrays, bit for bit, the arrays
outlive the handle untouched by its destruction, and arrays that are too
short, misaligned, overlapping or host memory are refused before any
device work."""
import ctypes

import numpy as np
import pytest

import paper_1201_5029_amd as sl
import synth

pytestmark = pytest.mark.gpu


def _hip():
    sl.load()                                   # the library's own runtime is loaded
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return hip


def _alloc(hip, nbytes):
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), nbytes) == 0
    return p.value


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_caller_buffers_equal_owned(precision):
    hip = _hip()
    r = synth.preheat(n=24, order=4, dt=0.005, precision=precision, seed=31)
    n, nf = r["n"], r["nfields"]
    nbytes = nf * n ** 3 * (8 if precision == "f64" else 4)
    bufs = [_alloc(hip, nbytes) for _ in range(4)]
    try:
        src = sl.from_recipe(r)                 # the device vacuum state of the recipe
        phi, pi = src.get_fields()
        eta, a, p_a = src.background()
        src.close()
        own = sl.Lattice(n, nf, r["L"], precision=precision, mpl=r["mpl"])
        ext = sl.Lattice(n, nf, r["L"], precision=precision, mpl=r["mpl"], buffers=bufs)
        for lat in (own, ext):
            lat.set_potential(r["potential"], r["params"])
            lat.set_fields(phi, pi, a, p_a)
        assert own.tile() == ext.tile()
        for lat in (own, ext):
            lat.evolve(40, r["dt"], r["order"])
        fo, po = own.get_fields()
        fe, pe = ext.get_fields()
        assert np.array_equal(fo, fe) and np.array_equal(po, pe)
        assert own.background() == ext.background()
        # the state lives in the caller's arrays: the current buffer holds the
        # storage-precision momenta (drift pending, so compare the momenta);
        # FP32 storage holds each momentum's remainder around the handle's
        # FP64 homogeneous offset, so there the difference is one constant
        # per field
        ext.synchronize()
        host = np.empty(nf * n ** 3, dtype=np.float64 if precision == "f64" else np.float32)
        pis = []
        for k in (1, 3):
            assert hip.hipMemcpy(host.ctypes.data, bufs[k], nbytes, 2) == 0
            # device layout [z][field][y][x] -> [field][z][y][x]
            pis.append(host.copy().reshape(n, nf, n, n).transpose(1, 0, 2, 3).astype(np.float64))
        if precision == "f64":
            assert any(np.array_equal(x, pe) for x in pis)
        else:
            def offset_only(x):
                return all(np.ptp(pe[i] - x[i]) <= 1e-14 * max(1.0, np.abs(pe[i]).max())
                           for i in range(nf))
            assert any(offset_only(x) for x in pis)
        ext.close()
        own.close()
        assert hip.hipMemcpy(host.ctypes.data, bufs[1], nbytes, 2) == 0   # still valid
    finally:
        for b in bufs:
            hip.hipFree(b)


def test_caller_buffers_refused():
    """Arrays of 4 MB, so that no allocation granularity (at most 2 MB) can
    make a short array long enough."""
    hip = _hip()
    n, nf = 64, 2
    nbytes = nf * n ** 3 * 8
    big = _alloc(hip, 4 * nbytes + 64)
    short = _alloc(hip, nbytes // 2)
    host = np.zeros(nf * n ** 3)
    try:
        ok = [big + k * nbytes for k in range(4)]
        lat = sl.Lattice(n, nf, 10.0, buffers=ok)      # carved from one allocation
        lat.close()
        cases = [
            [ok[0], ok[1], ok[2], short],                   # too short
            [ok[0] + 8, ok[1], ok[2], ok[3]],               # misaligned
            [ok[0], ok[0] + nbytes // 2, ok[2], ok[3]],     # overlapping
            [ok[0], ok[1], ok[2], host.ctypes.data],        # host memory
            [ok[0], ok[1], ok[2], 0],                       # NULL
            [ok[0], ok[1], ok[2], big + 4 * nbytes - 64],   # runs past its allocation
        ]
        for bufs in cases:
            with pytest.raises(sl.SymlatError) as e:
                sl.Lattice(n, nf, 10.0, buffers=bufs)
            assert e.value.status == 1
    finally:
        hip.hipFree(big)
        hip.hipFree(short)
