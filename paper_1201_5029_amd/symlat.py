"""ctypes binding of libsymlat (include/symlat.h).

Argument marshalling only: every lattice computation runs in the HIP
kernels of the library.  Loading fails loudly if the built library is
missing; there is no fallback.
"""
import ctypes
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsymlat.so")

SL_OK, SL_E_INVALID, SL_E_NOMEM, SL_E_DEVICE, SL_E_STATE, SL_E_NONFINITE, SL_E_UNSTABLE = range(7)
STATUS_NAMES = {0: "SL_OK", 1: "SL_E_INVALID", 2: "SL_E_NOMEM", 3: "SL_E_DEVICE",
                4: "SL_E_STATE", 5: "SL_E_NONFINITE", 6: "SL_E_UNSTABLE"}
PRECISION = {"f64": 0, "f32": 1}
POTENTIAL = {"free": 0, "chaotic2": 1, "oscillon": 2, "qball": 3}
FLUCT = {"none": 0, "vacuum": 1, "white": 2}

#: every symbol the header declares (checked by the CPU test suite)
EXPORTS = (
    "sl_lattice_create", "sl_lattice_create_with_buffers", "sl_lattice_destroy", "sl_set_potential",
    "sl_init_fluctuations", "sl_evolve", "sl_energies", "sl_spectrum",
    "sl_get_fields", "sl_set_fields", "sl_get_background", "sl_synchronize",
    "sl_footprint_bytes", "sl_transient_bytes", "sl_last_error", "sl_composition_weights",
    "sl_stability_limit", "sl_set_kernel_timing", "sl_kernel_timing",
    "sl_get_tile", "sl_set_tile", "sl_set_chaining", "sl_hbm_copy_bench",
    "sl_batch_create", "sl_batch_destroy", "sl_batch_add", "sl_batch_remove",
    "sl_batch_count", "sl_batch_step", "sl_batch_synchronize", "sl_device_memory",
    "sl_autotune", "sl_autotune_forget", "sl_set_stencil", "sl_get_stencil",
    "sl_linear_create", "sl_linear_destroy", "sl_linear_set_potential",
    "sl_linear_set_stencil", "sl_linear_set_fields", "sl_linear_evolve",
    "sl_linear_get_fields", "sl_linear_get_background", "sl_linear_classes",
    "sl_linear_synchronize", "sl_linear_set_kernel_timing", "sl_linear_kernel_timing",
    "sl_batch_autotune", "sl_spectra", "sl_set_history", "sl_get_history",
    "sl_batch_set_grid", "sl_batch_get_grid", "sl_spectrum_noalloc", "sl_batch_time_pass",
)

#: Members of the cubic stencil family of eq. (2.7): (centre, face, edge,
#: corner) weights.  "19" and "27" are the members with isotropic leading
#: error (c1 = 2 c2 + 8 c3) without and with corner weights.
STENCILS = {
    "7": (-6.0, 1.0, 0.0, 0.0),
    "19": (-4.0, 1.0 / 3.0, 1.0 / 6.0, 0.0),
    "27": (-128.0 / 30.0, 14.0 / 30.0, 3.0 / 30.0, 1.0 / 30.0),
}


class SymlatError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nfields", ctypes.c_int32), ("L", ctypes.c_double),
                ("precision", ctypes.c_int32), ("expansion", ctypes.c_int32),
                ("mpl", ctypes.c_double), ("a0", ctypes.c_double),
                ("rho_rad0", ctypes.c_double), ("rho_mat0", ctypes.c_double)]


class Energies(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("eta", "a", "p_a", "hubble", "rho", "pressure", "w_eos",
                 "friedmann_residual", "h_total", "pot")] + \
               [(k, ctypes.c_double * 8) for k in ("kin", "grad", "mean", "var")]


_lib = None


def load():
    """Load libsymlat.so from the package directory (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsymlat.so is not built: run paper_1201_5029_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I32, I64, U64 = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                           ctypes.c_int64, ctypes.c_uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "sl_lattice_create": (I32, [ctypes.POINTER(Config), P, ctypes.POINTER(P)]),
        "sl_lattice_create_with_buffers": (I32, [ctypes.POINTER(Config), P, P, P, P, P,
                                                 ctypes.POINTER(P)]),
        "sl_lattice_destroy": (I32, [P]),
        "sl_set_potential": (I32, [P, I32, dp, I32]),
        "sl_init_fluctuations": (I32, [P, dp, dp, I32, D, U64]),
        "sl_evolve": (I32, [P, I64, D, I32]),
        "sl_energies": (I32, [P, ctypes.POINTER(Energies)]),
        "sl_spectrum": (I32, [P, I32, I32, dp, dp, ctypes.POINTER(ctypes.c_int64)]),
        "sl_spectrum_noalloc": (I32, [P, I32, I32, dp, dp, ctypes.POINTER(ctypes.c_int64)]),
        "sl_get_fields": (I32, [P, P, P]),
        "sl_set_fields": (I32, [P, P, P, D, D]),
        "sl_get_background": (I32, [P, dp, dp, dp]),
        "sl_synchronize": (I32, [P]),
        "sl_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config)]),
        "sl_transient_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config)]),
        "sl_last_error": (ctypes.c_char_p, []),
        "sl_composition_weights": (I32, [I32, dp, I32]),
        "sl_stability_limit": (D, [I32]),
        "sl_set_kernel_timing": (I32, [P, I32]),
        "sl_kernel_timing": (I32, [P, ctypes.POINTER(I64), dp]),
        "sl_get_tile": (I32, [P] + [ctypes.POINTER(I32)] * 5),
        "sl_set_tile": (I32, [P, I32, I32, I32, I32]),
        "sl_set_chaining": (I32, [P, I32]),
        "sl_hbm_copy_bench": (I32, [ctypes.c_size_t, I32, dp]),
        "sl_batch_create": (I32, [P, ctypes.POINTER(P)]),
        "sl_batch_destroy": (I32, [P]),
        "sl_batch_add": (I32, [P, P]),
        "sl_batch_remove": (I32, [P, P]),
        "sl_batch_count": (I32, [P, ctypes.POINTER(I32)]),
        "sl_batch_set_grid": (I32, [P, I32]),
        "sl_batch_get_grid": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "sl_batch_step": (I32, [P, I64, D, I32]),
        "sl_batch_synchronize": (I32, [P]),
        "sl_device_memory": (I32, [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "sl_autotune": (I32, [P, I32, I32, I32] + [ctypes.POINTER(I32)] * 4 + [dp]),
        "sl_autotune_forget": (I32, []),
        "sl_set_stencil": (I32, [P, dp]),
        "sl_get_stencil": (I32, [P, dp]),
        "sl_linear_create": (I32, [ctypes.POINTER(Config), P, ctypes.POINTER(P)]),
        "sl_linear_destroy": (I32, [P]),
        "sl_linear_set_potential": (I32, [P, I32, dp, I32]),
        "sl_linear_set_stencil": (I32, [P, dp]),
        "sl_linear_set_fields": (I32, [P, P, P, D]),
        "sl_linear_evolve": (I32, [P, I64, D, I32]),
        "sl_linear_get_fields": (I32, [P, P, P]),
        "sl_linear_get_background": (I32, [P, dp, dp, dp, dp, dp]),
        "sl_linear_classes": (I32, [P, ctypes.POINTER(I64)]),
        "sl_linear_synchronize": (I32, [P]),
        "sl_linear_set_kernel_timing": (I32, [P, I32]),
        "sl_linear_kernel_timing": (I32, [P, ctypes.POINTER(I64), dp, dp, dp]),
        "sl_batch_autotune": (I32, [P, I32, dp]),
        "sl_batch_time_pass": (I32, [P, I32, dp]),
        "sl_spectra": (I32, [P, I32, I32, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int64), dp]),
        "sl_set_history": (I32, [P, I64]),
        "sl_get_history": (I32, [P, dp, dp, dp, dp, I64, ctypes.POINTER(I64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != SL_OK:
        msg = load().sl_last_error()
        raise SymlatError(status, msg.decode() if msg else "")


def _dvec(values, n):
    """n doubles for the C side; a length other than n is refused here, since
    the library reads exactly n values."""
    values = list(values)
    if len(values) != n:
        raise ValueError("expected %d values, got %d" % (n, len(values)))
    arr = (ctypes.c_double * max(n, 1))()
    for i, v in enumerate(values):
        arr[i] = float(v)
    return arr


def make_config(n, nfields, L, precision="f64", expand=True, mpl=1.0, a0=1.0,
                rho_rad0=0.0, rho_mat0=0.0):
    return Config(int(n), int(nfields), float(L), PRECISION[precision],
                  1 if expand else 0, float(mpl), float(a0), float(rho_rad0),
                  float(rho_mat0))


def composition_weights(order):
    lib = load()
    buf = (ctypes.c_double * 32)()
    s = lib.sl_composition_weights(int(order), buf, 32)
    if s < 0:
        raise SymlatError(SL_E_INVALID, "unknown order %r" % order)
    return [buf[i] for i in range(s)]


def stability_limit(order):
    return load().sl_stability_limit(int(order))


def hbm_copy_bench(nbytes, iters=20):
    """Achieved read+write GB/s of a plain device copy of nbytes."""
    g = ctypes.c_double()
    _check(load().sl_hbm_copy_bench(int(nbytes), int(iters), ctypes.byref(g)))
    return g.value


def footprint_bytes(**cfg):
    """Device bytes a lattice of this configuration holds while it lives."""
    return int(load().sl_footprint_bytes(ctypes.byref(make_config(**cfg))))


def transient_bytes(**cfg):
    """Most device bytes one call on such a lattice allocates while it runs."""
    return int(load().sl_transient_bytes(ctypes.byref(make_config(**cfg))))


def autotune_forget():
    _check(load().sl_autotune_forget())


def device_memory():
    """(free, total) device bytes."""
    f, t = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().sl_device_memory(ctypes.byref(f), ctypes.byref(t)))
    return f.value, t.value


class Lattice:
    """One lattice handle.  ``stream`` is an optional hipStream_t (int);
    ``buffers`` optional device addresses (ints) of the caller's four field
    arrays (phi0, pi0, phi1, pi1), which the handle then uses without owning
    them (sl_lattice_create_with_buffers)."""

    def __init__(self, n, nfields, L, precision="f64", expand=True, mpl=1.0, a0=1.0,
                 rho_rad0=0.0, rho_mat0=0.0, stream=None, buffers=None):
        self._lib = load()
        self.n, self.nfields, self.L = int(n), int(nfields), float(L)
        self.precision = precision
        self.cfg = make_config(n, nfields, L, precision, expand, mpl, a0, rho_rad0, rho_mat0)
        h = ctypes.c_void_p()
        if buffers is None:
            _check(self._lib.sl_lattice_create(ctypes.byref(self.cfg),
                                               ctypes.c_void_p(stream or 0), ctypes.byref(h)))
        else:
            b = [ctypes.c_void_p(int(x) if x else 0) for x in buffers]
            if len(b) != 4:
                raise ValueError("buffers: four device addresses (phi0, pi0, phi1, pi1)")
            _check(self._lib.sl_lattice_create_with_buffers(
                ctypes.byref(self.cfg), ctypes.c_void_p(stream or 0), *b, ctypes.byref(h)))
        self._h = h

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.sl_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- model and state --------------------------------------------------
    def set_potential(self, kind, params):
        params = list(params)
        _check(self._lib.sl_set_potential(self._h, POTENTIAL[kind], _dvec(params, len(params)),
                                          len(params)))

    def set_stencil(self, c):
        """Laplacian weights (centre, face, edge, corner): a name of
        STENCILS or a 4-sequence."""
        c = STENCILS[c] if isinstance(c, str) else tuple(float(v) for v in c)
        if len(c) != 4:
            raise ValueError("a stencil has 4 weights")
        _check(self._lib.sl_set_stencil(self._h, _dvec(c, 4)))

    def stencil(self):
        buf = (ctypes.c_double * 4)()
        _check(self._lib.sl_get_stencil(self._h, buf))
        return tuple(buf[i] for i in range(4))

    def init_fluctuations(self, phi0, pi0, kind="vacuum", amplitude=0.0, seed=0):
        _check(self._lib.sl_init_fluctuations(
            self._h, _dvec(phi0, self.nfields), _dvec(pi0, self.nfields), FLUCT[kind],
            float(amplitude), ctypes.c_uint64(int(seed) & (2 ** 64 - 1))))

    def set_fields(self, phi, pi, a=1.0, p_a=math.nan):
        shape = (self.nfields, self.n, self.n, self.n)
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(shape)
        pi = np.ascontiguousarray(pi, dtype=np.float64).reshape(shape)
        _check(self._lib.sl_set_fields(self._h, phi.ctypes.data, pi.ctypes.data,
                                       float(a), float(p_a)))

    def get_fields(self):
        shape = (self.nfields, self.n, self.n, self.n)
        phi = np.empty(shape, dtype=np.float64)
        pi = np.empty(shape, dtype=np.float64)
        _check(self._lib.sl_get_fields(self._h, phi.ctypes.data, pi.ctypes.data))
        return phi, pi

    def background(self):
        eta, a, pa = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self._lib.sl_get_background(self._h, ctypes.byref(eta), ctypes.byref(a),
                                           ctypes.byref(pa)))
        return eta.value, a.value, pa.value

    # -- evolution and observables ------------------------------------------
    def evolve(self, steps, dt, order=4):
        _check(self._lib.sl_evolve(self._h, int(steps), float(dt), int(order)))

    def synchronize(self):
        _check(self._lib.sl_synchronize(self._h))

    def energies(self):
        e = Energies()
        _check(self._lib.sl_energies(self._h, ctypes.byref(e)))
        out = {k: getattr(e, k) for k in ("eta", "a", "p_a", "hubble", "rho", "pressure",
                                          "w_eos", "friedmann_residual", "h_total", "pot")}
        for k in ("kin", "grad", "mean", "var"):
            out[k] = [getattr(e, k)[i] for i in range(self.nfields)]
        return out

    def spectrum(self, field, nbins):
        k = np.zeros(nbins)
        p = np.zeros(nbins)
        c = np.zeros(nbins, dtype=np.int64)
        _check(self._lib.sl_spectrum(self._h, int(field), int(nbins),
                                     k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return k, p, c

    def spectrum_noalloc(self, field, nbins):
        """spectrum() through the entry point that allocates no device
        memory (a static per-GPU scratch array; see the header's limits)."""
        k = np.zeros(nbins)
        p = np.zeros(nbins)
        c = np.zeros(nbins, dtype=np.int64)
        _check(self._lib.sl_spectrum_noalloc(self._h, int(field), int(nbins),
                                             k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return k, p, c

    def spectra(self, field, nbins):
        """(k_b, <|F|^2>_b, <rho>_b, <n>_b, counts, m_eff^2): field,
        energy-density and number-density spectra of one field."""
        dp = ctypes.POINTER(ctypes.c_double)
        k, pf, pe, pn = (np.zeros(nbins) for _ in range(4))
        c = np.zeros(nbins, dtype=np.int64)
        m2 = ctypes.c_double()
        _check(self._lib.sl_spectra(self._h, int(field), int(nbins), k.ctypes.data_as(dp),
                                    pf.ctypes.data_as(dp), pe.ctypes.data_as(dp),
                                    pn.ctypes.data_as(dp),
                                    c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    ctypes.byref(m2)))
        return k, pf, pe, pn, c, m2.value

    def set_history(self, capacity):
        """Record (eta, a, p_a, rho) at the end of each step, up to capacity."""
        _check(self._lib.sl_set_history(self._h, int(capacity)))

    def history(self, cap=None):
        """(eta, a, p_a, rho) arrays of the recorded steps; rho is the total
        density the library derives from the constraint."""
        n = ctypes.c_int64()
        _check(self._lib.sl_get_history(self._h, None, None, None, None, 0, ctypes.byref(n)))
        m = n.value if cap is None else min(n.value, int(cap))
        dp = ctypes.POINTER(ctypes.c_double)
        eta, a, pa, rho = np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(m)
        _check(self._lib.sl_get_history(self._h, eta.ctypes.data_as(dp), a.ctypes.data_as(dp),
                                        pa.ctypes.data_as(dp), rho.ctypes.data_as(dp), m,
                                        ctypes.byref(n)))
        return eta, a, pa, rho

    # -- launch shape and timing ---------------------------------------------
    def tile(self):
        """(tx lanes, vx sites per lane, ty rows, tz planes, pf pass mode)
        of the fused pass."""
        v = [ctypes.c_int32() for _ in range(5)]
        _check(self._lib.sl_get_tile(self._h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_tile(self, tx, vx=1, tz=0, pf=1):
        _check(self._lib.sl_set_tile(self._h, int(tx), int(vx), int(tz), int(pf)))

    def set_chaining(self, mode):
        """-1: automatic (default), 0: a stage finalize kernel after every
        pass, 1: fold it into the next pass (results are identical)."""
        _check(self._lib.sl_set_chaining(self._h, int(mode)))

    def autotune(self, reps=3, vx_only=0, pf_only=0):
        """Pick the fastest pass shape for this lattice (timed as real
        stages with frozen coefficients; the state is kept); returns
        ((tx, vx, tz, pf), best time of one stage in ms)."""
        v = [ctypes.c_int32() for _ in range(4)]
        ms = ctypes.c_double()
        _check(self._lib.sl_autotune(self._h, int(reps), int(vx_only), int(pf_only),
                                     *[ctypes.byref(x) for x in v], ctypes.byref(ms)))
        return tuple(x.value for x in v), ms.value

    def set_kernel_timing(self, enable):
        _check(self._lib.sl_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_timing(self):
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(self._lib.sl_kernel_timing(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


class Batch:
    """Many lattices advanced together by one fused pass per stage."""

    def __init__(self, stream=None):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.sl_batch_create(ctypes.c_void_p(stream or 0), ctypes.byref(h)))
        self._h = h
        self.members = []

    def add(self, lat):
        _check(self._lib.sl_batch_add(self._h, lat._h))
        self.members.append(lat)

    def remove(self, lat):
        _check(self._lib.sl_batch_remove(self._h, lat._h))
        self.members.remove(lat)

    def __len__(self):
        c = ctypes.c_int32()
        _check(self._lib.sl_batch_count(self._h, ctypes.byref(c)))
        return c.value

    def step(self, steps, dt, order=4):
        _check(self._lib.sl_batch_step(self._h, int(steps), float(dt), int(order)))

    def set_grid(self, workgroups):
        """0: one workgroup per tile; w > 0: the persistent form with
        min(w, tiles) workgroups striding through the tiles."""
        _check(self._lib.sl_batch_set_grid(self._h, int(workgroups)))

    def grid(self):
        """(requested, launched) workgroups of the batched pass."""
        r, l = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.sl_batch_get_grid(self._h, ctypes.byref(r), ctypes.byref(l)))
        return r.value, l.value

    def synchronize(self):
        _check(self._lib.sl_batch_synchronize(self._h))

    def autotune(self, reps=3):
        """Tune the members' pass shapes for the batched pass; returns the
        best pass time (ms)."""
        ms = ctypes.c_double()
        _check(self._lib.sl_batch_autotune(self._h, int(reps), ctypes.byref(ms)))
        return ms.value

    def time_pass(self, reps=3):
        """Time of one batched pass (ms) with the members' current shapes."""
        ms = ctypes.c_double()
        _check(self._lib.sl_batch_time_pass(self._h, int(reps), ctypes.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.sl_batch_destroy(self._h)
            self._h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Linear:
    """Linearized integrator: homogeneous background plus Fourier-space
    perturbations advanced through growth functions per k_eff^2 class."""

    def __init__(self, n, nfields, L, expand=True, mpl=1.0, a0=1.0, rho_rad0=0.0,
                 rho_mat0=0.0, stream=None):
        self._lib = load()
        self.n, self.nfields = int(n), int(nfields)
        cfg = make_config(n, nfields, L, "f64", expand, mpl, a0, rho_rad0, rho_mat0)
        h = ctypes.c_void_p()
        _check(self._lib.sl_linear_create(ctypes.byref(cfg), ctypes.c_void_p(stream or 0),
                                          ctypes.byref(h)))
        self._h = h

    def set_potential(self, kind, params):
        params = list(params)
        _check(self._lib.sl_linear_set_potential(self._h, POTENTIAL[kind],
                                                 _dvec(params, len(params)), len(params)))

    def set_stencil(self, c):
        c = STENCILS[c] if isinstance(c, str) else tuple(float(v) for v in c)
        _check(self._lib.sl_linear_set_stencil(self._h, _dvec(c, 4)))

    def set_fields(self, phi, pi, p_a=math.nan):
        shape = (self.nfields, self.n, self.n, self.n)
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(shape)
        pi = np.ascontiguousarray(pi, dtype=np.float64).reshape(shape)
        _check(self._lib.sl_linear_set_fields(self._h, phi.ctypes.data, pi.ctypes.data,
                                              float(p_a)))

    def evolve(self, steps, dt, order=4):
        _check(self._lib.sl_linear_evolve(self._h, int(steps), float(dt), int(order)))

    def get_fields(self):
        shape = (self.nfields, self.n, self.n, self.n)
        phi = np.empty(shape)
        pi = np.empty(shape)
        _check(self._lib.sl_linear_get_fields(self._h, phi.ctypes.data, pi.ctypes.data))
        return phi, pi

    def background(self):
        """(eta, a, p_a, phi0, pi0)."""
        v = [ctypes.c_double() for _ in range(3)]
        f0 = (ctypes.c_double * self.nfields)()
        p0 = (ctypes.c_double * self.nfields)()
        _check(self._lib.sl_linear_get_background(self._h, *[ctypes.byref(x) for x in v], f0, p0))
        return v[0].value, v[1].value, v[2].value, list(f0), list(p0)

    def classes(self):
        c = ctypes.c_int64()
        _check(self._lib.sl_linear_classes(self._h, ctypes.byref(c)))
        return c.value

    def synchronize(self):
        _check(self._lib.sl_linear_synchronize(self._h))

    def set_kernel_timing(self, enable):
        _check(self._lib.sl_linear_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_timing(self):
        """(growth launches, growth ms, background-table ms, apply ms)."""
        n = ctypes.c_int64()
        g, t, a = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self._lib.sl_linear_kernel_timing(self._h, ctypes.byref(n), ctypes.byref(g),
                                                 ctypes.byref(t), ctypes.byref(a)))
        return n.value, g.value, t.value, a.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.sl_linear_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reset_from_recipe(lat, r):
    """Re-initialise a lattice made for the recipe's configuration (size,
    fields, box, precision, expansion, m_pl, a0, stencil) for a new run of
    it: the potential and the initial state exactly as from_recipe sets
    them, the pass shape kept."""
    lat.set_potential(r["potential"], r["params"])
    lat.init_fluctuations(r["phi0"], r["pi0"], r["fluct"], r["amplitude"], r["seed"])
    return lat


def from_recipe(r, stream=None):
    """Lattice with potential set and initial state drawn from a workload
    recipe dict (see the synth module)."""
    lat = Lattice(r["n"], r["nfields"], r["L"], precision=r.get("precision", "f64"),
                  expand=r.get("expand", True), mpl=r["mpl"], a0=r.get("a0", 1.0),
                  stream=stream)
    lat.set_potential(r["potential"], r["params"])
    if r.get("stencil") is not None:
        lat.set_stencil(r["stencil"])
    lat.init_fluctuations(r["phi0"], r["pi0"], r["fluct"], r["amplitude"], r["seed"])
    return lat
