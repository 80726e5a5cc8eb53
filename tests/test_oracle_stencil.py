"""Pins of the oracle's stencils (Sec. 2.1, eq. (2.7), (2.8), (2.17)) and
potentials (Sec. 3) against closed forms, brute force and complex steps."""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth


def test_laplacian_plane_wave_eigenrelation():
    """D[exp(i k.x)] = -(sum_d 4 sin^2(k_d/2)) exp(i k.x) for the 7-point
    member of eq. (2.7): the lattice dispersion fixed for the method."""
    n = 12
    r = np.arange(n)
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    for kv in [(1, 0, 0), (0, 3, 0), (2, 5, 7), (6, 6, 6), (11, 1, 4)]:
        k = 2 * np.pi * np.array(kv) / n
        # phase reduced mod n in integers so that f is a plane wave to 1 ulp
        m = (kv[0] * x + kv[1] * y + kv[2] * z) % n
        f = np.exp(2j * np.pi * m / n)
        lam = -sum(4 * np.sin(kd / 2) ** 2 for kd in k)
        err = np.max(np.abs(oracle.lap(f) - lam * f))
        assert err <= 4e-15 * max(1.0, abs(lam))


def _brute_lap_G(f):
    n = f.shape[0]
    D = np.zeros_like(f)
    G = np.zeros_like(f)
    for z, y, x in itertools.product(range(n), repeat=3):
        c = f[z, y, x]
        acc, g = 0.0, 0.0
        for dz, dy, dx in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                           (0, 0, 1), (0, 0, -1)]:
            v = f[(z + dz) % n, (y + dy) % n, (x + dx) % n]
            acc += v
            g += (v - c) ** 2
        D[z, y, x] = acc - 6 * c
        G[z, y, x] = 0.5 * g
    return D, G


def test_laplacian_and_G_brute_force():
    f = np.random.default_rng(1).standard_normal((5, 5, 5))
    D, G = _brute_lap_G(f)
    np.testing.assert_allclose(oracle.lap(f), D, rtol=0, atol=1e-13)
    np.testing.assert_allclose(oracle.grad_energy(f), G, rtol=0, atol=1e-13)


def test_laplacian_axes_are_distinct():
    """An x-only wave must not be differentiated along z (catches a
    transposed axis)."""
    n = 8
    f = synth.plane_wave(n, (1, 0, 0))
    D = oracle.lap(f)
    lam = -4 * np.sin(np.pi / n) ** 2
    np.testing.assert_allclose(D, lam * f, atol=1e-14)
    # the wave varies along the last (x) axis only
    assert np.allclose(f[:, :, 0], f[0, 0, 0])


def test_stokes_identity():
    """sum_x phi D[phi] = -sum_x G[phi] on a periodic lattice, eq. (2.17)."""
    rng = np.random.default_rng(7)
    for n in (4, 7, 10):
        f = 1.0 + rng.standard_normal((n, n, n))
        lhs = np.sum(f * oracle.lap(f))
        rhs = -np.sum(oracle.grad_energy(f))
        scale = np.sum(np.abs(f * oracle.lap(f)))
        assert abs(lhs - rhs) <= 1e-13 * scale


POTS = [
    oracle.Potential("free", (1.0, 4.0, 0.25)),
    oracle.Potential("chaotic2", (1.0, synth.PREHEAT_G)),
    oracle.Potential("oscillon", (1.0, 1.0, 0.2)),
    oracle.Potential("qball", (1.0, -0.1, 1.0)),
]


@pytest.mark.parametrize("pot", POTS, ids=lambda p: p.kind)
def test_dV_is_complex_step_gradient_of_V(pot):
    rng = np.random.default_rng(3)
    phi = 0.1 + 0.5 * rng.standard_normal((pot.nfields, 6))
    dV = pot.dV(phi)
    h = 1e-30
    for i in range(pot.nfields):
        pc = phi.astype(complex)
        pc[i] += 1j * h
        cs = np.imag(pot.V(pc)) / h
        np.testing.assert_allclose(dV[i], cs, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("pot", POTS, ids=lambda p: p.kind)
def test_hessian_diag_is_complex_step_of_dV(pot):
    phi0 = [0.7, 0.3][: pot.nfields] if pot.nfields <= 2 else [0.7, 0.3, -0.2]
    d2 = pot.d2V_diag(phi0)
    h = 1e-30
    for i in range(pot.nfields):
        pc = np.array(phi0, dtype=complex)[:, None]
        pc[i] += 1j * h
        cs = np.imag(pot.dV(pc)[i, 0]) / h
        assert abs(d2[i] - cs) <= 1e-12 * max(1.0, abs(cs))


def test_qball_regular_at_origin():
    pot = oracle.Potential("qball", (1.0, -0.1, 1.0))
    z = np.zeros((2, 3))
    assert np.all(pot.V(z) == 0.0)
    assert np.all(pot.dV(z) == 0.0)
    # u ln u -> 0: the potential is continuous at the origin
    small = np.full((2, 1), 1e-150)
    assert abs(pot.V(small)[0]) < 1e-290


def _worked_values():
    path = os.path.join(os.path.dirname(__file__), "golden", "potential_worked_values.txt")
    rows = []
    with open(path) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            tok = line.split()
            kind, vals = tok[0], [float(t) for t in tok[1:]]
            nf = 1 if kind == "oscillon" else 2
            rows.append((kind, vals[:3], vals[3:3 + nf], vals[3 + nf], vals[4 + nf:]))
    return rows


@pytest.mark.parametrize("row", _worked_values(), ids=lambda r: "%s-%s" % (r[0], r[2]))
def test_oscillon_and_qball_worked_values(row):
    """Sec. 3.2 and 3.3 potentials at hand-computed points (fixture with the
    exact derivations): pins the coefficients lam/4 and g/6, the sign of
    each term, u = (phi1^2 + phi2^2)/2 and the 1 + K + K ln(u/M^2) factor of
    the Q-ball force, which the complex-step gradient pin cannot tell apart
    from a consistent slip in V and dV together."""
    kind, params, phi, V, dV = row
    pot = oracle.Potential(kind, params)
    f = np.array(phi, dtype=float).reshape(len(phi), 1)
    assert float(pot.V(f)[0]) == pytest.approx(V, rel=1e-13, abs=1e-15)
    np.testing.assert_allclose(pot.dV(f)[:, 0], dV, rtol=1e-13, atol=1e-15)


def test_chaotic_potential_closed_form():
    """Sec. 3.1: V = m^2 phi^2/2 + g^2 phi^2 psi^2 / 2 at a worked point."""
    pot = oracle.Potential("chaotic2", (2.0, 3.0))
    phi = np.array([[0.5], [2.0]])
    assert pot.V(phi)[0] == pytest.approx(0.5 * 2 * 0.25 + 0.5 * 3 * 0.25 * 4)


# ---------------------------------------------------------------------------
# The cubic stencil family of eq. (2.7): face, edge and corner weights
# ---------------------------------------------------------------------------

# c0 of the last (non-isotropic) member is filled in by _fix_family below;
# c1 = 1 - 4 c2 - 4 c3 keeps it in the family
FAMILY = [oracle.STENCIL_7, oracle.STENCIL_19, oracle.STENCIL_27,
          oracle.isotropic_stencil(-0.02), (None, 0.4, 0.1, 0.05)]


def _brute_symbol(c, k):
    """sum over the 27 offsets of weight(offset) exp(i k.offset), by class
    of the offset (number of nonzero components)."""
    tot = 0.0 + 0.0j
    for off in itertools.product((-1, 0, 1), repeat=3):
        cls = sum(1 for o in off if o)
        tot += c[cls] * np.exp(1j * np.dot(k, off))
    return tot


def _fix_family(c):
    # recompute c0 so that the last entry satisfies the zero-sum condition
    return (-(6 * c[1] + 12 * c[2] + 8 * c[3]), c[1], c[2], c[3])


FAMILY = [_fix_family(c) for c in FAMILY]


@pytest.mark.parametrize("c", FAMILY, ids=lambda c: "c3=%.3g" % c[3])
def test_family_conditions(c):
    assert oracle.stencil_ok(c)
    assert not oracle.stencil_ok((c[0] + 0.1, c[1], c[2], c[3]))


@pytest.mark.parametrize("c", FAMILY, ids=lambda c: "c3=%.3g" % c[3])
def test_general_stencil_plane_wave(c):
    """D[exp(i k.x)] equals the brute-force sum of weighted neighbour phases
    times the wave, and that sum equals the closed-form symbol."""
    n = 10
    r = np.arange(n)
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    for kv in [(1, 0, 0), (0, 3, 2), (2, 5, 7), (5, 5, 5), (9, 1, 4)]:
        k = 2 * np.pi * np.array(kv) / n   # (kz, ky, kx) order of the axes
        m = (kv[0] * z + kv[1] * y + kv[2] * x) % n
        f = np.exp(2j * np.pi * m / n)
        lam = _brute_symbol(c, k)
        assert abs(lam.imag) < 1e-14
        assert abs(oracle.stencil_symbol(c, *k) - lam.real) < 1e-13
        err = np.max(np.abs(oracle.lap(f, c) - lam.real * f))
        assert err <= 1e-13 * max(1.0, abs(lam.real))


def test_seven_point_symbol_is_sine_form():
    k = np.linspace(-np.pi, np.pi, 13)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    s = oracle.stencil_symbol(oracle.STENCIL_7, kz, ky, kx)
    np.testing.assert_allclose(-s, sum(4 * np.sin(q / 2) ** 2 for q in (kz, ky, kx)),
                               atol=1e-13)


@pytest.mark.parametrize("c", FAMILY, ids=lambda c: "c3=%.3g" % c[3])
def test_general_stencil_brute_force_and_stokes(c):
    """lap and G against explicit loops over all 26 neighbours, and the
    summation-by-parts identity sum f D[f] = -sum G[f] of eq. (2.17)."""
    f = np.random.default_rng(5).standard_normal((4, 5, 3))
    nz, ny, nx = f.shape
    D = np.zeros_like(f)
    G = np.zeros_like(f)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        acc, g = c[0] * f[z, y, x], 0.0
        for off in itertools.product((-1, 0, 1), repeat=3):
            cls = sum(1 for o in off if o)
            if cls == 0:
                continue
            v = f[(z + off[0]) % nz, (y + off[1]) % ny, (x + off[2]) % nx]
            acc += c[cls] * v
            g += c[cls] * (v - f[z, y, x]) ** 2
        D[z, y, x] = acc
        G[z, y, x] = 0.5 * g
    np.testing.assert_allclose(oracle.lap(f, c), D, rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.grad_energy(f, c), G, rtol=0, atol=1e-12)
    lhs = np.sum(f * oracle.lap(f, c))
    assert abs(lhs + np.sum(oracle.grad_energy(f, c))) <= 1e-12 * np.sum(np.abs(f * D))


def _anisotropy(c, kmag):
    """Largest difference of the symbol between the axis, face-diagonal and
    body-diagonal directions at the same |k|."""
    dirs = [np.array([1.0, 0, 0]), np.array([1.0, 1, 0]) / np.sqrt(2),
            np.array([1.0, 1, 1]) / np.sqrt(3), np.array([1.0, 2, 3]) / np.sqrt(14)]
    vals = [oracle.stencil_symbol(c, *(kmag * d)) for d in dirs]
    return max(vals) - min(vals), vals


def test_isotropic_members_have_k6_anisotropy():
    """For the isotropic members the direction dependence of the symbol
    starts at |k|^6 (halving |k| divides it by 64) and the symbol is
    -|k|^2 + |k|^4/12 up to O(k^6); for the 7-point member it starts at
    |k|^4 (factor 16)."""
    for c in (oracle.STENCIL_19, oracle.STENCIL_27, oracle.isotropic_stencil(0.1)):
        a1, v1 = _anisotropy(c, 0.2)
        a2, _ = _anisotropy(c, 0.1)
        assert 50 < a1 / a2 < 80
        for v in v1:
            assert abs(v - (-0.04 + 0.0016 / 12)) < 0.2 ** 6
    a1, _ = _anisotropy(oracle.STENCIL_7, 0.2)
    a2, _ = _anisotropy(oracle.STENCIL_7, 0.1)
    assert 14 < a1 / a2 < 18


def test_named_isotropic_members():
    assert oracle.STENCIL_19 == pytest.approx((-4.0, 1 / 3, 1 / 6, 0.0), abs=1e-15)
    assert oracle.STENCIL_27 == pytest.approx((-128 / 30, 14 / 30, 3 / 30, 1 / 30), abs=1e-15)


@pytest.mark.parametrize("c", FAMILY, ids=lambda c: "c3=%.3g" % c[3])
def test_max_keff2_is_a_zone_vertex(c):
    """The largest -symbol over a fine scan of the zone equals the vertex
    value returned (the symbol is multilinear in the cosines)."""
    k = np.linspace(-np.pi, np.pi, 41)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    scan = float(np.max(-oracle.stencil_symbol(c, kz, ky, kx)))
    assert abs(scan - oracle.stencil_max_keff2(c)) < 1e-12
    assert oracle.stencil_max_keff2(oracle.STENCIL_7) == pytest.approx(12.0)


def test_keff2_modes_matches_symbol():
    n = 6
    for c in (oracle.STENCIL_7, oracle.STENCIL_27):
        k2 = oracle.keff2_modes(n, c)
        for (a, b, d) in [(0, 0, 0), (1, 2, 3), (3, 3, 3), (5, 0, 1)]:
            k = 2 * np.pi * np.array([a, b, d]) / n
            assert abs(k2[a, b, d] + _brute_symbol(c, k).real) < 1e-13
