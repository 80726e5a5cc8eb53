"""Pins of the oracle's stencils (Sec. 2.1, eq. (2.7), (2.8), (2.17)) and
potentials (Sec. 3) against closed forms, brute force and complex steps."""
import itertools

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


def test_chaotic_potential_closed_form():
    """Sec. 3.1: V = m^2 phi^2/2 + g^2 phi^2 psi^2 / 2 at a worked point."""
    pot = oracle.Potential("chaotic2", (2.0, 3.0))
    phi = np.array([[0.5], [2.0]])
    assert pot.V(phi)[0] == pytest.approx(0.5 * 2 * 0.25 + 0.5 * 3 * 0.25 * 4)
