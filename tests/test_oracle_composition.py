"""Pins of the compositions (Sec. 2.3, eq. (2.42)-(2.45), Table 1): printed
constants, order conditions, the exact discrete linear map of a free field,
closed-form homogeneous solutions and convergence against high-accuracy
ODE solutions."""
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1_weights.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            o, i, v = line.split()
            rows.setdefault(int(o), {})[int(i)] = float(v)
    return rows


def test_table1_weights_match_paper():
    t = _table1()
    for order, n_half in ((6, 3), (8, 7)):
        w = oracle.composition_weights(order)
        assert len(w) == 2 * n_half + 1
        for i in range(1, n_half + 1):
            assert w[i - 1] == t[order][i]
            assert w[-i] == t[order][i]          # symmetry w_{s+1-i} = w_i
        assert w[n_half] == pytest.approx(1 - 2 * sum(t[order].values()), abs=1e-15)


def test_composition_constants():
    for order in (2, 4, 6, 8):
        assert sum(oracle.composition_weights(order)) == pytest.approx(1.0, abs=1e-14)
    z1, z0, _ = oracle.composition_weights(4)
    # triple jump: 2 z1 + z0 = 1 and 2 z1^3 + z0^3 = 0 (third-order condition)
    assert 2 * z1 ** 3 + z0 ** 3 == pytest.approx(0.0, abs=1e-14)
    assert z1 == pytest.approx(1.3512071919596578, rel=1e-15)
    assert z0 == pytest.approx(-1.7024143839193153, rel=1e-15)
    assert oracle.composition_weights(6)[3] == pytest.approx(1.3151863206839112, rel=1e-14)
    assert oracle.composition_weights(8)[7] == pytest.approx(-0.79688793935291646, rel=1e-13)
    # symmetric compositions satisfy sum w^3 = 0 (order >= 3 condition)
    for order in (4, 6, 8):
        assert sum(w ** 3 for w in oracle.composition_weights(order)) == pytest.approx(0, abs=1e-13)


def test_stability_limits():
    # leapfrog: omega h < 2 (textbook)
    assert oracle.stability_limit(2) == pytest.approx(2.0, abs=2e-5)
    # triple-jump (Forest-Ruth / Yoshida) 4th order: omega h < 1.5734
    assert oracle.stability_limit(4) == pytest.approx(1.5734, abs=2e-4)
    lim6, lim8 = oracle.stability_limit(6), oracle.stability_limit(8)
    assert 2.26 < lim6 < 2.28 and 3.38 < lim8 < 3.40


# ---------------------------------------------------------------------------
# Exact discrete linear map (free field, static background)
# ---------------------------------------------------------------------------

def _mode_map(h, order, omega2, a):
    """Per-mode product of stage matrices: drift phi += pi tau/a^2, kick
    pi -= (a^2 k^2/dx^2 + a^4 m^2) phi tau, in the order of eq. (2.48)."""
    M = np.broadcast_to(np.eye(2), omega2.shape + (2, 2)).copy()
    for w in oracle.composition_weights(order):
        t = w * h
        Dr = np.zeros(omega2.shape + (2, 2))
        Dr[..., 0, 0] = Dr[..., 1, 1] = 1
        Dr[..., 0, 1] = t / 2 / a ** 2
        K = np.zeros_like(Dr)
        K[..., 0, 0] = K[..., 1, 1] = 1
        K[..., 1, 0] = -t * omega2
        M = Dr @ K @ Dr @ M
    return M


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("a0", [1.0, 1.3])
def test_exact_linear_map(order, a0):
    """Static free field: every Fourier mode evolves by the product of the
    2x2 stage matrices; the lattice result equals FFT -> product -> iFFT."""
    n, L, m2, h, steps = 8, 5.0, 0.7, 0.05, 100
    pot = oracle.Potential("free", (m2,))
    lat = oracle.Lattice(n, L, pot, a0=a0, expand=False)
    phi, pi = synth.gaussian_state(n, 1, 11, phi_amp=1.0, pi_amp=1.0)
    lat.phi[...] = phi
    lat.pi[...] = pi
    lat.evolve(steps, h, order)

    f = np.fft.fftfreq(n) * n
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    keff2 = sum(4 * np.sin(np.pi * k / n) ** 2 for k in (kz, ky, kx))
    omega2 = a0 ** 2 * keff2 / lat.dx ** 2 + a0 ** 4 * m2
    M1 = _mode_map(h, order, omega2, a0)
    M = np.broadcast_to(np.eye(2), omega2.shape + (2, 2)).copy()
    for _ in range(steps):
        M = M1 @ M
    P, Q = np.fft.fftn(phi[0]), np.fft.fftn(pi[0])
    P2 = M[..., 0, 0] * P + M[..., 0, 1] * Q
    Q2 = M[..., 1, 0] * P + M[..., 1, 1] * Q
    np.testing.assert_allclose(lat.phi[0], np.fft.ifftn(P2).real, atol=1e-12 * np.abs(phi).max())
    np.testing.assert_allclose(lat.pi[0], np.fft.ifftn(Q2).real, atol=1e-12 * np.abs(pi).max())


def test_lattice_dispersion_continuum_limit():
    """A plane wave oscillates at omega^2 = m^2 + sum_d 4 sin^2(k_d dx/2)/dx^2
    in the dt -> 0 limit, with 4th-order error in dt."""
    n, L, m2 = 8, 4.0, 0.5
    kv = (1, 2, 0)
    dx = L / n
    omega = np.sqrt(m2 + sum(4 * np.sin(np.pi * k / n) ** 2 for k in kv) / dx ** 2)
    T = 2.0
    errs = []
    for steps in (40, 80):
        lat = oracle.Lattice(n, L, oracle.Potential("free", (m2,)), expand=False)
        lat.phi[0] = synth.plane_wave(n, kv)
        lat.evolve(steps, T / steps, 4)
        exact = np.cos(omega * T) * synth.plane_wave(n, kv)
        errs.append(np.abs(lat.phi[0] - exact).max())
    assert errs[1] < 1e-4
    slope = np.log2(errs[0] / errs[1])
    assert 3.8 < slope < 4.2


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_homogeneous_harmonic_closed_form(order):
    """phi(eta) = phi0 cos(m eta) + (pi0/m) sin(m eta) for a static
    homogeneous free field; error ~ dt^order."""
    m2, phi0, pi0, T = 2.0, 0.7, -0.3, 3.0
    m = np.sqrt(m2)
    exact = phi0 * np.cos(m * T) + pi0 / m * np.sin(m * T)
    errs = []
    base = {2: 100, 4: 25, 6: 12, 8: 8}[order]
    for steps in (base, 2 * base):
        lat = oracle.Lattice(4, 1.0, oracle.Potential("free", (m2,)), expand=False)
        lat.init_homogeneous([phi0], [pi0])
        lat.evolve(steps, T / steps, order)
        errs.append(abs(lat.phi[0, 0, 0, 0] - exact))
        # homogeneous: the Laplacian vanishes, every site identical
        assert np.ptp(lat.phi) == 0
    slope = np.log2(errs[0] / errs[1])
    assert order - 0.3 < slope < order + 0.6


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_anharmonic_oscillator_order(order):
    """Homogeneous oscillon potential (phi^6 term), static: convergence slope
    against DOP853 at rtol 1e-13 equals the composition order."""
    pot = oracle.Potential("oscillon", (1.0, 1.0, 0.2))
    phi0, T = 1.2, 2.0
    ref = solve_ivp(lambda t, y: [y[1], -pot.dV(np.array([[y[0]]]))[0, 0]],
                    (0, T), [phi0, 0.0], method="DOP853", rtol=1e-13, atol=1e-15)
    exact = ref.y[0, -1]
    base = {2: 200, 4: 40, 6: 10, 8: 5}[order]
    errs = []
    for steps in (base, 2 * base):
        lat = oracle.Lattice(4, 1.0, pot, expand=False)
        lat.init_homogeneous([phi0], [0.0])
        lat.evolve(steps, T / steps, order)
        errs.append(abs(lat.phi[0, 0, 0, 0] - exact))
    slope = np.log2(errs[0] / errs[1])
    assert order - 0.4 < slope < order + 0.8, (errs, slope)


# ---------------------------------------------------------------------------
# Expanding background: closed forms and a homogeneous ODE reference
# ---------------------------------------------------------------------------

def test_radiation_only_closed_form():
    """Fields zero, radiation only: a(eta) = a0 + sqrt(rho_r/(3 m_pl^2)) eta
    exactly (radiation does not enter the equations of motion)."""
    rho_r, mpl = 0.8, 1.3
    lat = oracle.Lattice(4, 1.0, oracle.Potential("free", (1.0,)), mpl=mpl,
                         rho_rad0=rho_r)
    lat.init_fluctuations([0.0], [0.0], "none", 0.0, 0)
    lat.evolve(37, 0.05, 4)
    expect = 1.0 + np.sqrt(rho_r / (3 * mpl ** 2)) * lat.eta
    assert lat.a == pytest.approx(expect, rel=1e-14)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_matter_only_closed_form(order):
    """Fields zero, matter only: a = a0 + a0' eta + rho_m eta^2 / (12 m_pl^2)
    exactly, each exact flow being exact for a constant force."""
    rho_m, mpl, a0 = 0.6, 0.8, 1.0
    lat = oracle.Lattice(4, 1.0, oracle.Potential("free", (1.0,)), mpl=mpl,
                         a0=a0, rho_mat0=rho_m)
    lat.init_fluctuations([0.0], [0.0], "none", 0.0, 0)
    ap0 = -lat.p_a / (6 * lat.VL * mpl ** 2)
    assert ap0 == pytest.approx(np.sqrt(a0 * rho_m / (3 * mpl ** 2)), rel=1e-14)
    lat.evolve(25, 0.08, order)
    eta = lat.eta
    assert lat.a == pytest.approx(a0 + ap0 * eta + rho_m * eta ** 2 / (12 * mpl ** 2), rel=1e-13)


def _homog_ode(pot, mpl, rho_m):
    """Per-site homogeneous system: phi' = pi/a^2, pi' = -a^4 V',
    a' = -q/(6 m^2), q' = pi^2/a^3 - 4 a^3 V - rho_m, with q = p_a / V_L."""
    def f(t, y):
        phi, pi, a, q = y
        V = pot.V(np.array([[phi]]))[0]
        dV = pot.dV(np.array([[phi]]))[0, 0]
        return [pi / a ** 2, -a ** 4 * dV, -q / (6 * mpl ** 2),
                pi ** 2 / a ** 3 - 4 * a ** 3 * V - rho_m]
    return f


@pytest.mark.parametrize("order", [4, 6])
def test_homogeneous_expanding_field_vs_ode(order):
    pot = oracle.Potential("free", (1.0,))
    mpl, rho_m, T = 0.7, 0.05, 2.0
    lat0 = oracle.Lattice(4, 1.0, pot, mpl=mpl, rho_mat0=rho_m)
    lat0.init_fluctuations([1.0], [0.2], "none", 0.0, 0)
    y0 = [1.0, 0.2, 1.0, lat0.p_a / lat0.VL]
    ref = solve_ivp(_homog_ode(pot, mpl, rho_m), (0, T), y0, method="DOP853",
                    rtol=1e-13, atol=1e-15).y[:, -1]
    base = {4: 40, 6: 16}[order]
    errs = []
    for steps in (base, 2 * base):
        lat = lat0.copy()
        lat.evolve(steps, T / steps, order)
        got = np.array([lat.phi[0, 0, 0, 0], lat.pi[0, 0, 0, 0], lat.a, lat.p_a / lat.VL])
        errs.append(np.abs(got - ref).max())
    slope = np.log2(errs[0] / errs[1])
    assert order - 0.4 < slope < order + 0.8, (errs, slope)


def _flow_vector_field(lat0):
    """Sum of the three flows' vector fields (each flow is exactly linear in
    tau, so increment/tau is its generator; pinned to dH by complex step in
    the flow tests)."""
    nf, n = lat0.nf, lat0.n
    size = nf * n ** 3

    def unpack(y):
        l = lat0.copy()
        l.phi = y[:size].reshape(nf, n, n, n).copy()
        l.pi = y[size:2 * size].reshape(nf, n, n, n).copy()
        l.a, l.p_a = y[-2], y[-1]
        return l

    def pack(l):
        return np.concatenate([l.phi.ravel(), l.pi.ravel(), [l.a, l.p_a]])

    def f(t, y):
        base = unpack(y)
        out = np.zeros_like(y)
        for flow in ("flow_H1", "flow_H2", "flow_H3"):
            l = unpack(y)
            getattr(l, flow)(1.0)
            out += pack(l) - pack(base)
        return out

    return f, pack, unpack


@pytest.mark.parametrize("order", [4, 6])
def test_full_lattice_4cubed_vs_ode(order):
    """Full 4^3 two-field lattice with gradients, potential coupling and
    self-consistent expansion converges to the Hamiltonian ODE at the
    composition's order."""
    pot = oracle.Potential("chaotic2", (1.0, 4.0))
    lat0 = oracle.Lattice(4, 3.0, pot, mpl=0.8, rho_mat0=0.02, rho_rad0=0.01)
    phi, pi = synth.gaussian_state(4, 2, 17, phi_base=[1.0, 0.1], phi_amp=0.1, pi_amp=0.1)
    lat0.phi[...] = phi
    lat0.pi[...] = pi
    lat0.solve_constraint()
    f, pack, _ = _flow_vector_field(lat0)
    T = 1.0
    ref = solve_ivp(f, (0, T), pack(lat0), method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    base = {4: 20, 6: 10}[order]
    errs = []
    for steps in (base, 2 * base):
        lat = lat0.copy()
        lat.evolve(steps, T / steps, order)
        errs.append(np.abs(pack(lat) - ref).max())
    slope = np.log2(errs[0] / errs[1])
    assert order - 0.5 < slope < order + 1.0, (errs, slope)


@pytest.mark.parametrize("order", [4, 6])
def test_exact_linear_map_27_point(order):
    """Same pin for the isotropic 27-point member of eq. (2.7): the mode
    frequency is set by its symbol, written here as the brute-force sum of
    weighted neighbour phases."""
    import itertools
    c = oracle.STENCIL_27
    n, L, m2, h, steps = 6, 4.0, 0.7, 0.05, 60
    lat = oracle.Lattice(n, L, oracle.Potential("free", (m2,)), expand=False, stencil=c)
    phi, pi = synth.gaussian_state(n, 1, 12, phi_amp=1.0, pi_amp=1.0)
    lat.phi[...] = phi
    lat.pi[...] = pi
    lat.evolve(steps, h, order)
    f = np.fft.fftfreq(n) * n
    lam = np.zeros((n, n, n))
    for iz, iy, ix in itertools.product(range(n), repeat=3):
        k = 2 * np.pi * np.array([f[iz], f[iy], f[ix]]) / n
        tot = 0.0
        for off in itertools.product((-1, 0, 1), repeat=3):
            tot += c[sum(1 for o in off if o)] * np.cos(np.dot(k, off))
        lam[iz, iy, ix] = tot
    omega2 = -lam / lat.dx ** 2 + m2
    M1 = _mode_map(h, order, omega2, 1.0)
    M = np.broadcast_to(np.eye(2), omega2.shape + (2, 2)).copy()
    for _ in range(steps):
        M = M1 @ M
    P, Q = np.fft.fftn(phi[0]), np.fft.fftn(pi[0])
    np.testing.assert_allclose(lat.phi[0], np.fft.ifftn(M[..., 0, 0] * P + M[..., 0, 1] * Q).real,
                               atol=1e-12 * np.abs(phi).max())
    np.testing.assert_allclose(lat.pi[0], np.fft.ifftn(M[..., 1, 0] * P + M[..., 1, 1] * Q).real,
                               atol=1e-12 * np.abs(pi).max())
