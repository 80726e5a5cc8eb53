"""Geometric pins of the oracle's map (Sec. 2.3): time reversibility,
symplecticity by a complex-step Jacobian, bounded energy error without
expansion, conservation of the Friedmann constraint with expansion and the
matter-like scaling of a homogeneous massive field (Sec. 3.1)."""
import numpy as np
import pytest

import oracle
import synth


def _chaotic(n=4, expand=True, seed=3):
    pot = oracle.Potential("chaotic2", (1.0, 40.0))
    lat = oracle.Lattice(n, 5.0, pot, mpl=1.03, rho_mat0=0.01)
    lat.expand = expand
    phi, pi = synth.gaussian_state(n, 2, seed, phi_base=[1.0, 0.0], phi_amp=0.05, pi_amp=0.05)
    lat.phi[...] = phi
    lat.pi[...] = pi
    lat.solve_constraint()
    return lat


@pytest.mark.parametrize("order", [2, 4, 6])
def test_time_reversibility(order):
    lat = _chaotic()
    l = lat.copy()
    l.evolve(20, 0.02, order)
    assert np.abs(l.phi - lat.phi).max() > 1e-4       # it did move
    l.evolve(20, -0.02, order)
    np.testing.assert_allclose(l.phi, lat.phi, rtol=0, atol=1e-13)
    np.testing.assert_allclose(l.pi, lat.pi, rtol=0, atol=1e-13)
    assert l.a == pytest.approx(lat.a, rel=1e-13)
    assert l.p_a == pytest.approx(lat.p_a, rel=1e-13)


@pytest.mark.parametrize("pot", [oracle.Potential("oscillon", (1.0, 1.0, 0.2)),
                                 oracle.Potential("qball", (1.0, -0.1, 1.0))],
                         ids=lambda p: p.kind)
def test_symplectic_jacobian(pot):
    """J^T Omega J = Omega for one composed step of the full expanding map,
    in the canonical variables (phi, a ; pi, p_a), J by complex step."""
    n = 4 if pot.nfields == 1 else 3
    lat = oracle.Lattice(n, 3.0, pot, mpl=0.9, rho_mat0=0.05, rho_rad0=0.02)
    phi, pi = synth.gaussian_state(n, pot.nfields, 9, phi_base=[0.6] * pot.nfields,
                                   phi_amp=0.1, pi_amp=0.1)
    lat.phi[...] = phi
    lat.pi[...] = pi
    lat.solve_constraint()
    size = pot.nfields * n ** 3

    def pack(l):
        return np.concatenate([l.phi.ravel(), [l.a], l.pi.ravel(), [l.p_a]])

    def run(z):
        l = lat.copy()
        l.phi = z[:size].reshape(lat.phi.shape).copy()
        l.a = z[size]
        l.pi = z[size + 1:2 * size + 1].reshape(lat.pi.shape).copy()
        l.p_a = z[-1]
        l.step(0.05, 4)
        return pack(l)

    z0 = pack(lat).astype(complex)
    dim = z0.size
    J = np.zeros((dim, dim))
    h = 1e-30
    for j in range(dim):
        z = z0.copy()
        z[j] += 1j * h
        J[:, j] = np.imag(run(z)) / h
    half = dim // 2
    Om = np.zeros((dim, dim))
    Om[:half, half:] = np.eye(half)
    Om[half:, :half] = -np.eye(half)
    resid = J.T @ Om @ J - Om
    assert np.abs(resid).max() < 1e-11 * max(1.0, np.abs(J).max() ** 2)


@pytest.mark.parametrize("order", [2, 4])
def test_bounded_energy_static(order):
    """Without expansion the field energy oscillates with amplitude ~ dt^p
    and shows no secular drift over many steps."""
    pot = oracle.Potential("oscillon", (1.0, 1.0, 0.2))

    def run(h, steps):
        lat = oracle.Lattice(6, 6.0, pot, expand=False)
        phi, pi = synth.gaussian_state(6, 1, 21, phi_base=[0.8], phi_amp=0.05, pi_amp=0.0)
        lat.phi[...] = phi
        lat.pi[...] = pi
        E0 = lat.hamiltonian()
        dev = []
        for _ in range(steps):
            lat.step(h, order)
            dev.append(lat.hamiltonian() - E0)
        return np.array(dev) / abs(E0)

    dev1 = run(0.1, 2000)
    dev2 = run(0.05, 4000)
    amp1, amp2 = np.abs(dev1).max(), np.abs(dev2).max()
    assert amp1 < 1e-2
    ratio = np.log2(amp1 / amp2)
    assert order - 0.5 < ratio < order + 0.7, (amp1, amp2)
    # no secular drift: the second half is not larger than the first half
    half = len(dev2) // 2
    assert np.abs(dev2[half:]).max() < 1.5 * np.abs(dev2[:half]).max()


def test_friedmann_constraint_conserved():
    """With self-consistent expansion the residual curvature eq. (3.1)
    stays bounded and shrinks as dt^4 at 4th order (two-field preheating
    model at 8^3, one unit of conformal time)."""
    cfg = synth.preheat(n=8)
    pot = oracle.Potential(cfg["potential"], cfg["params"])
    worst = []
    for dt in (0.005, 0.0025):
        lat = oracle.Lattice(8, cfg["L"], pot, mpl=cfg["mpl"])
        lat.init_fluctuations(cfg["phi0"], cfg["pi0"], "vacuum", 1e-3, cfg["seed"])
        assert lat.energies()["friedmann_residual"] < 1e-13
        r = []
        for _ in range(4):
            lat.evolve(int(round(0.25 / dt)), dt, 4)
            r.append(lat.energies()["friedmann_residual"])
        # bounded: no growth from the first to the last quarter
        assert max(r) < 1e-7 and r[-1] < 2 * r[0]
        worst.append(max(r))
    assert 3.5 < np.log2(worst[0] / worst[1]) < 4.6
    assert lat.a > 1.5


def test_matter_like_scaling():
    """A homogeneous massive field in an expanding background behaves like
    matter: a^(-3/2) / H is nearly constant once oscillations dominate
    (Sec. 3.1, discussion of its Fig. 1a)."""
    pot = oracle.Potential("free", (1.0,))
    lat = oracle.Lattice(4, 1.0, pot, mpl=1.0)
    lat.init_fluctuations([0.3], [0.0], "none", 0.0, 0)
    vals = []
    for _ in range(400):
        lat.evolve(10, 0.01, 4)
        e = lat.energies()
        vals.append(lat.a ** -1.5 / e["hubble"])
    v = np.array(vals)
    # average over many oscillations (period 2 pi in physical time)
    early, late = v[100:200].mean(), v[300:400].mean()
    assert abs(late / early - 1) < 0.02
    assert lat.a > 1.5
