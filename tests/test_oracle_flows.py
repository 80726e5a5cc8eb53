"""Pins of the exact sub-flows (Sec. 2.3, eq. (2.46)-(2.47)) and the
observables (eq. (2.16), (2.18), (2.19), (3.1)) against complex-step
derivatives of the Hamiltonian and the Friedmann equations."""
import numpy as np
import pytest

import oracle
import synth

H_CS = 1e-30


def _lattice(pot=None, expand=True, rho_rad0=0.3, rho_mat0=0.2, n=4, seed=5,
             stencil=oracle.STENCIL_7):
    pot = pot or oracle.Potential("chaotic2", (1.0, 3.0))
    lat = oracle.Lattice(n, 2.0, pot, mpl=0.9, a0=1.3, rho_rad0=rho_rad0,
                         rho_mat0=rho_mat0, expand=expand, stencil=stencil)
    phi, pi = synth.gaussian_state(n, pot.nfields, seed, phi_base=[0.8] + [0.3] * (pot.nfields - 1),
                                   phi_amp=0.2, pi_amp=0.3)
    lat.phi[...] = phi
    lat.pi[...] = pi
    lat.p_a = -2.7
    return lat


def _cs_grad_field(lat, part, which):
    """Complex-step d H_part / d(which) for every lattice entry."""
    base = dict(a=complex(lat.a), p_a=complex(lat.p_a),
                phi=lat.phi.astype(complex), pi=lat.pi.astype(complex))
    arr = base[which]
    out = np.zeros(arr.shape)
    for idx in np.ndindex(arr.shape):
        kw = dict(base)
        a2 = arr.copy()
        a2[idx] += 1j * H_CS
        kw[which] = a2
        out[idx] = np.imag(lat.ham_parts(**kw)[part]) / H_CS
    return out


def _cs_grad_scalar(lat, part, which):
    kw = dict(a=complex(lat.a), p_a=complex(lat.p_a),
              phi=lat.phi.astype(complex), pi=lat.pi.astype(complex))
    kw[which] = kw[which] + 1j * H_CS
    return np.imag(lat.ham_parts(**kw)[part]) / H_CS


POTS = [oracle.Potential("chaotic2", (1.0, 3.0)),
        oracle.Potential("oscillon", (1.0, 1.0, 0.2)),
        oracle.Potential("qball", (1.0, -0.1, 1.0)),
        oracle.Potential("free", (1.0, 2.0, 0.5))]


@pytest.mark.parametrize("pot,stencil", [(p, oracle.STENCIL_7) for p in POTS]
                         + [(POTS[0], oracle.STENCIL_27), (POTS[2], oracle.STENCIL_19)],
                         ids=lambda v: getattr(v, "kind", None) or "c3=%g" % v[3])
def test_flows_are_hamiltonian_vector_fields(pot, stencil):
    """Each flow's increment / tau equals the Hamiltonian vector field of its
    part of eq. (2.46): H1 drives a, H2 drives phi and p_a, H3 drives pi and
    p_a (brute-force complex step over every lattice entry)."""
    lat = _lattice(pot, stencil=stencil)
    tau = 0.37

    # H1: a' = dH1/dp_a, nothing else moves
    l1 = lat.copy()
    l1.flow_H1(tau)
    assert (l1.a - lat.a) / tau == pytest.approx(_cs_grad_scalar(lat, 0, "p_a"), rel=1e-13)
    assert l1.p_a == lat.p_a
    assert np.array_equal(l1.phi, lat.phi) and np.array_equal(l1.pi, lat.pi)

    # H2: phi' = dH2/dpi, p_a' = -dH2/da, a and pi fixed
    l2 = lat.copy()
    l2.flow_H2(tau)
    np.testing.assert_allclose((l2.phi - lat.phi) / tau,
                               _cs_grad_field(lat, 1, "pi"), rtol=1e-12, atol=1e-14)
    assert (l2.p_a - lat.p_a) / tau == pytest.approx(-_cs_grad_scalar(lat, 1, "a"), rel=1e-12)
    assert l2.a == lat.a and np.array_equal(l2.pi, lat.pi)

    # H3: pi' = -dH3/dphi, p_a' = -dH3/da, a and phi fixed
    l3 = lat.copy()
    l3.flow_H3(tau)
    np.testing.assert_allclose((l3.pi - lat.pi) / tau,
                               -_cs_grad_field(lat, 2, "phi"), rtol=1e-11, atol=1e-12)
    assert (l3.p_a - lat.p_a) / tau == pytest.approx(-_cs_grad_scalar(lat, 2, "a"), rel=1e-11)
    assert l3.a == lat.a and np.array_equal(l3.phi, lat.phi)

    # the three parts do not depend on the variables their flows move
    assert _cs_grad_scalar(lat, 1, "p_a") == 0 and _cs_grad_scalar(lat, 2, "p_a") == 0
    assert np.all(_cs_grad_field(lat, 2, "pi") == 0)
    assert np.all(_cs_grad_field(lat, 1, "phi") == 0)


@pytest.mark.parametrize("flow", ["flow_H1", "flow_H2", "flow_H3"])
def test_flow_inverse(flow):
    lat = _lattice()
    l = lat.copy()
    getattr(l, flow)(0.21)
    getattr(l, flow)(-0.21)
    assert l.a == pytest.approx(lat.a, rel=1e-15, abs=1e-15)
    assert l.p_a == pytest.approx(lat.p_a, rel=1e-14)
    np.testing.assert_allclose(l.phi, lat.phi, rtol=0, atol=1e-14)
    np.testing.assert_allclose(l.pi, lat.pi, rtol=0, atol=1e-13)


def test_static_mode_freezes_background():
    lat = _lattice(expand=False)
    l = lat.copy()
    l.evolve(3, 0.01, 4)
    assert l.a == lat.a and l.p_a == lat.p_a


def test_constraint_gives_zero_hamiltonian_and_residual():
    """p_a from H = 0 (eq. (2.20)) satisfies the first Friedmann equation
    (2.18) built from eq. (2.16) with G for the gradient energy: ties the
    Hamiltonian's phi D phi form to rho through the Stokes identity."""
    lat = _lattice()
    lat.solve_constraint()
    e = lat.energies()
    assert lat.p_a < 0 and e["hubble"] > 0
    assert abs(e["h_total"]) <= 1e-12 * abs(lat.p_a) ** 2 / (12 * lat.VL * lat.mpl ** 2)
    assert e["friedmann_residual"] < 1e-13


@pytest.mark.parametrize("pot", POTS, ids=lambda p: p.kind)
def test_second_friedmann_equation(pot):
    """a'' from Hamilton's equations equals +a^3 <rho - 3P>/(6 m_pl^2) plus
    the matter term (the '+' reading of eq. (2.19)); pins the pressure."""
    lat = _lattice(pot)
    VL, m2 = lat.VL, lat.mpl ** 2
    # a' = dH/dp_a = -p_a/(6 V_L m^2)  =>  a'' = -p_a'/(6 V_L m^2), p_a' = -dH/da
    dHda = sum(_cs_grad_scalar(lat, k, "a") for k in range(3))
    app_eom = dHda / (6 * VL * m2)
    e = lat.energies()
    app_fried = lat.a ** 3 * (e["rho"] - 3 * e["pressure"]) / (6 * m2) \
        + lat.rho_mat0 / (6 * m2)
    assert app_eom == pytest.approx(app_fried, rel=1e-12)


def test_energy_terms_on_plane_wave():
    """rho and P on a static plane wave with known averages:
    <(grad phi)^2> = A^2 k_eff^2 / (2 dx^2), <pi^2> = B^2/2."""
    n, A, B = 8, 0.3, 0.4
    pot = oracle.Potential("free", (0.0,))
    lat = oracle.Lattice(n, 4.0, pot, expand=False)
    lat.phi[0] = synth.plane_wave(n, (1, 2, 0), A)
    lat.pi[0] = synth.plane_wave(n, (0, 0, 3), B)
    e = lat.energies()
    keff2 = 4 * np.sin(np.pi / n) ** 2 + 4 * np.sin(2 * np.pi / n) ** 2
    grad = A * A * keff2 / 2 / lat.dx ** 2 / 2
    kin = B * B / 2 / 2
    assert e["kin"][0] == pytest.approx(kin, rel=1e-13)
    assert e["grad"][0] == pytest.approx(grad, rel=1e-13)
    assert e["rho"] == pytest.approx(kin + grad, rel=1e-13)
    assert e["pressure"] == pytest.approx(kin - grad / 3, rel=1e-13)
    assert e["mean"][0] == pytest.approx(0.0, abs=1e-15)
    assert e["var"][0] == pytest.approx(A * A / 2, rel=1e-13)
