"""Pins of the linearized-integrator oracle (Sec. 2.2 and Sec. 2.4, eq.
(2.49)-(2.50)): the Hessian against complex steps and the printed V^(2) of
the chaotic model, the background against the nonlinear lattice with no
perturbation, the free static field against the nonlinear lattice (the
problem is linear there), agreement with the nonlinear lattice to second
order in the amplitude, conservation of the symplectic form of the
perturbations, and time reversibility."""
import numpy as np
import pytest

import oracle
import synth

POTS = [oracle.Potential("chaotic2", (1.0, 3.0)),
        oracle.Potential("oscillon", (1.0, 1.0, 0.2)),
        oracle.Potential("qball", (1.0, -0.1, 1.0)),
        oracle.Potential("free", (1.0, 2.0, 0.5))]


@pytest.mark.parametrize("pot", POTS, ids=lambda p: p.kind)
def test_hessian_is_complex_step_of_dV(pot):
    phi0 = [0.7, 0.3, -0.2][: pot.nfields]
    H = pot.hessian(phi0)
    h = 1e-30
    for j in range(pot.nfields):
        pc = np.array(phi0, dtype=complex)[:, None]
        pc[j] += 1j * h
        col = np.imag(pot.dV(pc)[:, 0]) / h
        np.testing.assert_allclose(H[:, j], col, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(H, H.T, rtol=0, atol=0)
    np.testing.assert_allclose(np.diag(H), pot.d2V_diag(phi0), rtol=1e-14)


def test_chaotic_second_order_potential_printed_form():
    """Sec. 2.2 prints V^(2) of V = m^2 phi^2/2 + g^2 phi^2 chi^2/2 as
    m^2 dphi^2/2 + g^2 dphi^2 chi0^2/2 + 2 g^2 phi0 chi0 dphi dchi
    + g^2 phi0^2 dchi^2/2; the oracle's Hessian gives delta^T H delta / 2."""
    m2, g2 = 1.7, 2.3
    pot = oracle.Potential("chaotic2", (m2, g2))
    phi0, chi0 = 0.6, -0.4
    H = pot.hessian([phi0, chi0])
    rng = np.random.default_rng(8)
    for _ in range(5):
        d = rng.standard_normal(2)
        printed = (0.5 * m2 * d[0] ** 2 + 0.5 * g2 * d[0] ** 2 * chi0 ** 2
                   + 2 * g2 * phi0 * chi0 * d[0] * d[1] + 0.5 * g2 * phi0 ** 2 * d[1] ** 2)
        assert 0.5 * d @ H @ d == pytest.approx(printed, rel=1e-14)


def _lin_and_nonlin(pot, n=6, L=3.0, expand=True, amp=1e-3, seed=21, a0=1.0,
                    stencil=oracle.STENCIL_7, **kw):
    base = [0.8, 0.3, 0.1][: pot.nfields]
    pibase = [0.05, -0.02, 0.01][: pot.nfields]
    phi, pi = synth.gaussian_state(n, pot.nfields, seed, phi_base=base, phi_amp=amp,
                                   pi_base=pibase, pi_amp=amp)
    lin = oracle.LinearLattice(n, L, pot, mpl=0.7, a0=a0, expand=expand, stencil=stencil, **kw)
    lin.set_fields(phi, pi)
    non = oracle.Lattice(n, L, pot, mpl=0.7, a0=a0, expand=expand, stencil=stencil, **kw)
    non.phi[...] = phi
    non.pi[...] = pi
    return lin, non, phi, pi


@pytest.mark.parametrize("order", [4, 6])
def test_background_equals_homogeneous_nonlinear_lattice(order):
    """With no perturbation the linear background is the nonlinear lattice
    with homogeneous fields (H3 split in halves only changes rounding)."""
    pot = oracle.Potential("chaotic2", (1.0, 3.0))
    lin, non, _, _ = _lin_and_nonlin(pot, n=4, amp=0.0, rho_rad0=0.02, rho_mat0=0.03)
    non.solve_constraint()
    assert lin.p_a == pytest.approx(non.p_a, rel=1e-14)
    lin.evolve(60, 0.05, order)
    non.evolve(60, 0.05, order)
    assert lin.a == pytest.approx(non.a, rel=1e-13)
    assert lin.p_a == pytest.approx(non.p_a, rel=1e-12)
    np.testing.assert_allclose(lin.phi0, non.phi[:, 0, 0, 0], rtol=1e-12)
    np.testing.assert_allclose(lin.pi0, non.pi[:, 0, 0, 0], rtol=1e-11, atol=1e-14)
    assert np.all(lin.dPhi == 0) and np.all(lin.dPi == 0)


@pytest.mark.parametrize("stencil", [oracle.STENCIL_7, oracle.STENCIL_27], ids=["7", "27"])
def test_free_static_field_equals_nonlinear(stencil):
    """A free field in a static background is linear: both integrators
    apply the same drift-kick-drift to every mode."""
    pot = oracle.Potential("free", (0.8, 1.9))
    lin, non, _, _ = _lin_and_nonlin(pot, expand=False, amp=0.3, a0=1.3, stencil=stencil)
    lin.evolve(80, 0.04, 4)
    non.evolve(80, 0.04, 4)
    phi, pi = lin.fields()
    np.testing.assert_allclose(phi, non.phi, rtol=0, atol=1e-12 * np.abs(non.phi).max())
    np.testing.assert_allclose(pi, non.pi, rtol=0, atol=1e-12 * np.abs(non.pi).max())


@pytest.mark.parametrize("pot", POTS[:3], ids=lambda p: p.kind)
def test_agrees_with_nonlinear_to_second_order(pot):
    """Expanding background: the linear result differs from the nonlinear
    lattice by O(amp^2), so the perturbation error per unit amplitude
    halves when the amplitude halves."""
    errs = []
    for amp in (2e-3, 1e-3):
        lin, non, phi, _ = _lin_and_nonlin(pot, amp=amp)
        non.solve_constraint()
        lin.evolve(40, 0.02, 4)
        non.evolve(40, 0.02, 4)
        lphi, lpi = lin.fields()
        dl = lphi - lphi.mean(axis=(1, 2, 3), keepdims=True)
        dn = non.phi - non.phi.mean(axis=(1, 2, 3), keepdims=True)
        errs.append(np.abs(dl - dn).max() / np.abs(dn).max())
    assert errs[0] < 0.05
    assert 1.7 < errs[0] / errs[1] < 2.3


def test_symplectic_form_of_perturbations_conserved():
    """The perturbation map is a linear Hamiltonian flow: sum_x (dphi_u
    dpi_v - dpi_u dphi_v) is the same before and after the evolution."""
    pot = oracle.Potential("chaotic2", (1.0, 3.0))
    lu, _, _, _ = _lin_and_nonlin(pot, amp=1e-2, seed=1)
    lv, _, _, _ = _lin_and_nonlin(pot, amp=1e-2, seed=2)
    # same background for both (the map depends on it), different perturbations
    lv.phi0, lv.pi0, lv.a, lv.p_a = lu.phi0.copy(), lu.pi0.copy(), lu.a, lu.p_a

    def form(a, b):
        pa, qa = a.fields()
        pb, qb = b.fields()
        da, ea = pa - pa.mean(axis=(1, 2, 3), keepdims=True), qa - qa.mean(axis=(1, 2, 3), keepdims=True)
        db, eb = pb - pb.mean(axis=(1, 2, 3), keepdims=True), qb - qb.mean(axis=(1, 2, 3), keepdims=True)
        return float(np.sum(da * eb - ea * db)), float(np.sum(np.abs(da * eb)))

    w0, s0 = form(lu, lv)
    lu.evolve(30, 0.03, 6)
    lv.evolve(30, 0.03, 6)
    w1, _ = form(lu, lv)
    assert abs(w1 - w0) <= 1e-11 * s0


def test_linear_reversibility():
    pot = oracle.Potential("chaotic2", (1.0, 3.0))
    lin, _, _, _ = _lin_and_nonlin(pot, amp=1e-2)
    phi0, pi0 = lin.fields()
    a0, pa0 = lin.a, lin.p_a
    lin.evolve(25, 0.03, 4)
    lin.evolve(25, -0.03, 4)
    phi1, pi1 = lin.fields()
    np.testing.assert_allclose(phi1, phi0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(pi1, pi0, rtol=0, atol=1e-12)
    assert lin.a == pytest.approx(a0, rel=1e-13) and lin.p_a == pytest.approx(pa0, rel=1e-12)
