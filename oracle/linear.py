"""FP64 oracle of the linearized integrator (Sec. 2.2 and the perturbed
splitting of Sec. 2.4).

Test infrastructure only (see the package docstring).

The fields are split into a homogeneous part and a perturbation whose
lattice sum vanishes, eq. (2.21)-(2.22).  Keeping the Hamiltonian to second
order in the perturbation, eq. (2.34), and letting the perturbation act on
nothing else (the paper drops H^(2) from the background equations), gives:

* the background (a, p_a, phi0_i, pi0_i) with pi0_i = a^2 phi0_i' per
  site, eq. (2.32), evolved by eq. (2.35)-(2.36);
* the perturbations evolved mode by mode in Fourier space, eq. (2.38), with
  k_eff^2 minus the lattice Laplacian's eigenvalue and the potential term
  a^4 H(phi0) dPhi, H the Hessian of V at the homogeneous point (the
  gradient of V^(2), eq. (2.26)).

The second-order map, eq. (2.50), splits the Hamiltonian into the five
parts of eq. (2.49): H1 (p_a^2 term), H2 (background kinetic + fluids),
H3 (background potential), H4 (perturbation kinetic), H5 (perturbation
gradient + potential), and applies

    H1(t/2) H2(t/2) H3(t/2) H4(t/2) H5(t) H4(t/2) H3(t/2) H2(t/2) H1(t/2)

in this time order (the product is palindromic), each flow exactly, with
every right-hand side frozen at the flow's start.  Compositions use the
same weights as the nonlinear integrator.  This oracle evolves every
Fourier mode of the lattice separately (no grouping of equal k_eff^2).
"""
import math

import numpy as np

from .lattice import STENCIL_7, keff2_modes, stencil_ok, composition_weights


class LinearLattice:
    """Background and Fourier-space perturbations of the linearized system.

    Perturbation modes are stored as dPhi[i] = FFT(delta phi_i) and
    dPi[i] = FFT(delta pi_i) (numpy's unnormalised forward transform over
    the [z][y][x] axes)."""

    def __init__(self, n, L, potential, mpl=1.0, a0=1.0, rho_rad0=0.0,
                 rho_mat0=0.0, expand=True, stencil=STENCIL_7):
        if not stencil_ok(stencil):
            raise ValueError("stencil coefficients outside the family of eq. (2.7)")
        self.n = int(n)
        self.L = float(L)
        self.dx = self.L / self.n
        self.VL = float(self.n) ** 3
        self.pot = potential
        self.nf = potential.nfields
        self.mpl = float(mpl)
        self.rho_rad0 = float(rho_rad0)
        self.rho_mat0 = float(rho_mat0)
        self.expand = bool(expand)
        self.c = tuple(float(v) for v in stencil)
        self.keff2 = keff2_modes(self.n, self.c)
        self.a = float(a0)
        self.p_a = 0.0
        self.eta = 0.0
        self.phi0 = np.zeros(self.nf)
        self.pi0 = np.zeros(self.nf)
        shape = (self.nf, self.n, self.n, self.n)
        self.dPhi = np.zeros(shape, dtype=complex)
        self.dPi = np.zeros(shape, dtype=complex)

    # --- state ------------------------------------------------------------
    def set_fields(self, phi, pi, p_a=None):
        """Split lattice fields into the homogeneous means and perturbations
        with zero lattice sum; p_a from the background constraint when
        None."""
        phi = np.asarray(phi, dtype=np.float64)
        pi = np.asarray(pi, dtype=np.float64)
        self.phi0 = np.array([float(np.mean(phi[i])) for i in range(self.nf)])
        self.pi0 = np.array([float(np.mean(pi[i])) for i in range(self.nf)])
        for i in range(self.nf):
            self.dPhi[i] = np.fft.fftn(phi[i] - self.phi0[i])
            self.dPi[i] = np.fft.fftn(pi[i] - self.pi0[i])
            self.dPhi[i][0, 0, 0] = 0.0
            self.dPi[i][0, 0, 0] = 0.0
        self.eta = 0.0
        if p_a is None:
            self.solve_constraint()
        else:
            self.p_a = float(p_a)

    def fields(self):
        """Lattice fields phi0 + delta phi, pi0 + delta pi (real arrays)."""
        phi = np.stack([self.phi0[i] + np.fft.ifftn(self.dPhi[i]).real for i in range(self.nf)])
        pi = np.stack([self.pi0[i] + np.fft.ifftn(self.dPi[i]).real for i in range(self.nf)])
        return phi, pi

    def background_energy(self, a=None):
        """H^(0) without its p_a term: V_L (sum pi0^2/(2 a^2) + a^4 V(phi0))
        + V_L rho_gamma0 + a V_L rho_m0: H1 + H2 + H3 of eq. (2.49)."""
        a = self.a if a is None else a
        V = float(self.pot.V(self.phi0.reshape(self.nf, 1))[0])
        return (self.VL * (float(np.sum(self.pi0 ** 2)) / (2.0 * a * a) + a ** 4 * V)
                + self.VL * self.rho_rad0 + a * self.VL * self.rho_mat0)

    def solve_constraint(self):
        """p_a from H^(0) = 0 on the expanding branch (p_a < 0)."""
        if not self.expand:
            self.p_a = 0.0
            return
        E0 = self.background_energy()
        if E0 < 0:
            raise ValueError("background constraint has no real p_a")
        self.p_a = -math.sqrt(12.0 * self.VL * self.mpl ** 2 * E0)

    # --- exact flows of eq. (2.49) ----------------------------------------
    def flow_H1(self, tau):
        if self.expand:
            self.a = self.a - self.p_a * tau / (6.0 * self.VL * self.mpl ** 2)

    def flow_H2(self, tau):
        """phi0 += pi0 tau / a^2; p_a += V_L (sum pi0^2 / a^3 - rho_m0) tau."""
        a = self.a
        if self.expand:
            self.p_a = self.p_a + self.VL * (float(np.sum(self.pi0 ** 2)) / a ** 3
                                             - self.rho_mat0) * tau
        self.phi0 = self.phi0 + self.pi0 * (tau / (a * a))

    def flow_H3(self, tau):
        """pi0 -= a^4 dV(phi0) tau; p_a -= 4 a^3 V_L V(phi0) tau."""
        a = self.a
        f = self.phi0.reshape(self.nf, 1)
        if self.expand:
            V = float(self.pot.V(f)[0])
            self.p_a = self.p_a - 4.0 * a ** 3 * self.VL * V * tau
        self.pi0 = self.pi0 - a ** 4 * self.pot.dV(f)[:, 0] * tau

    def flow_H4(self, tau):
        """dPhi += dPi tau / a^2 (every mode)."""
        self.dPhi = self.dPhi + self.dPi * (tau / (self.a * self.a))

    def flow_H5(self, tau):
        """dPi -= (a^2 k_eff^2 / dx^2 dPhi + a^4 H(phi0) dPhi) tau."""
        a = self.a
        H = self.pot.hessian(self.phi0)
        force = np.empty_like(self.dPhi)
        for i in range(self.nf):
            f = a * a * self.keff2 / self.dx ** 2 * self.dPhi[i]
            for j in range(self.nf):
                f = f + a ** 4 * H[i, j] * self.dPhi[j]
            force[i] = f
        self.dPi = self.dPi - force * tau

    def phi2(self, tau):
        h = 0.5 * tau
        self.flow_H1(h)
        self.flow_H2(h)
        self.flow_H3(h)
        self.flow_H4(h)
        self.flow_H5(tau)
        self.flow_H4(h)
        self.flow_H3(h)
        self.flow_H2(h)
        self.flow_H1(h)

    def step(self, h, order):
        for w in composition_weights(order):
            self.phi2(w * h)
        self.eta = self.eta + h

    def evolve(self, steps, h, order):
        for _ in range(int(steps)):
            self.step(h, order)
