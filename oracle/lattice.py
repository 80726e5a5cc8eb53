"""FP64 oracle of the nonlinear symplectic lattice step (Sec. 2.1 and 2.3).

Test infrastructure only (see the package docstring).

Notation follows the paper: n^3 periodic sites with spacing dx = L/n,
V_L = n^3 (the lattice volume in units of dx^3), scale factor a with
canonical momentum p_a, fields phi_i with momenta pi_i = a^2 phi_i',
conformal time eta, reduced Planck mass m_pl.  Arrays are indexed
[field][z][y][x].

Readings of points the paper leaves open:

* the Laplacian coefficients c_d of eq. (2.7) are the 7-point member
  (c0 = -6, c1 = 1, c2 = c3 = 0); G of eq. (2.8) uses the same coefficients;
* the potential enters the Hamiltonian once per site (outside the field sum);
* the triple-jump z0 of eq. (2.44) is -2^(1/3) / (2 - 2^(1/3)) at 4th order;
* the initial p_a solves the constraint H = 0 on the expanding branch.
"""
import math

import numpy as np

from . import rng as _rng

# ---------------------------------------------------------------------------
# Composition weights, Sec. 2.3
# ---------------------------------------------------------------------------

#: Table 1, 6th order (s = 7): w1..w3; w4 = 1 - 2 (w1 + w2 + w3).
TABLE1_ORDER6 = (0.78451361047755726382, 0.23557321335935813368,
                 -1.17767998417887100695)
#: Table 1, 8th order (s = 15): w1..w7; w8 = 1 - 2 sum(w1..w7).
TABLE1_ORDER8 = (0.74167036435061295345, -0.40910082580003159400,
                 0.19075471029623837995, -0.57386247111608226666,
                 0.29906418130365592384, 0.33462491824529818378,
                 0.31529309239676659663)


def composition_weights(order):
    """Stage weights w_1..w_s of the symmetric composition of second-order
    maps (Sec. 2.3, eq. (2.45) and Table 1; 4th order by the triple-jump
    recursion eq. (2.43)-(2.44) applied once to the second-order map)."""
    if order == 2:
        return [1.0]
    if order == 4:
        c = 2.0 ** (1.0 / 3.0)
        z1 = 1.0 / (2.0 - c)
        z0 = -c / (2.0 - c)
        return [z1, z0, z1]
    if order in (6, 8):
        half = list(TABLE1_ORDER6 if order == 6 else TABLE1_ORDER8)
        mid = 1.0 - 2.0 * sum(half)
        return half + [mid] + half[::-1]
    raise ValueError("order must be 2, 4, 6 or 8")


# ---------------------------------------------------------------------------
# Stencils, Sec. 2.1 eq. (2.7)-(2.8)
# ---------------------------------------------------------------------------

#: 7-point member of the family of eq. (2.7): (c0, c1, c2, c3) = weights of
#: the centre, the 6 face, the 12 edge and the 8 corner neighbours.
STENCIL_7 = (-6.0, 1.0, 0.0, 0.0)


def _neighbour_classes():
    """Offsets of the 26 neighbours grouped by class: 1 = face (one nonzero
    component), 2 = edge (two), 3 = corner (three)."""
    out = {1: [], 2: [], 3: []}
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                k = abs(dz) + abs(dy) + abs(dx)
                if k:
                    out[k].append((dz, dy, dx))
    return out


_NEIGHBOURS = _neighbour_classes()


def _shifted(f, off):
    """f(x + off) on the periodic lattice (arrays indexed [..., z, y, x])."""
    dz, dy, dx = off
    return np.roll(f, (-dz, -dy, -dx), axis=(-3, -2, -1))


def lap(f, c=STENCIL_7):
    """D[f](x) of eq. (2.7): c0 f(x) + sum over the neighbour classes of
    c_class times the sum of f over that class, periodic."""
    out = c[0] * f
    for cls in (1, 2, 3):
        if c[cls] != 0.0:
            acc = np.zeros_like(f)
            for off in _NEIGHBOURS[cls]:
                acc = acc + _shifted(f, off)
            out = out + c[cls] * acc
    return out


def grad_energy(f, c=STENCIL_7):
    """G[f](x) of eq. (2.8) with the coefficients of D: one half of the sum
    over neighbours of c_class (f(nbr) - f(x))^2."""
    out = np.zeros_like(f)
    for cls in (1, 2, 3):
        if c[cls] != 0.0:
            acc = np.zeros_like(f)
            for off in _NEIGHBOURS[cls]:
                d = _shifted(f, off) - f
                acc = acc + d * d
            out = out + c[cls] * acc
    return 0.5 * out


def stencil_symbol(c, kz, ky, kx):
    """Eigenvalue of D on the plane wave exp(i k.x) with k in lattice units
    (radians per site): c0 + 2 c1 sum cos + 4 c2 sum_{d<e} cos cos +
    8 c3 prod cos.  For the 7-point member it equals -sum 4 sin^2(k_d/2)."""
    cz, cy, cx = np.cos(kz), np.cos(ky), np.cos(kx)
    return (c[0] + 2.0 * c[1] * (cz + cy + cx)
            + 4.0 * c[2] * (cz * cy + cz * cx + cy * cx)
            + 8.0 * c[3] * cz * cy * cx)


def stencil_ok(c, tol=1e-12):
    """The family's two conditions: D annihilates constants (c0 + 6 c1 +
    12 c2 + 8 c3 = 0) and tends to the Laplacian (c1 + 4 c2 + 4 c3 = 1)."""
    return (abs(c[0] + 6 * c[1] + 12 * c[2] + 8 * c[3]) <= tol
            and abs(c[1] + 4 * c[2] + 4 * c[3] - 1.0) <= tol)


def isotropic_stencil(c3):
    """Member of the family whose leading (k^4) error term is isotropic:
    Taylor-expanding the symbol gives, at fourth order,
    S4 (c1/12 + c2/3 + c3/3) + P (c2 + 2 c3) with S4 = sum k_d^4 and
    P = sum_{d<e} k_d^2 k_e^2, which is a multiple of |k|^4 = S4 + 2P when
    c1 = 2 c2 + 8 c3.  With the two family conditions this leaves c3 free:
    c1 = 1/3 + 4 c3, c2 = 1/6 - 2 c3, c0 = -4 - 8 c3 (and the symbol is
    -|k|^2 + |k|^4/12 + O(k^6) for every member)."""
    c3 = float(c3)
    return (-4.0 - 8.0 * c3, 1.0 / 3.0 + 4.0 * c3, 1.0 / 6.0 - 2.0 * c3, c3)


#: 19-point (no corners) and 27-point isotropic members, c3 = 0 and 1/30.
STENCIL_19 = isotropic_stencil(0.0)
STENCIL_27 = isotropic_stencil(1.0 / 30.0)


def stencil_max_keff2(c):
    """Largest -symbol over the Brillouin zone.  The symbol is multilinear
    in (cos kz, cos ky, cos kx) in [-1, 1]^3, so its extremes sit at the 8
    vertices k_d in {0, pi}."""
    best = -np.inf
    for kz in (0.0, np.pi):
        for ky in (0.0, np.pi):
            for kx in (0.0, np.pi):
                best = max(best, -float(stencil_symbol(c, kz, ky, kx)))
    return best


# ---------------------------------------------------------------------------
# Potentials (Sec. 3 models, in program units)
# ---------------------------------------------------------------------------

class Potential:
    """V(phi_1..phi_N), dV/dphi_i and the Hessian diagonal.

    kinds and parameter vectors:
      'free'      (m_1^2, ..., m_N^2):  V = sum_i m_i^2 phi_i^2 / 2
      'chaotic2'  (m^2, G):             V = m^2 phi^2/2 + G phi^2 chi^2 / 2
                                        (Sec. 3.1 potential with G = g^2)
      'oscillon'  (m^2, lam, g):        V = m^2 phi^2/2 - lam phi^4/4
                                        + g phi^6/6   (Sec. 3.2 form)
      'qball'     (m^2, K, M^2):        u = (phi_1^2 + phi_2^2)/2 = |Phi|^2,
                                        V = m^2 u (1 + K ln(u/M^2))
                                        (Sec. 3.3 without the |Phi|^6 and
                                        H^2 terms); V = dV = 0 at u = 0.
    All functions accept complex arrays so that complex-step derivatives
    can be taken through them.
    """

    NFIELDS = {"chaotic2": 2, "oscillon": 1, "qball": 2}
    NPARAMS = {"chaotic2": 2, "oscillon": 3, "qball": 3}

    def __init__(self, kind, params, nfields=None):
        params = tuple(float(p) for p in params)
        if kind == "free":
            nfields = len(params) if nfields is None else nfields
            if len(params) != nfields:
                raise ValueError("free potential needs one m^2 per field")
        elif kind in self.NFIELDS:
            if nfields is not None and nfields != self.NFIELDS[kind]:
                raise ValueError("wrong field count for %s" % kind)
            nfields = self.NFIELDS[kind]
            if len(params) != self.NPARAMS[kind]:
                raise ValueError("wrong parameter count for %s" % kind)
        else:
            raise ValueError("unknown potential " + kind)
        self.kind, self.params, self.nfields = kind, params, nfields

    @staticmethod
    def _u_log(u, M2):
        """(mask, ln(u/M^2)) with the log evaluated only where u > 0."""
        pos = np.real(u) > 0
        safe = np.where(pos, u, M2)
        return pos, np.log(safe / M2)

    def V(self, phi):
        k, p = self.kind, self.params
        if k == "free":
            return sum(0.5 * p[i] * phi[i] ** 2 for i in range(self.nfields))
        if k == "chaotic2":
            m2, G = p
            f, c = phi[0], phi[1]
            return 0.5 * m2 * f ** 2 + 0.5 * G * f ** 2 * c ** 2
        if k == "oscillon":
            m2, lam, g = p
            f = phi[0]
            return 0.5 * m2 * f ** 2 - 0.25 * lam * f ** 4 + g / 6.0 * f ** 6
        m2, K, M2 = p
        u = 0.5 * (phi[0] ** 2 + phi[1] ** 2)
        pos, lg = self._u_log(u, M2)
        return np.where(pos, m2 * u * (1.0 + K * lg), 0.0 * u)

    def dV(self, phi):
        """Array [field][...] of dV/dphi_i."""
        k, p = self.kind, self.params
        if k == "free":
            return np.stack([p[i] * phi[i] for i in range(self.nfields)])
        if k == "chaotic2":
            m2, G = p
            f, c = phi[0], phi[1]
            return np.stack([f * (m2 + G * c ** 2), G * f ** 2 * c])
        if k == "oscillon":
            m2, lam, g = p
            f = phi[0]
            return np.stack([m2 * f - lam * f ** 3 + g * f ** 5])
        m2, K, M2 = p
        u = 0.5 * (phi[0] ** 2 + phi[1] ** 2)
        pos, lg = self._u_log(u, M2)
        fac = np.where(pos, m2 * (1.0 + K + K * lg), 0.0 * u)
        return np.stack([fac * phi[0], fac * phi[1]])

    def d2V_diag(self, phi0):
        """d^2V/dphi_i^2 at a homogeneous point phi0 (sequence of floats)."""
        k, p = self.kind, self.params
        phi0 = [float(v) for v in phi0]
        if k == "free":
            return [p[i] for i in range(self.nfields)]
        if k == "chaotic2":
            m2, G = p
            f, c = phi0
            return [m2 + G * c * c, G * f * f]
        if k == "oscillon":
            m2, lam, g = p
            f = phi0[0]
            return [m2 - 3.0 * lam * f * f + 5.0 * g * f ** 4]
        m2, K, M2 = p
        u = 0.5 * (phi0[0] ** 2 + phi0[1] ** 2)
        if u <= 0.0:
            raise ValueError("Q-ball mass undefined at |Phi| = 0")
        base = m2 * (1.0 + K + K * math.log(u / M2))
        return [base + m2 * K * phi0[0] ** 2 / u, base + m2 * K * phi0[1] ** 2 / u]

    def d2V_sites(self, phi):
        """Array [field][...] of d^2V/dphi_i^2 at every site of phi."""
        k, p = self.kind, self.params
        if k == "free":
            return np.stack([p[i] + 0.0 * phi[i] for i in range(self.nfields)])
        if k == "chaotic2":
            m2, G = p
            f, c = phi[0], phi[1]
            return np.stack([m2 + G * c * c, G * f * f])
        if k == "oscillon":
            m2, lam, g = p
            f = phi[0]
            return np.stack([m2 - 3.0 * lam * f * f + 5.0 * g * f ** 4])
        m2, K, M2 = p
        u = 0.5 * (phi[0] ** 2 + phi[1] ** 2)
        pos, lg = self._u_log(u, M2)
        base = m2 * (1.0 + K + K * lg)
        safe = np.where(pos, u, 1.0)
        return np.stack([np.where(pos, base + m2 * K * phi[i] ** 2 / safe, 0.0 * u)
                         for i in range(2)])

    def hessian(self, phi0):
        """Matrix d^2V/dphi_i dphi_j at a homogeneous point phi0: the
        quadratic form of V^(2), eq. (2.26), is delta^T H delta / 2."""
        k, p = self.kind, self.params
        phi0 = [float(v) for v in phi0]
        nf = self.nfields
        H = np.zeros((nf, nf))
        if k == "free":
            for i in range(nf):
                H[i, i] = p[i]
        elif k == "chaotic2":
            m2, G = p
            f, c = phi0
            H[0, 0] = m2 + G * c * c
            H[0, 1] = H[1, 0] = 2.0 * G * f * c
            H[1, 1] = G * f * f
        elif k == "oscillon":
            m2, lam, g = p
            f = phi0[0]
            H[0, 0] = m2 - 3.0 * lam * f * f + 5.0 * g * f ** 4
        else:
            m2, K, M2 = p
            u = 0.5 * (phi0[0] ** 2 + phi0[1] ** 2)
            if u <= 0.0:
                raise ValueError("Q-ball Hessian undefined at |Phi| = 0")
            base = m2 * (1.0 + K + K * math.log(u / M2))
            for i in range(2):
                for j in range(2):
                    H[i, j] = (base if i == j else 0.0) + m2 * K * phi0[i] * phi0[j] / u
        return H


# ---------------------------------------------------------------------------
# The lattice and its exact flows
# ---------------------------------------------------------------------------

class Lattice:
    """State (a, p_a, phi_i, pi_i, eta) of the discretised system, Sec. 2.1.

    ``expand=False`` freezes the background: a stays at a0, the H1 flow is
    the identity and p_a is not updated (static-space limit m_pl -> inf).
    """

    def __init__(self, n, L, potential, mpl=1.0, a0=1.0, rho_rad0=0.0,
                 rho_mat0=0.0, expand=True, dtype=np.float64, stencil=STENCIL_7):
        if not stencil_ok(stencil):
            raise ValueError("stencil coefficients outside the family of eq. (2.7)")
        self.c = tuple(float(v) for v in stencil)
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
        shape = (self.nf, self.n, self.n, self.n)
        self.phi = np.zeros(shape, dtype=dtype)
        self.pi = np.zeros(shape, dtype=dtype)
        self.a = float(a0)
        self.p_a = 0.0
        self.eta = 0.0

    def copy(self):
        c = Lattice.__new__(Lattice)
        c.__dict__.update(self.__dict__)
        c.phi = self.phi.copy()
        c.pi = self.pi.copy()
        return c

    # --- Hamiltonian, eq. (2.20) and its split eq. (2.46) -----------------
    def ham_parts(self, a=None, p_a=None, phi=None, pi=None):
        """(H1, H2, H3) of eq. (2.46) at the given (or current) state."""
        a = self.a if a is None else a
        p_a = self.p_a if p_a is None else p_a
        phi = self.phi if phi is None else phi
        pi = self.pi if pi is None else pi
        VL, m2pl, dx2 = self.VL, self.mpl ** 2, self.dx ** 2
        H1 = -p_a ** 2 / (12.0 * VL * m2pl)
        H2 = np.sum(pi * pi) / (2.0 * a * a) \
            + VL * self.rho_rad0 + a * VL * self.rho_mat0
        grad = sum(np.sum(phi[i] * lap(phi[i], self.c)) for i in range(self.nf))
        H3 = -a * a * grad / (2.0 * dx2) + a ** 4 * np.sum(self.pot.V(phi))
        return H1, H2, H3

    def hamiltonian(self, **kw):
        H1, H2, H3 = self.ham_parts(**kw)
        return (H1 if self.expand else 0.0) + H2 + H3

    # --- exact flows, eq. (2.47) -------------------------------------------
    def flow_H1(self, tau):
        """a -> a - p_a tau / (6 V_L m_pl^2)."""
        if self.expand:
            self.a = self.a - self.p_a * tau / (6.0 * self.VL * self.mpl ** 2)

    def flow_H2(self, tau):
        """p_a -> p_a + (sum pi^2 / a^3 - V_L rho_m0) tau,
        phi -> phi + pi tau / a^2 (both from the start state)."""
        a = self.a
        if self.expand:
            S2 = np.sum(self.pi * self.pi)
            self.p_a = self.p_a + (S2 / a ** 3 - self.VL * self.rho_mat0) * tau
        self.phi = self.phi + self.pi * (tau / (a * a))

    def flow_H3(self, tau):
        """p_a -> p_a + sum_x [sum_i a phi_i D phi_i / dx^2 - 4 a^3 V] tau,
        pi_i -> pi_i + (a^2 D phi_i / dx^2 - a^4 dV/dphi_i) tau."""
        a, dx2 = self.a, self.dx ** 2
        D = np.stack([lap(self.phi[i], self.c) for i in range(self.nf)])
        dV = self.pot.dV(self.phi)
        if self.expand:
            S3 = a * np.sum(self.phi * D) / dx2 \
                - 4.0 * a ** 3 * np.sum(self.pot.V(self.phi))
            self.p_a = self.p_a + S3 * tau
        self.pi = self.pi + (a * a * D / dx2 - a ** 4 * dV) * tau

    # --- second-order map and compositions -----------------------------------
    def phi2(self, tau):
        """Phi^(2)(tau) = H1(tau/2) H2(tau/2) H3(tau) H2(tau/2) H1(tau/2),
        eq. (2.48), applied in this time order (the map is palindromic)."""
        self.flow_H1(0.5 * tau)
        self.flow_H2(0.5 * tau)
        self.flow_H3(tau)
        self.flow_H2(0.5 * tau)
        self.flow_H1(0.5 * tau)

    def step(self, h, order):
        """One composed step: Phi2(w_1 h) ... Phi2(w_s h), then eta += h."""
        for w in composition_weights(order):
            self.phi2(w * h)
        self.eta = self.eta + h

    def evolve(self, steps, h, order):
        for _ in range(int(steps)):
            self.step(h, order)

    # --- constraint and observables -------------------------------------------
    def solve_constraint(self):
        """p_a from H = 0 on the expanding branch (a' > 0, so p_a < 0)."""
        if not self.expand:
            self.p_a = 0.0
            return
        _, H2, H3 = self.ham_parts(p_a=0.0)
        E0 = H2 + H3
        if E0 < 0:
            raise ValueError("constraint H = 0 has no real p_a (E0 < 0)")
        self.p_a = -math.sqrt(12.0 * self.VL * self.mpl ** 2 * E0)

    def energies(self):
        """Volume averages of eq. (2.16), the Hubble rate, the residual
        curvature eq. (3.1) and the total Hamiltonian eq. (2.20)."""
        a, dx2 = self.a, self.dx ** 2
        kin = [float(np.mean(self.pi[i] ** 2)) / (2.0 * a ** 6)
               for i in range(self.nf)]
        grad = [float(np.mean(grad_energy(self.phi[i], self.c))) / (2.0 * a * a * dx2)
                for i in range(self.nf)]
        pot = float(np.mean(self.pot.V(self.phi)))
        rho = sum(kin) + sum(grad) + pot
        pres = sum(kin) - sum(grad) / 3.0 - pot
        rho_tot = rho + self.rho_rad0 / a ** 4 + self.rho_mat0 / a ** 3
        if self.expand:
            hub = -self.p_a / (6.0 * self.VL * self.mpl ** 2 * a * a)
            resid = abs(rho_tot / (3.0 * self.mpl ** 2 * hub * hub) - 1.0)
        else:
            hub, resid = 0.0, float("nan")
        mean = [float(np.mean(self.phi[i])) for i in range(self.nf)]
        var = [float(np.var(self.phi[i])) for i in range(self.nf)]
        return dict(eta=self.eta, a=a, p_a=self.p_a, hubble=hub, rho=rho,
                    pressure=pres, w_eos=pres / rho if rho != 0 else float("nan"),
                    friedmann_residual=resid, h_total=float(self.hamiltonian()),
                    kin=kin, grad=grad, pot=pot, mean=mean, var=var)

    # --- initial state, Sec. 2.4 (Gaussian modes in place of the paper's
    #     convolution method) ------------------------------------------------
    def init_homogeneous(self, phi0, pi0):
        for i in range(self.nf):
            self.phi[i][...] = phi0[i]
            self.pi[i][...] = pi0[i]

    def init_fluctuations(self, phi0, pi0, kind, amplitude, seed):
        """Homogeneous phi0, pi0 plus Gaussian fluctuations, then p_a from
        the constraint.  kind: 'none', 'vacuum' or 'white'."""
        self.init_homogeneous(phi0, pi0)
        if kind == "vacuum":
            m2eff = self.pot.d2V_diag(phi0)
            for i in range(self.nf):
                self.phi[i] += vacuum_field(self.n, self.L, m2eff[i],
                                            amplitude, seed, i, self.nf, self.c)
        elif kind == "white":
            for i in range(self.nf):
                self.phi[i] += white_field(self.n, amplitude, seed, i)
        elif kind != "none":
            raise ValueError(kind)
        self.eta = 0.0
        self.solve_constraint()


def _mode_indices(n):
    """Integer mode components n_z, n_y, n_x in [0, n) and their linear
    index (z slowest)."""
    r = np.arange(n, dtype=np.int64)
    nz, ny, nx = np.meshgrid(r, r, r, indexing="ij")
    return nz, ny, nx, (nz * n + ny) * n + nx


def keff2_modes(n, c=STENCIL_7):
    """k_eff^2 of every mode (n_z, n_y, n_x): minus the stencil's symbol at
    k_d = 2 pi n_d / N; for the 7-point member written as
    sum_d 4 sin^2(pi n_d / N)."""
    nz, ny, nx, _ = _mode_indices(n)
    if tuple(c) == STENCIL_7:
        return sum(4.0 * np.sin(np.pi * m / n) ** 2 for m in (nz, ny, nx))
    t = 2.0 * np.pi / n
    return -stencil_symbol(c, t * nz, t * ny, t * nx)


def vacuum_field(n, L, m2eff, eps, seed, field, nfields, c=STENCIL_7):
    """delta phi(x_j) = sum_n f_n exp(2 pi i n.j / N) with
    E|f_n|^2 = eps^2 / (2 omega_n L^3), omega_n^2 = k_eff^2/dx^2 + m_eff^2,
    k_eff^2 of the stencil (keff2_modes); f_0 = 0; f_{-n} = conj(f_n);
    self-conjugate modes real.  Each +-n pair draws its normals at the
    canonical (smaller linear index) member."""
    dx = L / n
    nz, ny, nx, idx = _mode_indices(n)
    neg = ((-nz) % n * n + (-ny) % n) * n + (-nx) % n
    canon = np.minimum(idx, neg)
    keff2 = keff2_modes(n, c)
    w2 = keff2 / dx ** 2 + m2eff
    w = np.sqrt(np.where(w2 > 0, w2, 1.0))
    P = np.where(w2 > 0, eps ** 2 / (2.0 * w * L ** 3), 0.0)
    P.flat[0] = 0.0
    nsites = n ** 3
    g1 = _rng.normals(seed, field, nsites, canon, 0)
    g2 = _rng.normals(seed, field, nsites, canon, 1)
    selfc = idx == neg
    fc = np.sqrt(P / 2.0) * (g1 + 1j * g2)
    f = np.where(idx == canon, fc, np.conj(fc))
    f = np.where(selfc, np.sqrt(P) * g1 + 0j, f)
    dphi = np.fft.ifftn(f) * nsites
    return dphi.real


def white_field(n, amp, seed, field):
    """delta phi(x) = A (g(x) - mean_x g), g i.i.d. normal keyed by site."""
    idx = np.arange(n ** 3, dtype=np.int64)
    g = _rng.normals(seed, field, n ** 3, idx, 0).reshape(n, n, n)
    return amp * (g - np.mean(g))


# ---------------------------------------------------------------------------
# Spectrum (Sec. 2.4 post-processing; |n| rounded half away from zero)
# ---------------------------------------------------------------------------

def spectrum_bins(n):
    """(bin index, |n| ) for every mode; bin = |n| rounded half away from
    zero, decided in integers: smallest b with |n|^2 <= b^2 + b."""
    f = np.rint(np.fft.fftfreq(n) * n).astype(np.int64)
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    m = kz * kz + ky * ky + kx * kx
    b = np.floor(np.sqrt(m.astype(np.float64))).astype(np.int64)
    b = b + (m > b * b + b)
    return b, np.sqrt(m.astype(np.float64)), m


def spectrum(field, L, nbins):
    """F = FFT(phi)/N^3; P_b = mean |F_n|^2 over modes with bin b,
    k_b = 2 pi mean|n| / L, counts.  The n = 0 mode is excluded; modes with
    bin >= nbins are dropped; empty bins report zeros."""
    n = field.shape[-1]
    F = np.fft.fftn(field) / n ** 3
    pw = (F.real ** 2 + F.imag ** 2).ravel()
    b, kn, m = spectrum_bins(n)
    b, kn, m = b.ravel(), kn.ravel(), m.ravel()
    keep = (m > 0) & (b < nbins)
    cnt = np.bincount(b[keep], minlength=nbins)[:nbins]
    ps = np.bincount(b[keep], weights=pw[keep], minlength=nbins)[:nbins]
    ks = np.bincount(b[keep], weights=kn[keep], minlength=nbins)[:nbins]
    with np.errstate(invalid="ignore", divide="ignore"):
        P = np.where(cnt > 0, ps / np.maximum(cnt, 1), 0.0)
        k = np.where(cnt > 0, 2.0 * np.pi * ks / np.maximum(cnt, 1) / L, 0.0)
    return k, P, cnt.astype(np.int64)


def mode_spectra(lat, field, nbins):
    """Field, energy-density and number-density spectra of one field
    (the post-processing spectra of Sec. 2.4; the paper refers to the
    LATTICEEASY definitions without printing them; the forms below are
    written in the paper's variables).  With F_n = FFT(phi_i)/N^3 and
    P_n = FFT(pi_i)/N^3,
    k_eff^2(n) of the lattice's stencil and m_eff^2 the lattice mean of
    d^2V/dphi_i^2:

      rho_n   = |P_n|^2/(2 a^6) + (k_eff^2/(2 a^2 dx^2) + m_eff^2/2) |F_n|^2
      omega_n = sqrt(k_eff^2/(a^2 dx^2) + m_eff^2),  n_n = rho_n / omega_n

    (n_n = 0 where omega_n^2 <= 0).  rho_n is mode n's share of the
    quadratic energy density; summed over n != 0 it is the kinetic, gradient
    and m_eff^2 energy of the fluctuations.  Binned as spectrum(): returns
    k_b, and per bin the means of |F_n|^2, rho_n, n_n, the counts and
    m_eff^2."""
    n = lat.n
    a, dx2 = lat.a, lat.dx ** 2
    F = np.fft.fftn(lat.phi[field]) / n ** 3
    P = np.fft.fftn(lat.pi[field]) / n ** 3
    m2 = float(np.mean(lat.pot.d2V_sites(lat.phi)[field]))
    k2 = keff2_modes(n, lat.c)
    f2 = F.real ** 2 + F.imag ** 2
    p2 = P.real ** 2 + P.imag ** 2
    rho = p2 / (2.0 * a ** 6) + (k2 / (2.0 * a * a * dx2) + 0.5 * m2) * f2
    w2 = k2 / (a * a * dx2) + m2
    num = np.where(w2 > 0, rho / np.sqrt(np.where(w2 > 0, w2, 1.0)), 0.0)
    b, kn, m = spectrum_bins(n)
    b, kn, m = b.ravel(), kn.ravel(), m.ravel()
    keep = (m > 0) & (b < nbins)
    cnt = np.bincount(b[keep], minlength=nbins)[:nbins]

    def binmean(v):
        sm = np.bincount(b[keep], weights=v.ravel()[keep], minlength=nbins)[:nbins]
        return np.where(cnt > 0, sm / np.maximum(cnt, 1), 0.0)

    k = np.where(cnt > 0, 2.0 * np.pi * binmean(kn) / lat.L, 0.0)
    return k, binmean(f2), binmean(rho), binmean(num), cnt.astype(np.int64), m2


# ---------------------------------------------------------------------------
# Linear stability of a composition (free field, static background)
# ---------------------------------------------------------------------------

def linear_stage_matrix(tau, omega2):
    """One second-order map on a single mode (phi, pi) of a free field with
    a = 1: drift tau/2, kick tau * omega^2, drift tau/2 (eq. (2.48) with H1
    trivial)."""
    Dr = np.array([[1.0, tau / 2.0], [0.0, 1.0]])
    K = np.array([[1.0, 0.0], [-tau * omega2, 1.0]])
    return Dr @ K @ Dr


def stability_limit(order, step=1e-5, xmax=6.0):
    """Largest omega*h such that the composed one-mode map has
    |trace| <= 2 at every scanned value up to it (uniform scan)."""
    ws = composition_weights(order)
    x = np.arange(1, int(round(xmax / step)) + 1) * step
    m00, m01, m10, m11 = (np.ones_like(x), np.zeros_like(x),
                          np.zeros_like(x), np.ones_like(x))
    for w in ws:
        t = w * x
        # stage matrix Dr(t/2) K(t) Dr(t/2) with omega^2 = 1, written out
        s00 = 1.0 - t * t / 2.0
        s01 = t - t ** 3 / 4.0
        s10 = -t
        s11 = 1.0 - t * t / 2.0
        m00, m01, m10, m11 = (s00 * m00 + s01 * m10, s00 * m01 + s01 * m11,
                              s10 * m00 + s11 * m10, s10 * m01 + s11 * m11)
    bad = np.nonzero(np.abs(m00 + m11) > 2.0)[0]
    return float(x[bad[0] - 1]) if bad.size else float(xmax)
