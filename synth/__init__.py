"""Seeded synthetic inputs shared by the oracle-side tests and the library
tests.

This module holds no arithmetic of the lattice method: it only draws
seeded random arrays (numpy PCG64) and records the workload recipes
(lattice sizes, model parameters in program units, seeds) that the tests
and the benchmark use.  The unit conversions below are readings of the
paper's model descriptions, stated once here so that both sides read the
same numbers.
"""
import math

import numpy as np

# ---------------------------------------------------------------------------
# Random lattice states
# ---------------------------------------------------------------------------


def gaussian_state(n, nfields, seed, phi_base=None, phi_amp=1e-3,
                   pi_base=None, pi_amp=1e-3):
    """phi_i = phi_base_i + phi_amp * N(0,1), pi_i = pi_base_i + pi_amp *
    N(0,1) on an n^3 lattice, float64 arrays [field][z][y][x]."""
    rng = np.random.default_rng(seed)
    phi_base = np.zeros(nfields) if phi_base is None else np.asarray(phi_base, float)
    pi_base = np.zeros(nfields) if pi_base is None else np.asarray(pi_base, float)
    shape = (nfields, n, n, n)
    phi = phi_base[:, None, None, None] + phi_amp * rng.standard_normal(shape)
    pi = pi_base[:, None, None, None] + pi_amp * rng.standard_normal(shape)
    return np.ascontiguousarray(phi), np.ascontiguousarray(pi)


def plane_wave(n, kvec, amp=1.0, phase=0.0):
    """amp * cos(2 pi k.x / n + phase) on an n^3 lattice ([z][y][x], kvec in
    (kx, ky, kz) integer units)."""
    r = np.arange(n)
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    kx, ky, kz = kvec
    return amp * np.cos(2.0 * np.pi * (kx * x + ky * y + kz * z) / n + phase)


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

#: inflaton vev unit of the two-field preheating benchmark, in units of the
#: non-reduced Planck mass M_p
PHI0_IN_MP = 0.193
#: coupling ratio g^2/m^2 of that benchmark
G2_OVER_M2 = 2.5e5
#: inflaton mass in units of M_p (the benchmark's customary value)
M_IN_MP = 1.0e-6

#: m_pl (reduced Planck mass) in program units phi / phi0:
#: m_pl = M_p / sqrt(8 pi) = 1 / (0.193 sqrt(8 pi))
PREHEAT_MPL = 1.0 / (PHI0_IN_MP * math.sqrt(8.0 * math.pi))
#: G = g^2 phi0^2 / m^2 in program units (x in 1/m, fields in phi0)
PREHEAT_G = G2_OVER_M2 * PHI0_IN_MP ** 2
#: vacuum amplitude eps = m / phi0 in program units
PREHEAT_EPS = M_IN_MP / PHI0_IN_MP


def preheat(n=32, order=4, dt=0.005, steps=200, precision="f64",
            L=10.0, seed=20120123, phi0=1.0):
    """Two-field chaotic preheating V = m^2 phi^2/2 + g^2 phi^2 chi^2/2."""
    return dict(workload="preheat", n=n, L=L, nfields=2, potential="chaotic2",
                params=(1.0, PREHEAT_G), mpl=PREHEAT_MPL, a0=1.0,
                phi0=(phi0, 0.0), pi0=(0.0, 0.0), fluct="vacuum",
                amplitude=PREHEAT_EPS, seed=seed, dt=dt, order=order,
                steps=steps, precision=precision, expand=True)


def oscillon(n=128, steps=5000, precision="f32"):
    """Single-field oscillon V = phi^2/2 - lam phi^4/4 + g phi^6/6."""
    lam_phys = 2.8125e-6
    m_over_mpl = 5.0e-6
    return dict(workload="oscillon", n=n, L=64.0, nfields=1,
                potential="oscillon", params=(1.0, 1.0, 0.2),
                mpl=math.sqrt(lam_phys) / m_over_mpl, a0=1.0, phi0=(0.8,),
                pi0=(0.0,), fluct="white", amplitude=1e-4, seed=20120124,
                dt=0.005, order=4, steps=steps, precision=precision,
                expand=True)


def qball(n=512, steps=3000, precision="f32"):
    """Curvaton Q-ball, Phi = (phi1 + i phi2)/sqrt(2), |Phi| = 1e-2 rotating
    with angular-momentum ratio 0.5."""
    f1 = math.sqrt(2.0) * 1e-2
    return dict(workload="qball", n=n, L=100.0, nfields=2, potential="qball",
                params=(1.0, -0.1, 1.0), mpl=1.0, a0=1.0, phi0=(f1, 0.0),
                pi0=(0.0, 0.5 * f1), fluct="white", amplitude=1e-6,
                seed=20120127, dt=0.005, order=6, steps=steps,
                precision=precision, expand=True)


def delta_n_scan(nruns=96, steps=500, seed=20120125):
    """Batched ensemble: phi0 = 1 + k 1e-5, k in [-48, 48), sizes drawn
    uniformly from {32, 64, 96}, per-run seeds."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice([32, 64, 96], size=nruns)
    runs = []
    for j in range(nruns):
        k = j - nruns // 2
        r = preheat(n=int(sizes[j]), order=4, dt=0.005, steps=steps,
                    precision="f32", seed=20120200 + j, phi0=1.0 + k * 1e-5)
        runs.append(r)
    return runs


def poisson_arrivals(nruns, rate, seed=20120126):
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=nruns))
