"""FP64 oracle of the separate-universe (Delta N) read-out of a scan over
initial homogeneous values (Sec. 2.4 and Sec. 4).

Test infrastructure only (see the package docstring).

A run's background is recorded after every composed step.  The total
density on a run's time slice is the one the constraint H = 0 implies:
the first Friedmann equation (2.18) with the Hubble rate of the H1 flow,
H = a'/a^2 and a' = -p_a / (6 V_L m_pl^2), gives rho = 3 m_pl^2 H^2.  The
uniform-density e-fold count of a run is ln a on the slice where that
density first reaches a common reference value, found between two
recorded steps by linear interpolation of ln a in ln rho (exact when rho
is a power law of a over the interval).
"""
import math

import numpy as np


def constraint_density(a, p_a, n, mpl):
    """rho = 3 m_pl^2 H^2 with H = -p_a / (6 V_L m_pl^2 a^2), V_L = n^3."""
    VL = float(n) ** 3
    out = []
    for ak, pk in zip(np.atleast_1d(a), np.atleast_1d(p_a)):
        hub = -float(pk) / (6.0 * VL * mpl * mpl * float(ak) * float(ak))
        out.append(3.0 * mpl * mpl * hub * hub)
    return np.array(out)


def evolve_recording(lat, steps, h, order):
    """Advance an oracle Lattice step by step; returns arrays (eta, a, p_a,
    rho) taken after each composed step."""
    eta, a, p_a = [], [], []
    for _ in range(int(steps)):
        lat.step(h, order)
        eta.append(lat.eta)
        a.append(lat.a)
        p_a.append(lat.p_a)
    rho = constraint_density(a, p_a, lat.n, lat.mpl)
    return np.array(eta), np.array(a), np.array(p_a), rho


def efolds_at_density(a, rho, rho_ref):
    """ln a where rho first falls to rho_ref or below (records in step
    order).  NaN if it never does; ln a of the first record if that one is
    already at or below rho_ref."""
    prev = None
    for k in range(len(a)):
        if rho[k] <= rho_ref:
            if prev is None:
                return math.log(a[k])
            la0, la1 = math.log(a[prev]), math.log(a[k])
            lr0, lr1 = math.log(rho[prev]), math.log(rho[k])
            # ln a as a straight line in ln rho through the two records
            return la0 + (la1 - la0) * (math.log(rho_ref) - lr0) / (lr1 - lr0)
        prev = k
    return float("nan")
