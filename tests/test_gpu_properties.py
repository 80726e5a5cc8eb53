"""Properties of the method checked on the GPU path directly, without the
oracle: the convergence order of each composition on a lattice plane wave
whose exact solution is known in closed form (a free field in a static
background oscillates at omega^2 = m^2 + sum_d 4 sin^2(pi k_d / n) / dx^2),
and the bounded, non-drifting energy error of a symplectic map on a
nonlinear lattice without expansion, shrinking with the step as the order
says."""
import math

import numpy as np
import pytest

import paper_1201_5029_amd as sl
from gpu_util import say

pytestmark = pytest.mark.gpu


def _plane_wave_error(order, dt, n=8, L=8.0, k=(1, 2, 0), m2=1.0, amp=1e-2, T=2.0):
    dx = L / n
    z, y, x = np.indices((n, n, n))
    phase = 2 * math.pi * (k[0] * x + k[1] * y + k[2] * z) / n
    omega = math.sqrt(m2 + sum(4 * math.sin(math.pi * kd / n) ** 2 for kd in k) / dx ** 2)
    g = sl.Lattice(n, 1, L, precision="f64", expand=False)
    g.set_potential("free", (m2,))
    g.set_fields((amp * np.cos(phase))[None], np.zeros((1, n, n, n)), 1.0, 0.0)
    g.evolve(int(round(T / dt)), dt, order)
    phi, _ = g.get_fields()
    g.close()
    exact = amp * np.cos(phase) * math.cos(omega * T)
    return float(np.abs(phi[0] - exact).max() / amp)


@pytest.mark.parametrize("order,dts", [(2, (0.05, 0.025, 0.0125)), (4, (0.1, 0.05, 0.025)),
                                       (6, (0.2, 0.1, 0.05)), (8, (0.2, 0.1))])
def test_convergence_order_on_a_plane_wave(order, dts):
    err = [_plane_wave_error(order, dt) for dt in dts]
    slopes = [math.log2(err[i] / err[i + 1]) for i in range(len(err) - 1)]
    say("order", order, "errors", err, "slopes", slopes)
    assert all(abs(s - order) < 0.15 for s in slopes)


def _energy_drift(dt, T=20.0, n=12, L=12.0, seed=5):
    rng = np.random.default_rng(seed)
    phi = (0.8 + 0.05 * rng.standard_normal((n, n, n)))[None]
    g = sl.Lattice(n, 1, L, precision="f64", expand=False, mpl=335.41)
    g.set_potential("oscillon", (1.0, 1.0, 0.2))
    g.set_fields(phi, np.zeros_like(phi), 1.0, 0.0)
    h0 = g.energies()["h_total"]
    dev = []
    for _ in range(int(round(T / dt)) // 10):
        g.evolve(10, dt, 4)
        dev.append(abs(g.energies()["h_total"] - h0) / abs(h0))
    g.close()
    half = len(dev) // 2
    return max(dev[:half]), max(dev[half:])


def test_energy_error_bounded_without_expansion():
    coarse = _energy_drift(0.1)
    fine = _energy_drift(0.05)
    say("energy error (first half, second half): dt 0.1", coarse, "dt 0.05", fine)
    # bounded: no growth from the first half of the run to the second
    assert coarse[1] < 2 * coarse[0] and fine[1] < 2 * fine[0]
    # and shrinking with the step like a 4th-order method (16x per halving)
    assert max(coarse) / max(fine) > 8
    assert max(coarse) < 1e-4
