"""Pins of the oracle's initial-state generator (vacuum and white Gaussian
fluctuations, constraint solve) and of its field spectrum."""
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import rng
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for k, hexval in rows:
        k = int(k)
        assert rng.splitmix64_scalar(k * rng.GAMMA) == int(hexval, 16)
        # vectorised form, counter convention key = seed + (c + 1) GAMMA
        v = rng.splitmix64(rng.keys_for(0, np.array([k - 1], dtype=np.uint64)))[0]
        assert int(v) == int(hexval, 16)


def test_uniforms_and_normals():
    u = rng.uniforms(12345, np.arange(200000, dtype=np.uint64))
    assert u.min() > 0 and u.max() <= 1
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    g = rng.normals(777, 0, 10 ** 6, np.arange(10 ** 6), 0)
    assert abs(g.mean()) < 5e-3 and abs(g.var() - 1) < 6e-3
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # draws are a pure function of (seed, field, index, component)
    g2 = rng.normals(777, 0, 10 ** 6, np.arange(10, 20), 0)
    np.testing.assert_array_equal(g2, g[10:20])
    assert not np.array_equal(rng.normals(777, 0, 10 ** 6, np.arange(10), 1), g[:10])


def _mode_power(n, L, m2eff, eps):
    f = np.fft.fftfreq(n) * n
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    keff2 = sum(4 * np.sin(np.pi * k / n) ** 2 for k in (kz, ky, kx))
    w = np.sqrt(keff2 / (L / n) ** 2 + m2eff)
    P = eps ** 2 / (2 * w * L ** 3)
    P[0, 0, 0] = 0
    return P, keff2


def test_vacuum_field_statistics():
    """E|f_n|^2 = eps^2/(2 omega_n L^3): the ratio |f_n|^2 / P_n averages to
    one (chi-square with 2 dof per complex pair), the zero mode vanishes,
    the field is real and depends only on the seed."""
    n, L, m2, eps, seed = 16, 10.0, 1.0, 1e-3, 99
    d = oracle.lattice.vacuum_field(n, L, m2, eps, seed, 0, 1)
    assert d.dtype == np.float64 and d.shape == (n, n, n)
    F = np.fft.fftn(d) / n ** 3
    P, _ = _mode_power(n, L, m2, eps)
    assert abs(F[0, 0, 0]) < 1e-15 * np.abs(F).max() * n ** 3
    ratio = (np.abs(F) ** 2 / np.where(P > 0, P, 1))[P > 0]
    # each mode's |f|^2/P is chi^2_2/2 (complex) or chi^2_1 (self-conjugate)
    assert abs(ratio.mean() - 1) < 0.05
    # Hermitian symmetry makes the inverse transform real to rounding
    nz = np.fft.ifftn(F * n ** 3)
    assert np.abs(nz.imag).max() < 1e-12 * np.abs(nz.real).max()
    np.testing.assert_array_equal(d, oracle.lattice.vacuum_field(n, L, m2, eps, seed, 0, 1))
    assert not np.array_equal(d, oracle.lattice.vacuum_field(n, L, m2, eps, seed + 1, 0, 1))
    # the second field draws an independent sequence
    d1 = oracle.lattice.vacuum_field(n, L, m2, eps, seed, 1, 2)
    assert abs(np.corrcoef(d.ravel(), d1.ravel())[0, 1]) < 0.05


def test_vacuum_shell_chi_square():
    """Per shell, sum |f|^2/P over m modes ~ Gamma: a chi-square test on the
    shell means."""
    n, L, m2, eps = 24, 8.0, 2.0, 1.0
    d = oracle.lattice.vacuum_field(n, L, m2, eps, 4242, 0, 1)
    F = np.fft.fftn(d) / n ** 3
    P, keff2 = _mode_power(n, L, m2, eps)
    r = np.abs(F) ** 2 / np.where(P > 0, P, 1)
    b, _, m = oracle.lattice.spectrum_bins(n)
    zs = []
    for shell in range(1, 10):
        sel = (b == shell) & (m > 0)
        cnt = sel.sum()
        # pairs are not independent: effective independent count is cnt/2
        zs.append((r[sel].mean() - 1) * np.sqrt(cnt / 2))
    chi2 = float(np.sum(np.square(zs)))
    assert stats.chi2.sf(chi2, len(zs)) > 1e-3


def test_white_field():
    n, A = 12, 1e-4
    d = oracle.lattice.white_field(n, A, 5, 0)
    assert abs(d.mean()) < 1e-20
    assert d.std() == pytest.approx(A, rel=0.1)


def test_init_constraint_and_parseval():
    cfg = synth.preheat(n=16)
    pot = oracle.Potential(cfg["potential"], cfg["params"])
    lat = oracle.Lattice(16, cfg["L"], pot, mpl=cfg["mpl"])
    lat.init_fluctuations(cfg["phi0"], cfg["pi0"], "vacuum", cfg["amplitude"], cfg["seed"])
    e = lat.energies()
    assert e["friedmann_residual"] < 1e-14
    # mean of each field is the homogeneous value (f_0 = 0)
    assert e["mean"][0] == pytest.approx(1.0, abs=1e-15)
    assert abs(e["mean"][1]) < 1e-18
    # Parseval: sum of the spectrum over bins is the variance
    k, P, c = oracle.spectrum(lat.phi[1], cfg["L"], 64)
    assert np.sum(c * P) == pytest.approx(np.var(lat.phi[1]), rel=1e-12)


def test_spectrum_single_plane_wave():
    n, L, A = 16, 6.0, 0.5
    f = synth.plane_wave(n, (3, 0, 0), A) + 2.0
    k, P, c = oracle.spectrum(f, L, 20)
    nz = np.nonzero(P > 1e-20 * P.max())[0]
    assert list(nz) == [3]
    # two modes (+-3) of |F|^2 = A^2/4 each, averaged over the shell
    assert c[3] * P[3] == pytest.approx(A * A / 2, rel=1e-13)
    # k_b is 2 pi / L times the mean |n| of the shell's modes (brute force)
    norms = []
    for a in range(-8, 8):
        for b in range(-8, 8):
            for d in range(-8, 8):
                r = (a * a + b * b + d * d) ** 0.5
                if 2.5 < r < 3.5:
                    norms.append(r)
    assert c[3] == len(norms)
    assert k[3] == pytest.approx(2 * np.pi * np.mean(norms) / L, rel=1e-13)
    assert c[0] == 0 and P[0] == 0           # the mean is excluded


def test_spectrum_bin_rule_and_counts():
    b, kn, m = oracle.lattice.spectrum_bins(8)
    # |n|^2 = 2 (|n| = 1.41) rounds to 1; |n|^2 = 3 (1.73) rounds to 2;
    # |n|^2 = b^2 + b is the last value of bin b
    assert set(b[m == 2].ravel()) == {1}
    assert set(b[m == 3].ravel()) == {2}
    assert set(b[m == 6].ravel()) == {2} and set(b[m == 8].ravel()) == {3}
    assert set(b[m == 12].ravel()) == {3} and set(b[m == 13].ravel()) == {4}
    # bin 1 holds |n|^2 in {1, 2}: 6 + 12 modes; bin 2 holds {3, 4, 5, 6}:
    # 8 + 6 + 24 + 24 modes (all components within [-4, 4) for n = 8)
    _, _, c = oracle.spectrum(np.zeros((8, 8, 8)), 1.0, 8)
    assert c[1] == 6 + 12 and c[2] == 8 + 6 + 24 + 24


@pytest.mark.parametrize("n", [7, 8])
def test_spectrum_parseval_random(n):
    f = np.random.default_rng(n).standard_normal((n, n, n))
    nb = int(np.ceil(np.sqrt(3) * n / 2)) + 2
    _, P, c = oracle.spectrum(f, 1.0, nb)
    assert np.sum(c * P) == pytest.approx(np.var(f), rel=1e-12)


def test_vacuum_field_27_point_uses_its_own_dispersion():
    """With the 27-point member the mode power follows that stencil's
    frequencies: the normalised |f_n|^2 / P_n averages to one with P_n from
    the stencil's symbol (computed here by brute force over the offsets),
    and not with the 7-point frequencies at the high modes."""
    import itertools
    c = oracle.STENCIL_27
    n, L, m2, eps, seed = 16, 4.0, 1.0, 1e-3, 77
    d = oracle.lattice.vacuum_field(n, L, m2, eps, seed, 0, 1, c)
    F = np.fft.fftn(d) / n ** 3
    f = np.fft.fftfreq(n) * n
    keff2 = np.zeros((n, n, n))
    for iz, iy, ix in itertools.product(range(n), repeat=3):
        k = 2 * np.pi * np.array([f[iz], f[iy], f[ix]]) / n
        keff2[iz, iy, ix] = -sum(c[sum(1 for o in off if o)] * np.cos(np.dot(k, off))
                                 for off in itertools.product((-1, 0, 1), repeat=3))
    w = np.sqrt(keff2 / (L / n) ** 2 + m2)
    P = eps ** 2 / (2 * w * L ** 3)
    P[0, 0, 0] = 0
    ratio = (np.abs(F) ** 2 / np.where(P > 0, P, 1))[P > 0]
    assert abs(ratio.mean() - 1) < 0.05
    P7, k7 = _mode_power(n, L, m2, eps)
    hi = (k7 > 8) & (P7 > 0)
    assert abs((np.abs(F) ** 2 / np.where(P7 > 0, P7, 1))[hi].mean() - 1) > 0.1
