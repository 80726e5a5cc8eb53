"""Seeded sweep over lattice sizes (4 .. 40, odd and even), potential
families and field counts, the 7- and 27-point stencils and pass shapes
(lanes, sites per lane, z-chunk, prefetch depth): each case advances 5
steps of 4th order on the GPU and in the oracle from one synthetic state,
FP64 with self-consistent expansion; fields, momenta, a and p_a within the
FP64 gate.  The cases are drawn once from a fixed seed."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_state, gpu_lattice, oracle_lattice, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10

# (potential, parameters, homogeneous fields, m_pl)
MODELS = [
    ("chaotic2", (1.0, 9312.25), (1.0, 0.0), 1.0335292),
    ("oscillon", (1.0, 1.0, 0.2), (0.8,), 335.41),
    ("qball", (1.0, -0.1, 1.0), (math.sqrt(2) * 1e-2, 0.0), 1.0),
    ("free", (0.9, 1.6, 2.5), (0.1, 0.2, 0.3), 1.0),
]


def _cases(count=24, seed=20120299):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind, params, base, mpl = MODELS[int(rng.integers(len(MODELS)))]
        nf = len(base)
        n = int(rng.integers(4, 41))
        st27 = bool(rng.random() < 0.3)
        vxs = [1] if nf > 2 else [v for v in (1, 2, 4) if n % v == 0 and not (st27 and v == 4)]
        vx = int(rng.choice(vxs))
        tx = int(rng.choice([16, 32, 64]))
        pf = 1 if (nf > 2 or st27) else int(rng.choice([1, 2]))
        tz = int(rng.integers(0, n + 1))           # 0: chosen from the occupancy
        out.append((kind, params, base, mpl, n, "27" if st27 else None, (tx, vx, tz, pf)))
    return out


CASES = _cases()


def _cases_lanes(count=16, seed=20120298):
    """Cases for the lane count along x: 8 lanes (32 rows of the workgroup),
    a whole row per tile (n / vx lanes, often not a power of two, with the
    last 256 mod tx lanes idle) or any count in [8, 64]; half of the sizes
    multiples of 4, with 4 sites per lane where the case allows it."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        kind, params, base, mpl = MODELS[int(rng.integers(len(MODELS)))]
        nf = len(base)
        n = int(4 * rng.integers(1, 11)) if rng.random() < 0.5 else int(rng.integers(4, 41))
        st27 = bool(rng.random() < 0.3)
        vxs = [1] if nf > 2 else [v for v in (1, 2, 4) if n % v == 0 and not (st27 and v == 4)]
        vx = 4 if 4 in vxs else int(rng.choice(vxs))
        pf = 1 if (nf > 2 or st27) else int(rng.choice([1, 2]))
        tz = int(rng.integers(0, n + 1))
        row = n // vx
        tx = [8, row if 8 <= row <= 64 else 8, int(rng.integers(8, 65))][k % 3]
        out.append((kind, params, base, mpl, n, "27" if st27 else None, (tx, vx, tz, pf)))
    return out


CASES_LANES = _cases_lanes()


def _cases_nontemporal(count=10, seed=20120297):
    """Cases for the pass modes with non-temporal result stores (pf = 5, 6:
    depth 1 or 2 plus 4), which the 7-point pass runs for up to two fields
    with 2 or 4 sites per lane."""
    rng = np.random.default_rng(seed)
    models = [m for m in MODELS if len(m[2]) <= 2]
    out = []
    for _ in range(count):
        kind, params, base, mpl = models[int(rng.integers(len(models)))]
        n = int(2 * rng.integers(2, 21))
        vx = 4 if (n % 4 == 0 and rng.random() < 0.6) else 2
        tx = int(rng.choice([8, 16, 32, 64])) if vx == 4 else int(rng.choice([16, 32, 64]))
        pf = int(rng.choice([5, 6]))
        tz = int(rng.integers(0, n + 1))
        out.append((kind, params, base, mpl, n, None, (tx, vx, tz, pf)))
    return out


CASES_NT = _cases_nontemporal()


def _run_case(case, spec, seed):
    kind, params, base, mpl, n, stencil, tile = spec
    nf = len(base)
    L = 0.5 * n                                    # dx = 0.5
    scale = max(abs(b) for b in base)
    phi, pi = synth.gaussian_state(n, nf, seed, phi_base=list(base),
                                   phi_amp=1e-3 * scale, pi_amp=1e-3 * scale)
    o = oracle_lattice(n, L, kind, params, phi, pi, mpl=mpl,
                       stencil=oracle.STENCIL_27 if stencil else None)
    g = gpu_lattice(n, L, kind, params, phi, pi, mpl=mpl, tile=tile, stencil=stencil)
    say("sweep case", case, kind, "n", n, "stencil", stencil or "7", "tile", tile, "->", g.tile())
    g.evolve(5, 0.005, 4)
    o.evolve(5, 0.005, 4)
    ef, ep, ea, epa, _ = compare_state(g, o)
    say("  errors", ef, ep, ea, epa)
    assert max(ef, ep, ea, epa) <= FP64_TOL
    g.close()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sweep(case):
    _run_case(case, CASES[case], 9000 + case)


@pytest.mark.parametrize("case", range(len(CASES_LANES)))
def test_sweep_lanes(case):
    _run_case(case, CASES_LANES[case], 9100 + case)


@pytest.mark.parametrize("case", range(len(CASES_NT)))
def test_sweep_nontemporal(case):
    _run_case(case, CASES_NT[case], 9200 + case)


@pytest.mark.parametrize("case", list(range(0, len(CASES), 3)) +
                         list(range(len(CASES), len(CASES) + len(CASES_NT), 2)))
def test_sweep_fp32_storage(case):
    """Every third case with FP32 field storage: relative L2 error of the
    fields and momenta within the FP32 gate (1e-4)."""
    from gpu_util import rel_l2
    kind, params, base, mpl, n, stencil, tile = (CASES + CASES_NT)[case]
    nf = len(base)
    L = 0.5 * n
    scale = max(abs(b) for b in base)
    phi, pi = synth.gaussian_state(n, nf, 9000 + case, phi_base=list(base),
                                   phi_amp=1e-3 * scale, pi_amp=1e-3 * scale)
    o = oracle_lattice(n, L, kind, params, phi, pi, mpl=mpl,
                       stencil=oracle.STENCIL_27 if stencil else None)
    g = gpu_lattice(n, L, kind, params, phi, pi, precision="f32", mpl=mpl, tile=tile,
                    stencil=stencil)
    g.evolve(5, 0.005, 4)
    o.evolve(5, 0.005, 4)
    gphi, gpi = g.get_fields()
    e1, e2 = rel_l2(gphi, o.phi), rel_l2(gpi, o.pi)
    say("sweep fp32 case", case, kind, n, stencil or "7", g.tile(), e1, e2)
    assert max(e1, e2) <= 1e-4
    g.close()
