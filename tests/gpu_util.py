"""Helpers shared by the GPU tests: build the oracle and the library lattice
from the same synthetic state, and the error measures of the parity gates
(per array: max |diff| / max |ref| and ||diff||_2 / ||ref||_2)."""
import math
import sys

import numpy as np

import oracle
import paper_1201_5029_amd as sl


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_lattice(n, L, kind, params, phi, pi, mpl=1.0, a0=1.0, rho_rad0=0.0,
                   rho_mat0=0.0, expand=True, p_a=None, stencil=None):
    pot = oracle.Potential(kind, params)
    lat = oracle.Lattice(n, L, pot, mpl=mpl, a0=a0, rho_rad0=rho_rad0,
                         rho_mat0=rho_mat0, expand=expand,
                         stencil=oracle.STENCIL_7 if stencil is None else stencil)
    lat.phi[...] = phi
    lat.pi[...] = pi
    if p_a is None:
        lat.solve_constraint()
    else:
        lat.p_a = p_a
    return lat


def gpu_lattice(n, L, kind, params, phi, pi, precision="f64", mpl=1.0, a0=1.0,
                rho_rad0=0.0, rho_mat0=0.0, expand=True, p_a=math.nan, tile=None,
                stencil=None):
    g = sl.Lattice(n, phi.shape[0], L, precision=precision, expand=expand, mpl=mpl,
                   a0=a0, rho_rad0=rho_rad0, rho_mat0=rho_mat0)
    g.set_potential(kind, params)
    if stencil is not None:
        g.set_stencil(stencil)
    if tile is not None:
        g.set_tile(*tile)
    g.set_fields(phi, pi, a0, p_a)
    return g


def max_rel(got, ref):
    """max over arrays of max|got - ref| / max|ref| (arrays = first axis)."""
    worst = 0.0
    for g, r in zip(got, ref):
        scale = np.abs(r).max()
        if scale == 0:
            scale = 1.0
        worst = max(worst, float(np.abs(g - r).max() / scale))
    return worst


def rel_l2(got, ref):
    worst = 0.0
    for g, r in zip(got, ref):
        nr = np.linalg.norm(r)
        if nr == 0:
            nr = 1.0
        worst = max(worst, float(np.linalg.norm(g - r) / nr))
    return worst


def fluct_rel_l2(got, ref):
    """rel-L2 of the fluctuation part of each array (its own lattice mean
    removed), worst array: ||(g - <g>) - (r - <r>)||_2 / ||r - <r>||_2.  In
    the linear regime the homogeneous value dominates the full-field
    measure; this one sees the error of the perturbations themselves."""
    worst = 0.0
    for g, r in zip(got, ref):
        dr = r - r.mean()
        nr = np.linalg.norm(dr)
        if nr == 0:
            continue
        worst = max(worst, float(np.linalg.norm((g - g.mean()) - dr) / nr))
    return worst


def compare_state(g, o):
    """(field error, momentum error, rel error of a, rel error of p_a)."""
    phi, pi = g.get_fields()
    eta, a, pa = g.background()
    ea = abs(a - o.a) / abs(o.a)
    ep = abs(pa - o.p_a) / max(abs(o.p_a), 1e-300) if o.p_a != 0 else abs(pa)
    return max_rel(phi, o.phi), max_rel(pi, o.pi), ea, ep, (phi, pi, eta, a, pa)
