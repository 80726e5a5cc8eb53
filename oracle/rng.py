"""Counter-based normal deviates for the oracle's initial states.

Test infrastructure only (see the package docstring).

* SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014): the state advances by the
  odd constant GAMMA and each output is the state passed through the
  published two-multiply finaliser.  The k-th output (k >= 1) from a seed is
  therefore ``mix(seed + k * GAMMA)``, which makes the generator
  counter-based: any draw can be made independently of traversal order.
* Uniforms take the top 53 bits: u = ((x >> 11) + 1) * 2**-53, in (0, 1].
* Normals use the Box-Muller transform (Box & Muller 1958):
  g = sqrt(-2 ln u1) * cos(2 pi u2).

Counter layout: draw ``r`` (0/1 = first/second uniform) of component ``c``
(0/1 = real/imaginary part) for field ``i`` at linear index ``idx`` of an
``nsites``-entry array uses counter 4*(i*nsites + idx) + 2*c + r, i.e. key
``seed + (counter + 1) * GAMMA`` (mod 2**64).
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
_M64 = (1 << 64) - 1


def splitmix64_scalar(key):
    """Finaliser of SplitMix64 on one Python int (reference form)."""
    z = key & _M64
    z = ((z ^ (z >> 30)) * MIX1) & _M64
    z = ((z ^ (z >> 27)) * MIX2) & _M64
    return z ^ (z >> 31)


def splitmix64(keys):
    """Vectorised finaliser on a uint64 array (wrap-around arithmetic)."""
    z = np.asarray(keys, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
    return z ^ (z >> np.uint64(31))


def keys_for(seed, counters):
    """seed + (counter + 1) * GAMMA mod 2**64 for a uint64 counter array."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return np.uint64(seed & _M64) + (c + np.uint64(1)) * np.uint64(GAMMA)


def uniforms(seed, counters):
    x = splitmix64(keys_for(seed, counters))
    return ((x >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53


def normals(seed, field, nsites, idx, comp):
    """Box-Muller normal for (field, linear index array, component)."""
    idx = np.asarray(idx, dtype=np.uint64)
    base = np.uint64(4) * (np.uint64(field) * np.uint64(nsites) + idx) \
        + np.uint64(2 * comp)
    u1 = uniforms(seed, base)
    u2 = uniforms(seed, base + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
