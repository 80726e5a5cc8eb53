"""Plain, slow FP64 CPU oracle of the symplectic FRW lattice method of
Sainio, "PyCOOL - a Cosmological Object-Oriented Lattice code written in
Python" (arXiv:1201.5029).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the test suite, the smoke check of the entry module and the CPU-baseline
leg of the benchmark script may use it.  It shares no code with the HIP
library; the one thing both sides see is the seeded input module ``synth``,
which holds no arithmetic of the method.

The oracle applies the paper's exact sub-flows one by one, in the order the
composition prescribes, with no merging, fusion or lazy bookkeeping:

* ``lattice``   stencils, potentials, the Hamiltonian and its three-way
                split, the exact flows, the second-order map, the Yoshida /
                Table 1 compositions, observables, spectrum, initial state.
* ``linear``    the linearized integrator: homogeneous background plus
                Fourier-space perturbations, every mode evolved on its own.
* ``rng``       the counter-based SplitMix64 generator and Box-Muller normals,
                written from their published definitions.
* ``deltan``    the separate-universe read-out of a scan: the constraint's
                total density along a run and the uniform-density e-folds.

Every function is pinned by a ``-m "not gpu"`` test against a closed form, an
invariant, a printed constant or brute force; see the test modules named
``test_oracle_*``.
"""
from .lattice import (  # noqa: F401
    TABLE1_ORDER6, TABLE1_ORDER8, composition_weights, lap, grad_energy,
    Potential, Lattice, spectrum, stability_limit, linear_stage_matrix,
    STENCIL_7, STENCIL_19, STENCIL_27, isotropic_stencil, stencil_symbol,
    stencil_ok, stencil_max_keff2, keff2_modes, mode_spectra,
)
from .linear import LinearLattice  # noqa: F401
from . import deltan, rng  # noqa: F401
