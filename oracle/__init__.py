"""CPU oracle for the spherical-harmonic x discontinuous-Galerkin VFP operator.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy
restatement of the method of Schween, Schulze & Reville (arXiv 2501.05110):
the real spherical-harmonic system matrices (Sec. 2.1), the advection-reaction
form (Sec. 2.2), and the assembled DG system M dzeta/dt + D zeta = h
(Sec. 3, eq. definition-mass-and-dg-matrix) with upwind fluxes (eq.
definition-upwind-flux) and weak boundary fluxes (eq. definition-boundary-flux,
eq. continuous-bc), advanced by the classical fourth-order Runge-Kutta method.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code, tables or constants with the
HIP library in ``paper_2501_05110_amd``; the two meet only through the seeded
input generators in ``paper_2501_05110_amd.workloads`` (which hold no method
arithmetic).

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms
and invariants that the paper fixes, except where a docstring says
"parity unpinned".
"""

from . import sh, dg  # noqa: F401
