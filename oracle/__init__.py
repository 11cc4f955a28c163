"""CPU FP64 oracle for the boundary-element Poisson-Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything here.
The product library (``paper_1309_4018_amd``) never imports, links or calls
this package, and this package never imports the product library; the two
share only the seeded input generators of ``synth``.

Contents (each module cites the passages it follows):
  quadrature    Dunavant triangle rules, Gauss-Legendre
  geometry      flat-panel geometry and Gauss points
  integrals     Green's functions, panel integrals, semi-analytic self term
  bem           dense-direct assembly (single and multi surface), RHS,
                reaction potential, solvation energy
  gmres         restarted GMRES
  closed_forms  Born, Born-Debye-Hueckel, Kirkwood, concentric spheres
  adjoint       exact discrete gradients dE/dq, dE/dkappa, dE/deps
  refinement    Richardson extrapolation and observed order
"""

from .bem import ENERGY_FACTOR, KE, Oracle, Params, Solution
from .gmres import gmres

__all__ = ["Oracle", "Params", "Solution", "gmres", "KE", "ENERGY_FACTOR"]
