"""CPU FP64 oracle for the SIPG variable-viscosity viscous operator and the
SIPG Poisson operator of Schussnig, Fehn, Pacheco and Kronbichler,
"Higher-Order Discontinuous Galerkin Splitting Schemes for Fluids with
Variable Viscosity" (arXiv 2506.14424).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP library is checked against.  Only the test suite, the
smoke check of the package entry point and the CPU-baseline leg of the
benchmark may import it; the library never calls it, and it shares no code
with the library (the seeded generators in ``workloads`` are the only common
inputs).

What it computes, and from which passage:

* the discrete space: tensor-product Lagrange polynomials of degree k on
  each hexahedron (Sec. 4, the spaces V_h^u and V_h^p), with nodes at the
  k+1 Gauss-Legendre points and the same points as quadrature rule;
* the viscous bilinear form v_h^e of Sec. 4.1 (paragraph "Viscous Step") with
  the SIPG fluxes u = {{u}}, tau_1 = {{nu grad u}} - tau [[u]], tau_2 = tau_1^T,
  plus the mass term (gamma_0/dt)(v, u) of the viscous step, the mirror
  principle at the boundary;
* the SIPG Poisson form of the pressure step (Sec. 4.1, paragraph
  "Pressure Step") with a coercive penalty sign;
* the penalty-step form (Sec. 4.3, "Consistent Stabilization"): mass plus
  divergence and normal-continuity penalties;
* the viscosity laws of Sec. 2 (generalised Newtonian law) and smooth
  prescribed fields, evaluated pointwise at quadrature points (Sec. 4.1);
* the matrix diagonal, a Chebyshev-accelerated Jacobi preconditioner and a
  flexible CG with FP64 outer iteration (Sec. 5.3);
* the hp-multigrid V-cycle preconditioner of Sec. 5.3 (degree lowered from
  k to 1, then mesh coarsening, Chebyshev-Jacobi smoothing on every level),
  in ``multigrid``;
* the Picard update of the viscosity from the velocity (Sec. 4.1,
  eq. viscosity_pointwise) on every multigrid level and the Aitken-relaxed
  fixed-point iteration of the nonlinear viscous step (Sec. 5.1, Alg. 1),
  in ``picard``.

Two evaluation modes: ``assemble`` builds the global sparse matrix cell by
cell and face by face (small meshes); ``apply`` evaluates the same quadrature
sums directly on a vector, one batch of cells or faces at a time (any size).

Parity status: every function is pinned by tests under ``tests/`` marked
``not gpu`` (symmetry, definiteness, null spaces, polynomial reproduction,
patch tests on curved meshes, Laplacian reduction, convergence order,
independent brute-force quadrature).
"""

from .basis import gauss_points, lagrange_values, lagrange_derivatives
from .mesh import Mesh
from .laws import viscosity
from .forms import Problem, assemble, apply, diagonal, load_vector
from . import solvers

__all__ = [
    "gauss_points", "lagrange_values", "lagrange_derivatives", "Mesh", "viscosity",
    "Problem", "assemble", "apply", "diagonal", "load_vector", "solvers",
]
