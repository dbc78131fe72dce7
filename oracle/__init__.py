"""CPU FP64 oracle of the X-FFT solver (Gehrig & Schneider, arXiv 2601.02172).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU path is checked against.  Only the test suite, the smoke
check of the package entry point and the CPU-baseline leg of the benchmark may
import it; the product path never calls it and shares no code with it.

What it computes (voxel units, h = 1; Sec. 2 and Sec. 3 of the paper):

* ``kuhn``        -- the reference voxel, its six P1 tetrahedra and their
                     barycentric gradients (Sec. 3, division of the voxel
                     into six P1 elements; node numbering matrix Y).
* ``quadrature``  -- the degree-2 four-point rule on (sub)tetrahedra (Sec. 3,
                     subdivision integration) and a degree-3 rule for checks.
* ``xfem``        -- snapping, cut detection, enriched node set J, subdivision
                     of cut elements along the linearised interface, modified
                     abs enrichment, internal scaling D0, element matrices
                     (eqs. X-FEM space, modified abs enrichment, scaling factors,
                     Kapp_q, b_q, Sapp_q).
* ``system``      -- global assembly (CSR) and a matrix-free element loop of the
                     scaled system, right-hand side and average stress (eqs.
                     linearSystem_element, resVector, average stress).
* ``green``       -- the constant-coefficient preconditioner A11^0 inverted in
                     Fourier space; its symbol is taken from the FFT of the
                     assembled stencil (eqs. constantCoefficientPreconditioner,
                     GreenHermitian).
* ``solver``      -- the displacement-based linear CG of Algorithm 1 with the
                     stopping criterion of eq. stoppingCriterion, the basic,
                     Barzilai-Borwein and nonlinear CG schemes with the step
                     size of eq. stepsize, and a dense least-squares solve for
                     tiny grids.
* ``homogenize``  -- effective stiffness from the average stress, the energy
                     form and its closed-form derivative with respect to the
                     per-phase Lame parameters.
* ``accuracy``    -- the accuracy measures of Sec. 4.1: relative error and the
                     L^2 norm of local strain and stress fields by the
                     discretisation's own quadrature (eqs. relError,
                     L2NormGauss).
"""

from .kuhn import CORNERS, kuhn_tets, bary_gradients
from .quadrature import degree2_rule, degree3_rule
from .xfem import Discretization
from .system import System
from .green import GreenOperator
from .solver import pcg, dense_solve
from .homogenize import effective_stiffness, solve_loads, energy_stiffness, lame_gradient

__all__ = [
    "CORNERS", "kuhn_tets", "bary_gradients", "degree2_rule", "degree3_rule",
    "Discretization", "System", "GreenOperator", "pcg", "dense_solve",
    "effective_stiffness", "solve_loads", "energy_stiffness", "lame_gradient",
]
