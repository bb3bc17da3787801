"""FP64 CPU oracle of the grand-potential ternary phase-field lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test-suite, the smoke check of the
package entry point and the CPU-baseline leg of the benchmark may import it.
The GPU library never imports, links or calls anything here, and nothing here
imports the GPU library: the two share no code.  Inputs (initial fields and
parameters) are passed in as arrays and plain numbers.

Written from Verdier, Cartalade & Plapp, "Grand-potential phase field
simulations of droplet growth and sedimentation in a two-phase ternary fluid"
(arXiv 2409.03401):

* ``lattices``  – velocity sets (Section 3, Tables tab:D2Q9 / tab:D3Q19, plus
                  the D2Q5 / D3Q7 reading for the scalar fields).
* ``model``     – thermodynamics of Section 2 (interpolation p, double well,
                  dimensionless grand potentials, closure, source term).
* ``lbm``       – the discrete map: initialisation, one time step (Section 3,
                  Eqs. LBE_FluidFlow ... Moment0_c_alpha), moments, diagnostics.
* ``analytic``  – closed forms used to pin the oracle: tanh interface profile
                  (Eq. tanh), the ternary diffusion-couple similarity solution
                  (Section 4.1, Eqs. Stefan ... Solution_Mu), Poiseuille flow.

Every array computation runs in float64; passing complex128 inputs runs the
same arithmetic on complex numbers, which gives exact directional derivatives
by the complex-step method (Squire & Trapp, SIAM Rev. 40 (1998) 110) because
the step uses only +, -, *, / and index permutations.
"""

from . import lattices, model, lbm, analytic  # noqa: F401
