"""Plain FP64 CPU oracle for the spectral-element right-hand side.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.

The oracle is a slow, literal NumPy/SciPy restatement of the discretisation in
Tissaoui, Guimond, Giraldo & Marras, "Accelerating Simulations of Tropical
Cyclones using Adaptive Mesh Refinement" (arXiv 2410.21607):

* ``gll``       Legendre-Gauss-Lobatto nodes, weights, derivative and
                interpolation matrices (Section 3, tensor-product basis).
* ``mesh``      hexahedral column mesh, unique-node numbering by coordinate,
                hanging nodes and the interpolation matrix Z (Section 3.1).
* ``euler``     pointwise thermodynamics and the strong-form right-hand side
                of the perturbation equations (Section 2, eqs. mass_split,
                mom_split, ent_split).
* ``assembly``  direct stiffness summation with the modified (hanging-node)
                rule: scatter Z, gather Z^T, lumped mass (Section 3.1).
* ``timestep``  explicit third-order Runge-Kutta stages (Section 5).
* ``amr``       threshold refinement / coarsening flags (Section 4.1).
* ``adapt``     one adaptation pass of the column quadtree (split, 2:1
                balance, merge) and the transfer of the solution onto it.
* ``terrain``   terrain-following (mapped) hexahedra: discrete metrics, the
                chain-rule derivatives, mapped lumped masses and the surface
                boundary rule.
* ``mlp``       small multilayer perceptron used by the refinement forecaster.
* ``metrics``   floor-scaled relative L2 error and maximum wind.

Every function states the passage it follows.  It shares no code, table or
constant generator with the HIP path; the only shared module is ``synth``
(seeded input generation), which holds none of the method's arithmetic.
"""

from . import gll, mesh, euler, assembly, timestep, amr, adapt, metrics, terrain  # noqa: F401
