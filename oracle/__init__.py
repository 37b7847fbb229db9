"""FP64 CPU oracle for the lattice Boltzmann transport pipeline (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
import this package.  The product path (``paper_1410_1921_amd``) never does.  The C
source ``lbm_oracle.c`` shares no code, table or constant with the HIP library.

Parity status of each function (what pins it, in ``tests/test_oracle_*.py``):

* ``splitmix64`` -- published SplitMix64 outputs for seed 0 (golden file).
* ``lens_volume`` -- closed forms (containment, tangency, equal spheres) and a
  Monte-Carlo estimate.
* ``reconstruct`` -- brute-force re-check of the acceptance rules over every accepted
  pair and of the stop rule; porosity reached.
* ``label18`` -- ``scipy.ndimage.label`` with the 18-neighbour structure on masks
  whose y/z faces are solid, plus hand cases for the periodic wrap.
* ``chords13`` -- closed values on boxes, slabs and single voxels, and an independent
  pure-Python walk on tiny masks.
* ``edt2`` -- ``scipy.ndimage.distance_transform_edt`` and O(N^6) brute force.
* ``mis`` -- slit widths (odd H gives H, even gives H-1), single balls, brute force.
* ``flow_solve`` -- exact discrete slit (plane Poiseuille) permeability, square duct
  series solution, tube (Eq. 27) convergence, mass and momentum balance, mirror
  symmetry, Stokes linearity.
* ``knudsen_solve`` -- exact straight-duct flux (tortuosity 1 at tau = 1), parallel
  columns with different tau, mass conservation, swap and linearity.
* ``knudsen_diffusivity`` / ``fc`` -- the paper's printed D_K(60 nm, 323 K) and the
  coefficient 64/(3 pi) of Eq. 28.
* ``k_kozeny_carman`` (Eq. 17) -- worked examples computed by hand
  (``tests/golden/props_worked_examples.txt``) and Carman's hydraulic-radius form with
  the Kozeny constant 5 and the sphere's surface-to-volume ratio taken numerically from
  ``sphere_volume``.
* ``lattice_diffusivity``, ``time_step``, ``deff_physical``, ``k_physical``, ``m2_to_mD``
  (Eq. 15), ``tortuosity`` (Eq. 16), ``bruggeman_alpha`` (Section 4.2) -- worked examples;
  tortuosity 1 of a straight duct at tau = 1 and its closed form at tau = 1.4; channels
  of reference pores diffusing at eps D_K(d_ref); alpha and tortuosity consistent; a
  physical slit's permeability independent of the voxel size.
* ``collide19_mrt`` / ``flow_solve(collision=MRT)`` -- the inverse of Q against the
  paper's printed Appendix A table (golden file; its misprinted row 6 noted), mass and
  momentum conservation, equal rates reducing to BGK, and the tau-independent slit
  permeability (H^2 + 1/2)/12 that the rates of Eq. 7 imply.
* ``nn_oracle`` (the learned warm start, not part of the paper's method) --
  ``conv3d`` against ``scipy.ndimage.correlate``, every backward against central finite
  differences, pooling / upsampling adjointness.
"""
from .oracle import *  # noqa: F401,F403
