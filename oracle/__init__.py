"""Plain FP64 CPU oracle for the HOBI-PB boundary-integral method (arXiv 1301.5914).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it, to check and to time the HIP implementation.  It shares no code
with the HIP path (no kernels, headers, constants or helpers); both sides receive the
same seeded input arrays.

Modules, in the order of the method:

* ``quadrature``  -- the 4-point Gauss-Radau triangle rule (Section 2.2) and the
  Gauss-Legendre tensor rule with the Duffy-type regularising map (Section 2.3).
* ``geometry``    -- flat to curved triangles: cubic edge arcs, the constructive
  (r,s)->(u,v)->x map, the 10-node interpolated patch, Jacobians and normals
  (Section 2.2, eqs. eqrs2uv and eqintepolation).
* ``kernels``     -- Green's functions and the kernels K1..K4 (Section 2.1, eq_potential,
  Eq_Ls).
* ``operator``    -- mesh validation, node setup, source terms S1/S2 (Eq_Ss), the
  discrete matrix-vector product (eqdbef3 to eqdbef6) and the solvation energy
  (solvation_energy, Section 2.5).
* ``gmres``       -- restarted GMRES (the Krylov solver named in the abstract and in the
  parallel pseudocode table).
* ``kirkwood``    -- Kirkwood's analytic sphere solutions (closed form and series), the
  error norm eqerror and the order eqeorder (Section 3.1).
* ``solve``       -- the whole pipeline of the parallel pseudocode table, run serially.
* ``lobi``        -- the lower-order scheme: flat triangles, centroid collocation and
  one-point quadrature (Section 2.4, eqdbef1/eqdbef2).
* ``treecode``    -- a cluster-particle treecode over a binary cluster tree for the regular sum
  (polynomial interpolation of the Green's functions in the source point), the
  reference of the GPU's optional fast matvec.
* ``field``       -- potential and field at points off the surface from the
  representation formulas (Section 2.1, eqbim_1/eqbim_2) combined into the kernels of
  eq. solvation_energy.

Readings taken where the paper is silent or garbled are listed in each function's
docstring.  The geometric construction (arc tangents, node normals, the centroid node, the
choice of Gauss-Radau rule) is a reading of a garbled passage with no worked example; it is
pinned by closed forms (exactness of the rule, the error orders of the arcs on a circle and
of the elements on spheres, area and volume, watertightness, Kirkwood convergence), not by
values the paper prints.
"""

FOUR_PI = 12.566370614359172953850573533118
# Coulomb constant in kcal*A/(mol*e^2) (CHARMM's value); converts e^2/A to kcal/mol.
COULOMB_KCAL = 332.0716
