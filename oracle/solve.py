"""The whole solve of the parallel pseudocode table (Section 2.6), run serially.

Order: validate and curve the surface, store the quadrature data (routines (2)-(4)),
source terms (routine (1)), GMRES on A u = (S1, S2) (routine (5) inside), solvation
energy (routine (6)).  Outputs phi and dphi/dn in kcal/(mol e) and kcal/(mol e A)
(internal values times 4 pi C) and E_sol in kcal/mol.
"""
from __future__ import annotations

import numpy as np

from . import COULOMB_KCAL, FOUR_PI
from .gmres import diagonal_scaling, gmres, gmres_scaled
from .operator import check_charges_inside, diagonal, matvec, setup, solvation_energy, sources


def solve(xyz, nrm, tri, qpos, q, eps1=1.0, eps2=80.0, kappa=0.1257,
          rtol=1e-6, restart=200, max_iter=200, st=None, workers=1, diag_scaling=2):
    """diag_scaling, the right preconditioner of GMRES: 2 (default) Jacobi, the inverse of A's
    own diagonal (operator.diagonal); 1 (or True) the two row blocks' constants; 0 (or False)
    none, A u = b as written."""
    eps = eps2 / eps1
    if st is None:
        st = setup(xyz, nrm, tri)
    qpos = np.asarray(qpos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).ravel()
    check_charges_inside(st, qpos)
    S1, S2 = sources(st.xyz, st.nrm, qpos, q, eps1)
    b = np.concatenate([S1, S2])
    A = lambda v: matvec(st, v, kappa, eps, workers=workers)
    if diag_scaling:
        dinv = 1.0 / diagonal(st, kappa, eps) if int(diag_scaling) == 2 else diagonal_scaling(st.nv, eps)
        u, its, rel, conv = gmres_scaled(A, b, dinv, rtol, restart, max_iter)
    else:
        u, its, rel, conv = gmres(A, b, rtol, restart, max_iter)
    true_rel = float(np.linalg.norm(b - matvec(st, u, kappa, eps, workers=workers)) / np.linalg.norm(b))
    E = solvation_energy(st, u, qpos, q, kappa, eps)
    nv = st.nv
    scale = FOUR_PI * COULOMB_KCAL
    return dict(u=u, phi=scale * u[:nv], dphi=scale * u[nv:], energy=E, iterations=its,
                est_residual=rel, true_residual=true_rel, converged=conv, setup=st, b=b)
