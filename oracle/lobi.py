"""Lower-order scheme (LOBI-PB, the paper's "low-order scheme" subsection, eqdbef1/eqdbef2):
flat triangles, one collocation point and one quadrature point per triangle, its centroid.

Test infrastructure only: plain numpy FP64, written from the equations; nothing in the
product path imports it.

Unknowns: u = (phi_1..phi_Nf, dphi_1..dphi_Nf) at the Nf centroids, in internal units
(the Green's functions carry their 1/(4 pi); phi in e/A), and

  (Au)_i      = 1/2 (1 + eps) phi_i        - sum_{j != i} W_j [K1(c_i, c_j) dphi_j + K2(c_i, c_j) phi_j]
  (Au)_{i+Nf} = 1/2 (1 + 1/eps) dphi_i     - sum_{j != i} W_j [K3(c_i, c_j) dphi_j + K4(c_i, c_j) phi_j]

Readings (the subsection is brief):
* W_j is the area of flat triangle j; the unknowns and the kernels are taken constant on it;
* the normal at centroid c_j is the flat triangle's unit normal (its orientation is the
  stored, counter-clockwise-from-outside vertex order);
* the subsection drops a triangle's contribution where the kernel is singular; read as the
  self term j = i only, where the collocation point and the quadrature point coincide
  (Section 2.4);
* the source terms are those of the higher-order scheme, evaluated at the centroids with
  the face normals; the energy uses the same one-point rule at the charges.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import COULOMB_KCAL, FOUR_PI
from .gmres import diagonal_scaling, gmres, gmres_scaled
from .kernels import kernels, kernels_12
from .operator import ChargeOutsideError, sources, validate_mesh


@dataclasses.dataclass
class LobiSetup:
    c: np.ndarray   # [nf,3] centroids (collocation and quadrature points)
    n: np.ndarray   # [nf,3] unit face normals
    W: np.ndarray   # [nf] triangle areas

    @property
    def nf(self):
        return self.c.shape[0]


def setup(xyz, nrm, tri) -> LobiSetup:
    """Flat triangles: centroids, unit normals and areas (the mesh is validated as for
    the higher-order scheme)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    validate_mesh(xyz, nrm, tri)
    tri = np.asarray(tri, dtype=np.int64)
    A, B, C = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(B - A, C - A)
    area2 = np.linalg.norm(cr, axis=1)
    return LobiSetup((A + B + C) / 3.0, cr / area2[:, None], 0.5 * area2)


def matvec(st: LobiSetup, u, kappa, eps, rows=None):
    """y = A u (all 2 Nf rows), or the pair (rows i, i+Nf) for each i in ``rows``."""
    nf = st.nf
    u = np.asarray(u, dtype=np.float64)
    phi, dphi = u[:nf], u[nf:]
    idx = np.arange(nf) if rows is None else np.asarray(rows)
    s1 = np.empty(idx.shape[0])
    s2 = np.empty(idx.shape[0])
    for r, i in enumerate(idx):
        others = np.arange(nf) != i
        K1, K2, K3, K4 = kernels(st.c[i], st.n[i], st.c[others], st.n[others], kappa, eps)
        W = st.W[others]
        s1[r] = np.sum(W * (K1 * dphi[others] + K2 * phi[others]))
        s2[r] = np.sum(W * (K3 * dphi[others] + K4 * phi[others]))
    top = 0.5 * (1.0 + eps) * phi[idx] - s1
    bot = 0.5 * (1.0 + 1.0 / eps) * dphi[idx] - s2
    if rows is None:
        return np.concatenate([top, bot])
    return np.stack([top, bot])


def double_layer_row_sums(st: LobiSetup):
    """sum_{j != i} W_j dG0(c_i, c_j)/dn_j for every i: the one-point discrete double layer
    of a unit density at the collocation points (-1/2 on a smooth closed surface)."""
    out = np.empty(st.nf)
    for i in range(st.nf):
        d = st.c[i] - st.c
        r = np.linalg.norm(d, axis=1)
        r[i] = 1.0
        term = st.W * np.sum(d * st.n, axis=1) / (FOUR_PI * r ** 3)
        term[i] = 0.0
        out[i] = np.sum(term)
    return out


def reaction_potential(st: LobiSetup, u, points, kappa, eps):
    nf = st.nf
    phi, dphi = u[:nf], u[nf:]
    out = np.empty(points.shape[0])
    for k in range(points.shape[0]):
        K1, K2 = kernels_12(points[k], st.c, st.n, kappa, eps)
        out[k] = np.sum(st.W * (K1 * dphi + K2 * phi))
    return out


def solvation_energy(st: LobiSetup, u, qpos, q, kappa, eps):
    """E_sol = 1/2 sum_k q_k phi_reac(x_k) in kcal/mol, one-point rule on every triangle."""
    pr = reaction_potential(st, u, qpos, kappa, eps)
    return 0.5 * FOUR_PI * COULOMB_KCAL * float(np.sum(q * pr))


def solid_angle_fraction(st: LobiSetup, points):
    out = np.empty(points.shape[0])
    for k in range(points.shape[0]):
        d = points[k] - st.c
        r = np.linalg.norm(d, axis=1)
        out[k] = -np.sum(st.W * np.sum(d * st.n, axis=1) / (FOUR_PI * r ** 3))
    return out


def solve(xyz, nrm, tri, qpos, q, eps1=1.0, eps2=80.0, kappa=0.1257, rtol=1e-6, restart=200,
          max_iter=200, st=None, diag_scaling=True):
    """The whole lower-order solve: sources at the centroids, GMRES (on the diagonally
    scaled system by default, as oracle.solve), energy."""
    eps = eps2 / eps1
    if st is None:
        st = setup(xyz, nrm, tri)
    qpos = np.asarray(qpos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).ravel()
    if np.any(solid_angle_fraction(st, qpos) < 0.5):
        raise ChargeOutsideError("charge outside the surface")
    S1, S2 = sources(st.c, st.n, qpos, q, eps1)
    b = np.concatenate([S1, S2])
    A = lambda v: matvec(st, v, kappa, eps)
    if diag_scaling:
        u, its, rel, conv = gmres_scaled(A, b, diagonal_scaling(st.nf, eps), rtol, restart, max_iter)
    else:
        u, its, rel, conv = gmres(A, b, rtol, restart, max_iter)
    E = solvation_energy(st, u, qpos, q, kappa, eps)
    nf = st.nf
    scale = FOUR_PI * COULOMB_KCAL
    return dict(u=u, phi=scale * u[:nf], dphi=scale * u[nf:], energy=E, iterations=its,
                est_residual=rel, converged=conv, setup=st, b=b)
