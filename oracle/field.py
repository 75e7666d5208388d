"""Potential and field at points off the surface, from the representation formulas.

Test infrastructure only: plain numpy FP64; nothing in the product path imports it.

The representation formulas of Section 2.1 (eqbim_1 for x in the solute Omega_1, eqbim_2
for x in the solvent Omega_2) give the potential anywhere once the surface unknowns are
known.  With the jump conditions phi_2 = phi_1 and eps2 dphi_2/dnu = eps1 dphi_1/dnu on
the surface (so dphi_2/dnu = dphi_1/dnu / eps, eps = eps2 / eps1), and using that each
formula vanishes on the other side of the surface, the two combine into one surface
integral, the reaction potential of eq. solvation_energy,

  R(x) = int [K1(x, y) dphi_1/dnu(y) + K2(x, y) phi_1(y)] dS_y,

and, with S1(x) = sum_k q_k G0(x, x_k) / eps1 (the source term of eq. Eq_Ss, 1/eps1
reading),

  x in Omega_1:  phi(x) = S1(x) + R(x)
  x in Omega_2:  phi(x) = (S1(x) + R(x)) / eps.

(Inside: eqbim_1 plus eps times eqbim_2, whose value is 0 there.  Outside: eqbim_2 plus
1/eps times eqbim_1, whose value is 0 there.)  The field is E = -grad phi.  The side of x
is read from the double layer of a unit density, -1 inside and 0 outside: x is inside when
the solid-angle fraction -int dG0/dnu_y dS_y exceeds 1/2.

Everything here is written with the Green's functions and their derivatives themselves
(eq. eq_potential), with d = x - y, r = |d|, a = exp(-kappa r):

  G0 = 1/(4 pi r),  Gk = a/(4 pi r)
  dG0/dnu_y = (d.n_y)/(4 pi r^3),  dGk/dnu_y = a (1 + kappa r)(d.n_y)/(4 pi r^3)
  grad_x G0 = -d/(4 pi r^3),  grad_x Gk = -a (1 + kappa r) d/(4 pi r^3)
  grad_x dG0/dnu_y = [n_y - 3 (d.n_y) d / r^2]/(4 pi r^3)
  grad_x dGk/dnu_y = a [(1 + kappa r) n_y - (3 + 3 kappa r + kappa^2 r^2)(d.n_y) d / r^2]/(4 pi r^3)

and K1 = G0 - Gk, K2 = eps dGk/dnu_y - dG0/dnu_y (eq. Eq_Ls).  The surface integral uses
the quadrature of the energy: the 4-point rule on every triangle (higher-order method) or
the centroid rule (lower-order method); there is no near-singular treatment, so a point
within about one edge length of the surface gets that rule's error.

Reading: a charge closer than COINCIDENT to the point is left out of that point's S1 and
grad S1 (the potential and field at an atom are then those of the other charges plus the
reaction terms; q_k times the reaction field at x_k is the solvation force on atom k).
"""
from __future__ import annotations

import numpy as np

from . import FOUR_PI
from .lobi import LobiSetup
from .operator import Setup

COINCIDENT = 1e-6   # A


def surface_nodes(st, u):
    """(y, n_y, w, dphi, phi) over the quadrature nodes of a solved surface: the 4
    regular nodes of every curved triangle with the vertex unknowns interpolated linearly
    (Section 2.2), or the centroids with their own unknowns (Section 2.4)."""
    u = np.asarray(u, dtype=np.float64)
    if isinstance(st, LobiSetup):
        nf = st.nf
        return st.c, st.n, st.W, u[nf:], u[:nf]
    if isinstance(st, Setup):
        nv = st.nv
        dphi = (u[nv:][st.tri] @ st.L.T).ravel()
        phi = (u[:nv][st.tri] @ st.L.T).ravel()
        return st.y.reshape(-1, 3), st.ny.reshape(-1, 3), st.w.ravel(), dphi, phi
    raise TypeError("unknown setup type")


def node_sums(pts, y, ny, w, dphi, phi, kappa, eps):
    """(R, grad R, solid-angle fraction) at each point from the given quadrature nodes
    (positions y, normals ny, weights w, interpolated dphi and phi)."""
    R = np.empty(pts.shape[0])
    gR = np.empty((pts.shape[0], 3))
    frac = np.empty(pts.shape[0])
    for k in range(pts.shape[0]):
        d = pts[k] - y
        r = np.linalg.norm(d, axis=1)
        dny = np.sum(d * ny, axis=1)
        a = np.exp(-kappa * r)
        z = kappa * r
        c3 = FOUR_PI * r ** 3
        G0 = 1.0 / (FOUR_PI * r)
        Gk = a / (FOUR_PI * r)
        dG0 = dny / c3
        dGk = a * (1.0 + z) * dny / c3
        K1 = G0 - Gk
        K2 = eps * dGk - dG0
        R[k] = np.sum(w * (K1 * dphi + K2 * phi))
        gG0 = -d / c3[:, None]
        gGk = -(a * (1.0 + z) / c3)[:, None] * d
        q = (dny / (r * r))[:, None]
        gdG0 = (ny - 3.0 * q * d) / c3[:, None]
        gdGk = (a / c3)[:, None] * ((1.0 + z)[:, None] * ny - (3.0 + 3.0 * z + z * z)[:, None] * q * d)
        gK1 = gG0 - gGk
        gK2 = eps * gdGk - gdG0
        gR[k] = np.sum(w[:, None] * (gK1 * dphi[:, None] + gK2 * phi[:, None]), axis=0)
        frac[k] = -np.sum(w * dG0)
    return R, gR, frac


def reaction_terms(st, u, points, kappa, eps):
    """(R, grad R, solid-angle fraction) at each point, internal units."""
    y, ny, w, dphi, phi = surface_nodes(st, u)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    return node_sums(pts, y, ny, w, dphi, phi, kappa, eps)


def coulomb_terms(points, qpos, q, eps1):
    """(S1, grad S1) at each point: sum_k q_k G0(x, x_k) / eps1 and its gradient, charges
    closer than COINCIDENT left out."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    qpos = np.asarray(qpos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).ravel()
    S = np.zeros(pts.shape[0])
    gS = np.zeros((pts.shape[0], 3))
    for k in range(q.shape[0]):
        d = pts - qpos[k]
        r = np.linalg.norm(d, axis=1)
        use = r >= COINCIDENT
        rr = np.where(use, r, 1.0)
        S += np.where(use, q[k] / (FOUR_PI * rr), 0.0)
        gS += np.where(use, -q[k] / (FOUR_PI * rr ** 3), 0.0)[:, None] * d
    return S / eps1, gS / eps1


def potential_and_field(st, u, points, qpos, q, eps1, eps2, kappa):
    """Total potential and field at each point (internal units), with the parts:
    dict(phi, field, reac, reac_field, inside, frac)."""
    eps = eps2 / eps1
    R, gR, frac = reaction_terms(st, u, points, kappa, eps)
    S, gS = coulomb_terms(points, qpos, q, eps1)
    inside = frac > 0.5
    scale = np.where(inside, 1.0, 1.0 / eps)
    phi = scale * (S + R)
    grad = scale[:, None] * (gS + gR)
    return dict(phi=phi, field=-grad, reac=R, reac_field=-gR, inside=inside, frac=frac)
