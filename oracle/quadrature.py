"""Quadrature rules on the unit right triangle T = {r, s >= 0, r + s <= 1} (area 1/2).

* Regular triangles: the 4-point Gauss-Radau rule (Section 2.2, N_GR = 4).  The paper
  cites Akin's table, which is not available; the reading used here is the collapsed
  (Duffy/Stroud) product rule anchored at local vertex 1: in the collapsed coordinates
  (u, v) with r = u(1 - v), s = u v, dr ds = u du dv, the u-direction uses the 2-point
  Gauss-Jacobi rule for the weight u on [0, 1] (the interior nodes of the 3-point
  Radau rule) and the v-direction the 2-point Gauss-Legendre rule.  Exact for all
  polynomials of degree <= 3.
* Singular triangles: the tensor product of N_GL-point Gauss-Legendre rules on the unit
  square with the map r = (1 - y) x, s = y x whose Jacobian is x (Section 2.3; the
  printed domain "0 <= x,y <= 0" is read as [0,1]^2).  This map sends the whole edge
  x = 0 to the singular vertex (r,s) = (0,0) and cancels an O(1/|x - y|) singularity.
"""
from __future__ import annotations

import numpy as np
import scipy.special


def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre nodes and weights on [0, 1] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_jacobi_u_01(n: int):
    """n-point Gauss rule on [0, 1] for the weight function u (weights sum to 1/2)."""
    # shifted Jacobi weight (1-x)^(p-q) x^(q-1) with p = q = 2  ->  weight x
    x, w = scipy.special.roots_sh_jacobi(n, 2.0, 2.0)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def gauss_radau_triangle():
    """The 4-point regular-triangle rule: arrays r[4], s[4], w[4] with sum(w) = 1/2.

    Node order: u outer, v inner, i.e. (u0,v0), (u0,v1), (u1,v0), (u1,v1).
    """
    u, wu = gauss_jacobi_u_01(2)
    v, wv = gauss_legendre_01(2)
    r, s, w = [], [], []
    for a in range(2):
        for b in range(2):
            r.append(u[a] * (1.0 - v[b]))
            s.append(u[a] * v[b])
            w.append(wu[a] * wv[b])
    return np.array(r), np.array(s), np.array(w)


def duffy_gauss_legendre(ngl: int = 4):
    """The singular-triangle rule: (ngl^2) nodes r = (1-y)x, s = yx, weight gx*gy*x.

    The singular point is the local vertex (r, s) = (0, 0).  Node order: x outer, y inner.
    """
    g, gw = gauss_legendre_01(ngl)
    r, s, w = [], [], []
    for a in range(ngl):
        for b in range(ngl):
            x, y = g[a], g[b]
            r.append((1.0 - y) * x)
            s.append(y * x)
            w.append(gw[a] * gw[b] * x)
    return np.array(r), np.array(s), np.array(w)
