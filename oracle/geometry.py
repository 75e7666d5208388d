"""Flat to curved triangles (Section 2.2), written out step by step in FP64.

The paper's construction, in its order:

1. Every straight edge between two vertices is replaced by a cubic arc
   x(t) = c0 + c1 t + c2 t^2 + c3 t^3 fixed by the two end points and their unit
   normals.  Reading (the paper gives the 12 conditions but not the tangent lengths):
   the arc is the cubic Hermite curve whose end tangents lie in the tangent planes of
   the end normals, along the projection of the chord d = Q - P, with common length
   m = 2|d| / (1 + cos(theta/2)), cos(theta) = nP . nQ.  On a circular arc this is the
   4 R tan(theta/4) tangent of the best cubic circle approximation.
2. The normal along an arc (eq. eqcurvature is garbled and undefined at inflexions).
   Reading: the linear blend (1-t) nP + t nQ projected orthogonal to the arc's tangent
   and normalised.  For a planar arc this is the principal normal the paper asks for.
3. The constructive point map (eq. eqrs2uv and the three steps after it): (r, s) ->
   u = r + s, v = s / (r + s); Y1 on arc X1X2 and Y2 on arc X1X3 at parameter u (with
   their normals); the point is the arc Y1Y2 at parameter v.
4. The 10-point interpolated element (eq. eqintepolation): the map is applied at the
   10 lattice points (i/3, j/3) of the unit right triangle and the patch is the cubic
   Lagrange interpolant x(r, s) = sum_k N_k(r, s) x_k.  Reading: the standard P3
   Lagrange basis (the Zauhar-Morgan table the paper refers to is not available).
5. Quadrature data (Section 2.2): J = |x_r x x_s| and the node normal (x_r x x_s)/J.

Nodes are stored in the order of their barycentric multi-indices ``ALPHA`` below;
(r, s) = (alpha_2 / 3, alpha_3 / 3).
"""
from __future__ import annotations

import numpy as np


class GeometryError(ValueError):
    """Raised when the curved-edge construction is undefined (e.g. normal along edge)."""


# Barycentric multi-indices (a1, a2, a3), a1 + a2 + a3 = 3, for L = (1-r-s, r, s).
ALPHA = np.array([
    [3, 0, 0], [0, 3, 0], [0, 0, 3],      # vertices X1, X2, X3
    [2, 1, 0], [1, 2, 0],                 # edge X1X2 at r = 1/3, 2/3
    [2, 0, 1], [1, 0, 2],                 # edge X1X3 at s = 1/3, 2/3
    [0, 2, 1], [0, 1, 2],                 # edge X2X3
    [1, 1, 1],                            # centroid
], dtype=np.int64)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _dot(a, b):
    return np.sum(a * b, axis=-1, keepdims=True)


def arc_coefficients(P, nP, Q, nQ):
    """Coefficients c0..c3 of the cubic arc from P (normal nP) to Q (normal nQ).

    All arguments are [..., 3] arrays; the arcs are built independently.
    """
    P, nP, Q, nQ = (np.asarray(a, dtype=np.float64) for a in (P, nP, Q, nQ))
    d = Q - P
    ell = np.linalg.norm(d, axis=-1, keepdims=True)
    if not np.all(ell > 0.0):
        raise GeometryError("zero-length arc")
    c = np.clip(_dot(nP, nQ), -1.0, 1.0)
    m = 2.0 * ell / (1.0 + np.sqrt((1.0 + c) / 2.0))
    tP = d - _dot(d, nP) * nP
    tQ = d - _dot(d, nQ) * nQ
    if np.any(np.linalg.norm(tP, axis=-1, keepdims=True) < 1e-12 * ell) or \
            np.any(np.linalg.norm(tQ, axis=-1, keepdims=True) < 1e-12 * ell):
        raise GeometryError("vertex normal parallel to an edge chord")
    TP = m * _unit(tP)
    TQ = m * _unit(tQ)
    return P, TP, 3.0 * d - 2.0 * TP - TQ, TP + TQ - 2.0 * d


def arc_point(P, nP, Q, nQ, t):
    """Point and unit normal at parameter t in [0, 1] (a scalar) on the arcs P -> Q."""
    P, nP, Q, nQ = (np.asarray(a, dtype=np.float64) for a in (P, nP, Q, nQ))
    if t == 0.0:
        return P.copy(), nP.copy()
    if t == 1.0:
        return Q.copy(), nQ.copy()
    c0, c1, c2, c3 = arc_coefficients(P, nP, Q, nQ)
    x = c0 + c1 * t + c2 * t * t + c3 * t * t * t
    dx = c1 + 2.0 * c2 * t + 3.0 * c3 * t * t
    tau = _unit(dx)
    nb = (1.0 - t) * nP + t * nQ
    n = _unit(nb - _dot(nb, tau) * tau)
    return x, n


def point_map(X, N, r, s):
    """The constructive map (r, s) -> point on the curved element (Section 2.2, 3 steps).

    X, N: [..., 3, 3] vertex positions and unit normals in each triangle's stored
    order; (r, s) scalars.  Returns [..., 3].
    """
    X = np.asarray(X, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    if r == 0.0 and s == 0.0:
        return X[..., 0, :].copy()
    u = r + s
    v = s / (r + s)
    Y1, nY1 = arc_point(X[..., 0, :], N[..., 0, :], X[..., 1, :], N[..., 1, :], u)
    Y2, nY2 = arc_point(X[..., 0, :], N[..., 0, :], X[..., 2, :], N[..., 2, :], u)
    x, _ = arc_point(Y1, nY1, Y2, nY2, v)
    return x


def patch_nodes(X, N):
    """The 10 nodes x_k of each curved element, in ``ALPHA`` order ([..., 10, 3])."""
    X = np.asarray(X, dtype=np.float64)
    out = np.empty(X.shape[:-2] + (10, 3))
    for k, a in enumerate(ALPHA):
        if a[0] == 3:
            out[..., k, :] = X[..., 0, :]
        elif a[1] == 3:
            out[..., k, :] = X[..., 1, :]
        elif a[2] == 3:
            out[..., k, :] = X[..., 2, :]
        else:
            out[..., k, :] = point_map(X, N, a[1] / 3.0, a[2] / 3.0)
    return out


def p3_basis(r, s):
    """Cubic Lagrange basis on the 10 lattice nodes: N, dN/dr, dN/ds, each [10].

    N_alpha = prod_b prod_{p < alpha_b} (3 L_b - p) / (p + 1), L = (1 - r - s, r, s);
    d/dr = d/dL2 - d/dL1 and d/ds = d/dL3 - d/dL1.
    """
    L = np.array([1.0 - r - s, r, s])
    val = np.ones(10)
    dL = np.zeros((10, 3))
    for k, a in enumerate(ALPHA):
        factors = []   # per barycentric b: (value, derivative wrt L_b)
        for b in range(3):
            f, df = 1.0, 0.0
            for p in range(a[b]):
                g = (3.0 * L[b] - p) / (p + 1.0)
                dg = 3.0 / (p + 1.0)
                f, df = f * g, df * g + f * dg
            factors.append((f, df))
        val[k] = factors[0][0] * factors[1][0] * factors[2][0]
        dL[k, 0] = factors[0][1] * factors[1][0] * factors[2][0]
        dL[k, 1] = factors[0][0] * factors[1][1] * factors[2][0]
        dL[k, 2] = factors[0][0] * factors[1][0] * factors[2][1]
    return val, dL[:, 1] - dL[:, 0], dL[:, 2] - dL[:, 0]


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def eval_patch(nodes10, r, s):
    """Position, Jacobian J = |x_r x x_s| and unit normal of the patches at (r, s).

    nodes10: [..., 10, 3]; (r, s) scalars.
    """
    Nv, Nr, Ns = p3_basis(r, s)
    x = np.einsum("k,...kc->...c", Nv, nodes10)
    xr = np.einsum("k,...kc->...c", Nr, nodes10)
    xs = np.einsum("k,...kc->...c", Ns, nodes10)
    c = _cross(xr, xs)
    J = np.linalg.norm(c, axis=-1)
    return x, J, c / J[..., None]


def rotate_nodes(nodes10, k):
    """Relabel the element so that its stored vertex k becomes local vertex 1.

    The cubic patch is the same surface; only the barycentric labels rotate
    cyclically (new L'_b = L_{(k + b) mod 3}).
    """
    lookup = {tuple(a): i for i, a in enumerate(ALPHA)}
    perm = []
    for a in ALPHA:
        stored = [0, 0, 0]
        for b in range(3):
            stored[(k + b) % 3] = a[b]
        perm.append(lookup[tuple(stored)])
    return nodes10[..., perm, :]
