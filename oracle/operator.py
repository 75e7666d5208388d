"""Discrete HOBI-PB operator: validation, setup, sources, matvec, solvation energy.

Unknowns (Section 2.2): u = (phi_1..phi_Nv, dphi_1..dphi_Nv) at the Nv vertices, in
internal units (the Green's functions carry their 1/(4 pi); phi in e/A).

The matrix-vector product is eqdbef3/eqdbef4 (regular triangles, 4-point Gauss-Radau)
plus eqdbef5/eqdbef6 (singular triangles, 16-point Gauss-Legendre with the Duffy map):

  (Au)_i      = 1/2 (1 + eps) phi_i
                - sum_{j not incident to i} sum_m sum_n W_jmn [K1 dphi_jn + K2 phi_jn]
                - sum_{j incident to i}     sum_m sum_n W_jmn [K1 dphi_jn + K2 phi_jn]
  (Au)_{i+Nv} = 1/2 (1 + 1/eps) dphi_i  - (the same sums with K3, K4)

Readings (the paper is ambiguous here):
* the diagonal term printed in both the regular and the singular formula is counted
  once;
* "regular triangles of vertex i" = every triangle that does not have i as a vertex;
  the singular ones are those that do (Section 2.3, first paragraph);
* W_jmn = w_m J_j(r_m, s_m) L_n(r_m, s_m) with L the linear barycentric weights of the
  three vertex unknowns (the unknowns live only at vertices, Section 2.2);
* the target normal n_x at vertex i is the input vertex normal;
* the source terms carry 1/eps1 (eq. eq1 has eps1 on its left side):
  S1 = (1/eps1) sum_k q_k G0(x, x_k), S2 = (1/eps1) sum_k q_k dG0(x, x_k)/dnx;
* a singular triangle is re-labelled cyclically so that vertex i is its local vertex 1,
  re-using the 10 nodes built in the stored order.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import COULOMB_KCAL, FOUR_PI
from .geometry import GeometryError, eval_patch, patch_nodes, rotate_nodes
from .kernels import kernels, kernels_12
from .quadrature import duffy_gauss_legendre, gauss_radau_triangle


class MeshError(ValueError):
    pass


class ChargeOutsideError(ValueError):
    pass


def validate_mesh(xyz, nrm, tri):
    """Closed, consistently oriented 2-manifold with unit normals; returns normals.

    Every directed edge must occur exactly once and its reverse exactly once; every
    triangle must be non-degenerate; every triangle must be counter-clockwise with respect
    to the sum of its vertex normals (the outward normals of the surface statement, Section
    2.2); normals must be unit to 1e-6 (they are then renormalised).
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    nrm = np.asarray(nrm, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    nv = xyz.shape[0]
    if xyz.ndim != 2 or xyz.shape[1] != 3 or nrm.shape != xyz.shape:
        raise MeshError("xyz/nrm must be [nv,3]")
    if tri.ndim != 2 or tri.shape[1] != 3 or tri.shape[0] < 4:
        raise MeshError("tri must be [nf,3] with nf >= 4")
    if not (np.all(np.isfinite(xyz)) and np.all(np.isfinite(nrm))):
        raise MeshError("non-finite input")
    if tri.min() < 0 or tri.max() >= nv:
        raise MeshError("vertex index out of range")
    ln = np.linalg.norm(nrm, axis=1)
    if np.any(np.abs(ln - 1.0) > 1e-6):
        raise MeshError("normals are not unit length")
    nrm = nrm / ln[:, None]
    edges = {}
    for t, (a, b, c) in enumerate(tri):
        if a == b or b == c or a == c:
            raise MeshError("repeated vertex in triangle")
        for e in ((a, b), (b, c), (c, a)):
            if e in edges:
                raise MeshError("directed edge used twice (non-manifold or misoriented)")
            edges[e] = t
    for (a, b) in edges:
        if (b, a) not in edges:
            raise MeshError("open edge")
    used = np.zeros(nv, dtype=bool)
    used[tri.ravel()] = True
    if not used.all():
        raise MeshError("unreferenced vertex")
    A, B, C = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(B - A, C - A)
    area2 = np.linalg.norm(cr, axis=1)
    scale = np.maximum(np.linalg.norm(B - A, axis=1), np.linalg.norm(C - A, axis=1)) ** 2
    if np.any(area2 <= 1e-12 * scale):
        raise MeshError("degenerate triangle")
    ns = nrm[tri[:, 0]] + nrm[tri[:, 1]] + nrm[tri[:, 2]]
    disagree = int(np.count_nonzero(np.einsum("ij,ij->i", cr, ns) <= 0.0))
    if disagree > 0:
        raise MeshError(f"orientation of {disagree} triangles disagrees with their vertex normals")
    return nrm


@dataclasses.dataclass
class Setup:
    xyz: np.ndarray       # [nv,3] targets
    nrm: np.ndarray       # [nv,3] target normals (unit)
    tri: np.ndarray       # [nf,3]
    patch: np.ndarray     # [nf,10,3] curved-element nodes
    y: np.ndarray         # [nf,4,3] regular quadrature nodes
    ny: np.ndarray        # [nf,4,3] node normals
    w: np.ndarray         # [nf,4] w_m * J
    L: np.ndarray         # [4,3] linear interpolation weights at the regular nodes
    ys: np.ndarray        # [nf,3,16,3] singular nodes, per local singular vertex k
    nys: np.ndarray       # [nf,3,16,3]
    ws: np.ndarray        # [nf,3,16] w * x * J
    Ls: np.ndarray        # [16,3] linear weights in the rotated frame
    incident: list        # incident[i] = sorted triangle ids having vertex i

    @property
    def nv(self):
        return self.xyz.shape[0]

    @property
    def nf(self):
        return self.tri.shape[0]


def setup(xyz, nrm, tri, ngl: int = 4) -> Setup:
    """Routines (2)-(4) of Section 2.6: curve the triangles, store the quadrature data."""
    xyz = np.asarray(xyz, dtype=np.float64)
    nrm = validate_mesh(xyz, nrm, tri)
    tri = np.asarray(tri, dtype=np.int64)
    nf = tri.shape[0]
    rr, ss, ww = gauss_radau_triangle()
    rd, sd, wd = duffy_gauss_legendre(ngl)
    nsg = rd.shape[0]
    X = xyz[tri]                     # [nf,3,3] stored vertex order
    N = nrm[tri]
    try:
        patch = patch_nodes(X, N)    # [nf,10,3]
    except GeometryError as e:
        raise MeshError(str(e)) from e
    y = np.empty((nf, 4, 3))
    ny = np.empty((nf, 4, 3))
    w = np.empty((nf, 4))
    for m in range(4):
        x, J, n = eval_patch(patch, rr[m], ss[m])
        y[:, m], ny[:, m], w[:, m] = x, n, ww[m] * J
    ys = np.empty((nf, 3, nsg, 3))
    nys = np.empty((nf, 3, nsg, 3))
    ws = np.empty((nf, 3, nsg))
    for k in range(3):
        rot = rotate_nodes(patch, k)
        for m in range(nsg):
            x, J, n = eval_patch(rot, rd[m], sd[m])
            ys[:, k, m], nys[:, k, m], ws[:, k, m] = x, n, wd[m] * J
    L = np.stack([1.0 - rr - ss, rr, ss], axis=1)
    Ls = np.stack([1.0 - rd - sd, rd, sd], axis=1)
    incident = [[] for _ in range(xyz.shape[0])]
    for j in range(nf):
        for v in tri[j]:
            incident[v].append(j)
    return Setup(xyz, nrm, tri, patch, y, ny, w, L, ys, nys, ws, Ls, incident)


def sources(xyz, nrm, qpos, q, eps1):
    """S1, S2 at the vertices (eq. Eq_Ss, with the 1/eps1 reading)."""
    S1 = np.zeros(xyz.shape[0])
    S2 = np.zeros(xyz.shape[0])
    for k in range(q.shape[0]):
        d = xyz - qpos[k]
        r = np.linalg.norm(d, axis=1)
        S1 += q[k] / (FOUR_PI * r)
        S2 += -q[k] * np.einsum("ij,ij->i", d, nrm) / (FOUR_PI * r ** 3)
    return S1 / eps1, S2 / eps1


def _row(st: Setup, i, phi, dphi, kappa, eps):
    """Integral part of rows i and i+Nv: (sum of K1/K2 terms, sum of K3/K4 terms)."""
    x, nx = st.xyz[i], st.nrm[i]
    inc = st.incident[i]
    reg = np.ones(st.nf, dtype=bool)
    reg[inc] = False
    # regular triangles, 4-point rule (eqdbef3, eqdbef4)
    tv = st.tri[reg]                            # [M,3]
    K1, K2, K3, K4 = kernels(x, nx, st.y[reg], st.ny[reg], kappa, eps)   # [M,4]
    dphi_m = dphi[tv] @ st.L.T                  # [M,4] interpolated at the nodes
    phi_m = phi[tv] @ st.L.T
    W = st.w[reg]
    s1 = np.sum(W * (K1 * dphi_m + K2 * phi_m))
    s2 = np.sum(W * (K3 * dphi_m + K4 * phi_m))
    # singular triangles, Duffy + Gauss-Legendre (eqdbef5, eqdbef6)
    for j in inc:
        k = int(np.nonzero(st.tri[j] == i)[0][0])
        verts = st.tri[j][[k, (k + 1) % 3, (k + 2) % 3]]
        K1, K2, K3, K4 = kernels(x, nx, st.ys[j, k], st.nys[j, k], kappa, eps)
        dphi_m = st.Ls @ dphi[verts]
        phi_m = st.Ls @ phi[verts]
        W = st.ws[j, k]
        s1 += np.sum(W * (K1 * dphi_m + K2 * phi_m))
        s2 += np.sum(W * (K3 * dphi_m + K4 * phi_m))
    return s1, s2


_POOL_STATE = {}


def _rows_worker(args):
    lo, hi = args
    st, phi, dphi, kappa, eps = _POOL_STATE["job"]
    return [_row(st, i, phi, dphi, kappa, eps) for i in range(lo, hi)]


def _integral_rows(st, phi, dphi, kappa, eps, rows, workers):
    """(s1, s2) for each row; optionally spread over forked worker processes."""
    if workers <= 1 or len(rows) < 64:
        return [_row(st, i, phi, dphi, kappa, eps) for i in rows]
    import multiprocessing as mp
    _POOL_STATE["job"] = (st, phi, dphi, kappa, eps)
    rows = list(rows)
    step = max(1, len(rows) // (4 * workers))
    spans = [(rows[a], rows[min(a + step, len(rows)) - 1] + 1) for a in range(0, len(rows), step)]
    contiguous = all(rows[i + 1] == rows[i] + 1 for i in range(len(rows) - 1))
    if not contiguous:
        return [_row(st, i, phi, dphi, kappa, eps) for i in rows]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_rows_worker, spans)
    _POOL_STATE.clear()
    return [v for p in parts for v in p]


def diagonal(st: Setup, kappa, eps):
    """The diagonal of A (eqdbef3/eqdbef4): 1/2 (1 + eps) and 1/2 (1 + 1/eps) minus each vertex's
    singular terms on its own unknowns (K2 on phi_i in row i, K3 on dphi_i in row i + Nv, over
    its incident triangles with the Duffy rule).  The regular sum does not touch a vertex's
    own unknowns: they enter only the nodes of its incident triangles, which are singular."""
    nv = st.nv
    d = np.concatenate([np.full(nv, 0.5 * (1.0 + eps)), np.full(nv, 0.5 * (1.0 + 1.0 / eps))])
    for i in range(nv):
        x, nx = st.xyz[i], st.nrm[i]
        for j in st.incident[i]:
            k = int(np.nonzero(st.tri[j] == i)[0][0])
            _, K2, K3, _ = kernels(x, nx, st.ys[j, k], st.nys[j, k], kappa, eps)
            W = st.ws[j, k] * st.Ls[:, 0]           # weight of the target's own (local 0) unknown
            d[i] -= np.sum(W * K2)
            d[nv + i] -= np.sum(W * K3)
    # a non-positive entry (not met on the surfaces tried) is replaced by the row block's constant
    const = np.concatenate([np.full(nv, 0.5 * (1.0 + eps)), np.full(nv, 0.5 * (1.0 + 1.0 / eps))])
    return np.where(np.isfinite(d) & (d > 0.0), d, const)


def matvec(st: Setup, u, kappa, eps, rows=None, workers: int = 1):
    """y = A u (all 2Nv rows), or the pair (rows i, i+Nv) for each i in ``rows``."""
    nv = st.nv
    u = np.asarray(u, dtype=np.float64)
    phi, dphi = u[:nv], u[nv:]
    idx = np.arange(nv) if rows is None else np.asarray(rows)
    sums = _integral_rows(st, phi, dphi, kappa, eps, [int(i) for i in idx], workers)
    s1 = np.array([a for a, _ in sums])
    s2 = np.array([b for _, b in sums])
    top = 0.5 * (1.0 + eps) * phi[idx] - s1
    bot = 0.5 * (1.0 + 1.0 / eps) * dphi[idx] - s2
    if rows is None:
        return np.concatenate([top, bot])
    return np.stack([top, bot])


def reaction_potential(st: Setup, u, points, kappa, eps):
    """phi_reac at interior points: the integral of eq. solvation_energy, regular rule on
    every triangle (the charges are inside, so no triangle is singular for them)."""
    nv = st.nv
    phi, dphi = u[:nv], u[nv:]
    dphi_m = dphi[st.tri] @ st.L.T
    phi_m = phi[st.tri] @ st.L.T
    out = np.empty(points.shape[0])
    for k in range(points.shape[0]):
        K1, K2 = kernels_12(points[k], st.y, st.ny, kappa, eps)
        out[k] = np.sum(st.w * (K1 * dphi_m + K2 * phi_m))
    return out


def solvation_energy(st: Setup, u, qpos, q, kappa, eps):
    """E_sol = 1/2 sum_k q_k phi_reac(x_k), converted to kcal/mol."""
    pr = reaction_potential(st, u, qpos, kappa, eps)
    return 0.5 * FOUR_PI * COULOMB_KCAL * float(np.sum(q * pr))


def solid_angle_fraction(st: Setup, points):
    """-sum over all regular nodes of w dG0/dny at each point: 1 inside, 0 outside."""
    out = np.empty(points.shape[0])
    for k in range(points.shape[0]):
        d = points[k] - st.y
        r = np.linalg.norm(d, axis=-1)
        out[k] = -np.sum(st.w * np.sum(d * st.ny, axis=-1) / (FOUR_PI * r ** 3))
    return out


def check_charges_inside(st: Setup, qpos):
    frac = solid_angle_fraction(st, qpos)
    if np.any(frac < 0.5):
        raise ChargeOutsideError("charge outside the surface")
    return frac


def dense_matrix(st: Setup, kappa, eps):
    """Assemble A column by column (A e_1 ... A e_2Nv); only for tiny meshes."""
    n = 2 * st.nv
    A = np.empty((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        A[:, c] = matvec(st, e, kappa, eps)
    return A
