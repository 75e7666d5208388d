"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only produces data: surface meshes with vertex normals and charge sets.
It contains none of the boundary-integral arithmetic (no kernels, no quadrature, no
curved patches), so that the oracle and the HIP path can both consume its output
without sharing any of the method's code.

Workloads (the paper's datasets -- MSMS surfaces of protein 1ajj and CHARMM22 charges --
are not available, so seeded synthetic stand-ins with the same structure are used):

* ``icosphere``: uniform icosahedral triangulation projected to a sphere, with exact
  sphere normals at the vertices (the "ico" triangulation the paper uses for its
  spherical-cavity tests, Section 3.3).
* ``kirkwood_centered``: one +1 e charge at the centre of a 2 A sphere (the spherical
  cavity test of Section 3.2, Table 1).
* ``kirkwood_offcenter``: 8 charges in r < 2.5 A inside a 4 A sphere, seeded.
* ``molecule``: protein-like surface made of packed atoms (see ``molecule_surface``).
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np


@dataclasses.dataclass
class Problem:
    """One solve request: surface, charges and dielectric constants."""

    xyz: np.ndarray      # [nv, 3] float64, vertex positions (A)
    nrm: np.ndarray      # [nv, 3] float64, unit outward vertex normals
    tri: np.ndarray      # [nf, 3] int32, counter-clockwise seen from outside
    qpos: np.ndarray     # [nc, 3] float64, charge positions (A)
    q: np.ndarray        # [nc] float64, charges (e)
    eps1: float = 1.0
    eps2: float = 80.0
    kappa: float = 0.1257
    name: str = ""

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nf(self) -> int:
        return int(self.tri.shape[0])

    @property
    def nc(self) -> int:
        return int(self.q.shape[0])


# --------------------------------------------------------------------------------------
# Icosahedral triangulation
# --------------------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Icosphere with 20*4**level triangles and 10*4**level+2 vertices.

    Each subdivision splits every triangle into four through its edge midpoints, which
    are pushed out to the unit sphere.  Returns (xyz, nrm, tri) with exact sphere
    normals and counter-clockwise triangles seen from outside.
    """
    v, f = _icosahedron()
    for _ in range(level):
        verts = list(v)
        cache: dict = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = verts[a] + verts[b]
                m = m / np.linalg.norm(m)
                idx = len(verts)
                verts.append(m)
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        v = np.array(verts)
        f = np.array(nf, dtype=np.int64)
    nrm = v / np.linalg.norm(v, axis=1, keepdims=True)
    xyz = nrm * radius + np.asarray(center, dtype=np.float64)
    # orient counter-clockwise seen from outside
    a, b, c = xyz[f[:, 0]], xyz[f[:, 1]], xyz[f[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c - 3 * np.asarray(center))
    f[s < 0] = f[s < 0][:, ::-1]
    return xyz, nrm.copy(), f.astype(np.int32)


# --------------------------------------------------------------------------------------
# Kirkwood sphere workloads
# --------------------------------------------------------------------------------------

def kirkwood_centered(level: int = 3, radius: float = 2.0, kappa: float = 0.1257,
                      eps1: float = 1.0, eps2: float = 80.0) -> Problem:
    """Unit charge at the centre of a sphere (Section 3.2 spherical cavity)."""
    xyz, nrm, tri = icosphere(level, radius)
    return Problem(xyz, nrm, tri, np.zeros((1, 3)), np.ones(1), eps1, eps2, kappa,
                   name=f"kirkwood_centered_L{level}")


def offcenter_charges(n: int = 8, rmax: float = 2.5, seed: int = 2):
    """n charges uniform in the ball r < rmax, |q| ~ U[0.1, 1.0] with a random sign."""
    rng = np.random.default_rng(seed)
    pos = []
    while len(pos) < n:
        c = rng.uniform(-rmax, rmax, size=3)
        if np.dot(c, c) < rmax * rmax:
            pos.append(c)
    mag = rng.uniform(0.1, 1.0, size=n)
    sgn = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    return np.array(pos), mag * sgn


def kirkwood_offcenter(level: int = 3, radius: float = 4.0, kappa: float = 0.1257,
                       eps1: float = 1.0, eps2: float = 80.0, seed: int = 2,
                       nq: int = 8) -> Problem:
    """Eight seeded charges inside a 4 A sphere (eccentric-charge test, Section 3.3)."""
    xyz, nrm, tri = icosphere(level, radius)
    qpos, q = offcenter_charges(nq, 2.5, seed)
    return Problem(xyz, nrm, tri, qpos, q, eps1, eps2, kappa,
                   name=f"kirkwood_offcenter_L{level}")


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded random FP64 vector (e.g. a matvec input)."""
    return np.random.default_rng(seed).standard_normal(n)


# --------------------------------------------------------------------------------------
# Protein-like synthetic molecules: packed atoms, Gaussian density, marching tetrahedra
# --------------------------------------------------------------------------------------

DENSITY_DECAY = 2.3


def pack_atoms(n: int, ball_radius: float, seed: int, min_spacing: float = 1.4,
               radius_range=(1.2, 2.0), charge_sigma: float = 0.4, max_tries: int = 10_000_000):
    """Random sequential addition of n atom centres in a ball (rejecting candidates closer
    than ``min_spacing`` to an accepted centre), radii ~ U(radius_range), partial charges
    ~ N(0, charge_sigma) shifted so that the net charge is an integer."""
    rng = np.random.default_rng(seed)
    cell = min_spacing
    grid: dict = {}
    centers = []
    tries = 0
    R2 = ball_radius * ball_radius
    while len(centers) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("packing did not finish")
        c = rng.uniform(-ball_radius, ball_radius, size=3)
        if np.dot(c, c) > R2:
            continue
        key = tuple(np.floor(c / cell).astype(int))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        d = c - centers[j]
                        if np.dot(d, d) < min_spacing * min_spacing:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            grid.setdefault(key, []).append(len(centers))
            centers.append(c)
    centers = np.array(centers)
    radii = rng.uniform(radius_range[0], radius_range[1], size=n)
    q = rng.normal(0.0, charge_sigma, size=n)
    q -= (q.sum() - np.round(q.sum())) / n
    return centers, radii, q


class _AtomGrid:
    """Cell list of atoms for evaluating the density and its gradient at points."""

    def __init__(self, centers, radii, decay=DENSITY_DECAY, tol=1e-10):
        self.c = centers
        self.r = radii
        self.decay = decay
        # exp(-decay (d^2/r^2 - 1)) < tol beyond d = r sqrt(1 + ln(1/tol)/decay)
        self.cut = float(np.max(radii) * np.sqrt(1.0 + np.log(1.0 / tol) / decay))
        self.cell = self.cut
        self.lo = centers.min(axis=0) - self.cut
        keys = np.floor((centers - self.lo) / self.cell).astype(np.int64)
        self.cells: dict = {}
        for i, k in enumerate(map(tuple, keys)):
            self.cells.setdefault(k, []).append(i)

    def eval(self, pts, grad=False):
        pts = np.asarray(pts, dtype=np.float64)
        rho = np.zeros(pts.shape[0])
        g = np.zeros_like(pts) if grad else None
        keys = np.floor((pts - self.lo) / self.cell).astype(np.int64)
        order = np.lexsort(keys.T[::-1])
        ks = keys[order]
        bounds = np.flatnonzero(np.any(np.diff(ks, axis=0) != 0, axis=1)) + 1
        starts = np.r_[0, bounds]
        ends = np.r_[bounds, len(order)]
        for s, e in zip(starts, ends):
            k = ks[s]
            idx = order[s:e]
            atoms = []
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        atoms += self.cells.get((k[0] + dx, k[1] + dy, k[2] + dz), [])
            if not atoms:
                continue
            atoms = np.array(atoms)
            d = pts[idx, None, :] - self.c[None, atoms, :]
            r2 = self.r[atoms] ** 2
            w = np.exp(-self.decay * (np.sum(d * d, axis=-1) / r2 - 1.0))
            rho[idx] = w.sum(axis=1)
            if grad:
                g[idx] = np.einsum("pa,pac->pc", -2.0 * self.decay * w / r2, d)
        return (rho, g) if grad else rho


# the six tetrahedra of a cube along its main diagonal (one per axis permutation): a
# consistent split, so neighbouring cubes cut their shared faces the same way
_KUHN = []
for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
    p = [np.zeros(3, dtype=np.int64)]
    for ax in perm:
        q_ = p[-1].copy()
        q_[ax] += 1
        p.append(q_)
    _KUHN.append(np.array(p))


def _tet_table():
    """Per sign pattern (bit a set = local vertex a inside): list of triangles as triples
    of tet edges (pairs of local vertices), and one (inside, outside) vertex pair used to
    orient them."""
    table = {}
    for mask in range(16):
        inside = [a for a in range(4) if mask >> a & 1]
        outside = [a for a in range(4) if not mask >> a & 1]
        if len(inside) in (0, 4):
            table[mask] = ([], None)
        elif len(inside) in (1, 3):
            lone = inside[0] if len(inside) == 1 else outside[0]
            others = [a for a in range(4) if a != lone]
            tris = [[(lone, others[0]), (lone, others[1]), (lone, others[2])]]
            ref = (inside[0], outside[0])
            table[mask] = (tris, ref)
        else:
            a, b = inside
            c, d = outside
            tris = [[(a, c), (a, d), (b, d)], [(a, c), (b, d), (b, c)]]
            table[mask] = (tris, (a, c))
    return table


_TET_TABLE = _tet_table()


def marching_tetrahedra(func, lo, h, shape, iso_shift=1e-9):
    """Watertight triangulation of {func > 0} on the grid lo + h * (i, j, k).

    func: callable on [n, 3] points -> values (positive inside).  Returns (verts, tris,
    edge_keys) with triangles oriented so that their normals point outside.
    """
    nx, ny, nz = shape
    gx = lo[0] + h * np.arange(nx)
    gy = lo[1] + h * np.arange(ny)
    gz = lo[2] + h * np.arange(nz)
    vals = np.empty(shape)
    for i in range(nx):
        P = np.stack(np.meshgrid(np.full(1, gx[i]), gy, gz, indexing="ij"), axis=-1).reshape(-1, 3)
        vals[i] = func(P).reshape(ny, nz)
    # keep grid values off the iso level so that no crossing sits exactly on a grid point
    vals = np.where(np.abs(vals) < iso_shift, np.where(vals < 0, -iso_shift, iso_shift), vals)
    gid = lambda i, j, k: (i * ny + j) * nz + k
    I, J, K = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    edge_a, edge_b, tri_edges_all = [], [], []
    n_edges_total = 0
    tri_list = []
    for tet in _KUHN:
        cid = [gid(I + t[0], J + t[1], K + t[2]) for t in tet]              # 4 x ncube
        fv = [vals.ravel()[c] for c in cid]
        mask = sum((fv[a] > 0).astype(np.int64) << a for a in range(4))
        for m in range(1, 15):
            tris, ref = _TET_TABLE[m]
            sel = np.flatnonzero(mask == m)
            if sel.size == 0:
                continue
            for tri in tris:
                ids = []
                for (a, b) in tri:
                    ga, gb = cid[a][sel], cid[b][sel]
                    ids.append(np.stack([np.minimum(ga, gb), np.maximum(ga, gb)], axis=1))
                ia, ib = ref
                tri_list.append((np.stack(ids, axis=1), cid[ia][sel], cid[ib][sel]))
    edges = np.concatenate([t[0].reshape(-1, 2) for t in tri_list])
    uniq, inv = np.unique(edges, axis=0, return_inverse=True)
    inv = inv.ravel()
    fa = vals.ravel()[uniq[:, 0]]
    fb = vals.ravel()[uniq[:, 1]]
    t = fa / (fa - fb)

    def coords(g):
        k = g % nz
        j = (g // nz) % ny
        i = g // (ny * nz)
        return np.stack([gx[i], gy[j], gz[k]], axis=1)

    pa, pb = coords(uniq[:, 0]), coords(uniq[:, 1])
    verts = pa + t[:, None] * (pb - pa)
    tris = inv.reshape(-1, 3)
    refin = np.concatenate([t_[1] for t_ in tri_list])
    refout = np.concatenate([t_[2] for t_ in tri_list])
    nrm = np.cross(verts[tris[:, 1]] - verts[tris[:, 0]], verts[tris[:, 2]] - verts[tris[:, 0]])
    flip = np.einsum("ij,ij->i", nrm, coords(refout) - coords(refin)) < 0
    tris[flip] = tris[flip][:, ::-1]
    return verts, tris, (uniq, pa, pb, fa, fb)


class _EdgeCollapser:
    """Edge collapses on a closed oriented triangle mesh.  An edge (u, v) may be merged into
    one point only when its end points share exactly the two vertices opposite to it (the
    link condition), so the mesh stays a closed 2-manifold."""

    def __init__(self, xyz, tri):
        self.xyz = np.array(xyz, dtype=np.float64)
        self.tri = [list(t) for t in np.asarray(tri)]
        self.vt = [set() for _ in range(self.xyz.shape[0])]
        for t, (a, b, c) in enumerate(self.tri):
            self.vt[a].add(t), self.vt[b].add(t), self.vt[c].add(t)
        self.alive = np.ones(len(self.tri), dtype=bool)

    def neigh(self, v):
        out = set()
        for t in self.vt[v]:
            out.update(self.tri[t])
        out.discard(v)
        return out

    def edges(self):
        live = np.asarray([t for t, ok in zip(self.tri, self.alive) if ok])
        E = np.concatenate([live[:, [i, (i + 1) % 3]] for i in range(3)])
        return np.unique(np.sort(E, axis=1), axis=0)

    def link_ok(self, u, v):
        shared = self.vt[u] & self.vt[v]
        if len(shared) != 2:
            return False
        opp = set()
        for t in shared:
            opp.update(self.tri[t])
        opp -= {u, v}
        return len(opp) == 2 and self.neigh(u) & self.neigh(v) == opp

    def ring(self, u, v):
        """Triangles that survive the collapse of (u, v) and change shape."""
        return (self.vt[u] | self.vt[v]) - (self.vt[u] & self.vt[v])

    def corners(self, t, u, v, p):
        return [p if w in (u, v) else self.xyz[w] for w in self.tri[t]]

    def collapse(self, u, v, p):
        for t in self.vt[u] & self.vt[v]:
            self.alive[t] = False
            for w in self.tri[t]:
                self.vt[w].discard(t)
        for t in list(self.vt[v]):
            self.tri[t] = [u if w == v else w for w in self.tri[t]]
            self.vt[u].add(t)
        self.vt[v] = set()
        self.xyz[u] = p

    def result(self):
        tri = np.asarray([t for t, ok in zip(self.tri, self.alive) if ok], dtype=np.int64)
        used = np.unique(tri)
        remap = -np.ones(self.xyz.shape[0], dtype=np.int64)
        remap[used] = np.arange(used.size)
        return self.xyz[used], remap[tri]


def collapse_short_edges(xyz, tri, min_len):
    """Removes edges shorter than ``min_len`` by merging their end points at the midpoint,
    when the link condition holds and no surviving triangle around the edge turns over.
    Returns (xyz, tri) with unused vertices dropped."""
    m = _EdgeCollapser(xyz, tri)

    def tnormal(P):
        return np.cross(P[1] - P[0], P[2] - P[0])

    changed = True
    while changed:
        changed = False
        E = m.edges()
        L = np.linalg.norm(m.xyz[E[:, 0]] - m.xyz[E[:, 1]], axis=1)
        order = np.argsort(L)
        order = order[L[order] < min_len]
        touched = set()
        for e in order:
            u, v = int(E[e, 0]), int(E[e, 1])
            if u in touched or v in touched or not m.link_ok(u, v):
                continue
            p = 0.5 * (m.xyz[u] + m.xyz[v])
            ok = True
            for t in m.ring(u, v):
                before = tnormal([m.xyz[w] for w in m.tri[t]])
                after = tnormal(m.corners(t, u, v, p))
                if np.dot(before, after) <= 0.0 or np.linalg.norm(after) <= 1e-12 * np.dot(before, before) ** 0.5:
                    ok = False
                    break
            if not ok:
                continue
            m.collapse(u, v, p)
            touched.update((u, v))
            touched.update(m.neigh(u))
            changed = True
    return m.result()


def _fold_cosine(verts, tri, nrm):
    """Smallest cosine between a triangle's face normal and its three vertex normals."""
    A, B, C = verts[tri[:, 0]], verts[tri[:, 1]], verts[tri[:, 2]]
    fn = np.cross(B - A, C - A)
    fn /= np.maximum(np.linalg.norm(fn, axis=1, keepdims=True), 1e-300)
    return np.min(np.stack([np.einsum("ij,ij->i", fn, nrm[tri[:, k]]) for k in range(3)], axis=1), axis=1)


def _surface_normals(ag, verts):
    _, g = ag.eval(verts, grad=True)
    return -g / np.linalg.norm(g, axis=1, keepdims=True)


def remove_folds(ag, verts, tri, cos_min: float = 0.3, passes: int = 6):
    """Removes folded triangles (face normal against a vertex normal, cosine below
    ``cos_min``: creases of the density narrower than the marching grid resolves).  Each
    pass first flips the edges of folded triangles where the flip raises the smaller fold
    cosine of the pair, then collapses the shortest edge of the folds left, at its midpoint
    moved onto rho = 1, when no triangle around it ends up below both ``cos_min`` and its
    old fold cosine."""
    verts = np.array(verts, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64).copy()
    for _ in range(passes):
        nrm = _surface_normals(ag, verts)
        fc = _fold_cosine(verts, tri, nrm)
        if fc.min() >= cos_min:
            break

        def fcos(a, b, c, P=None, N=None):
            return float(_fold_cosine(verts, np.array([[a, b, c]]), nrm)[0])

        # flips
        edge_of = {}
        for t, (a, b, c) in enumerate(tri):
            edge_of[(a, b)] = t
            edge_of[(b, c)] = t
            edge_of[(c, a)] = t
        for t1 in np.nonzero(fc < cos_min)[0]:
            best = None
            for k in range(3):
                a, b, c = tri[t1][k], tri[t1][(k + 1) % 3], tri[t1][(k + 2) % 3]
                t2 = edge_of.get((b, a))
                if t2 is None:
                    continue
                d = [w for w in tri[t2] if w != a and w != b][0]
                if c == d or (c, d) in edge_of or (d, c) in edge_of:
                    continue
                old = min(fcos(*tri[t1]), fcos(*tri[t2]))
                new = min(fcos(a, d, c), fcos(d, b, c))
                if new > old + 1e-3 and (best is None or new > best[0]):
                    best = (new, a, b, c, d, t2)
            if best is None:
                continue
            _, a, b, c, d, t2 = best
            for e in ((a, b), (b, c), (c, a), (b, a), (a, d), (d, b)):
                edge_of.pop(e, None)
            tri[t1] = (a, d, c)
            tri[t2] = (d, b, c)
            for t in (t1, t2):
                x, y, z = tri[t]
                edge_of[(x, y)] = t
                edge_of[(y, z)] = t
                edge_of[(z, x)] = t
        # collapses
        fc = _fold_cosine(verts, tri, nrm)
        m = _EdgeCollapser(verts, tri)
        touched = set()
        for t in np.argsort(fc):
            if fc[t] >= cos_min:
                break
            if not m.alive[t]:
                continue
            es = [(m.tri[t][k], m.tri[t][(k + 1) % 3]) for k in range(3)]
            es.sort(key=lambda e: float(np.sum((m.xyz[e[0]] - m.xyz[e[1]]) ** 2)))
            for u, v in es:
                if u in touched or v in touched or not m.link_ok(u, v):
                    continue
                p = _project_to_iso(ag, (0.5 * (m.xyz[u] + m.xyz[v]))[None, :])[0]
                pn = _surface_normals(ag, p[None, :])[0]
                ok = True
                for s_ in m.ring(u, v):
                    P = m.corners(s_, u, v, p)
                    fn = np.cross(P[1] - P[0], P[2] - P[0])
                    ln = np.linalg.norm(fn)
                    if ln <= 0.0:
                        ok = False
                        break
                    new = min(np.dot(fn, pn if w in (u, v) else nrm[w]) for w in m.tri[s_]) / ln
                    if new < min(cos_min, fcos(*m.tri[s_])):
                        ok = False
                        break
                if ok:
                    m.collapse(u, v, p)
                    touched.update((u, v))
                    touched.update(m.neigh(u))
                    break
        verts, tri = m.result()
    return verts, tri


def delaunay_flips(xyz, tri, nrm, max_passes: int = 20):
    """Flips interior edges whose two opposite angles sum to more than pi (the Delaunay
    criterion on the surface), when the flipped pair stays counter-clockwise with respect
    to the vertex normals and the new edge does not exist yet.  Removes the obtuse
    'cap' triangles marching tetrahedra produces."""
    tri = np.array(tri, dtype=np.int64)
    edge_of = {}
    for t, (a, b, c) in enumerate(tri):
        edge_of[(a, b)] = t
        edge_of[(b, c)] = t
        edge_of[(c, a)] = t

    def angle(p, q, r):   # angle at p
        u, v = q - p, r - p
        return np.arctan2(np.linalg.norm(np.cross(u, v)), np.dot(u, v))

    def ok_tri(a, b, c):
        n = np.cross(xyz[b] - xyz[a], xyz[c] - xyz[a])
        return np.dot(n, nrm[a] + nrm[b] + nrm[c]) > 0.0

    for _ in range(max_passes):
        flipped = 0
        for (a, b), t1 in list(edge_of.items()):
            if a > b or edge_of.get((a, b)) != t1:
                continue
            t2 = edge_of.get((b, a))
            if t2 is None:
                continue
            c = [w for w in tri[t1] if w != a and w != b][0]
            d = [w for w in tri[t2] if w != a and w != b][0]
            if c == d or (c, d) in edge_of or (d, c) in edge_of:
                continue
            if angle(xyz[c], xyz[a], xyz[b]) + angle(xyz[d], xyz[a], xyz[b]) <= np.pi + 1e-9:
                continue
            if not (ok_tri(a, d, c) and ok_tri(d, b, c)):
                continue
            for e in ((a, b), (b, c), (c, a), (b, a), (a, d), (d, b)):
                edge_of.pop(e, None)
            tri[t1] = (a, d, c)
            tri[t2] = (d, b, c)
            for t in (t1, t2):
                x, y, z = tri[t]
                edge_of[(x, y)] = t
                edge_of[(y, z)] = t
                edge_of[(z, x)] = t
            flipped += 1
        if flipped == 0:
            break
    return tri


def _project_to_iso(ag, verts, steps: int = 8):
    """Newton steps along the gradient onto rho = 1."""
    for _ in range(steps):
        rho, g = ag.eval(verts, grad=True)
        verts = verts - ((rho - 1.0) / np.sum(g * g, axis=1))[:, None] * g
    return verts


def tangential_smooth(ag, verts, tri, iters: int = 2, lam: float = 0.5):
    """Moves every vertex a fraction ``lam`` of the way to the centroid of its neighbours,
    within the tangent plane of the iso-surface, then back onto rho = 1; evens out the
    short edges and thin triangles that survive edge collapse."""
    nv = verts.shape[0]
    E = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    E = np.unique(np.concatenate([E, E[:, ::-1]]), axis=0)
    deg = np.bincount(E[:, 0], minlength=nv).astype(np.float64)
    for _ in range(iters):
        acc = np.zeros_like(verts)
        np.add.at(acc, E[:, 0], verts[E[:, 1]])
        d = acc / deg[:, None] - verts
        _, g = ag.eval(verts, grad=True)
        n = g / np.linalg.norm(g, axis=1, keepdims=True)
        d -= np.einsum("ij,ij->i", d, n)[:, None] * n
        verts = _project_to_iso(ag, verts + lam * d, steps=6)
    return verts


def fill_cavities(verts, tri):
    """Drops the closed components whose enclosed signed volume (outward normals) is not
    positive: buried cavities of the density, which become part of the solute.  Outer
    surfaces, also of separate blobs, enclose positive volume and are kept."""
    tri = np.asarray(tri)
    nv = verts.shape[0]
    parent = np.arange(nv)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b, c in tri:
        for u, v in ((a, b), (b, c)):
            ru, rv = find(u), find(v)
            if ru != rv:
                parent[ru] = rv
    root = np.array([find(i) for i in range(nv)])[tri[:, 0]]
    A, B, C = verts[tri[:, 0]], verts[tri[:, 1]], verts[tri[:, 2]]
    vol6 = np.einsum("ij,ij->i", A, np.cross(B, C))
    keep_root = {r for r in np.unique(root) if vol6[root == r].sum() > 0.0}
    keep = np.array([r in keep_root for r in root])
    tri = tri[keep]
    used = np.unique(tri)
    remap = -np.ones(nv, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return verts[used], remap[tri]


def crease_normals(verts, tri, nrm, cos_min: float = 0.3, passes: int = 3):
    """At the vertices of triangles still folded against their vertex normals (fold cosine
    below ``cos_min``), replaces the density-gradient normal by the area-weighted mean of
    the incident face normals: in a crease narrower than the triangles, the gradient
    describes the crease wall, not the triangulated surface the patches are built on."""
    nrm = np.array(nrm, dtype=np.float64)
    A, B, C = verts[tri[:, 0]], verts[tri[:, 1]], verts[tri[:, 2]]
    fnw = np.cross(B - A, C - A)
    vn = np.zeros_like(verts)
    for k in range(3):
        np.add.at(vn, tri[:, k], fnw)
    vn /= np.linalg.norm(vn, axis=1, keepdims=True)
    done = np.zeros(verts.shape[0], dtype=bool)
    for _ in range(passes):
        bad = _fold_cosine(verts, tri, nrm) < cos_min
        vs = np.unique(tri[bad])
        vs = vs[~done[vs]]
        if vs.size == 0:
            break
        nrm[vs] = vn[vs]
        done[vs] = True
    return nrm


def orientation_flips(verts, tri, nrm, passes: int = 4):
    """Flips an edge of each triangle still oriented against the sum of its vertex normals
    (a fold in a pinch of the density narrower than the grid, where neighbouring normals
    point apart), choosing among its three edges the flip whose two new triangles both
    agree with their vertex normals, with the larger of the smaller agreement; a flip that
    would duplicate an edge is skipped.  Surfaces without such triangles are unchanged."""
    tri = np.array(tri, dtype=np.int64)

    def agree(a, b, c):
        n = np.cross(verts[b] - verts[a], verts[c] - verts[a])
        return float(np.dot(n, nrm[a] + nrm[b] + nrm[c]) / max(np.linalg.norm(n), 1e-300))

    for _ in range(passes):
        A, B, C = verts[tri[:, 0]], verts[tri[:, 1]], verts[tri[:, 2]]
        bad = np.nonzero(np.einsum("ij,ij->i", np.cross(B - A, C - A), nrm[tri].sum(axis=1)) <= 0.0)[0]
        if bad.size == 0:
            break
        edge_of = {}
        for t, (a, b, c) in enumerate(tri):
            edge_of[(a, b)] = t
            edge_of[(b, c)] = t
            edge_of[(c, a)] = t
        for t1 in bad:
            if agree(*tri[t1]) > 0.0:      # fixed by an earlier flip of this pass
                continue
            best = None
            for k in range(3):
                a, b, c = tri[t1][k], tri[t1][(k + 1) % 3], tri[t1][(k + 2) % 3]
                t2 = edge_of.get((b, a))
                if t2 is None:
                    continue
                d = [w for w in tri[t2] if w != a and w != b][0]
                if c == d or (c, d) in edge_of or (d, c) in edge_of:
                    continue
                new = min(agree(a, d, c), agree(d, b, c))
                if new > 0.0 and (best is None or new > best[0]):
                    best = (new, a, b, c, d, t2)
            if best is None:
                continue
            _, a, b, c, d, t2 = best
            for e in ((a, b), (b, c), (c, a), (b, a), (a, d), (d, b)):
                edge_of.pop(e, None)
            tri[t1] = (a, d, c)
            tri[t2] = (d, b, c)
            for t in (t1, t2):
                x, y, z = tri[t]
                edge_of[(x, y)] = t
                edge_of[(y, z)] = t
                edge_of[(z, x)] = t
    return tri


def molecule_surface(centers, radii, grid: float = 0.5, pad: float = 3.0, decay=DENSITY_DECAY,
                     refine_steps: int = 30, collapse: float = 0.25, smooth: int = 2, flips: bool = True,
                     folds: bool = True, cavities: bool = False):
    """Iso-surface rho = 1 of rho(x) = sum_i exp(-decay (|x - c_i|^2 / r_i^2 - 1)), by
    marching tetrahedra on a grid of spacing ``grid`` over the bounding box padded by
    ``pad``.  Vertices are moved onto the iso-surface along their grid edge (bisection
    on the exact density); edges shorter than ``collapse * grid`` are collapsed (the
    slivers marching tetrahedra leaves near grid points) and the merged points projected
    back onto the surface; ``smooth`` rounds of tangential smoothing and Delaunay flips
    then remove the thin triangles left over, and ``folds`` removes triangles folded across
    creases; normals are -grad rho / |grad rho|, except at the vertices of folds that
    remain (face-averaged there), and a last edge flip turns each triangle still against
    the sum of its vertex normals.  Buried cavities (closed components enclosing negative
    volume) are filled unless ``cavities``."""
    ag = _AtomGrid(centers, radii, decay)
    lo = centers.min(axis=0) - radii.max() - pad
    hi = centers.max(axis=0) + radii.max() + pad
    shape = tuple(int(np.ceil((hi[d] - lo[d]) / grid)) + 1 for d in range(3))
    verts, tris, (uniq, pa, pb, fa, fb) = marching_tetrahedra(lambda P: ag.eval(P) - 1.0, lo, grid, shape)
    # bisection along each grid edge on the exact density (fa > 0 inside or fb > 0 inside)
    a_in = fa > 0
    pin = np.where(a_in[:, None], pa, pb)
    pout = np.where(a_in[:, None], pb, pa)
    lo_t = np.zeros(len(pin))
    hi_t = np.ones(len(pin))
    for _ in range(refine_steps):
        mid = 0.5 * (lo_t + hi_t)
        inside = ag.eval(pin + mid[:, None] * (pout - pin)) > 1.0
        lo_t = np.where(inside, mid, lo_t)
        hi_t = np.where(inside, hi_t, mid)
    tm = 0.5 * (lo_t + hi_t)
    verts = pin + tm[:, None] * (pout - pin)
    if not cavities:
        verts, tris = fill_cavities(verts, tris)
    if collapse > 0:
        verts, tris = collapse_short_edges(verts, tris, collapse * grid)
        verts = _project_to_iso(ag, verts)     # merged points back onto rho = 1
    if smooth > 0:
        verts = tangential_smooth(ag, verts, np.asarray(tris), iters=smooth)
    if folds:
        verts, tris = remove_folds(ag, verts, tris)
    _, g = ag.eval(verts, grad=True)
    nrm = -g / np.linalg.norm(g, axis=1, keepdims=True)
    if flips:
        tris = delaunay_flips(verts, tris, nrm)
    if folds:
        nrm = crease_normals(verts, np.asarray(tris), nrm)
        tris = orientation_flips(verts, tris, nrm)
    return verts, nrm, tris.astype(np.int32)


ATOM_VOLUME = 8.5   # A^3 per atom (hydrogens included) at protein density


def protein_ball_radius(n_atoms: int) -> float:
    """Radius of the ball holding n atoms at protein density (about 10 A for 500 atoms)."""
    return float((3.0 * n_atoms * ATOM_VOLUME / (4.0 * math.pi)) ** (1.0 / 3.0))


def molecule(n_atoms: int = 500, seed: int = 3, grid: float = 0.5, ball_radius=None,
             eps1: float = 1.0, eps2: float = 80.0, kappa: float = 0.1257) -> Problem:
    """Protein-like test molecule: atoms packed at protein density (unless ``ball_radius``
    is given), the Gaussian-density surface marched on ``grid``, one partial charge at
    every atom centre."""
    R = protein_ball_radius(n_atoms) if ball_radius is None else ball_radius
    c, r, q = pack_atoms(n_atoms, R, seed)
    xyz, nrm, tri = molecule_surface(c, r, grid=grid)
    return Problem(xyz, nrm, tri, c, q, eps1, eps2, kappa, name=f"molecule_{n_atoms}_s{seed}")


# Surfaces too slow to generate on the fly, stored by meshes/make_meshes.py (positions and
# triangles; the atoms and normals are recomputed here from the same generator).
MESH_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "meshes")
STORED_MOLECULES = {
    # 5000 atoms at protein density, marched at 0.4 A: 267,718 triangles, 133,859 vertices
    "molecule_5000_s4_g0.4": {"n_atoms": 5000, "seed": 4, "grid": 0.4},
}


def stored_molecule(name: str = "molecule_5000_s4_g0.4", eps1: float = 1.0, eps2: float = 80.0,
                    kappa: float = 0.1257) -> Problem:
    """A protein-like molecule of STORED_MOLECULES: the stored surface positions and
    triangles, the atoms and charges from pack_atoms with the same seed, and the vertex
    normals as molecule_surface computes them (-grad rho / |grad rho|, face-averaged at the
    vertices of remaining folds).  Raises if the stored vertices do not lie on the density
    iso-surface of those atoms."""
    spec = STORED_MOLECULES[name]
    d = np.load(os.path.join(MESH_DIR, name + ".npz"))
    xyz = np.ascontiguousarray(d["xyz"], dtype=np.float64)
    tri = np.ascontiguousarray(d["tri"], dtype=np.int32)
    n = spec["n_atoms"]
    c, r, q = pack_atoms(n, protein_ball_radius(n), spec["seed"])
    ag = _AtomGrid(c, r)
    rho, g = ag.eval(xyz, grad=True)
    if np.max(np.abs(rho - 1.0)) > 1e-8:
        raise ValueError(f"{name}: stored vertices are not on the density iso-surface of its atoms")
    nrm = -g / np.linalg.norm(g, axis=1, keepdims=True)
    nrm = crease_normals(xyz, tri.astype(np.int64), nrm)
    return Problem(xyz, nrm, tri, c, q, eps1, eps2, kappa, name=name)


def mesh_quality(xyz, tri):
    """(min angle in degrees, number of connected components, Euler characteristic)."""
    A, B, C = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]

    def ang(u, v):
        c = np.einsum("ij,ij->i", u, v) / (np.linalg.norm(u, axis=1) * np.linalg.norm(v, axis=1))
        return np.degrees(np.arccos(np.clip(c, -1, 1)))

    amin = np.minimum(np.minimum(ang(B - A, C - A), ang(A - B, C - B)), ang(A - C, B - C))
    nv = xyz.shape[0]
    parent = np.arange(nv)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b, c in tri:
        for u, v in ((a, b), (b, c)):
            ru, rv = find(u), find(v)
            if ru != rv:
                parent[ru] = rv
    comps = len({find(i) for i in range(nv)})
    edges = np.unique(np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]), axis=1), axis=0)
    euler = nv - edges.shape[0] + tri.shape[0]
    return float(amin.min()), comps, int(euler)
