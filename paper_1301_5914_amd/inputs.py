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
