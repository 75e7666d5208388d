"""Writes the stored protein-like surfaces of this folder (positions and triangles only).

The large protein-like workload -- 5000 atoms packed at protein density (seed 4), the
Gaussian density surface marched on a 0.4 A grid (267,718 triangles, 133,859 vertices) --
takes about nine minutes to generate on one core, so its surface is stored; the atoms and
the vertex normals are recomputed from the same generator when it is loaded
(`inputs.stored_molecule`), which checks them against this file's positions.

Usage: python -m paper_1301_5914_amd.meshes.make_meshes [name ...]
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def write(name: str) -> str:
    from paper_1301_5914_amd import inputs
    spec = inputs.STORED_MOLECULES[name]
    p = inputs.molecule(spec["n_atoms"], seed=spec["seed"], grid=spec["grid"])
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, xyz=p.xyz, tri=p.tri.astype(np.int32))
    return path


if __name__ == "__main__":
    from paper_1301_5914_amd import inputs
    for n in (sys.argv[1:] or list(inputs.STORED_MOLECULES)):
        print(write(n), flush=True)
