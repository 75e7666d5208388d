"""Writes tests/golden/tree_*.npz: the treecode oracle's matvec (oracle/treecode.py) on the
seeded surfaces and vectors of the GPU treecode parity test, with the far-pair count.
Calls only oracle/ and the seeded input generators.  Usage (from the repository root):
``PYTHONPATH=. python tests/golden/make_tree_golden.py``; about a minute per case."""
import os

import numpy as np

from oracle import operator as O
from oracle import treecode as T
from paper_1301_5914_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
SEED = 21

# name: (surface recipe, theta, degree, leaf); recipe = (level, kappa, eps1) of kirkwood_offcenter
CASES = {
    "L4_k0.1257_n4_leaf256": ((4, 0.1257, 1.0), 0.6, 4, 256),
    "L4_k0_n3_leaf192": ((4, 0.0, 2.0), 0.7, 3, 192),
}


def surface(recipe):
    level, kappa, eps1 = recipe
    return inputs.kirkwood_offcenter(level, kappa=kappa, eps1=eps1)


def main():
    for name, (recipe, theta, degree, leaf) in CASES.items():
        p = surface(recipe)
        st = O.setup(p.xyz, p.nrm, p.tri)
        u = inputs.random_vector(2 * p.nv, SEED)
        y, nfar = T.matvec(st, u, p.kappa, p.eps2 / p.eps1, theta=theta, degree=degree, leaf=leaf, batch=512)
        np.savez(os.path.join(HERE, f"tree_{name}.npz"), y=y, nfar=np.int64(nfar), theta=theta,
                 degree=np.int64(degree), leaf=np.int64(leaf), seed=np.int64(SEED))
        print(name, nfar, flush=True)


if __name__ == "__main__":
    main()
