"""Writes tests/golden/tree_*.npz: the treecode oracle's matvec (oracle/treecode.py) on the
seeded surfaces and vectors of the GPU treecode parity test, with the counts of accepted
(batch, cluster) and near (batch, leaf) pairs.
Calls only oracle/ and the seeded input generators.  Usage (from the repository root):
``PYTHONPATH=. python tests/golden/make_tree_golden.py [--lower-order-only]``; about a
minute per case."""
import os

import numpy as np

from oracle import lobi as LO
from oracle import operator as O
from oracle import treecode as T
from paper_1301_5914_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
SEED = 21

# name: (surface recipe, theta, degree, leaf, batch); recipe = (level, kappa, eps1) of
# kirkwood_offcenter
CASES = {
    "L4_k0.1257_n4_leaf256_b256": ((4, 0.1257, 1.0), 0.6, 4, 256, 256),
    "L4_k0_n3_leaf192_b128": ((4, 0.0, 2.0), 0.7, 3, 192, 128),
    "L4_k1_n5_leaf64_b512": ((4, 1.0, 4.0), 0.8, 5, 64, 512),
}


# lower-order scheme: name: (surface recipe, theta, degree, leaf, batch)
LOBI_CASES = {
    "L4_k0.1257_n4_leaf64_b128": ((4, 0.1257, 1.0), 0.7, 4, 64, 128),
}


def surface(recipe):
    level, kappa, eps1 = recipe
    return inputs.kirkwood_offcenter(level, kappa=kappa, eps1=eps1)


def main(lobi_only=False):
    for name, (recipe, theta, degree, leaf, batch) in ({} if lobi_only else CASES).items():
        p = surface(recipe)
        st = O.setup(p.xyz, p.nrm, p.tri)
        u = inputs.random_vector(2 * p.nv, SEED)
        y, nfar = T.matvec(st, u, p.kappa, p.eps2 / p.eps1, theta=theta, degree=degree, leaf=leaf, batch=batch)
        nnear = sum(len(n) for n in T.partition(st, theta, leaf, batch).near)
        np.savez(os.path.join(HERE, f"tree_{name}.npz"), y=y, nfar=np.int64(nfar), nnear=np.int64(nnear), theta=theta,
                 degree=np.int64(degree), leaf=np.int64(leaf), batch=np.int64(batch), seed=np.int64(SEED))
        print(name, nfar, nnear, flush=True)
    for name, (recipe, theta, degree, leaf, batch) in LOBI_CASES.items():
        p = surface(recipe)
        ls = LO.setup(p.xyz, p.nrm, p.tri)
        u = inputs.random_vector(2 * p.nf, SEED)
        y, nfar = T.matvec_lobi(ls, p.xyz, p.tri, u, p.kappa, p.eps2 / p.eps1, theta=theta, degree=degree, leaf=leaf,
                                batch=batch)
        np.savez(os.path.join(HERE, f"tree_lobi_{name}.npz"), y=y, nfar=np.int64(nfar), theta=theta,
                 degree=np.int64(degree), leaf=np.int64(leaf), batch=np.int64(batch), seed=np.int64(SEED))
        print("lower-order", name, nfar, flush=True)


if __name__ == "__main__":
    import sys
    main(lobi_only="--lower-order-only" in sys.argv)
