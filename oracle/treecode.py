"""Treecode approximation of the dense regular sum (the O(N^2) part of eqdbef3/eqdbef4).

Test infrastructure only: plain numpy FP64; nothing in the product path imports it.

The paper's CPU time grows as O(N^2) with the number of elements (Section 3, protein
1ajj), and it names fast summation (treecode or fast multipole, its refs. on TABI-PB) as
the way past that.  This module is one such scheme, a cluster-particle treecode over a
binary cluster tree with polynomial interpolation of the Green's functions in the source
point; it is the reference the GPU version is checked against, both taking the same
partition and rules, written out here:

* Order: vertices and triangles in Morton order over the vertices' bounding box: each
  coordinate mapped to [0, 1] by (x - lo) / (hi - lo) (an extent of 0 read as 1), clamped,
  multiplied by 2097151 and truncated to 21 bits; the bits interleaved with x lowest; a
  stable sort (ties keep the input order).  A triangle's position is its vertex
  centroid (a + b + c) / 3; its 4 regular nodes stay together in the rule's order.
* Leaves: consecutive runs of `leaf` nodes in that order; batches: consecutive runs of
  `batch` target vertices in vertex order.  Each cluster and batch has the bounding box of
  its points, its centre and its radius (half the box diagonal).
* Cluster tree: the leaves are level 0; level l + 1 joins neighbours 2i and 2i + 1 of level l
  into one cluster over both node ranges, a last cluster without a neighbour moving up
  unchanged; the single cluster left is the root.
* A (batch, cluster) pair is accepted (far) when rb + rc <= theta |cb - cc| and no target of
  the batch is a vertex of a triangle of the cluster (so an incident triangle, which
  belongs to the singular rule, is never approximated).  Each batch walks the tree from
  the root: an accepted cluster is taken by its proxies, a rejected leaf is summed
  directly (near), a rejected parent is opened into its two children.  The accepted and
  near clusters of a batch cover every node once.
* Near pairs: the direct regular sum, incident triangles masked (as operator.matvec).
* Far pairs: the Green's functions interpolated in the source point y by the tensor
  Lagrange basis L_k on the (n+1)^3 Chebyshev points of the second kind of the cluster's
  box (grown by GROW of its diagonal on every side):
      G(x, y) ~ sum_k G(x, s_k) L_k(y),   dG/dnu_y(x, y) ~ sum_k G(x, s_k) grad L_k(y).n_y,
  so that with Gamma = w dphi, Phi = w phi at the nodes (the linear interpolation of the
  vertex unknowns, Section 2.2) and the proxy charges
      Q0_k  = sum_j  Gamma_j L_k(y_j) - Phi_j grad L_k(y_j).n_j
      Qk_k  = sum_j -Gamma_j L_k(y_j) + eps Phi_j grad L_k(y_j).n_j
      Qk2_k = sum_j -Gamma_j L_k(y_j) / eps + Phi_j grad L_k(y_j).n_j
  the two rows of a far pair are
      sum_k G0(x, s_k) Q0_k + Gk(x, s_k) Qk_k,   sum_k dG0/dnu_x(x, s_k) Q0_k + dGk/dnu_x(x, s_k) Qk2_k
  (K1 = G0 - Gk, K2 = eps dGk/dnu_y - dG0/dnu_y, K3 = dG0/dnu_x - dGk/dnu_x / eps,
  K4 = d2Gk/dnu_x dnu_y - d2G0/dnu_x dnu_y, eq. Eq_Ls).  The charges of every cluster,
  parent or leaf, are these sums over its own nodes.
The singular correction and the diagonal are those of operator.matvec.  theta = 0 makes
every pair near, and the result is the dense matvec.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import FOUR_PI
from .kernels import kernels
from .operator import Setup, matvec as dense_matvec

GROW = 1e-6


def _spread(v):
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    out = np.zeros_like(v)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def morton_order(pts, lo, hi):
    ext = np.where(hi - lo > 0, hi - lo, 1.0)
    f = np.clip((pts - lo) / ext, 0.0, 1.0)
    q = (f * 2097151.0).astype(np.uint64)
    code = _spread(q[:, 0]) | (_spread(q[:, 1]) << np.uint64(1)) | (_spread(q[:, 2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


@dataclasses.dataclass
class Partition:
    vorder: np.ndarray     # [nv] targets in order (caller's vertex ids)
    torder: np.ndarray     # [nf] triangles in order
    clusters: list         # (first, last + 1) in ordered node positions; leaves first
    children: list         # per cluster: None (leaf) or its two children's indices
    nleaf: int
    batches: list          # (first, last + 1) in ordered target positions
    far: list              # per batch: accepted cluster indices
    near: list             # per batch: rejected leaf indices


def cluster_tree(nn, leaf):
    """Clusters (leaves first, then each level's parents) and their children."""
    clusters = [(a, min(a + leaf, nn)) for a in range(0, nn, leaf)]
    children = [None] * len(clusters)
    level = list(range(len(clusters)))
    while len(level) > 1:
        up = []
        for i in range(0, len(level), 2):
            if i + 1 < len(level):
                l, r = level[i], level[i + 1]
                clusters.append((clusters[l][0], clusters[r][1]))
                children.append((l, r))
                up.append(len(clusters) - 1)
            else:
                up.append(level[i])
        level = up
    return clusters, children, level[0]


def partition(st: Setup, theta, leaf, batch):
    xyz, tri = st.xyz, st.tri
    lo, hi = xyz.min(axis=0), xyz.max(axis=0)
    vorder = morton_order(xyz, lo, hi)
    cen = (xyz[tri[:, 0]] + xyz[tri[:, 1]] + xyz[tri[:, 2]]) / 3.0
    torder = morton_order(cen, lo, hi)
    vrank = np.empty(st.nv, dtype=np.int64)
    vrank[vorder] = np.arange(st.nv)
    y = st.y[torder].reshape(-1, 3)
    tv = vrank[tri[torder]]                       # [nf,3] ordered vertex ranks
    nn = y.shape[0]
    clusters, children, root = cluster_tree(nn, leaf)
    nleaf = (nn + leaf - 1) // leaf
    batches = [(a, min(a + batch, st.nv)) for a in range(0, st.nv, batch)]
    tx = xyz[vorder]

    def sphere(p):
        blo, bhi = p.min(axis=0), p.max(axis=0)
        return 0.5 * (blo + bhi), 0.5 * np.linalg.norm(bhi - blo)

    cs = [sphere(y[a:b]) for a, b in clusters]
    cv = [(tv[a // 4:(b + 3) // 4].min(), tv[a // 4:(b + 3) // 4].max()) for a, b in clusters]
    far, near = [], []
    for a, b in batches:
        cb, rb = sphere(tx[a:b])
        fa, ne = [], []
        stack = [root]
        while stack:
            c = stack.pop()
            touches = cv[c][1] >= a and cv[c][0] <= b - 1
            if not touches and rb + cs[c][1] <= theta * np.linalg.norm(cb - cs[c][0]):
                fa.append(c)
            elif children[c] is None:
                ne.append(c)
            else:
                stack.extend(children[c][::-1])
        far.append(fa)
        near.append(ne)
    return Partition(vorder, torder, clusters, children, nleaf, batches, far, near)


def cheb_points(lo, hi, n):
    """n + 1 Chebyshev points of the second kind on [lo, hi] (lo, hi: arrays of 3)."""
    t = np.cos(np.pi * np.arange(n + 1) / n)
    return 0.5 * (lo + hi)[:, None] + 0.5 * (hi - lo)[:, None] * t[None, :]     # [3, n+1]


def lagrange_1d(p, t):
    """l_a(t) and l_a'(t), a = 0..n, for points p [n+1] at abscissae t [m] (product form)."""
    n1 = p.shape[0]
    L = np.ones((t.shape[0], n1))
    D = np.zeros((t.shape[0], n1))
    for a in range(n1):
        others = [m for m in range(n1) if m != a]
        for m in others:
            L[:, a] *= (t - p[m]) / (p[a] - p[m])
        for q in others:
            term = np.full(t.shape[0], 1.0 / (p[a] - p[q]))
            for m in others:
                if m != q:
                    term *= (t - p[m]) / (p[a] - p[m])
            D[:, a] += term
    return L, D


def basis(y, ny, n):
    """(s [P,3], L_k(y_j) [m,P], grad L_k(y_j).n_j [m,P]) of the cluster with nodes y,
    normals ny: the proxy points of its grown box and the tensor basis at its nodes."""
    blo, bhi = y.min(axis=0), y.max(axis=0)
    g = GROW * np.linalg.norm(bhi - blo) + 1e-12
    p = cheb_points(blo - g, bhi + g, n)
    L = [None] * 3
    D = [None] * 3
    for d in range(3):
        L[d], D[d] = lagrange_1d(p[d], y[:, d])
    Lk = np.einsum("ja,jb,jc->jabc", L[0], L[1], L[2]).reshape(y.shape[0], -1)
    Gk = (np.einsum("ja,jb,jc->jabc", D[0], L[1], L[2]) * ny[:, 0, None, None, None]
          + np.einsum("ja,jb,jc->jabc", L[0], D[1], L[2]) * ny[:, 1, None, None, None]
          + np.einsum("ja,jb,jc->jabc", L[0], L[1], D[2]) * ny[:, 2, None, None, None]).reshape(y.shape[0], -1)
    s = np.stack(np.meshgrid(p[0], p[1], p[2], indexing="ij"), axis=-1).reshape(-1, 3)
    return s, Lk, Gk


def proxies(y, ny, gam, phi, eps, n):
    """(s [P,3], Q0, Qk, Qk2 [P]) of one cluster (nodes y, normals ny, strengths)."""
    s, Lk, Gk = basis(y, ny, n)
    Q0 = gam @ Lk - phi @ Gk
    Qk = -(gam @ Lk) + eps * (phi @ Gk)
    Qk2 = -(gam @ Lk) / eps + phi @ Gk
    return s, Q0, Qk, Qk2


def matvec(st: Setup, u, kappa, eps, theta=0.5, degree=5, leaf=256, batch=128):
    """y = A u with the regular sum taken by the treecode (singular part and diagonal as
    operator.matvec), and the count of accepted (batch, cluster) pairs."""
    nv = st.nv
    u = np.asarray(u, dtype=np.float64)
    phi_v, dphi_v = u[:nv], u[nv:]
    part = partition(st, theta, leaf, batch)
    # dense = diagonal - (regular + singular); regular part alone from the regular rule
    y_dense = dense_matvec(st, u, kappa, eps)
    tri_o = st.tri[part.torder]
    y = st.y[part.torder].reshape(-1, 3)
    ny = st.ny[part.torder].reshape(-1, 3)
    w = st.w[part.torder].ravel()
    gam = w * (dphi_v[tri_o] @ st.L.T).ravel()
    phn = w * (phi_v[tri_o] @ st.L.T).ravel()
    node_tri = np.repeat(tri_o, 4, axis=0)        # caller vertex ids of each node's triangle
    tx = st.xyz[part.vorder]
    tn = st.nrm[part.vorder]
    reg = np.zeros((nv, 2))                       # exact regular sums (masked), ordered targets
    tree = np.zeros((nv, 2))                      # the treecode's regular sums
    cache = {}
    for i, (a, b) in enumerate(part.batches):
        for c in part.far[i]:
            p, q = part.clusters[c]
            if c not in cache:
                cache[c] = proxies(y[p:q], ny[p:q], gam[p:q], phn[p:q], eps, degree)
            s, Q0, Qk, Qk2 = cache[c]
            for t in range(a, b):
                d = tx[t] - s
                r = np.linalg.norm(d, axis=1)
                e = np.exp(-kappa * r)
                dnx = d @ tn[t]
                g0 = 1.0 / (FOUR_PI * r)
                tree[t, 0] += np.sum(g0 * Q0 + e * g0 * Qk)
                tree[t, 1] += np.sum(-dnx / (FOUR_PI * r ** 3) * (Q0 + e * (1.0 + kappa * r) * Qk2))
        for c in part.near[i]:
            p, q = part.clusters[c]
            for t in range(a, b):
                keep = ~np.any(node_tri[p:q] == part.vorder[t], axis=1)
                K1, K2, K3, K4 = kernels(tx[t], tn[t], y[p:q][keep], ny[p:q][keep], kappa, eps)
                tree[t, 0] += np.sum(K1 * gam[p:q][keep] + K2 * phn[p:q][keep])
                tree[t, 1] += np.sum(K3 * gam[p:q][keep] + K4 * phn[p:q][keep])
    # the same dense regular sum, for swapping it out of y_dense
    for t in range(nv):
        keep = ~np.any(node_tri == part.vorder[t], axis=1)
        K1, K2, K3, K4 = kernels(tx[t], tn[t], y[keep], ny[keep], kappa, eps)
        reg[t, 0] = np.sum(K1 * gam[keep] + K2 * phn[keep])
        reg[t, 1] = np.sum(K3 * gam[keep] + K4 * phn[keep])
    out = y_dense.copy()
    idx = part.vorder
    out[idx] += reg[:, 0] - tree[:, 0]
    out[nv + idx] += reg[:, 1] - tree[:, 1]
    return out, int(sum(len(f) for f in part.far))


def field_terms(st, u, points, kappa, eps, theta=0.5, degree=5, leaf=256, batch=256):
    """(R, grad R, solid-angle fraction) at each point (as field.reaction_terms) with the
    surface sum taken by the treecode, and the counts of accepted (batch, cluster) and near
    (batch, leaf) pairs.  The points are ordered by the Morton rule over their own bounding
    box and cut into batches of `batch`; each batch walks the cluster tree of the matvec's
    partition with the acceptance test rb + rc <= theta |cb - cc| alone (the points are off
    the surface).  Accepted clusters use, with d = x - s_k and a = exp(-kappa r),
        R      ~ sum_k G0 Q0_k + Gk Qk_k,
        grad R ~ -sum_k d/(4 pi r^3) (Q0_k + a (1 + kappa r) Qk_k),
        frac   ~ sum_k G0 Qs_k,  Qs_k = -sum_j w_j grad L_k(y_j).n_j
    (the solid angle is the double layer of the unit density, so its charge is the
    normal-derivative part with weight -w); near leaves are summed directly."""
    from .field import node_sums, surface_nodes

    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    xyz, tri = st.xyz, st.tri
    cen = (xyz[tri[:, 0]] + xyz[tri[:, 1]] + xyz[tri[:, 2]]) / 3.0
    torder = morton_order(cen, xyz.min(axis=0), xyz.max(axis=0))   # the matvec's node order
    y0, ny0, w0, dphi0, phi0 = surface_nodes(st, u)
    idx = (4 * torder[:, None] + np.arange(4)[None, :]).ravel()
    y, ny, w, dphi, phi = y0[idx], ny0[idx], w0[idx], dphi0[idx], phi0[idx]
    gam, phn = w * dphi, w * phi
    clusters, children, root = cluster_tree(y.shape[0], leaf)

    def sphere(p):
        blo, bhi = p.min(axis=0), p.max(axis=0)
        return 0.5 * (blo + bhi), 0.5 * np.linalg.norm(bhi - blo)

    cs = [sphere(y[a:b]) for a, b in clusters]
    porder = morton_order(pts, pts.min(axis=0), pts.max(axis=0))
    tp = pts[porder]
    R = np.zeros(pts.shape[0])
    gR = np.zeros((pts.shape[0], 3))
    frac = np.zeros(pts.shape[0])
    cache = {}
    nfar = nnear = 0
    for a0 in range(0, pts.shape[0], batch):
        b0 = min(a0 + batch, pts.shape[0])
        cb, rb = sphere(tp[a0:b0])
        stack = [root]
        while stack:
            c = stack.pop()
            a, b = clusters[c]
            if rb + cs[c][1] <= theta * np.linalg.norm(cb - cs[c][0]):
                nfar += 1
                if c not in cache:
                    s, Lk, Gk = basis(y[a:b], ny[a:b], degree)
                    cache[c] = (s, gam[a:b] @ Lk - phn[a:b] @ Gk, -(gam[a:b] @ Lk) + eps * (phn[a:b] @ Gk),
                                -(w[a:b] @ Gk))
                s, Q0, Qk, Qs = cache[c]
                for t in range(a0, b0):
                    d = tp[t] - s
                    r = np.linalg.norm(d, axis=1)
                    e = np.exp(-kappa * r)
                    g0 = 1.0 / (FOUR_PI * r)
                    R[t] += np.sum(g0 * Q0 + e * g0 * Qk)
                    gR[t] -= np.sum((d / (FOUR_PI * r ** 3)[:, None]) * (Q0 + e * (1.0 + kappa * r) * Qk)[:, None],
                                    axis=0)
                    frac[t] += np.sum(g0 * Qs)
            elif children[c] is None:
                nnear += 1
                r_, g_, f_ = node_sums(tp[a0:b0], y[a:b], ny[a:b], w[a:b], dphi[a:b], phi[a:b], kappa, eps)
                R[a0:b0] += r_
                gR[a0:b0] += g_
                frac[a0:b0] += f_
            else:
                stack.extend(children[c][::-1])
    out_R, out_g, out_f = np.empty_like(R), np.empty_like(gR), np.empty_like(frac)
    out_R[porder], out_g[porder], out_f[porder] = R, gR, frac
    return out_R, out_g, out_f, nfar, nnear


def matvec_lobi(ls, xyz, tri, u, kappa, eps, theta=0.5, degree=5, leaf=256, batch=128):
    """y = A u of the lower-order scheme (oracle.lobi.matvec, Section 2.4) with its regular
    sum taken by the treecode, and the count of accepted (batch, cluster) pairs.  Sites and
    nodes are the centroids, in the Morton order of the triangles (as `partition`); leaves,
    tree and batches as for the higher-order scheme.  A centroid's own node is the only one
    left out of its row, so a cluster is never accepted for a batch whose sites overlap its
    nodes.  There is no singular part: y = diagonal - (tree sums)."""
    nf = ls.nf
    u = np.asarray(u, dtype=np.float64)
    cen = (xyz[tri[:, 0]] + xyz[tri[:, 1]] + xyz[tri[:, 2]]) / 3.0
    order = morton_order(cen, xyz.min(axis=0), xyz.max(axis=0))
    y, ny, W = ls.c[order], ls.n[order], ls.W[order]
    phi, dphi = u[:nf][order], u[nf:][order]
    gam, phn = W * dphi, W * phi
    clusters, children, root = cluster_tree(nf, leaf)

    def sphere(p):
        blo, bhi = p.min(axis=0), p.max(axis=0)
        return 0.5 * (blo + bhi), 0.5 * np.linalg.norm(bhi - blo)

    cs = [sphere(y[a:b]) for a, b in clusters]
    tree = np.zeros((nf, 2))
    cache = {}
    nfar = 0
    for a0 in range(0, nf, batch):
        b0 = min(a0 + batch, nf)
        cb, rb = sphere(y[a0:b0])
        stack = [root]
        while stack:
            c = stack.pop()
            p, q = clusters[c]
            touches = q - 1 >= a0 and p <= b0 - 1
            if not touches and rb + cs[c][1] <= theta * np.linalg.norm(cb - cs[c][0]):
                nfar += 1
                if c not in cache:
                    cache[c] = proxies(y[p:q], ny[p:q], gam[p:q], phn[p:q], eps, degree)
                s, Q0, Qk, Qk2 = cache[c]
                for t in range(a0, b0):
                    d = y[t] - s
                    r = np.linalg.norm(d, axis=1)
                    e = np.exp(-kappa * r)
                    dnx = d @ ny[t]
                    g0 = 1.0 / (FOUR_PI * r)
                    tree[t, 0] += np.sum(g0 * Q0 + e * g0 * Qk)
                    tree[t, 1] += np.sum(-dnx / (FOUR_PI * r ** 3) * (Q0 + e * (1.0 + kappa * r) * Qk2))
            elif children[c] is None:
                for t in range(a0, b0):
                    keep = np.arange(p, q) != t
                    K1, K2, K3, K4 = kernels(y[t], ny[t], y[p:q][keep], ny[p:q][keep], kappa, eps)
                    tree[t, 0] += np.sum(K1 * gam[p:q][keep] + K2 * phn[p:q][keep])
                    tree[t, 1] += np.sum(K3 * gam[p:q][keep] + K4 * phn[p:q][keep])
            else:
                stack.extend(children[c][::-1])
    out = np.empty(2 * nf)
    out[order] = 0.5 * (1.0 + eps) * phi - tree[:, 0]
    out[nf + order] = 0.5 * (1.0 + 1.0 / eps) * dphi - tree[:, 1]
    return out, nfar
