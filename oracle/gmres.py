"""Restarted GMRES(m) (Saad & Schultz), the Krylov solver the paper uses.

Reading (the paper states neither tolerance, restart length, initial guess nor
preconditioner): x0 = 0, no preconditioner, modified Gram-Schmidt Arnoldi with one
re-orthogonalisation pass when the new column's norm drops by more than 1/sqrt(2),
Givens rotations for the Hessenberg least-squares problem, stop when the estimated
||b - A x|| / ||b|| <= rtol or after max_iter matrix-vector products.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, rtol=1e-6, restart=200, max_iter=200):
    """Returns (x, iterations, estimated relative residual, converged)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0, True
    total = 0
    rel = 1.0
    while True:
        r = b - matvec(x) if total > 0 else b.copy()
        beta = np.linalg.norm(r)
        rel = beta / bnorm
        if rel <= rtol or total >= max_iter:
            return x, total, rel, rel <= rtol
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k_used = 0
        done = False
        for k in range(m):
            w = matvec(V[k])
            total += 1
            wnorm0 = np.linalg.norm(w)
            for j in range(k + 1):
                H[j, k] = np.dot(w, V[j])
                w = w - H[j, k] * V[j]
            if np.linalg.norm(w) < wnorm0 / np.sqrt(2.0):
                for j in range(k + 1):
                    c = np.dot(w, V[j])
                    H[j, k] += c
                    w = w - c * V[j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0.0:
                V[k + 1] = w / H[k + 1, k]
            for j in range(k):
                a, bb = H[j, k], H[j + 1, k]
                H[j, k] = cs[j] * a + sn[j] * bb
                H[j + 1, k] = -sn[j] * a + cs[j] * bb
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            rel = abs(g[k + 1]) / bnorm
            k_used = k + 1
            if rel <= rtol or total >= max_iter or den == 0.0:
                done = True
                break
        yk = np.zeros(k_used)
        for i in range(k_used - 1, -1, -1):
            yk[i] = (g[i] - np.dot(H[i, i + 1:k_used], yk[i + 1:])) / H[i, i]
        x = x + V[:k_used].T @ yk
        if done:
            return x, total, rel, rel <= rtol


def diagonal_scaling(nv, eps):
    """1 / the diagonal coefficients of the two row blocks of eqdbef3/eqdbef4 (and of the
    lower-order eqdbef1/eqdbef2): 1/(1/2 (1 + eps)) on the phi unknowns, 1/(1/2 (1 + 1/eps))
    on the dphi unknowns."""
    return np.concatenate([np.full(nv, 1.0 / (0.5 * (1.0 + eps))), np.full(nv, 1.0 / (0.5 * (1.0 + 1.0 / eps)))])


def gmres_scaled(matvec, b, dinv, rtol=1e-6, restart=200, max_iter=200):
    """GMRES on the second-kind form with both diagonal blocks the identity: the unknowns
    are scaled, A D^-1 y = b with D the diagonal coefficients and u = D^-1 y (right
    scaling, so the residual GMRES estimates is still ||b - A u|| / ||b||).  The discrete
    solution is the same; only the Krylov iteration differs (reading: the paper names the
    equations well-posed of the second kind and runs GMRES on them without giving their
    scaling).  Returns (u, iterations, estimated relative residual, converged)."""
    dinv = np.asarray(dinv, dtype=np.float64)
    y, its, rel, conv = gmres(lambda v: matvec(dinv * v), b, rtol, restart, max_iter)
    return dinv * y, its, rel, conv

