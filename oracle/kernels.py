"""Green's functions and the kernels K1..K4 of the well-posed formulation (Section 2.1).

G0(x, y) = 1 / (4 pi r) and Gk(x, y) = exp(-kappa r) / (4 pi r), r = |x - y|
(eq. eq_potential).  With d = x - y, a = exp(-kappa r), z = kappa r:

  dG0/dny = (d.ny) / (4 pi r^3)            dGk/dny = a (1 + z) (d.ny) / (4 pi r^3)
  dG0/dnx = -(d.nx) / (4 pi r^3)           dGk/dnx = -a (1 + z) (d.nx) / (4 pi r^3)
  d2G0/dnx dny = (nx.ny) / (4 pi r^3) - 3 (d.nx)(d.ny) / (4 pi r^5)
  d2Gk/dnx dny = a (1 + z)(nx.ny) / (4 pi r^3) - a (3 + 3z + z^2)(d.nx)(d.ny) / (4 pi r^5)

The kernels (eq. Eq_Ls), with eps = eps2 / eps1 (reading: the printed eps1/eps2 is
inverted; only eps2/eps1 makes the exact sphere solution satisfy eqbim_3/eqbim_4):

  K1 = G0 - Gk,                      K2 = eps dGk/dny - dG0/dny,
  K3 = dG0/dnx - (1/eps) dGk/dnx,    K4 = d2Gk/dnx dny - d2G0/dnx dny.

The differences cancel for small kappa r.  They are evaluated through the exact
rewriting f0 = 1 - a, f1 = 1 - a (1 + z), f2 = 3 - a (3 + 3z + z^2):

  K1 = f0 / (4 pi r)
  K2 = (d.ny) / (4 pi r^3) ((eps - 1) - eps f1)
  K3 = -(d.nx) / (4 pi r^3) ((1 - 1/eps) + f1 / eps)
  K4 = [-(nx.ny) f1 + (d.nx)(d.ny) f2 / r^2] / (4 pi r^3)

with f0 from expm1 and f1, f2 from their Taylor series when z < 0.5.
"""
from __future__ import annotations

import math

import numpy as np

from . import FOUR_PI

_SERIES_Z = 0.5
_NTERMS = 26


def f0(z):
    """1 - exp(-z)."""
    return -np.expm1(-np.asarray(z, dtype=np.float64))


def _series(z, coef):
    """sum_{k=2}^{_NTERMS-1} coef(k) z^k / k!, by Horner's rule in z."""
    out = np.zeros_like(z)
    for k in range(_NTERMS - 1, 1, -1):
        out = out * z + coef(k) / math.factorial(k)
    return out * z * z


def f1(z):
    """1 - exp(-z) (1 + z) = sum_{k>=2} (-1)^k (k - 1) z^k / k!."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = 1.0 - np.exp(-z) * (1.0 + z)
    small = z < _SERIES_Z
    if np.any(small):
        out = np.where(small, 0.0, out)
        out[small] = _series(z[small], lambda k: (-1.0) ** k * (k - 1))
    return out


def f2(z):
    """3 - exp(-z) (3 + 3z + z^2) = sum_{k>=2} (-1)^(k+1) (k - 1)(k - 3) z^k / k!."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = 3.0 - np.exp(-z) * (3.0 + 3.0 * z + z * z)
    small = z < _SERIES_Z
    if np.any(small):
        out = np.where(small, 0.0, out)
        out[small] = _series(z[small], lambda k: (-1.0) ** (k + 1) * (k - 1) * (k - 3))
    return out


def _geom(x, nx, y, ny):
    d = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    dny = np.sum(d * ny, axis=-1)
    dnx = np.sum(d * nx, axis=-1) if nx is not None else None
    nxy = np.sum(np.asarray(nx) * np.asarray(ny), axis=-1) if nx is not None else None
    return d, r, dnx, dny, nxy


def kernels(x, nx, y, ny, kappa, eps):
    """K1, K2, K3, K4 at target x (normal nx) and source y (normal ny), broadcasting."""
    _, r, dnx, dny, nxy = _geom(x, nx, y, ny)
    z = kappa * r
    a0, a1, a2 = f0(z), f1(z), f2(z)
    r3 = FOUR_PI * r * r * r
    K1 = a0 / (FOUR_PI * r)
    K2 = dny / r3 * ((eps - 1.0) - eps * a1)
    K3 = -dnx / r3 * ((1.0 - 1.0 / eps) + a1 / eps)
    K4 = (-nxy * a1 + dnx * dny * a2 / (r * r)) / r3
    return K1, K2, K3, K4


def kernels_12(x, y, ny, kappa, eps):
    """K1 and K2 only (no target normal), for the reaction potential at charges."""
    _, r, _, dny, _ = _geom(x, None, y, ny)
    z = kappa * r
    K1 = f0(z) / (FOUR_PI * r)
    K2 = dny / (FOUR_PI * r * r * r) * ((eps - 1.0) - eps * f1(z))
    return K1, K2


# ---- the Green's functions themselves, written out (used to pin the kernels) ----------

def G0(x, y):
    r = np.linalg.norm(np.asarray(x) - np.asarray(y), axis=-1)
    return 1.0 / (FOUR_PI * r)


def Gk(x, y, kappa):
    r = np.linalg.norm(np.asarray(x) - np.asarray(y), axis=-1)
    return np.exp(-kappa * r) / (FOUR_PI * r)


def green_derivatives(x, nx, y, ny, kappa):
    """(dG/dny, dG/dnx, d2G/dnxdny) for G0 and for Gk, from the closed forms above."""
    d, r, dnx, dny, nxy = _geom(x, nx, y, ny)
    a = np.exp(-kappa * r)
    z = kappa * r
    r3 = FOUR_PI * r ** 3
    r5 = FOUR_PI * r ** 5
    g0 = (dny / r3, -dnx / r3, nxy / r3 - 3.0 * dnx * dny / r5)
    gk = (a * (1 + z) * dny / r3, -a * (1 + z) * dnx / r3,
          a * (1 + z) * nxy / r3 - a * (3 + 3 * z + z * z) * dnx * dny / r5)
    return g0, gk
