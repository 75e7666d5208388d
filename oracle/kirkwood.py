"""Kirkwood's analytic solution for point charges in a dielectric sphere, and error norms.

The paper validates against Kirkwood's sphere solutions (Section 3, "closed form for the
centred charge, spherical harmonics for eccentric charges") without printing them.
Derivation used here: inside the sphere (radius a, dielectric eps1) the potential is the
Coulomb field of the charges plus a regular harmonic series; outside (eps2, kappa) it is
a series in the decaying modified spherical Bessel functions k_n(kappa r).  Matching
phi and eps dphi/dr at r = a term by term for each Legendre order n gives, with
rho_n = z k_n'(z) / k_n(z) at z = kappa a (rho_n = -(n+1) when kappa = 0):

  D_n = eps1 n - eps2 rho_n,   f_n = (eps1 (n+1) + eps2 rho_n) / D_n
  phi_reac(x) = 1/(4 pi eps1) sum_n f_n sum_k q_k (rho_k |x|)^n / a^(2n+1) P_n(cos g_k)
  phi(a x^)   = 1/(4 pi) sum_n (2n+1)/D_n sum_k q_k rho_k^n / a^(n+1) P_n(cos g_k)
  dphi1/dn    = 1/(4 pi) sum_n (2n+1) eps2 rho_n / (eps1 a D_n) sum_k q_k rho_k^n / a^(n+1) P_n

The log-derivative comes from the three-term recurrence k_{n} = k_{n-2} + (2n-1)/z k_{n-1}:
R_0 = 1, R_n = k_{n-1}/k_n = 1 / (R_{n-1} + (2n-1)/z), rho_n = -z R_n - (n+1).
All potentials are in internal units (Green's functions with 1/(4 pi)); energies in
kcal/mol with the Coulomb constant of the package.
"""
from __future__ import annotations

import numpy as np

from . import COULOMB_KCAL, FOUR_PI


def log_derivative_kn(nmax, z):
    """rho_n = z k_n'(z) / k_n(z), n = 0..nmax (rho_n = -(n+1) at z = 0)."""
    n = np.arange(nmax + 1)
    if z == 0.0:
        return -(n + 1.0)
    R = np.empty(nmax + 1)
    R[0] = 1.0
    for k in range(1, nmax + 1):
        R[k] = 1.0 / (R[k - 1] + (2 * k - 1) / z)
    return -z * R - (n + 1.0)


def _legendre(nmax, x):
    """P_0..P_nmax at x (array), by the Bonnet recurrence; shape [nmax+1, *x.shape]."""
    x = np.asarray(x, dtype=np.float64)
    P = np.empty((nmax + 1,) + x.shape)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = x
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
    return P


def _coeffs(nmax, a, eps1, eps2, kappa):
    rho = log_derivative_kn(nmax, kappa * a)
    n = np.arange(nmax + 1)
    D = eps1 * n - eps2 * rho
    f = (eps1 * (n + 1) + eps2 * rho) / D
    return n, rho, D, f


def _cos_and_radius(points, qpos):
    rp = np.linalg.norm(points, axis=-1)
    rq = np.linalg.norm(qpos, axis=-1)
    up = np.where(rp[:, None] > 0, points / np.where(rp > 0, rp, 1.0)[:, None], 0.0)
    uq = np.where(rq[:, None] > 0, qpos / np.where(rq > 0, rq, 1.0)[:, None], 0.0)
    return rp, rq, up @ uq.T     # cos between each point and each charge


def surface_values(points, qpos, q, a, eps1, eps2, kappa, nmax=60):
    """Exact phi and dphi1/dn (internal units) at points on the sphere |x| = a."""
    n, rho, D, f = _coeffs(nmax, a, eps1, eps2, kappa)
    _, rq, cosg = _cos_and_radius(points, qpos)
    P = _legendre(nmax, cosg)                        # [n, npts, nq]
    radial = (rq[None, :] ** n[:, None]) / a ** (n[:, None] + 1)   # [n, nq], 0^0 = 1
    S = np.einsum("nk,npk,k->np", radial, P, q)       # [n, npts]
    phi = np.einsum("n,np->p", (2 * n + 1) / D, S) / FOUR_PI
    dphi = np.einsum("n,np->p", (2 * n + 1) * eps2 * rho / (eps1 * a * D), S) / FOUR_PI
    return phi, dphi


def _kn_ratio(nmax, x, x0):
    """k_n(x) / k_n(x0), n = 0..nmax, x >= x0 > 0: k_0 = (pi/2) e^-x / x and k_n = k_0 / prod_m R_m
    with R_m = k_{m-1} / k_m from the recurrence of log_derivative_kn."""
    def ratios(z):
        R = np.empty(nmax + 1)
        R[0] = 1.0
        for k in range(1, nmax + 1):
            R[k] = 1.0 / (R[k - 1] + (2 * k - 1) / z)
        return R
    out = (x0 / x) * np.exp(-(x - x0)) * np.cumprod(ratios(x0) / ratios(x))
    return out


def exterior_potential(points, qpos, q, a, eps1, eps2, kappa, nmax=60):
    """Exact phi_2 (internal units) at points with |x| >= a: the surface series of
    surface_values continued outwards by k_n(kappa r) / k_n(kappa a), or (a / r)^(n+1)
    when kappa = 0 (the decaying solutions of the screened and plain Laplace equations)."""
    n, rho, D, f = _coeffs(nmax, a, eps1, eps2, kappa)
    rp, rq, cosg = _cos_and_radius(points, qpos)
    P = _legendre(nmax, cosg)                        # [n, npts, nq]
    radial = (rq[None, :] ** n[:, None]) / a ** (n[:, None] + 1)
    S = np.einsum("nk,npk,k->np", radial, P, q)       # [n, npts]
    if kappa == 0.0:
        g = (a / rp[None, :]) ** (n[:, None] + 1)
    else:
        g = np.stack([_kn_ratio(nmax, kappa * r, kappa * a) for r in rp], axis=1)
    return np.einsum("n,np,np->p", (2 * n + 1) / D, S, g) / FOUR_PI


def reaction_potential(points, qpos, q, a, eps1, eps2, kappa, nmax=60):
    """Exact phi_reac (internal units) at interior points."""
    n, rho, D, f = _coeffs(nmax, a, eps1, eps2, kappa)
    rp, rq, cosg = _cos_and_radius(points, qpos)
    P = _legendre(nmax, cosg)
    rad = (rp[None, :, None] * rq[None, None, :]) ** n[:, None, None] / a ** (2 * n[:, None, None] + 1)
    return np.einsum("n,npk,npk,k->p", f, rad, P, q) / (FOUR_PI * eps1)


def solvation_energy(qpos, q, a, eps1, eps2, kappa, nmax=60):
    """Exact E_sol = 1/2 sum q_k phi_reac(x_k), kcal/mol."""
    pr = reaction_potential(qpos, qpos, q, a, eps1, eps2, kappa, nmax)
    return 0.5 * FOUR_PI * COULOMB_KCAL * float(np.sum(q * pr))


def centered_closed_form(q, a, eps1, eps2, kappa):
    """Single charge at the centre: (E kcal/mol, phi, dphi) with phi, dphi internal."""
    E = COULOMB_KCAL * q * q / (2.0 * a) * (1.0 / (eps2 * (1.0 + kappa * a)) - 1.0 / eps1)
    phi = q / (FOUR_PI * eps2 * (1.0 + kappa * a) * a)
    dphi = -q / (FOUR_PI * eps1 * a * a)
    return E, phi, dphi


def rel_max_error(num, exa):
    """e_phi of eq. eqerror: max |num - exa| / max |exa| over the unknowns."""
    return float(np.max(np.abs(num - exa)) / np.max(np.abs(exa)))


def order(coarse_mesh, fine_mesh, coarse_err, fine_err):
    """eq. eqeorder: log base (coarse_mesh / fine_mesh) of (coarse_err / fine_err).

    For boundary elements the paper's "mesh" is the density d (vertices per A^2); with
    h the edge length, an order p in h is an order p/2 in d.
    """
    return float(np.log(coarse_err / fine_err) / np.log(coarse_mesh / fine_mesh))
