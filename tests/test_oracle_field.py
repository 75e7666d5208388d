"""Pins of the off-surface potential and field oracle (representation formulas eqbim_1 /
eqbim_2 combined with the jump conditions, Section 2.1).  Each pin is fixed by something
other than the oracle's own formula: the reaction potential of the energy path (written
with the rewritten kernels), central differences of the potential, Born's and Kirkwood's
closed forms inside and outside the sphere, Gauss's law, and the lower-order scheme."""
import functools

import numpy as np
import pytest

from oracle import FOUR_PI
from oracle import field as F
from oracle import kirkwood as KW
from oracle import lobi as LO
from oracle import operator as O
from oracle.solve import solve as hobi_solve
from paper_1301_5914_amd import inputs


@functools.lru_cache(maxsize=None)
def _solved(kind, level, kappa):
    if kind == "born":
        p = inputs.kirkwood_centered(level, radius=2.0, kappa=kappa)
    else:
        p = inputs.kirkwood_offcenter(level, kappa=kappa)
    r = hobi_solve(p.xyz, p.nrm, p.tri, p.qpos, p.q, p.eps1, p.eps2, p.kappa, rtol=1e-10)
    return p, r


def _points(radii, n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v * np.asarray(radii)[:, None] if np.ndim(radii) else v * radii


def test_reaction_potential_equals_the_energy_path():
    """R from the Green's functions written out equals the reaction potential of the
    energy (rewritten, cancellation-free kernels K1, K2) at interior points."""
    p, r = _solved("off", 2, 0.1257)
    pts = _points(np.linspace(0.2, 2.8, 12), 12, 1)
    R, _, _ = F.reaction_terms(r["setup"], r["u"], pts, p.kappa, p.eps2 / p.eps1)
    ref = O.reaction_potential(r["setup"], r["u"], pts, p.kappa, p.eps2 / p.eps1)
    np.testing.assert_allclose(R, ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("kappa", [0.0, 0.1257])
def test_field_is_minus_the_gradient_of_the_potential(kappa):
    """Central differences (h = 1e-4 A) of phi and of R, inside and outside."""
    p, r = _solved("off", 2, kappa)
    pts = np.concatenate([_points(np.linspace(0.3, 2.5, 6), 6, 2), _points(np.linspace(5.5, 9.0, 6), 6, 3)])
    out = F.potential_and_field(r["setup"], r["u"], pts, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
    h = 1e-4
    for axis in range(3):
        e = np.zeros(3)
        e[axis] = h
        fp = F.potential_and_field(r["setup"], r["u"], pts + e, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
        fm = F.potential_and_field(r["setup"], r["u"], pts - e, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
        dphi = (fp["phi"] - fm["phi"]) / (2 * h)
        dR = (fp["reac"] - fm["reac"]) / (2 * h)
        np.testing.assert_allclose(-out["field"][:, axis], dphi, rtol=1e-6, atol=1e-9 * np.max(np.abs(dphi)))
        np.testing.assert_allclose(-out["reac_field"][:, axis], dR, rtol=1e-6, atol=1e-9 * np.max(np.abs(dR)))
    assert np.all(out["inside"][:6]) and not np.any(out["inside"][6:])


def test_born_sphere_inside_and_outside():
    """kappa = 0, unit charge at the centre of a 2 A sphere: inside, R is the constant
    q/(4 pi a) (1/eps2 - 1/eps1) with no field; outside, phi = q/(4 pi eps2 r) and
    E = q x/(4 pi eps2 r^3).  Errors fall under refinement."""
    errs = []
    for level in (1, 2):
        p, r = _solved("born", level, 0.0)
        a = 2.0
        inner = _points(np.linspace(0.1, 1.0, 8), 8, 4)
        outer = _points(np.linspace(3.0, 8.0, 8), 8, 5)
        fi = F.potential_and_field(r["setup"], r["u"], inner, p.qpos, p.q, p.eps1, p.eps2, 0.0)
        fo = F.potential_and_field(r["setup"], r["u"], outer, p.qpos, p.q, p.eps1, p.eps2, 0.0)
        R_exact = 1.0 / (FOUR_PI * a) * (1.0 / p.eps2 - 1.0 / p.eps1)
        ro = np.linalg.norm(outer, axis=1)
        phi_o = 1.0 / (FOUR_PI * p.eps2 * ro)
        E_o = outer / (FOUR_PI * p.eps2 * ro ** 3)[:, None]
        e = [np.max(np.abs(fi["reac"] / R_exact - 1)),
             np.max(np.linalg.norm(fi["reac_field"], axis=1)) * a / abs(R_exact),
             np.max(np.abs(fo["phi"] / phi_o - 1)),
             np.max(np.linalg.norm(fo["field"] - E_o, axis=1) / np.linalg.norm(E_o, axis=1))]
        errs.append(e)
        assert np.all(fi["inside"]) and not np.any(fo["inside"])
    errs = np.array(errs)
    assert np.all(errs[1] < 1e-3), errs
    assert np.all(errs[1] < errs[0] / 3), errs


def test_kirkwood_eccentric_charges_inside_and_outside():
    """kappa = 0.1257, eight charges: R and its field inside against Kirkwood's series
    (the field by central differences of the series), phi outside against the exterior
    series; errors fall under refinement."""
    errs = []
    for level in (1, 2):
        p, r = _solved("off", level, 0.1257)
        a = 4.0
        inner = _points(np.linspace(0.5, 2.5, 8), 8, 6)
        outer = _points(np.linspace(5.0, 10.0, 8), 8, 7)
        fi = F.potential_and_field(r["setup"], r["u"], inner, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
        fo = F.potential_and_field(r["setup"], r["u"], outer, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
        args = (p.qpos, p.q, a, p.eps1, p.eps2, p.kappa)
        R_ex = KW.reaction_potential(inner, *args)
        h = 1e-4
        gR = np.stack([(KW.reaction_potential(inner + h * np.eye(3)[k], *args)
                        - KW.reaction_potential(inner - h * np.eye(3)[k], *args)) / (2 * h) for k in range(3)], axis=1)
        phi_o = KW.exterior_potential(outer, *args)
        errs.append([np.max(np.abs(fi["reac"] - R_ex)) / np.max(np.abs(R_ex)),
                     np.max(np.abs(-fi["reac_field"] - gR)) / np.max(np.abs(gR)),
                     np.max(np.abs(fo["phi"] - phi_o)) / np.max(np.abs(phi_o))])
    errs = np.array(errs)
    assert np.all(errs[1] < [1e-2, 6e-2, 1e-2]), errs
    assert np.all(errs[1] < errs[0] / 3), errs


def test_gauss_law_outside():
    """kappa = 0: the flux of E through a sphere of radius 7 A around the molecule is
    Q / eps2 (charges in e, potentials in e/A with the 1/(4 pi) of G0)."""
    p, r = _solved("off", 2, 0.0)
    xs, ns, ts = inputs.icosphere(3, 7.0)
    P = xs[ts]
    cen = P.mean(axis=1)
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    # project the centroids onto the sphere and scale the flat areas to the sphere's total
    cen = 7.0 * cen / np.linalg.norm(cen, axis=1)[:, None]
    area *= 4 * np.pi * 49.0 / np.sum(area)
    out = F.potential_and_field(r["setup"], r["u"], cen, p.qpos, p.q, p.eps1, p.eps2, 0.0)
    flux = np.sum(area * np.sum(out["field"] * cen / 7.0, axis=1))
    Q = float(np.sum(p.q))
    assert abs(flux - Q / p.eps2) < 2e-3 * max(abs(Q), 1.0) / p.eps2 + 1e-4 * np.sum(np.abs(p.q)) / p.eps2, (flux, Q / p.eps2)


def test_lower_order_outside_the_born_sphere():
    """The same evaluation on a lower-order solution: phi outside the Born sphere is
    q/(4 pi eps2 r) to the scheme's first-order error, falling under refinement."""
    errs = []
    for level in (1, 2):
        p = inputs.kirkwood_centered(level, radius=2.0, kappa=0.0)
        r = LO.solve(p.xyz, p.nrm, p.tri, p.qpos, p.q, p.eps1, p.eps2, 0.0, rtol=1e-10)
        outer = _points(np.linspace(3.0, 8.0, 8), 8, 8)
        fo = F.potential_and_field(r["setup"], r["u"], outer, p.qpos, p.q, p.eps1, p.eps2, 0.0)
        ro = np.linalg.norm(outer, axis=1)
        errs.append(np.max(np.abs(fo["phi"] * FOUR_PI * p.eps2 * ro - 1)))
    assert errs[1] < errs[0] / 3 and errs[1] < 1e-3, errs


def test_coincident_charge_is_left_out():
    """At a charge's own position the Coulomb sum omits that charge (finite values), and
    the reaction part is the energy path's reaction potential there."""
    p, r = _solved("off", 2, 0.1257)
    out = F.potential_and_field(r["setup"], r["u"], p.qpos, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
    assert np.all(np.isfinite(out["phi"])) and np.all(np.isfinite(out["field"]))
    S_other = np.array([sum(p.q[j] / (FOUR_PI * p.eps1 * np.linalg.norm(p.qpos[k] - p.qpos[j]))
                            for j in range(len(p.q)) if j != k) for k in range(len(p.q))])
    ref = O.reaction_potential(r["setup"], r["u"], p.qpos, p.kappa, p.eps2 / p.eps1)
    np.testing.assert_allclose(out["phi"], S_other + ref, rtol=1e-12)
