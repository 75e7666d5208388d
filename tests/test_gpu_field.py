"""GPU parity of the potential and field off the surface (hobi_field) through the C ABI
against the FP64 oracle (oracle/field.py) on the same seeded inputs: FP64 to 1e-12 and
mixed to 1e-5 of each output's largest magnitude, the inside flags exactly, for both
methods, ragged point counts, the bench workload's full size, and every error status."""
import numpy as np
import pytest

from oracle import COULOMB_KCAL, FOUR_PI
from oracle import field as F
from oracle import lobi as LO
from oracle import operator as O
from paper_1301_5914_amd import hobi, inputs

pytestmark = pytest.mark.gpu

UNIT = FOUR_PI * COULOMB_KCAL
LOWER = hobi.HOBI_LOWER_ORDER


@pytest.fixture(scope="module")
def ctx():
    return hobi.Context(0)


def _points(p, n_in, n_out, seed, r_in, r_out):
    """Points inside (radius fractions of r_in) and outside (r_out[0] .. r_out[1]) of a
    surface centred near the origin, plus the charges themselves."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n_in + n_out, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    rad = np.r_[rng.uniform(0.05, 1.0, n_in) * r_in, rng.uniform(r_out[0], r_out[1], n_out)]
    return np.concatenate([v * rad[:, None], p.qpos])


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _check(got, ref, tol, label):
    for key in ("phi", "field", "reac", "reac_field"):
        err = _rel(got[key], UNIT * ref[key])
        print(f"  {label} {key} rel err {err:.3e}", flush=True)
        assert err <= tol, (key, err)
    np.testing.assert_array_equal(got["inside"], ref["inside"].astype(np.int32))


CASES = {
    "centered_L2": (inputs.kirkwood_centered(2), 1.5, (2.6, 6.0)),
    "offcenter_L2": (inputs.kirkwood_offcenter(2), 3.0, (5.0, 10.0)),
    "offcenter_L2_k0": (inputs.kirkwood_offcenter(2, kappa=0.0, eps1=2.0), 3.0, (5.0, 10.0)),
    "offcenter_L1_k1": (inputs.kirkwood_offcenter(1, kappa=1.0, eps1=4.0), 3.0, (5.0, 10.0)),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("method", [hobi.HOBI_HIGHER_ORDER, LOWER])
def test_field_matches_oracle(ctx, name, method):
    p, r_in, r_out = CASES[name]
    nu = p.nf if method == LOWER else p.nv
    st = LO.setup(p.xyz, p.nrm, p.tri) if method == LOWER else O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * nu, 11)
    pts = _points(p, 40, 40, 3, r_in, r_out)
    ref = F.potential_and_field(st, u, pts, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
    print(f"field case {name} method {method} points {pts.shape[0]}", flush=True)
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec, method=method)
        _check(g.field(u, pts), ref, tol, f"precision {prec}")


def test_field_molecule30(ctx):
    """The 30-atom protein-like surface: points at the atoms (inside) and on a shell 4 A
    beyond the atoms' extent (outside)."""
    p = inputs.molecule(30, seed=7)
    st = O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nv, 12)
    c = p.qpos.mean(axis=0)
    ext = np.max(np.linalg.norm(p.xyz - c, axis=1))
    rng = np.random.default_rng(5)
    v = rng.standard_normal((48, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    pts = np.concatenate([p.qpos, c + (ext + 4.0) * v])
    ref = F.potential_and_field(st, u, pts, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
    assert np.all(ref["inside"][:len(p.q)]) and not np.any(ref["inside"][len(p.q):])
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec)
        _check(g.field(u, pts), ref, tol, f"molecule30 precision {prec}")


@pytest.mark.parametrize("npts", [1, 63, 64, 65, 257, 1000])
def test_field_ragged_point_counts(ctx, npts):
    """Point counts around the slot sizes (256 points per FP32 slot, 128 per FP64 slot)."""
    p = inputs.kirkwood_offcenter(2)
    st = O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nv, 13)
    rng = np.random.default_rng(npts)
    v = rng.standard_normal((npts, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    pts = v * np.where(rng.random(npts) < 0.5, rng.uniform(0.2, 3.0, npts), rng.uniform(5.0, 9.0, npts))[:, None]
    ref = F.potential_and_field(st, u, pts, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec)
        _check(g.field(u, pts), ref, tol, f"np {npts} precision {prec}")


def test_field_of_the_solved_born_sphere(ctx):
    """End to end: the GPU's own solution of the Born sphere (kappa = 0), then phi and E
    outside against q/(4 pi eps2 r) (discretisation error of the L3 surface) and the
    reaction potential inside against the Born constant."""
    p = inputs.kirkwood_centered(3, kappa=0.0)
    g = hobi.Problem.from_inputs(ctx, p, rtol=1e-10)
    r = g.solve()
    u = np.concatenate([r["phi"], r["dphi"]]) / UNIT
    rng = np.random.default_rng(9)
    v = rng.standard_normal((32, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    outer = v * rng.uniform(3.0, 8.0, 32)[:, None]
    inner = v * rng.uniform(0.1, 1.0, 32)[:, None]
    fo = g.field(u, outer)
    fi = g.field(u, inner)
    ro = np.linalg.norm(outer, axis=1)
    phi_ex = UNIT / (FOUR_PI * p.eps2 * ro)
    E_ex = UNIT * outer / (FOUR_PI * p.eps2 * ro ** 3)[:, None]
    R_ex = UNIT / (FOUR_PI * 2.0) * (1.0 / p.eps2 - 1.0 / p.eps1)
    print("born outside", _rel(fo["phi"], phi_ex), _rel(fo["field"], E_ex), "inside", np.max(np.abs(fi["reac"] / R_ex - 1)), flush=True)
    assert _rel(fo["phi"], phi_ex) < 1e-4 and _rel(fo["field"], E_ex) < 1e-3
    assert np.max(np.abs(fi["reac"] / R_ex - 1)) < 1e-4
    assert np.all(fi["inside"] == 1) and np.all(fo["inside"] == 0)


def test_field_bench_workload_L6_sampled(ctx):
    """The default bench surface at full size (327680 nodes): a 32^3 potential map
    through the sphere and beyond, sampled points against the oracle point by point."""
    p = inputs.kirkwood_offcenter(6)
    st = O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nv, 14)
    ax = np.linspace(-7.9, 7.9, 32)
    pts = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    rad = np.linalg.norm(pts, axis=1)
    pts = pts[np.abs(rad - 4.0) > 0.6]           # keep off the surface (edge length ~0.1 A)
    rng = np.random.default_rng(2)
    sample = np.unique(np.r_[0:4, pts.shape[0] - 4:pts.shape[0], rng.integers(0, pts.shape[0], 40)])
    ref = F.potential_and_field(st, u, pts[sample], p.qpos, p.q, p.eps1, p.eps2, p.kappa)
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec)
        print(f"L6 map {pts.shape[0]} points precision {prec}", flush=True)
        out = g.field(u, pts)
        got = {k: v[sample] for k, v in out.items()}
        _check(got, ref, tol, f"L6 map precision {prec}")


def test_field_errors_and_empty(ctx):
    p = inputs.kirkwood_offcenter(1)
    g = hobi.Problem.from_inputs(ctx, p)
    u = inputs.random_vector(2 * p.nv, 1)
    out = g.field(u, np.zeros((0, 3)))
    assert out["phi"].shape == (0,)
    L = hobi.lib()
    pts = np.zeros((2, 3))
    assert L.hobi_field(g.handle, hobi._P(u.ctypes.data), 0, 2, None, None, None, None, None, None) == 1
    assert L.hobi_field(g.handle, hobi._P(u.ctypes.data), 0, -1, hobi._dptr(pts), None, None, None, None,
                        None) == 1
    assert L.hobi_field(g.handle, None, 0, 2, hobi._dptr(pts), None, None, None, None, None) == 1
    bad = np.array([[0.0, np.nan, 0.0]])
    assert L.hobi_field(g.handle, hobi._P(u.ctypes.data), 0, 1, hobi._dptr(bad), None, None, None, None,
                        None) == 7
    # all outputs NULL is allowed
    assert L.hobi_field(g.handle, hobi._P(u.ctypes.data), 0, 2, hobi._dptr(pts), None, None, None, None,
                        None) == 0
    # points so far away that kappa r could leave the FP64 exponential's range (2.5e6 here is
    # 2e7 A at kappa = 0.1257): rejected before any field sum; at kappa = 0 they are fine
    far = np.array([[0.0, 0.0, 0.0], [2.1e7, 0.0, 0.0]])
    assert L.hobi_field(g.handle, hobi._P(u.ctypes.data), 0, 2, hobi._dptr(far), None, None, None, None,
                        None) == 1
    near = np.array([[0.0, 0.0, 0.0], [1.9e7, 0.0, 0.0]])
    assert L.hobi_field(g.handle, hobi._P(u.ctypes.data), 0, 2, hobi._dptr(near), None, None, None, None,
                        None) == 0
    g0 = hobi.Problem(ctx, p.xyz, p.nrm, p.tri, p.qpos, p.q, p.eps1, p.eps2, 0.0)
    assert L.hobi_field(g0.handle, hobi._P(u.ctypes.data), 0, 2, hobi._dptr(far), None, None, None, None,
                        None) == 0
