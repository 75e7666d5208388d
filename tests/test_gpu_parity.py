"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded
inputs.  Bars: FP64 setup arrays 1e-13, FP64 matvec / solve / energy 1e-12 relative;
mixed precision 1e-5 relative on the solvation energy."""
import numpy as np
import pytest

from oracle import COULOMB_KCAL, FOUR_PI
from oracle import kirkwood as KW
from oracle import operator as O
from oracle.solve import solve as oracle_solve
from paper_1301_5914_amd import hobi, inputs

pytestmark = pytest.mark.gpu

SCALE = FOUR_PI * COULOMB_KCAL


@pytest.fixture(scope="module")
def ctx():
    return hobi.Context(0)


def _cases():
    return {
        "centered_L3": inputs.kirkwood_centered(3),
        "offcenter_L3": inputs.kirkwood_offcenter(3),
        "offcenter_L2_k0_eps1_2": inputs.kirkwood_offcenter(2, kappa=0.0, eps1=2.0),
        "offcenter_L2_k1": inputs.kirkwood_offcenter(2, kappa=1.0, eps1=4.0),
        "ico_L0": inputs.kirkwood_centered(0, radius=2.0),
        # small kappa: kappa r < 0.01 on every pair, where 1 - e, f1 and f2 cancel
        "offcenter_L3_k0.001": inputs.kirkwood_offcenter(3, kappa=0.001),
    }


CASES = _cases()


@pytest.fixture(scope="module")
def oracle_setups():
    return {k: O.setup(p.xyz, p.nrm, p.tri) for k, p in CASES.items()}


def _rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("name", list(CASES))
def test_setup_arrays_match(ctx, oracle_setups, name):
    p = CASES[name]
    print(f"case {name} nv={p.nv}", flush=True)
    g = hobi.Problem.from_inputs(ctx, p)
    y, ny, w = g.nodes()
    st = oracle_setups[name]
    assert np.max(np.abs(y - st.y)) <= 1e-13 * np.max(np.abs(st.y))
    assert np.max(np.abs(ny - st.ny)) <= 1e-13
    assert np.max(np.abs(w - st.w)) <= 1e-13 * np.max(st.w)
    S1, S2 = O.sources(st.xyz, st.nrm, p.qpos, p.q, p.eps1)
    assert _rel_inf(g.rhs(), np.concatenate([S1, S2])) <= 1e-13


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_fp64_matches_oracle(ctx, oracle_setups, name):
    p = CASES[name]
    print(f"case {name} nv={p.nv}", flush=True)
    g = hobi.Problem.from_inputs(ctx, p)
    st = oracle_setups[name]
    eps = p.eps2 / p.eps1
    for seed in (1, 2):
        u = inputs.random_vector(2 * p.nv, seed)
        y_or = O.matvec(st, u, p.kappa, eps)
        y = g.matvec(u)
        assert _rel_inf(y, y_or) <= 1e-12, (name, seed, _rel_inf(y, y_or))
    # a smooth vector (the exact Kirkwood data of a sphere centred at the origin)
    a = float(np.linalg.norm(p.xyz[0]))
    phi, dphi = KW.surface_values(p.xyz, p.qpos, p.q, a, p.eps1, p.eps2, p.kappa)
    u = np.concatenate([phi, dphi])
    assert _rel_inf(g.matvec(u), O.matvec(st, u, p.kappa, eps)) <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_mixed_close_to_oracle(ctx, oracle_setups, name):
    p = CASES[name]
    g = hobi.Problem.from_inputs(ctx, p, precision=hobi.HOBI_MIXED)
    st = oracle_setups[name]
    u = inputs.random_vector(2 * p.nv, 3)
    y_or = O.matvec(st, u, p.kappa, p.eps2 / p.eps1)
    err = _rel_inf(g.matvec(u), y_or)
    print(f"mixed matvec rel err {name}: {err:.3e}")
    assert err <= 1e-5


def test_matvec_level4_ragged_tiles(ctx):
    """2562 vertices: three 1024-target tiles with a ragged tail, 81920 nodes."""
    p = inputs.kirkwood_offcenter(4)
    st = O.setup(p.xyz, p.nrm, p.tri)
    g = hobi.Problem.from_inputs(ctx, p)
    u = inputs.random_vector(2 * p.nv, 4)
    rows = np.r_[0:40, p.nv - 40:p.nv, 1000:1040]
    y_or = O.matvec(st, u, p.kappa, p.eps2 / p.eps1, rows=rows)
    y = g.matvec(u)
    got = np.stack([y[rows], y[p.nv + rows]])
    assert _rel_inf(got, y_or) <= 1e-12


def test_identity_when_dielectrics_match(ctx):
    p = inputs.kirkwood_offcenter(2, kappa=0.0, eps1=3.0, eps2=3.0)
    for prec in (hobi.HOBI_FP64, hobi.HOBI_MIXED):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec)
        u = inputs.random_vector(2 * p.nv, 9)
        np.testing.assert_array_equal(g.matvec(u), u)


@pytest.mark.parametrize("scaled", [2, 1, 0])
def test_solve_fp64_fixed_iterations_matches_oracle(ctx, scaled):
    """Same number of GMRES iterations on both sides: same Krylov iterate to 1e-12, with the
    Jacobi preconditioner (default: A's own diagonal, the singular self terms included), with
    the row blocks' constant scaling and on A u = b as written."""
    p = inputs.kirkwood_offcenter(3)
    its = 4 if scaled else 6
    g = hobi.Problem.from_inputs(ctx, p, rtol=0.0, max_iter=its, restart=200, diag_scaling=scaled)
    r = g.solve(allow_noconv=True)
    assert r["status"] == "HOBI_E_NOCONV" and r["stats"]["iterations"] == its
    o = oracle_solve(p.xyz, p.nrm, p.tri, p.qpos, p.q, p.eps1, p.eps2, p.kappa, rtol=0.0,
                     max_iter=its, diag_scaling=scaled)
    assert o["iterations"] == its
    assert _rel_inf(r["phi"], o["phi"]) <= 1e-12
    assert _rel_inf(r["dphi"], o["dphi"]) <= 1e-12
    assert abs(r["energy"] / o["energy"] - 1) <= 1e-12


def test_scaled_and_unscaled_gmres_reach_the_same_solution(ctx):
    """Both forms of the iteration solve the same discrete system: solutions within the
    tolerance, true residuals below it, the scaled form in fewer matvecs."""
    p = inputs.kirkwood_offcenter(3)
    r = {}
    for scaled in (2, 1, 0):
        r[scaled] = hobi.Problem.from_inputs(ctx, p, rtol=1e-10, diag_scaling=scaled).solve()
        assert r[scaled]["stats"]["true_residual"] < 1e-10
    print("iterations Jacobi / scaled / unscaled", r[2]["stats"]["iterations"], r[1]["stats"]["iterations"],
          r[0]["stats"]["iterations"], flush=True)
    assert r[1]["stats"]["iterations"] < r[0]["stats"]["iterations"]
    assert r[2]["stats"]["iterations"] < r[0]["stats"]["iterations"]
    assert _rel_inf(r[1]["phi"], r[0]["phi"]) <= 1e-8
    assert _rel_inf(r[2]["phi"], r[0]["phi"]) <= 1e-8
    assert abs(r[1]["energy"] / r[0]["energy"] - 1) <= 1e-9


def test_solve_fp64_converged_matches_oracle(ctx):
    p = inputs.kirkwood_offcenter(2)
    g = hobi.Problem.from_inputs(ctx, p, rtol=1e-12)
    r = g.solve()
    o = oracle_solve(p.xyz, p.nrm, p.tri, p.qpos, p.q, p.eps1, p.eps2, p.kappa, rtol=1e-12)
    print("iterations gpu/oracle", r["stats"]["iterations"], o["iterations"])
    assert abs(r["energy"] / o["energy"] - 1) <= 1e-12
    assert _rel_inf(r["phi"], o["phi"]) <= 1e-11
    assert r["stats"]["true_residual"] < 1e-11


def test_config1_energy_against_closed_form(ctx):
    """Config 1 at rtol 1e-6, FP64 and mixed, against the oracle and Kirkwood."""
    p = inputs.kirkwood_centered(3)
    o = oracle_solve(p.xyz, p.nrm, p.tri, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
    E_exact, _, _ = KW.centered_closed_form(1.0, 2.0, 1.0, 80.0, 0.1257)
    for prec in (hobi.HOBI_FP64, hobi.HOBI_MIXED):
        r = hobi.Problem.from_inputs(ctx, p, precision=prec).solve()
        print("precision", prec, "E", r["energy"], "oracle", o["energy"], "its", r["stats"]["iterations"],
              o["iterations"])
        assert abs(r["energy"] / o["energy"] - 1) <= 1e-5
        assert abs(r["energy"] / E_exact - 1) <= 2e-5
        assert r["stats"]["converged"] == 1


def test_energy_entry_point(ctx):
    p = inputs.kirkwood_offcenter(2)
    st = O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nv, 11) * 1e-3
    g = hobi.Problem.from_inputs(ctx, p)
    e_or = O.solvation_energy(st, u, p.qpos, p.q, p.kappa, p.eps2 / p.eps1)
    assert abs(g.energy(u) / e_or - 1) <= 1e-12


def test_mixed_solve_energy_offcenter(ctx):
    p = inputs.kirkwood_offcenter(2)
    o = oracle_solve(p.xyz, p.nrm, p.tri, p.qpos, p.q, p.eps1, p.eps2, p.kappa)
    r = hobi.Problem.from_inputs(ctx, p, precision=hobi.HOBI_MIXED).solve()
    print("mixed E rel err", abs(r["energy"] / o["energy"] - 1))
    assert abs(r["energy"] / o["energy"] - 1) <= 1e-5


def test_deterministic(ctx):
    p = inputs.kirkwood_offcenter(3)
    for prec in (hobi.HOBI_FP64, hobi.HOBI_MIXED):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec)
        a = g.solve()
        b = g.solve()
        np.testing.assert_array_equal(a["phi"], b["phi"])
        assert a["energy"] == b["energy"]


def test_device_pointer_matvec(ctx):
    torch = pytest.importorskip("torch")
    p = inputs.kirkwood_offcenter(2)
    s = torch.cuda.Stream()
    tctx = hobi.Context(0, stream=s)
    g = hobi.Problem.from_inputs(tctx, p)
    u = inputs.random_vector(2 * p.nv, 5)
    with torch.cuda.stream(s):
        ud = torch.tensor(u, dtype=torch.float64, device="cuda")
        yd = torch.empty_like(ud)
        g.matvec(ud, out=yd)            # enqueued on s, after the tensors' creation
        y_dev = yd.cpu().numpy()        # ordered after the matvec on the same stream
    np.testing.assert_array_equal(y_dev, g.matvec(u))


def test_error_statuses(ctx):
    xyz, nrm, tri = inputs.icosphere(2, 2.0)
    q = np.ones(1)
    with pytest.raises(hobi.HobiError) as e:
        bad = tri.copy()
        bad[5] = bad[5][::-1]
        hobi.Problem(ctx, xyz, nrm, bad, np.zeros((1, 3)), q)
    assert e.value.name == "HOBI_E_MESH"
    with pytest.raises(hobi.HobiError) as e:
        hobi.Problem(ctx, xyz, nrm, tri[2:], np.zeros((1, 3)), q)
    assert e.value.name == "HOBI_E_MESH"
    with pytest.raises(hobi.HobiError) as e:
        hobi.Problem(ctx, xyz, nrm, tri, np.array([[0.0, 0.0, 2.5]]), q)
    assert e.value.name == "HOBI_E_CHARGE_OUTSIDE"
    with pytest.raises(hobi.HobiError) as e:
        x2 = xyz.copy()
        x2[3, 0] = np.nan
        hobi.Problem(ctx, x2, nrm, tri, np.zeros((1, 3)), q)
    assert e.value.name == "HOBI_E_NUMERIC"
    with pytest.raises(hobi.HobiError) as e:
        hobi.Problem(ctx, xyz, nrm, tri, np.zeros((1, 3)), q, eps1=-1.0)
    assert e.value.name == "HOBI_E_ARG"
    with pytest.raises(hobi.HobiError) as e:
        hobi.Problem(ctx, xyz, nrm, tri, np.zeros((1, 3)), q, diag_scaling=3)
    assert e.value.name == "HOBI_E_ARG"
    g = hobi.Problem(ctx, xyz, nrm, tri, np.zeros((1, 3)), q, max_iter=1, rtol=1e-12)
    with pytest.raises(hobi.HobiError) as e:
        g.solve()
    assert e.value.name == "HOBI_E_NOCONV"


@pytest.fixture(scope="module")
def mol30():
    return inputs.molecule(30, seed=7)


def test_molecule_matvec_matches_oracle(ctx, mol30):
    """Protein-like marched surface (30 atoms): FP64 to 1e-12 and mixed to 1e-5 on sampled
    rows of a random (sign-alternating) vector."""
    p = mol30
    print(f"molecule nv={p.nv} nf={p.nf}", flush=True)
    st = O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nv, 21)
    rng = np.random.default_rng(0)
    rows = np.unique(np.r_[0:30, p.nv - 30:p.nv, rng.integers(0, p.nv, 60)])
    y_or = O.matvec(st, u, p.kappa, p.eps2 / p.eps1, rows=rows)
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec)
        y = g.matvec(u)
        got = np.stack([y[rows], y[p.nv + rows]])
        err = _rel_inf(got, y_or)
        print("precision", prec, "rel err", err)
        assert err <= tol


def test_molecule_solve_mixed_matches_fp64(ctx, mol30):
    p = mol30
    r64 = hobi.Problem.from_inputs(ctx, p).solve()
    r32 = hobi.Problem.from_inputs(ctx, p, precision=hobi.HOBI_MIXED).solve()
    print("E fp64", r64["energy"], "its", r64["stats"]["iterations"], "E mixed", r32["energy"],
          "its", r32["stats"]["iterations"])
    assert abs(r32["energy"] / r64["energy"] - 1) <= 1e-5
    assert r64["stats"]["converged"] == 1 and r32["stats"]["converged"] == 1


# ---- the bench workloads at their full sizes, in the launch configuration bench.py times

@pytest.fixture(scope="module")
def l6():
    return inputs.kirkwood_offcenter(6)


def test_bench_workload_L6_sampled_rows(ctx, l6):
    """Default bench workload at full size (40962 vertices, 327680 nodes; 8 targets per lane,
    ~4096 XCD-remapped blocks): rows spread over the first and last target blocks, tile
    boundaries and random positions, against the oracle computed row by row."""
    p = l6
    st = O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nv, 31)
    rng = np.random.default_rng(1)
    rows = np.unique(np.r_[0:4, p.nv - 4:p.nv, 2046:2050, 16382:16386, rng.integers(0, p.nv, 16)])
    y_or = O.matvec(st, u, p.kappa, p.eps2 / p.eps1, rows=rows)
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec)
        y = g.matvec(u)
        got = np.stack([y[rows], y[p.nv + rows]])
        err = _rel_inf(got, y_or)
        print(f"L6 precision {prec} rel err {err:.3e}", flush=True)
        assert err <= tol


def test_bench_workload_L6_energy(ctx, l6):
    """Full L6 solves: mixed within 1e-5 of FP64 (the mixed-mode bar), FP64 within the
    discretisation error of the Kirkwood series (6e-5 measured at L6; O(h^2) from L1-L4)."""
    p = l6
    r64 = hobi.Problem.from_inputs(ctx, p, max_iter=400, restart=400).solve()
    r32 = hobi.Problem.from_inputs(ctx, p, precision=hobi.HOBI_MIXED, max_iter=400, restart=400).solve()
    E = KW.solvation_energy(p.qpos, p.q, 4.0, p.eps1, p.eps2, p.kappa)
    print("L6 E fp64", r64["energy"], "E mixed", r32["energy"], "Kirkwood", E, flush=True)
    assert abs(r32["energy"] / r64["energy"] - 1) <= 1e-5
    assert abs(r64["energy"] / E - 1) <= 2e-4


def test_config2_convergence_levels(ctx):
    """Config 2 on the GPU, icosphere L3-L6 in FP64 and mixed precision, solved to rtol 1e-9
    (FP64) and 1e-7 (mixed): e_phi, e_dphi (max error at the vertices over the max of the
    exact values, Section 3.1) and the energy error against the Kirkwood series, and their
    orders in h (h halves per level).  The orders stay near 2 (the oracle's L1-L4 run gives
    1.93 / 1.84 / 2.00 from L3 to L4); mixed precision follows FP64 until its matvec noise
    (about 1e-7 of a row) is reached."""
    a = 4.0
    errs = {}
    for lvl in (3, 4, 5, 6):
        p = inputs.kirkwood_offcenter(lvl)
        phi, dphi = KW.surface_values(p.xyz, p.qpos, p.q, a, p.eps1, p.eps2, p.kappa)
        E = KW.solvation_energy(p.qpos, p.q, a, p.eps1, p.eps2, p.kappa)
        for prec, rtol in ((hobi.HOBI_FP64, 1e-9), (hobi.HOBI_MIXED, 1e-7)):
            r = hobi.Problem.from_inputs(ctx, p, precision=prec, rtol=rtol, max_iter=400, restart=400).solve(
                allow_noconv=prec == hobi.HOBI_MIXED)
            errs[(lvl, prec)] = (KW.rel_max_error(r["phi"], SCALE * phi), KW.rel_max_error(r["dphi"], SCALE * dphi),
                                 abs(r["energy"] / E - 1), r["stats"]["iterations"])
    print("\n| level | precision | iterations | e_phi | e_dphi | energy | order phi | order dphi | order E |", flush=True)
    for prec, name in ((hobi.HOBI_FP64, "FP64"), (hobi.HOBI_MIXED, "mixed")):
        for lvl in (3, 4, 5, 6):
            e = errs[(lvl, prec)]
            o = ["", "", ""] if lvl == 3 else [f"{KW.order(2, 1, errs[(lvl - 1, prec)][k], e[k]):.2f}" for k in range(3)]
            print(f"| L{lvl} | {name} | {e[3]} | {e[0]:.3e} | {e[1]:.3e} | {e[2]:.3e} | {o[0]} | {o[1]} | {o[2]} |",
                  flush=True)
    for lvl in (4, 5, 6):
        f, c = errs[(lvl, hobi.HOBI_FP64)], errs[(lvl - 1, hobi.HOBI_FP64)]
        assert KW.order(2, 1, c[0], f[0]) > 1.6 and KW.order(2, 1, c[1], f[1]) > 1.6, lvl
        assert KW.order(2, 1, c[2], f[2]) > 1.8, lvl
        m = errs[(lvl, hobi.HOBI_MIXED)]
        assert abs(m[0] / f[0] - 1) < 0.05 and abs(m[2] / f[2] - 1) < 0.05, lvl


@pytest.fixture(scope="module")
def mol500():
    print("generating the 500-atom surface", flush=True)
    return inputs.molecule(500, seed=3)


def test_molecule500_sampled_rows_and_energy(ctx, mol500):
    """The 500-atom protein-like workload of `bench.py --workload molecule` at full size:
    FP64 rows to 1e-12 and mixed rows to 1e-5 against the oracle, and the mixed solve's
    energy within 1e-5 of FP64."""
    p = mol500
    print(f"molecule nv={p.nv} nf={p.nf}", flush=True)
    st = O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nv, 41)
    rng = np.random.default_rng(2)
    rows = np.unique(np.r_[0:4, p.nv - 4:p.nv, rng.integers(0, p.nv, 24)])
    y_or = O.matvec(st, u, p.kappa, p.eps2 / p.eps1, rows=rows)
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec)
        y = g.matvec(u)
        got = np.stack([y[rows], y[p.nv + rows]])
        err = _rel_inf(got, y_or)
        print(f"molecule500 precision {prec} rel err {err:.3e}", flush=True)
        assert err <= tol
    r64 = hobi.Problem.from_inputs(ctx, p, max_iter=400, restart=400).solve()
    r32 = hobi.Problem.from_inputs(ctx, p, precision=hobi.HOBI_MIXED, max_iter=400, restart=400).solve()
    print("molecule500 E fp64", r64["energy"], "its", r64["stats"]["iterations"], "E mixed", r32["energy"],
          flush=True)
    assert r64["stats"]["converged"] == 1 and r32["stats"]["converged"] == 1
    assert abs(r32["energy"] / r64["energy"] - 1) <= 1e-5


@pytest.fixture(scope="module")
def large():
    print("loading the stored 5000-atom surface", flush=True)
    return inputs.stored_molecule("molecule_5000_s4_g0.4")


def test_large_molecule_sampled_rows_and_energy(ctx, large):
    """The default bench workload at full size: 5000 atoms, 267,718 triangles, 133,859
    vertices, 1.43e11 pairs per matvec, in the launch configuration bench.py times (FP32
    kernel with 8 targets per lane, ~16 passes of node groups).  FP64 rows to 1e-12 and
    mixed rows to 1e-5 against the oracle computed row by row (first and last target
    slots, random rows), then full solves: the mixed energy within 1e-5 of the FP64 one."""
    p = large
    print(f"large molecule nv={p.nv} nf={p.nf}", flush=True)
    st = O.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nv, 51)
    rng = np.random.default_rng(5)
    rows = np.unique(np.r_[0:2, p.nv - 2:p.nv, rng.integers(0, p.nv, 8)])
    y_or = O.matvec(st, u, p.kappa, p.eps2 / p.eps1, rows=rows)
    print("oracle rows done", flush=True)
    res = {}
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec, max_iter=400, restart=400)
        y = g.matvec(u)
        got = np.stack([y[rows], y[p.nv + rows]])
        err = _rel_inf(got, y_or)
        print(f"large precision {prec} rows rel err {err:.3e}", flush=True)
        assert err <= tol
        res[prec] = g.solve()
        print(f"large precision {prec}: E {res[prec]['energy']:.10f} its {res[prec]['stats']['iterations']} "
              f"true residual {res[prec]['stats']['true_residual']:.2e}", flush=True)
        assert res[prec]["stats"]["converged"] == 1
        del g
    r64, r32 = res[hobi.HOBI_FP64], res[hobi.HOBI_MIXED]
    assert abs(r32["energy"] / r64["energy"] - 1) <= 1e-5


def test_library_and_oracle_reject_the_same_meshes(ctx):
    """Mesh validation of hobi_problem_create against the oracle's on the same inputs: a
    valid icosphere, two vertex normals turned inward (two triangles against their vertex
    normals), one reversed triangle, an open surface, normals of length 2, all normals
    inward; accepted or rejected alike, rejections with HOBI_E_MESH."""
    xyz, nrm, tri = inputs.icosphere(2, 2.0)
    a, b = int(tri[0, 0]), int(tri[0, 1])
    fold = nrm.copy()
    fold[[a, b]] *= -1.0
    rev = tri.copy()
    rev[5] = rev[5][::-1]
    cases = {"valid": (xyz, nrm, tri), "fold": (xyz, fold, tri), "reversed": (xyz, nrm, rev),
             "open": (xyz, nrm, tri[1:]), "long_normals": (xyz, 2.0 * nrm, tri), "inward": (xyz, -nrm, tri)}
    qpos, q = np.zeros((1, 3)), np.ones(1)
    for name, (x, n, t) in cases.items():
        try:
            O.validate_mesh(x, n, t)
            oracle_ok = True
        except O.MeshError:
            oracle_ok = False
        try:
            hobi.Problem(ctx, x, n, t, qpos, q)
            lib_ok = True
        except hobi.HobiError as e:
            assert e.name == "HOBI_E_MESH", (name, str(e))
            lib_ok = False
        print(f"mesh case {name}: oracle {'accepts' if oracle_ok else 'rejects'}, "
              f"library {'accepts' if lib_ok else 'rejects'}", flush=True)
        assert oracle_ok == lib_ok, name
        assert oracle_ok == (name == "valid")
