"""GPU parity of the lower-order method (centroid collocation on flat triangles) through the
C ABI against the FP64 lower-order oracle on the same seeded inputs.  Bars as for the
higher-order method: setup arrays 1e-13, FP64 matvec / solve / energy 1e-12 relative,
mixed 1e-5; the served result equals the single-problem result bit for bit."""
import time

import numpy as np
import pytest

from oracle import lobi as LO
from paper_1301_5914_amd import hobi, inputs

pytestmark = pytest.mark.gpu

LOWER = hobi.HOBI_LOWER_ORDER


@pytest.fixture(scope="module")
def ctx():
    return hobi.Context(0)


def _rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


CASES = {
    "centered_L3": inputs.kirkwood_centered(3),
    "offcenter_L3": inputs.kirkwood_offcenter(3),
    "offcenter_L2_k0_eps1_2": inputs.kirkwood_offcenter(2, kappa=0.0, eps1=2.0),
    "offcenter_L2_k1": inputs.kirkwood_offcenter(2, kappa=1.0, eps1=4.0),
    "ico_L0": inputs.kirkwood_centered(0, radius=2.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_lobi_setup_and_matvec_match_oracle(ctx, name):
    p = CASES[name]
    print(f"lobi case {name} nf={p.nf}", flush=True)
    st = LO.setup(p.xyz, p.nrm, p.tri)
    g = hobi.Problem.from_inputs(ctx, p, method=LOWER)
    y, ny, w = g.nodes()
    assert np.max(np.abs(y[:, 0] - st.c)) <= 1e-13 * np.max(np.abs(st.c))
    assert np.max(np.abs(ny[:, 0] - st.n)) <= 1e-13
    assert np.max(np.abs(w[:, 0] - st.W)) <= 1e-13 * np.max(st.W)
    S1, S2 = LO.sources(st.c, st.n, p.qpos, p.q, p.eps1)
    assert _rel_inf(g.rhs(), np.concatenate([S1, S2])) <= 1e-13
    eps = p.eps2 / p.eps1
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g.set_precision(prec)
        for seed in (1, 2):
            u = inputs.random_vector(2 * p.nf, seed)
            err = _rel_inf(g.matvec(u), LO.matvec(st, u, p.kappa, eps))
            print(f"   precision {prec} seed {seed} rel err {err:.3e}", flush=True)
            assert err <= tol


def test_lobi_identity_when_dielectrics_match(ctx):
    p = inputs.kirkwood_offcenter(2, kappa=0.0, eps1=3.0, eps2=3.0)
    for prec in (hobi.HOBI_FP64, hobi.HOBI_MIXED):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec, method=LOWER)
        u = inputs.random_vector(2 * p.nf, 9)
        np.testing.assert_array_equal(g.matvec(u), u)


def test_lobi_ragged_sizes_sampled_rows(ctx):
    """Icosphere L4 (5120 sites: two 2048-target blocks and a ragged third, 80 node blocks)
    and the 30-atom surface, rows at both ends and in between."""
    for p in (inputs.kirkwood_offcenter(4), inputs.molecule(30, seed=7)):
        st = LO.setup(p.xyz, p.nrm, p.tri)
        u = inputs.random_vector(2 * p.nf, 4)
        rows = np.unique(np.r_[0:20, p.nf - 20:p.nf, 2040:2056, np.random.default_rng(0).integers(0, p.nf, 40)])
        y_or = LO.matvec(st, u, p.kappa, p.eps2 / p.eps1, rows=rows)
        for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
            g = hobi.Problem.from_inputs(ctx, p, precision=prec, method=LOWER)
            y = g.matvec(u)
            err = _rel_inf(np.stack([y[rows], y[p.nf + rows]]), y_or)
            print(f"lobi nf={p.nf} precision {prec} rel err {err:.3e}", flush=True)
            assert err <= tol


def test_lobi_solve_matches_oracle(ctx):
    p = inputs.kirkwood_offcenter(2)
    r = hobi.Problem.from_inputs(ctx, p, rtol=1e-12, method=LOWER).solve()
    o = LO.solve(p.xyz, p.nrm, p.tri, p.qpos, p.q, p.eps1, p.eps2, p.kappa, rtol=1e-12)
    print("lobi iterations gpu/oracle", r["stats"]["iterations"], o["iterations"], "E", r["energy"], o["energy"])
    assert abs(r["energy"] / o["energy"] - 1) <= 1e-12
    assert _rel_inf(r["phi"], o["phi"]) <= 1e-11
    assert _rel_inf(r["dphi"], o["dphi"]) <= 1e-11
    rm = hobi.Problem.from_inputs(ctx, p, precision=hobi.HOBI_MIXED, method=LOWER).solve()
    assert abs(rm["energy"] / o["energy"] - 1) <= 1e-5
    assert r["stats"]["pairs_per_matvec"] == p.nf * p.nf


def test_lobi_served_equals_single_problem(ctx):
    sv = hobi.Server(ctx, hbm_budget_bytes=2 << 30, max_slots=8)
    p = inputs.kirkwood_offcenter(3)
    for prec in (hobi.HOBI_FP64, hobi.HOBI_MIXED):
        t = sv.submit(p, precision=prec, max_iter=200, method=LOWER)
        t0 = time.time()
        r = None
        while r is None:
            r = sv.poll(t, raise_errors=False)
            assert time.time() - t0 < 120
            time.sleep(0.002)
        ref = hobi.Problem.from_inputs(ctx, p, precision=prec, max_iter=200, restart=200, method=LOWER).solve()
        assert r["status"] == "HOBI_OK"
        assert r["phi"].shape == (p.nf,)
        np.testing.assert_array_equal(r["phi"], ref["phi"])
        np.testing.assert_array_equal(r["dphi"], ref["dphi"])
        assert r["energy"] == ref["energy"]
    sv.close()


def test_lobi_bench_workload_L6_sampled_rows(ctx):
    """The lower-order bench workload at full size (`bench.py --method lower`: 81920 sites
    and nodes, 8 targets per lane, the same pair plan as the timed run): rows at both ends,
    around slot boundaries and at random, against the oracle row by row, and the mixed
    energy against FP64."""
    p = inputs.kirkwood_offcenter(6)
    st = LO.setup(p.xyz, p.nrm, p.tri)
    u = inputs.random_vector(2 * p.nf, 32)
    rng = np.random.default_rng(3)
    rows = np.unique(np.r_[0:4, p.nf - 4:p.nf, 510:514, 40958:40962, rng.integers(0, p.nf, 24)])
    y_or = LO.matvec(st, u, p.kappa, p.eps2 / p.eps1, rows=rows)
    E = {}
    for prec, tol in ((hobi.HOBI_FP64, 1e-12), (hobi.HOBI_MIXED, 1e-5)):
        g = hobi.Problem.from_inputs(ctx, p, precision=prec, method=LOWER, max_iter=400, restart=400)
        y = g.matvec(u)
        err = _rel_inf(np.stack([y[rows], y[p.nf + rows]]), y_or)
        print(f"lobi L6 precision {prec} rel err {err:.3e}", flush=True)
        assert err <= tol
        E[prec] = g.solve()["energy"]
    assert abs(E[hobi.HOBI_MIXED] / E[hobi.HOBI_FP64] - 1) <= 1e-5
