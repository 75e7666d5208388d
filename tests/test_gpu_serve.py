"""The request server (continuous batching) through the C ABI: served results equal the
single-problem path, every request's result is bit-for-bit the same alone and in a mix,
admission respects the memory budget, graph replays equal eager launches, errors surface
per request."""
import time

import numpy as np
import pytest

from paper_1301_5914_amd import hobi, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return hobi.Context(0)


def _wait(sv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = sv.poll(t, raise_errors=False)
                if r is not None:
                    out[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(out)} of {len(tickets)} requests finished")
        time.sleep(0.002)
    return out


def _mix():
    return [
        (inputs.kirkwood_offcenter(2), dict(precision=hobi.HOBI_MIXED)),
        (inputs.kirkwood_centered(3), dict(precision=hobi.HOBI_FP64)),
        (inputs.kirkwood_offcenter(3, kappa=0.0, eps1=2.0), dict(precision=hobi.HOBI_MIXED)),
        (inputs.molecule(20, seed=4), dict(precision=hobi.HOBI_MIXED, eps1=4.0)),
        (inputs.kirkwood_offcenter(1, kappa=0.1257), dict(precision=hobi.HOBI_FP64, kappa=0.0)),
    ]


def test_served_equals_single_problem_path(ctx):
    """Alone in the server, a small request (same tile shape as the single-problem path)
    gives the single-problem solve's bits."""
    sv = hobi.Server(ctx, hbm_budget_bytes=2 << 30, max_slots=8)
    for prec, scaled in ((hobi.HOBI_FP64, 2), (hobi.HOBI_MIXED, 2), (hobi.HOBI_MIXED, 1), (hobi.HOBI_MIXED, 0)):
        p = inputs.kirkwood_offcenter(2)
        t = sv.submit(p, precision=prec, max_iter=200, diag_scaling=scaled)
        r = _wait(sv, [t])[t]
        ref = hobi.Problem.from_inputs(ctx, p, precision=prec, max_iter=200, restart=200,
                                       diag_scaling=scaled).solve()
        assert r["status"] == "HOBI_OK"
        assert r["stats"]["iterations"] == ref["stats"]["iterations"]
        np.testing.assert_array_equal(r["phi"], ref["phi"])
        np.testing.assert_array_equal(r["dphi"], ref["dphi"])
        assert r["energy"] == ref["energy"]
    sv.close()


@pytest.mark.parametrize("use_graph", [True, False])
def test_alone_equals_in_the_mix(ctx, use_graph):
    mix = _mix()
    sv = hobi.Server(ctx, hbm_budget_bytes=4 << 30, max_slots=16, use_graph=use_graph)
    alone = []
    for p, kw in mix:
        t = sv.submit(p, **kw)
        alone.append(_wait(sv, [t])[t])
    # all together, with staggered arrivals while others are running
    tickets = []
    for i, (p, kw) in enumerate(mix):
        tickets.append(sv.submit(p, **kw))
        if i % 2 == 1:
            time.sleep(0.01)
    mixed = _wait(sv, tickets)
    st = sv.stats()
    print("server stats", st)
    assert st["mean_batch"] > 1.0
    for a, t in zip(alone, tickets):
        b = mixed[t]
        assert a["status"] == b["status"] == "HOBI_OK"
        np.testing.assert_array_equal(a["phi"], b["phi"])
        np.testing.assert_array_equal(a["dphi"], b["dphi"])
        assert a["energy"] == b["energy"]
    sv.close()


def test_treecode_requests_equal_the_single_problem_path(ctx):
    """Treecode requests (their own matvec launches in each tick) give the bits of
    hobi_solve with the same parameters, alone and next to dense requests; a request with
    bad treecode parameters fails on its own."""
    tree = dict(tree_theta=0.8, tree_degree=4, tree_leaf=128, tree_batch=128)
    cases = [(inputs.kirkwood_offcenter(3), dict(precision=hobi.HOBI_MIXED, **tree)),
             (inputs.kirkwood_offcenter(3, kappa=0.0, eps1=2.0), dict(precision=hobi.HOBI_FP64, **tree)),
             (inputs.kirkwood_centered(3), dict(precision=hobi.HOBI_MIXED)),
             (inputs.kirkwood_offcenter(3), dict(precision=hobi.HOBI_MIXED, method=hobi.HOBI_LOWER_ORDER, **tree))]
    refs = []
    for p, kw in cases:
        g = hobi.Problem.from_inputs(ctx, p, max_iter=200, restart=200, **kw)
        assert kw.get("tree_theta", 0) == 0 or kw.get("method") == hobi.HOBI_LOWER_ORDER or \
            g.stats()["tree_far_pairs"] > 0
        refs.append(g.solve())
    for use_graph in (True, False):
        sv = hobi.Server(ctx, hbm_budget_bytes=4 << 30, max_slots=8, use_graph=use_graph)
        alone = _wait(sv, [sv.submit(cases[0][0], max_iter=200, **cases[0][1])])
        tickets = [sv.submit(p, max_iter=200, **kw) for p, kw in cases]
        bad = sv.submit(cases[0][0], max_iter=200, tree_theta=0.5, tree_degree=9)
        with pytest.raises(hobi.HobiError) as e:   # the defect correction needs a treecode
            sv.submit(cases[0][0], max_iter=200, tree_refine=1)
        assert e.value.status == 1
        out = _wait(sv, tickets + [bad])
        for r, ref in zip([next(iter(alone.values()))] + [out[t] for t in tickets], [refs[0]] + refs):
            assert r["status"] == "HOBI_OK"
            assert r["stats"]["iterations"] == ref["stats"]["iterations"]
            np.testing.assert_array_equal(r["phi"], ref["phi"])
            np.testing.assert_array_equal(r["dphi"], ref["dphi"])
            assert r["energy"] == ref["energy"]
        assert out[bad]["status"] == "HOBI_E_ARG"
        st = sv.stats()
        assert st["bytes_in_use"] == 0 and st["failed"] == 1
        sv.close()


def test_graph_replays_equal_eager_launches(ctx):
    mix = _mix()
    res = {}
    for use_graph in (True, False):
        sv = hobi.Server(ctx, hbm_budget_bytes=4 << 30, max_slots=16, use_graph=use_graph)
        ts = [sv.submit(p, **kw) for p, kw in mix]
        out = _wait(sv, ts)
        res[use_graph] = [out[t] for t in ts]
        sv.close()
    for a, b in zip(res[True], res[False]):
        np.testing.assert_array_equal(a["phi"], b["phi"])
        assert a["energy"] == b["energy"]


def test_admission_respects_the_budget(ctx):
    p = inputs.kirkwood_offcenter(3)
    probe = hobi.Server(ctx, hbm_budget_bytes=1 << 40, max_slots=1)
    t = probe.submit(p)
    _wait(probe, [t])
    one = probe.stats()["peak_bytes"]
    probe.close()
    sv = hobi.Server(ctx, hbm_budget_bytes=int(1.5 * one), max_slots=8)
    ts = [sv.submit(p) for _ in range(4)]
    out = _wait(sv, ts)
    st = sv.stats()
    assert st["peak_bytes"] <= 1.5 * one and st["completed"] == 4
    assert all(r["status"] == "HOBI_OK" for r in out.values())
    with pytest.raises(hobi.HobiError) as e:
        hobi.Server(ctx, hbm_budget_bytes=one // 2, max_slots=2).submit(p)
    assert e.value.name == "HOBI_E_OOM"
    sv.close()


def test_errors_are_reported_per_request(ctx):
    sv = hobi.Server(ctx, hbm_budget_bytes=2 << 30, max_slots=4)
    good = inputs.kirkwood_offcenter(2)
    bad = inputs.kirkwood_offcenter(2)
    bad.tri = bad.tri.copy()
    bad.tri[3] = bad.tri[3][::-1]
    outside = inputs.kirkwood_offcenter(2)
    outside.qpos = outside.qpos.copy()
    outside.qpos[0] = [0.0, 0.0, 9.0]
    ts = [sv.submit(good), sv.submit(bad), sv.submit(outside), sv.submit(good, max_iter=1, rtol=1e-14)]
    out = _wait(sv, ts)
    assert [out[t]["status"] for t in ts] == ["HOBI_OK", "HOBI_E_MESH", "HOBI_E_CHARGE_OUTSIDE", "HOBI_E_NOCONV"]
    with pytest.raises(hobi.HobiError):
        sv.poll(ts[0])   # already collected
    sv.close()


def test_served_energies_match_the_oracle(ctx):
    """Served solves against the FP64 oracle's solve of the same problem (rtol 1e-10 on the
    oracle's side): small protein-like molecules and spheres, mixed and FP64, several eps1
    and kappa, submitted together; energies within 1e-5 (the mixed-mode bar)."""
    from oracle.solve import solve as oracle_solve
    m3, m4 = inputs.molecule(3, seed=1), inputs.molecule(4, seed=2)
    cases = [(m3, dict(precision=hobi.HOBI_MIXED, eps1=1.0, kappa=0.1257)),
             (m4, dict(precision=hobi.HOBI_MIXED, eps1=4.0, kappa=0.0)),
             (m3, dict(precision=hobi.HOBI_FP64, eps1=2.0, kappa=0.1257)),
             (inputs.kirkwood_offcenter(3), dict(precision=hobi.HOBI_MIXED)),
             (inputs.kirkwood_offcenter(2), dict(precision=hobi.HOBI_MIXED, eps1=4.0, kappa=1.0)),
             (inputs.kirkwood_centered(2), dict(precision=hobi.HOBI_FP64, kappa=0.0))]
    sv = hobi.Server(ctx, hbm_budget_bytes=4 << 30, max_slots=8)
    ts = [sv.submit(p, max_iter=300, **kw) for p, kw in cases]
    out = _wait(sv, ts)
    sv.close()
    for (p, kw), t in zip(cases, ts):
        r = out[t]
        assert r["status"] == "HOBI_OK"
        o = oracle_solve(p.xyz, p.nrm, p.tri, p.qpos, p.q, kw.get("eps1", p.eps1), p.eps2, kw.get("kappa", p.kappa),
                         rtol=1e-10, max_iter=300, restart=300)
        err = abs(r["energy"] / o["energy"] - 1)
        print(f"served nv={p.nv} {kw}: E {r['energy']:.8f} oracle {o['energy']:.8f} rel {err:.2e}, "
              f"iterations {r['stats']['iterations']} / {o['iterations']}", flush=True)
        assert err <= 1e-5


def test_admission_respects_the_budget_with_treecode_requests(ctx):
    """Treecode requests are charged their treecode buffers before they run: with room for
    one and a half requests, four run one after another and the peak stays within the
    budget; a budget below one request's needs fails it with HOBI_E_OOM."""
    p = inputs.kirkwood_offcenter(3)
    tree = dict(tree_theta=0.7, tree_degree=4, tree_leaf=128, tree_batch=128)
    probe = hobi.Server(ctx, hbm_budget_bytes=1 << 40, max_slots=1)
    t = probe.submit(p, **tree)
    ref = _wait(probe, [t])[t]
    one = probe.stats()["peak_bytes"]
    probe.close()
    budget = int(1.5 * one)
    sv = hobi.Server(ctx, hbm_budget_bytes=budget, max_slots=8)
    ts = [sv.submit(p, **tree) for _ in range(4)]
    out = _wait(sv, ts)
    st = sv.stats()
    print("treecode budget test:", one, st, flush=True)
    assert st["peak_bytes"] <= budget and st["completed"] == 4 and st["bytes_in_use"] == 0
    for r in out.values():
        assert r["status"] == "HOBI_OK"
        np.testing.assert_array_equal(r["phi"], ref["phi"])
    sv.close()
    # room for the dense footprint but not the treecode buffers: fails alone
    probe2 = hobi.Server(ctx, hbm_budget_bytes=1 << 40, max_slots=1)
    t2 = probe2.submit(p)
    _wait(probe2, [t2])
    dense = probe2.stats()["peak_bytes"]
    probe2.close()
    assert dense < one
    small = hobi.Server(ctx, hbm_budget_bytes=dense, max_slots=2)
    try:
        tt = small.submit(p, **tree)
    except hobi.HobiError as e:        # refused at once: the dense footprint alone is over
        assert e.name == "HOBI_E_OOM"
    else:
        r = _wait(small, [tt])[tt]
        assert r["status"] == "HOBI_E_OOM"
        assert small.stats()["peak_bytes"] <= dense
    small.close()


def test_served_defect_correction_equals_hobi_solve(ctx):
    """tree_refine requests: each request's outer steps run between its ticks with the
    single-problem driver's arithmetic, so a served result is hobi_solve's bit for bit (the
    solution, the energy, the treecode matvecs, the outer steps and the dense residual),
    alone and in a mix with dense and plain treecode requests, with and without graphs."""
    tree = dict(tree_theta=0.9, tree_degree=3, tree_leaf=64, tree_batch=128)
    cases = [(inputs.kirkwood_offcenter(3), dict(precision=hobi.HOBI_MIXED, tree_refine=1, **tree)),
             (inputs.kirkwood_offcenter(3, kappa=0.0, eps1=2.0),
              dict(precision=hobi.HOBI_FP64, tree_refine=1, rtol=1e-9, **tree)),
             (inputs.kirkwood_offcenter(3), dict(precision=hobi.HOBI_MIXED, method=hobi.HOBI_LOWER_ORDER,
                                                 tree_refine=1, **tree)),
             (inputs.kirkwood_offcenter(2), dict(precision=hobi.HOBI_MIXED)),
             (inputs.kirkwood_offcenter(3), dict(precision=hobi.HOBI_MIXED, **tree))]
    refs = [hobi.Problem.from_inputs(ctx, p, max_iter=200, restart=200, **kw).solve() for p, kw in cases]
    for ref, (_, kw) in zip(refs, cases):
        steps = ref["stats"]["refine_steps"]
        print(f"single path: refine {kw.get('tree_refine', 0)} outer {steps} iterations {ref['stats']['iterations']} "
              f"residual {ref['stats']['true_residual']:.3e}", flush=True)
        assert steps >= 2 if kw.get("tree_refine") else steps == 0
    for use_graph in (True, False):
        sv = hobi.Server(ctx, hbm_budget_bytes=4 << 30, max_slots=8, use_graph=use_graph)
        alone = _wait(sv, [sv.submit(cases[0][0], max_iter=200, **cases[0][1])])
        tickets = [sv.submit(p, max_iter=200, **kw) for p, kw in cases]
        out = _wait(sv, tickets)
        for r, ref in zip([next(iter(alone.values()))] + [out[t] for t in tickets], [refs[0]] + refs):
            assert r["status"] == "HOBI_OK"
            for key in ("iterations", "refine_steps", "dense_matvecs"):
                assert r["stats"][key] == ref["stats"][key], key
            np.testing.assert_array_equal(r["phi"], ref["phi"])
            np.testing.assert_array_equal(r["dphi"], ref["dphi"])
            assert r["energy"] == ref["energy"]
            if ref["stats"]["refine_steps"]:
                assert r["stats"]["true_residual"] == ref["stats"]["true_residual"]
        st = sv.stats()
        assert st["bytes_in_use"] == 0 and st["failed"] == 0
        sv.close()

