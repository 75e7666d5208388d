"""Benchmark of the HOBI-PB hot path on one MI355X.

One step = one pass of the whole path on resident inputs: device setup (curved elements,
regular nodes, singular coefficients, source terms), restarted GMRES to ||r||/||b|| <= 1e-6
(every iteration one matvec: gather, dense pair kernel, singular correction + diagonal,
then Gram-Schmidt/Givens on the device) and the solvation energy.

Workload (default): the large protein-like surface -- 5000 atoms packed at protein density
(seed 4), partial charges N(0, 0.4) e at the atom centres, the Gaussian-density surface
marched on a 0.4 A grid (267,718 curved triangles, 133,859 vertices, 1,070,872 quadrature
nodes, 1.43e11 pairs per matvec), eps1 = 1, eps2 = 80, kappa = 0.1257 / A, mixed precision
(FP32 pair kernel, FP64 everywhere else).  The off-centre Kirkwood sphere at icosphere
level 6 is measured beside it (matvec and pair kernel, energy against the series).

Prints one JSON line: value = matvec (vertex, node) pairs evaluated per second over the
timed steps (G-pairs/s), with the dominant kernel's roofline, the FP64 oracle's rate on
the host cores and the GPU rows' error against the oracle's rows beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = {True: 58, False: 28}      # kappa > 0 / kappa = 0 (algorithmic count)
TRANS_PER_PAIR = {True: 2, False: 1}        # exp and rsqrt / rsqrt only
PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}  # published FP32 and FP64 vector peaks
CUS, CLOCK_HZ = 256, 2.4e9
FLOPS_PER_CLK_CU = {"mixed": 256.0, "fp64": 128.0}   # the peaks above per clock per CU
# HBM bytes per launch of the FP32 pair kernel on the default workload, from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE; each scaled by what it reads for a plain device copy
# of known size), valid only for the kernel sources they were taken on: keyed by the
# workload and a hash of those sources, else the bench reports null.
PAIR_TRAFFIC = {    # (workload, precision, sources sha16) -> (bytes per launch, profile file)
    ("large", "mixed", "b2c3fab00f3435cf"): (524756276, "profiles/pair_f32_kernel_molecule5000_hbm_counters.md"),
}
KERNEL_SOURCES = ("paper_1301_5914_amd/csrc/pair_tile.h", "paper_1301_5914_amd/csrc/pair_kernels.hip",
                  "paper_1301_5914_amd/csrc/hobi_device.h")

# Cycles of one wave64 transcendental instruction on a SIMD at 2.4 GHz, measured by the
# issue-rate probe (paper_1301_5914_amd/probes/issue_rate.hip, profiles/valu_issue_rate_probe.md);
# results per clock per compute unit = 4 SIMDs x 64 lanes / cycles.
TRANS_CYCLES_F32 = {"exp": 8.32, "rsq": 8.19}


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(args):
    from paper_1301_5914_amd import inputs
    if args.mesh:
        # a surface saved by a previous run of the same generator (xyz, nrm, tri, qpos, q)
        d = np.load(args.mesh)
        return inputs.Problem(d["xyz"], d["nrm"], d["tri"].astype(np.int32), d["qpos"], d["q"],
                              name=os.path.basename(args.mesh))
    if args.workload == "large":
        return inputs.stored_molecule("molecule_5000_s4_g0.4")
    if args.workload == "molecule":
        return inputs.molecule(args.atoms, seed=args.seed)
    return inputs.kirkwood_offcenter(args.level)


def surface_quality(prob):
    """The surface's smallest triangle angle, connected components and Euler characteristic
    (V - E + F: 2 per sphere-like component, 0 for a torus-like one)."""
    from paper_1301_5914_amd import inputs
    amin, comps, euler = inputs.mesh_quality(prob.xyz, prob.tri)
    return {"min_angle_deg": round(amin, 2), "components": comps, "euler_characteristic": euler}


def workload_name(args, prob):
    if args.mesh:
        return f"surface loaded from {prob.name} ({args.mesh_label or 'saved surface'}), {prob.nf} triangles"
    if args.workload == "large":
        return (f"large protein-like surface: 5000 atoms at protein density (seed 4), Gaussian density "
                f"marched at 0.4 A, {prob.nf} triangles, {prob.nv} vertices")
    if args.workload == "molecule":
        return (f"protein-like surface, {args.atoms} atoms (seed {args.seed}) at protein density, "
                f"Gaussian density marched at 0.5 A, {prob.nf} triangles")
    return f"off-centre Kirkwood sphere R=4 A, 8 charges, icosphere L{args.level}"


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, seconds: float, workers: int, lower: bool = False):
    """The FP64 oracle's matvec on a bounded sample of rows of the same workload.  Returns
    the baseline record and (u, rows, oracle rows) for the comparison with the GPU rows."""
    from paper_1301_5914_amd import inputs

    eps = prob.eps2 / prob.eps1
    t_setup = time.perf_counter()
    if lower:
        from oracle import lobi as LO
        st = LO.setup(prob.xyz, prob.nrm, prob.tri)
        n_sites, n_nodes = prob.nf, prob.nf

        def rows_fn(u, rows):
            return LO.matvec(st, u, prob.kappa, eps, rows=rows)
        cores = 1   # the lower-order oracle runs in one process
    else:
        from oracle import operator as O
        st = O.setup(prob.xyz, prob.nrm, prob.tri)
        n_sites, n_nodes = prob.nv, 4 * prob.nf

        def rows_fn(u, rows):
            return O.matvec(st, u, prob.kappa, eps, rows=rows, workers=workers)
        cores = workers
    t_setup = time.perf_counter() - t_setup
    u = inputs.random_vector(2 * n_sites, 1)
    rng = np.random.default_rng(0)

    def block(n):
        # a contiguous run of rows at a seeded offset (the oracle spreads a contiguous run
        # of rows over its worker processes)
        n = min(n, n_sites)
        a = int(rng.integers(0, n_sites - n + 1))
        return np.arange(a, a + n)
    # per-row cost measured with all workers busy, then a sample sized to ~`seconds`
    probe = block(4 * cores if cores > 1 else 4)
    t0 = time.perf_counter()
    rows_fn(u, probe)
    per_row = (time.perf_counter() - t0) / probe.size
    nrows = int(min(n_sites, max(probe.size, seconds / max(per_row, 1e-9))))
    rows = block(nrows)
    t0 = time.perf_counter()
    y_rows = rows_fn(u, rows)
    dt = time.perf_counter() - t0
    pairs = nrows * n_nodes
    rec = {"value": pairs / dt / 1e9, "unit": "G-pairs/s", "cores": cores, "kind": "oracle",
           "sample": f"{nrows} consecutive of {n_sites} matvec rows (x {n_nodes} nodes), {dt:.1f} s "
                     f"(oracle setup {t_setup:.1f} s, not timed)",
           "cpu_model": cpu_model(), "host_cpus_visible": len(os.sched_getaffinity(0)),
           "gpairs_per_s_per_core": pairs / dt / 1e9 / max(1, cores),
           "full_matvec_s_extrapolated": dt * n_sites / nrows}
    return rec, (u, rows, y_rows)


def rows_rel_err(y_gpu, sample):
    """max |GPU rows - oracle rows| / max |oracle rows| over the sampled row pairs."""
    u, rows, y_or = sample
    n = y_gpu.shape[0] // 2
    got = np.stack([y_gpu[rows], y_gpu[n + rows]])
    return float(np.max(np.abs(got - y_or)) / np.max(np.abs(y_or)))


def pair_roofline(precision: str, kappa_pos: bool, pairs: int, avg_ms: float, workload_key: str):
    """Roofline of the dominant kernel (the dense pair kernel): algorithmic flops per launch
    over the HIP-event average launch time, against the published vector peak; the
    mix-adjusted fraction charges each pair its transcendentals at the probed rate."""
    flops = FLOPS_PER_PAIR[kappa_pos] * pairs
    achieved = flops / (avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    out = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
           "traffic": None, "kernel": "pair_f32_kernel" if precision == "mixed" else "pair_f64_kernel",
           "flops_per_pair": FLOPS_PER_PAIR[kappa_pos]}
    if precision == "mixed" and TRANS_CYCLES_F32["exp"]:
        # clocks of one CU per pair: flops at 256 per clock, each transcendental at tau per clock
        tau_exp = 4 * 64 / TRANS_CYCLES_F32["exp"]
        tau_rsq = 4 * 64 / TRANS_CYCLES_F32["rsq"]
        clk = FLOPS_PER_PAIR[kappa_pos] / FLOPS_PER_CLK_CU["mixed"] + 1.0 / tau_rsq + (1.0 / tau_exp if kappa_pos else 0.0)
        pairs_max = CUS * CLOCK_HZ / clk
        out["mix_adjusted"] = {"pairs_per_s_ceiling": pairs_max, "tau_exp": tau_exp, "tau_rsq": tau_rsq,
                               "frac": pairs / (avg_ms * 1e-3) / pairs_max,
                               "source": "profiles/valu_issue_rate_probe.md"}
    key = (workload_key, precision, kernel_sources_hash())
    if key in PAIR_TRAFFIC:
        out["traffic"], out["traffic_source"] = PAIR_TRAFFIC[key]
    out["kernel_sources_sha16"] = key[2]
    return out


def l6_leg(ctx, stream, mixed):
    """The off-centre Kirkwood sphere at icosphere level 6 beside the headline workload: the
    matvec (median of 20 after 3 warm-ups), the pair kernel (HIP events) and a solve's energy
    against the Kirkwood series."""
    import torch
    from oracle import kirkwood as KW
    from paper_1301_5914_amd import hobi, inputs
    p = inputs.kirkwood_offcenter(6)
    pb = hobi.Problem.from_inputs(ctx, p, precision=hobi.HOBI_MIXED if mixed else hobi.HOBI_FP64,
                                  max_iter=400, restart=400)
    res = pb.solve()
    mv = matvec_median(pb, stream, 2 * p.nv)
    pb.reset_stats()
    u = torch.randn(2 * p.nv, dtype=torch.float64, device="cuda")
    y = torch.empty_like(u)
    for _ in range(20):
        pb.matvec(u, out=y)
    torch.cuda.synchronize()
    st = pb.stats()
    avg = st["ms_pair_kernel"] / max(1, st["pair_launches"])
    pairs = p.nv * 4 * p.nf
    E = KW.solvation_energy(p.qpos, p.q, 4.0, p.eps1, p.eps2, p.kappa)
    return {"workload": "off-centre Kirkwood sphere R=4 A, 8 charges, icosphere L6", "nv": p.nv, "nf": p.nf,
            "pairs_per_matvec": pairs, "matvec_ms_median": mv, "matvec_gpairs_per_s": pairs / (mv * 1e-3) / 1e9,
            "pair_kernel_ms": avg,
            "roofline": pair_roofline("mixed" if mixed else "fp64", True, pairs, avg, "kirkwood_L6"),
            "gmres_iterations": res["stats"]["iterations"], "solve_ms": res["stats"]["ms_solve"],
            "energy_rel_err_vs_kirkwood": abs(res["energy"] / E - 1)}


def matvec_median(pb, stream, n, reps=20, warm=3):
    """Median ms of hobi_matvec on device vectors (HIP events on the library's stream)."""
    import torch
    u = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(u)
    torch.cuda.synchronize()
    ms = []
    for i in range(reps + warm):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        pb.matvec(u, out=y)
        ev1.record(stream)
        ev1.synchronize()
        if i >= warm:
            ms.append(ev0.elapsed_time(ev1))
    return float(np.median(ms))


FIELD_FLOPS_PER_PAIR = {True: 60, False: 41}   # R, grad R and the solid angle per (point, node)


def map_points(prob, grid):
    """A grid^3 lattice over the surface's bounding box grown by 30% (inside and outside)."""
    lo, hi = prob.xyz.min(axis=0), prob.xyz.max(axis=0)
    c, h = 0.5 * (lo + hi), 0.65 * (hi - lo)
    axes = [np.linspace(c[k] - h[k], c[k] + h[k], grid) for k in range(3)]
    return np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)


def timed_map(pb, u, pts, reps=3):
    """hobi_field on pts: (outputs, median whole-call ms, median field-kernel ms)."""
    pb.field(u, pts[:1024])                       # work space and code warm-up
    times, kern = [], []
    out = None
    for _ in range(reps):
        pb.reset_stats()
        t0 = time.perf_counter()
        out = pb.field(u, pts)
        times.append((time.perf_counter() - t0) * 1e3)
        st = pb.stats()
        kern.append(st["ms_field_kernel"] / max(1, st["field_launches"]))
    return out, float(np.median(times)), float(np.median(kern))


def field_bench(pb, prob, grid, res, mixed, n_nodes):
    """Potential map: hobi_field on a grid^3 lattice over the surface's bounding box grown by
    30% (points inside and outside), for the solved surface of the last timed step."""
    from paper_1301_5914_amd import hobi
    unit = 4.0 * np.pi * 332.0716
    u = np.concatenate([res["phi"], res["dphi"]]) / unit
    pts = map_points(prob, grid)
    out, call_ms, k_ms = timed_map(pb, u, pts)
    pairs = pts.shape[0] * n_nodes
    flops = FIELD_FLOPS_PER_PAIR[prob.kappa > 0]
    achieved = flops * pairs / (k_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS["mixed" if mixed else "fp64"]
    # end-to-end cross-check: the energy from the reaction potential at the charges
    at_q = pb.field(u, prob.qpos)
    e_field = 0.5 * float(np.sum(prob.q * at_q["reac"]))
    return {"grid": grid, "points": int(pts.shape[0]), "pairs": int(pairs),
            "kernel_ms": k_ms, "kernel_gpairs_per_s": pairs / (k_ms * 1e-3) / 1e9,
            "call_ms_median": call_ms,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved / peak, "flops_per_pair": flops},
            "inside_fraction": float(np.mean(out["inside"])),
            "energy_from_field_rel": abs(e_field / res["energy"] - 1)}


def tree_bench(ctx, stream, prob, theta, degree, leaf, batch, mixed, dense_pb, dense_res, dense_mv_ms, pairs_mv,
               grid=0, lower=False, refine=(0.8, 3, 128, 128)):
    """The treecode form of the matvec on the same problem: matvec time (HIP events, median
    of 20), the dense pair count it replaces per second, its error against the dense matvec
    on a random vector, and the solve with it against the dense solve; then the dense system
    solved through a treecode of parameters `refine` (theta, degree, leaf, batch) by defect
    correction."""
    import torch
    from paper_1301_5914_amd import hobi
    pb = hobi.Problem.from_inputs(ctx, prob, precision=hobi.HOBI_MIXED if mixed else hobi.HOBI_FP64,
                                  method=hobi.HOBI_LOWER_ORDER if lower else hobi.HOBI_HIGHER_ORDER,
                                  tree_theta=theta, tree_degree=degree, tree_leaf=leaf, tree_batch=batch,
                                  max_iter=400, restart=400)
    st = pb.stats()
    u = torch.randn(2 * (prob.nf if lower else prob.nv), dtype=torch.float64, device="cuda")
    yt = torch.empty_like(u)
    yd = torch.empty_like(u)
    ms = []
    for i in range(23):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        pb.matvec(u, out=yt)
        ev1.record(stream)
        ev1.synchronize()
        if i >= 3:
            ms.append(ev0.elapsed_time(ev1))
    dense_pb.matvec(u, out=yd)
    torch.cuda.synchronize()
    err = float((yt - yd).abs().max() / yd.abs().max())
    pb.solve()                                        # warm-up
    res = [pb.solve() for _ in range(2)]
    mv = float(np.median(ms))
    # the dense system to the same rtol by defect correction with a treecode (tree_refine): its
    # accuracy only sets how many outer steps it takes, so a cheaper one than above serves
    r_theta, r_degree, r_leaf, r_batch = refine
    rp = hobi.Problem.from_inputs(ctx, prob, precision=hobi.HOBI_MIXED if mixed else hobi.HOBI_FP64,
                                  method=hobi.HOBI_LOWER_ORDER if lower else hobi.HOBI_HIGHER_ORDER,
                                  tree_theta=r_theta, tree_degree=r_degree, tree_leaf=r_leaf, tree_batch=r_batch,
                                  max_iter=400, restart=400, tree_refine=1)
    rp.solve()                                        # warm-up
    rr = [rp.solve() for _ in range(2)]
    del rp
    rs = rr[-1]["stats"]
    r_ms = float(np.mean([r["stats"]["ms_solve"] for r in rr]))
    refined = {"what": "the dense system A u = b by defect correction: treecode GMRES for each correction, "
                       "the dense matvec for each outer residual; it stops on the dense residual",
               "theta": r_theta, "degree": r_degree, "leaf": r_leaf, "batch": r_batch,
               "solve_ms": r_ms, "treecode_matvecs": rs["iterations"], "outer_steps": rs["refine_steps"],
               "dense_matvecs": rs["dense_matvecs"], "dense_true_residual": rs["true_residual"],
               "dense_solve_ms": dense_res["stats"]["ms_solve"],
               "dense_solve_true_residual": dense_res["stats"]["true_residual"],
               "speedup_over_dense_solve": dense_res["stats"]["ms_solve"] / r_ms,
               "energy_rel_diff_vs_dense": abs(rr[-1]["energy"] / dense_res["energy"] - 1)}
    fmap = None
    if grid > 0:
        # the potential map of the dense solution, with the treecode and with the dense sums
        unit = 4.0 * np.pi * 332.0716
        uu = np.concatenate([dense_res["phi"], dense_res["dphi"]]) / unit
        pts = map_points(prob, grid)
        od, d_call, d_kern = timed_map(dense_pb, uu, pts)
        ot, t_call, t_kern = timed_map(pb, uu, pts)
        fst = pb.stats()
        rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        fmap = {"grid": grid, "points": int(pts.shape[0]),
                "far_pairs": fst["field_tree_far_pairs"], "near_pairs": fst["field_tree_near_pairs"],
                "kernel_ms": t_kern, "call_ms_median": t_call, "dense_kernel_ms": d_kern,
                "dense_call_ms_median": d_call, "speedup_kernel": d_kern / t_kern, "speedup_call": d_call / t_call,
                "phi_rel_err_vs_dense": rel(ot["phi"], od["phi"]), "field_rel_err_vs_dense": rel(ot["field"], od["field"]),
                "inside_mismatches": int(np.sum(ot["inside"] != od["inside"]))}
    return {"theta": theta, "degree": degree, "leaf": leaf, "batch": batch, "map": fmap,
            "far_pairs": st["tree_far_pairs"], "near_pairs": st["tree_near_pairs"],
            "matvec_ms_median": mv, "dense_matvec_ms_median": dense_mv_ms,
            "speedup_over_dense_matvec": dense_mv_ms / mv,
            "equivalent_gpairs_per_s": pairs_mv / (mv * 1e-3) / 1e9,
            "matvec_rel_err_vs_dense": err,
            "gmres_iterations": res[-1]["stats"]["iterations"],
            "solve_ms": float(np.mean([r["stats"]["ms_solve"] for r in res])),
            "dense_solve_ms": dense_res["stats"]["ms_solve"],
            "energy_rel_diff_vs_dense": abs(res[-1]["energy"] / dense_res["energy"] - 1),
            "refined": refined}


def _make_molecule(n_atoms, seed):
    from paper_1301_5914_amd import inputs
    return inputs.molecule(int(n_atoms), seed=int(seed))


def build_pool(n_mol, min_atoms, max_atoms, seed, workers):
    """Seeded pool of protein-like molecules, atom counts log-uniform in [min, max]."""
    import multiprocessing as mp
    rng = np.random.default_rng(seed)
    atoms = np.round(np.exp(rng.uniform(np.log(min_atoms), np.log(max_atoms), n_mol))).astype(int)
    jobs = [(int(a), 1000 + i) for i, a in enumerate(atoms)]
    out = [None] * n_mol
    with mp.get_context("fork").Pool(max(1, min(workers, n_mol))) as pool:
        for done, (k, m) in enumerate(pool.imap_unordered(_make_molecule_job, list(enumerate(jobs)))):
            out[k] = m
            print(f"[bench] pool molecule {done + 1}/{n_mol}: {m.nf} triangles", file=sys.stderr, flush=True)
    return out


def load_or_build_pool(path, n_mol, min_atoms, max_atoms, seed, workers):
    """build_pool, or its molecules from `path` when that file holds the same pool (written
    there by an earlier run with the same arguments)."""
    from paper_1301_5914_amd import inputs
    key = np.array([n_mol, min_atoms, max_atoms, seed])
    if path and os.path.exists(path):
        d = np.load(path)
        if np.array_equal(d["key"], key):
            return [inputs.Problem(d[f"xyz{i}"], d[f"nrm{i}"], d[f"tri{i}"], d[f"qpos{i}"], d[f"q{i}"],
                                   name=f"pool{i}") for i in range(n_mol)]
    mols = build_pool(n_mol, min_atoms, max_atoms, seed, workers)
    if path:
        arrs = {"key": key}
        for i, m in enumerate(mols):
            arrs.update({f"xyz{i}": m.xyz, f"nrm{i}": m.nrm, f"tri{i}": m.tri, f"qpos{i}": m.qpos, f"q{i}": m.q})
        np.savez(path, **arrs)
    return mols


def _make_molecule_job(indexed_job):
    k, job = indexed_job
    return k, _make_molecule(*job)


def serve_bench(pool_mols, n_requests, seed, rate_factors, budget_bytes, max_slots, n_check, tree_theta=0.0,
                fp64_all=False, tree_degree=5, tree_leaf=256, tree_refine=0):
    """Poisson request streams through the continuous-batching server (mixed precision; with
    tree_theta > 0 every request takes the treecode of that theta, degree and leaf, and with
    tree_refine solves the dense system through it by defect correction): one stream per
    arrival-rate factor (the same requests, arrivals at that factor
    times the saturated rate of a 16-request burst).  The first factor's results are checked
    against the FP64 oracle (n_check requests) and, with fp64_all, every request's energy
    against a GPU FP64 solve of its (molecule, eps1, kappa)."""
    from paper_1301_5914_amd import hobi

    rng = np.random.default_rng(seed)

    def draw(k):
        out = []
        for _ in range(k):
            m = pool_mols[int(rng.integers(len(pool_mols)))]
            out.append((m, float(rng.choice([1.0, 2.0, 4.0])), float(rng.choice([0.0, 0.1257]))))
        return out

    ctx = hobi.Context(0)

    def submit(sv, req):
        m, e1, kap = req
        return sv.submit(m, precision=hobi.HOBI_MIXED, eps1=e1, kappa=kap, max_iter=400, tree_theta=tree_theta,
                         tree_degree=tree_degree, tree_leaf=tree_leaf, tree_refine=tree_refine)

    # saturated throughput: a burst submitted at once
    sv = hobi.Server(ctx, hbm_budget_bytes=budget_bytes, max_slots=max_slots)
    burst = draw(min(16, n_requests))
    t0 = time.perf_counter()
    ts = [submit(sv, r) for r in burst]
    left = set(ts)
    while left:
        for t in list(left):
            if sv.poll(t, raise_errors=False) is not None:
                left.discard(t)
        time.sleep(0.0005)
    sat = len(burst) / (time.perf_counter() - t0)
    sv.close()
    reqs = draw(n_requests)

    def stream(rate_factor):
        sv = hobi.Server(ctx, hbm_budget_bytes=budget_bytes, max_slots=max_slots)
        rate = rate_factor * sat
        arrivals = np.cumsum(np.random.default_rng([seed, int(round(rate_factor * 1000))]).exponential(
            1.0 / rate, n_requests))
        sub_time, lat, results = {}, [], {}
        i = 0
        start = time.perf_counter()
        while len(results) < n_requests:
            now = time.perf_counter() - start
            while i < n_requests and arrivals[i] <= now:
                t = submit(sv, reqs[i])
                sub_time[t] = (time.perf_counter(), i)
                i += 1
            for t in [t for t in sub_time if t not in results]:
                r = sv.poll(t, raise_errors=False)
                if r is not None:
                    results[t] = r
                    lat.append(time.perf_counter() - sub_time[t][0])
                    if len(results) % 32 == 0:
                        print(f"[bench] rate {rate_factor}: served {len(results)}/{n_requests}", file=sys.stderr,
                              flush=True)
            time.sleep(0.0002)
        wall = time.perf_counter() - start
        st = sv.stats()
        sv.close()
        pairs = sum(r["stats"]["pairs_per_matvec"] * r["stats"]["iterations"] for r in results.values())
        lat_ms = np.array(lat) * 1e3
        summary = {
            "rate_factor": rate_factor, "arrival_rate_per_s": rate,
            "converged": sum(1 for r in results.values() if r["status"] == "HOBI_OK"),
            "throughput_requests_per_s": n_requests / wall, "throughput_gpairs_per_s": pairs / wall / 1e9,
            "latency_ms_p50": float(np.percentile(lat_ms, 50)), "latency_ms_p99": float(np.percentile(lat_ms, 99)),
            "latency_ms_mean": float(lat_ms.mean()),
            "mean_active_per_tick": st["mean_batch"], "ticks": st["ticks"], "peak_hbm_bytes": st["peak_bytes"]}
        return summary, results, sub_time

    first, results, sub_time = stream(rate_factors[0])
    others = [stream(f)[0] for f in rate_factors[1:]]
    ok = first["converged"]
    # checks against the FP64 oracle: the served solution's energy recomputed by the oracle,
    # and the oracle's residual rows b - A u of the served solution (random rows), on
    # n_check requests with distinct (molecule, eps1, kappa), smallest molecules first
    # (single process: the GPU is initialised, so the oracle forks no workers here)
    from oracle import COULOMB_KCAL, FOUR_PI
    from oracle import operator as O
    seen, picks = set(), []
    for t in sorted(results, key=lambda t: (reqs[sub_time[t][1]][0].nf, t)):
        m, e1, kap = reqs[sub_time[t][1]]
        if (id(m), e1, kap) in seen or results[t]["status"] != "HOBI_OK":
            continue
        seen.add((id(m), e1, kap))
        picks.append(t)
        if len(picks) == n_check:
            break
    setups, checks = {}, []
    crng = np.random.default_rng(7)
    for t in picks:
        m, e1, kap = reqs[sub_time[t][1]]
        if id(m) not in setups:
            setups[id(m)] = O.setup(m.xyz, m.nrm, m.tri)
        st_or = setups[id(m)]
        eps = m.eps2 / e1
        r = results[t]
        u = np.concatenate([r["phi"], r["dphi"]]) / (FOUR_PI * COULOMB_KCAL)
        E_or = O.solvation_energy(st_or, u, m.qpos, m.q, kap, eps)
        S1, S2 = O.sources(st_or.xyz, st_or.nrm, m.qpos, m.q, e1)
        rows = np.sort(crng.choice(m.nv, min(32, m.nv), replace=False))
        Au = O.matvec(st_or, u, kap, eps, rows=rows)
        b = np.stack([S1[rows], S2[rows]])
        resid = float(np.max(np.abs(b - Au)) / max(np.max(np.abs(S1)), np.max(np.abs(S2))))
        checks.append({"nf": m.nf, "nc": m.nc, "eps1": e1, "kappa": kap, "its": r["stats"]["iterations"],
                       "E": r["energy"], "E_oracle_at_u": E_or, "energy_rel_err": abs(r["energy"] / E_or - 1),
                       "oracle_residual_rows": resid})
        print(f"[bench] oracle check {len(checks)}/{len(picks)}: {m.nf} triangles, energy {checks[-1]['energy_rel_err']:.1e}, "
              f"residual rows {resid:.1e}", file=sys.stderr, flush=True)
    # every request's energy against a GPU FP64 solve of its (molecule, eps1, kappa)
    fp64 = None
    if fp64_all:
        ref = {}
        for t in sorted(results, key=lambda t: sub_time[t][1]):
            m, e1, kap = reqs[sub_time[t][1]]
            key = (id(m), e1, kap)
            if key not in ref:
                pb = hobi.Problem(ctx, m.xyz, m.nrm, m.tri, m.qpos, m.q, e1, m.eps2, kap, precision=hobi.HOBI_FP64,
                                  max_iter=400, restart=400)
                res = pb.solve(allow_noconv=True)
                ref[key] = (res["energy"], res["status"] == "HOBI_OK")
                pb.close()
        errs = [abs(results[t]["energy"] / ref[(id(reqs[sub_time[t][1]][0]),) + reqs[sub_time[t][1]][1:]][0] - 1)
                for t in results if results[t]["status"] == "HOBI_OK"]
        fp64 = {"requests": len(errs), "combinations": len(ref),
                "fp64_converged": sum(1 for v in ref.values() if v[1]),
                "energy_rel_err_max": float(max(errs)), "energy_rel_err_median": float(np.median(errs)),
                "what": "|E_served / E_fp64 - 1| for every served request, E_fp64 a GPU FP64 solve (rtol 1e-6) "
                        "of the request's (molecule, eps1, kappa)"}
    sizes = [m.nf for m in pool_mols]
    return {
        "requests": n_requests, "tree_theta": tree_theta,
        "tree": ({"degree": tree_degree, "leaf": tree_leaf, "refine": tree_refine} if tree_theta > 0 else None),
        "converged": ok,
        "arrival_rate_per_s": first["arrival_rate_per_s"],
        "saturated_rate_per_s": sat, "rate_factor": first["rate_factor"],
        "throughput_requests_per_s": first["throughput_requests_per_s"],
        "throughput_gpairs_per_s": first["throughput_gpairs_per_s"],
        "latency_ms_p50": first["latency_ms_p50"], "latency_ms_p99": first["latency_ms_p99"],
        "latency_ms_mean": first["latency_ms_mean"],
        "mean_active_per_tick": first["mean_active_per_tick"], "ticks": first["ticks"],
        "peak_hbm_bytes": first["peak_hbm_bytes"],
        "budget_bytes": budget_bytes,
        "other_rates": others,
        "fp64_all": fp64,
        "pool": {"molecules": len(pool_mols), "triangles_min": int(min(sizes)), "triangles_max": int(max(sizes))},
        "oracle_checks": {
            "requests": len(checks),
            "energy_rel_err_max": max((c["energy_rel_err"] for c in checks), default=None),
            "residual_rows_max": max((c["oracle_residual_rows"] for c in checks), default=None),
            "what": "served solution u: |E_served / E_oracle(u) - 1| and max |b - A u| / max |b| over 32 "
                    "random oracle rows (FP64 oracle), distinct (molecule, eps1, kappa), smallest first",
            "checks": checks},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["large", "kirkwood", "molecule"], default="large",
                    help="large: the stored 5000-atom surface (default); kirkwood: the off-centre sphere at "
                         "--level; molecule: a generated protein-like surface of --atoms atoms")
    ap.add_argument("--level", type=int, default=6, help="icosphere level (kirkwood)")
    ap.add_argument("--atoms", type=int, default=500, help="atom count (molecule)")
    ap.add_argument("--seed", type=int, default=3, help="packing seed (molecule)")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--method", choices=["higher", "lower"], default="higher",
                    help="higher-order (curved, vertex unknowns) or lower-order (flat, centroid) scheme")
    ap.add_argument("--max-iter", type=int, default=400, help="GMRES iteration cap (unrestarted)")
    ap.add_argument("--mesh", default=None,
                    help="load the surface and charges from an .npz (xyz, nrm, tri, qpos, q) instead of generating")
    ap.add_argument("--mesh-label", default=None, help="description of the loaded surface for the JSON line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison solve in the other precision")
    ap.add_argument("--no-l6", action="store_true", help="skip the icosphere-L6 leg beside the workload")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests in the served stream (0: skip the serving measurement)")
    ap.add_argument("--serve-pool", type=int, default=8, help="distinct molecules the stream draws from")
    ap.add_argument("--serve-min-atoms", type=int, default=50)
    ap.add_argument("--serve-max-atoms", type=int, default=1000)
    ap.add_argument("--serve-rate", default="0.7",
                    help="arrival rate / saturated throughput; a comma-separated list runs one stream per factor "
                         "(the first is the reported one, the others go to serving.other_rates)")
    ap.add_argument("--serve-fp64-all", action="store_true",
                    help="check every served request's energy against a GPU FP64 solve of its problem")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-checks", type=int, default=16, help="served requests checked against the oracle")
    ap.add_argument("--serve-pool-cache", default=None,
                    help=".npz to load the molecule pool from (written there if absent or different)")
    ap.add_argument("--serve-tree-theta", type=float, default=0.0,
                    help="serve the stream with the treecode at this opening parameter (0: dense)")
    ap.add_argument("--serve-tree-degree", type=int, default=5)
    ap.add_argument("--serve-tree-leaf", type=int, default=256)
    ap.add_argument("--serve-tree-refine", action="store_true",
                    help="served treecode requests solve the dense system by defect correction (tree_refine)")
    ap.add_argument("--field-map", type=int, default=64,
                    help="potential map of grid^3 points after the timed steps (hobi_field); 0 = off")
    ap.add_argument("--tree-theta", type=float, default=0.7,
                    help="also time the treecode matvec and solve with this opening parameter (0: skip)")
    ap.add_argument("--tree-degree", type=int, default=5)
    ap.add_argument("--tree-leaf", type=int, default=256)
    ap.add_argument("--tree-batch", type=int, default=128)
    ap.add_argument("--refine-theta", type=float, default=0.8,
                    help="treecode of the defect-correction solve in the treecode leg (tree_refine)")
    ap.add_argument("--refine-degree", type=int, default=3)
    ap.add_argument("--refine-leaf", type=int, default=128)
    ap.add_argument("--refine-batch", type=int, default=128)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (the path runs on one device); --gpus must be 1"}))
        sys.exit(2)

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    prob = workload(args)
    progress(f"workload: {prob.nv} sites, {prob.nf} triangles")
    pool_mols = None
    # a one-GPU job gets a share of 16 host cores
    host_workers = max(1, min(16, len(os.sched_getaffinity(0))))
    if args.serve_requests > 0:
        pool_mols = load_or_build_pool(args.serve_pool_cache, args.serve_pool, args.serve_min_atoms,
                                       args.serve_max_atoms, 5, host_workers)
    cpu, sample = None, None
    if not args.no_cpu_baseline:
        # before any GPU call: the oracle forks worker processes
        cpu, sample = cpu_baseline(prob, args.cpu_seconds, host_workers, lower=args.method == "lower")
        progress(f"oracle baseline: {cpu['sample']}")

    import torch
    from oracle import kirkwood as KW
    from paper_1301_5914_amd import hobi

    mixed = args.precision == "mixed"
    stream = torch.cuda.Stream()          # kernels and their timing events share this stream
    ctx = hobi.Context(0, stream=stream, profiling=True)
    lower = args.method == "lower"
    n_sites = prob.nf if lower else prob.nv
    n_nodes = prob.nf if lower else 4 * prob.nf
    pb = hobi.Problem.from_inputs(ctx, prob, precision=hobi.HOBI_MIXED if mixed else hobi.HOBI_FP64,
                                  method=hobi.HOBI_LOWER_ORDER if lower else hobi.HOBI_HIGHER_ORDER,
                                  max_iter=args.max_iter, restart=args.max_iter)
    progress("problem created")

    def step():
        pb.set_dielectric(prob.eps1, prob.eps2, prob.kappa)
        return pb.solve()

    for _ in range(args.warmup):
        step()
    progress("warm-up done")
    pb.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kst = pb.stats()
    progress(f"timed steps done: {wall:.1f} s")

    pairs_mv = n_sites * n_nodes
    matvecs = sum(r["stats"]["iterations"] + 1 for r in results)   # + the true-residual matvec
    value = matvecs * pairs_mv / wall / 1e9
    avg_pair_ms = kst["ms_pair_kernel"] / max(1, kst["pair_launches"])
    E = results[-1]["energy"]
    E_exact = None
    if args.workload == "kirkwood" and not args.mesh:
        E_exact = KW.solvation_energy(prob.qpos, prob.q, 4.0, prob.eps1, prob.eps2, prob.kappa)
    wkey = ("large" if args.workload == "large" and not args.mesh else
            f"{args.workload}_{args.level if args.workload == 'kirkwood' else args.atoms}") + ("_lower" if lower else "")
    out = {
        "metric": "matvec G-pairs/s + GMRES solve time to 1e-6; serving p50/p99 latency",
        "value": value,
        "unit": "G-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-pairs/f64-accumulate" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": workload_name(args, prob),
                   "nv": prob.nv, "nf": prob.nf, "nc": prob.nc, "nodes": n_nodes, "pairs_per_matvec": pairs_mv,
                   "method": args.method,
                   "kappa": prob.kappa, "eps1": prob.eps1, "eps2": prob.eps2, "rtol": 1e-6,
                   "precision": args.precision,
                   "surface": surface_quality(prob)},
        "gmres_iterations": results[-1]["stats"]["iterations"],
        "gmres_converged": bool(results[-1]["stats"]["converged"]),
        "true_residual": results[-1]["stats"]["true_residual"],
        "solve_ms": float(np.mean([r["stats"]["ms_solve"] for r in results])),
        "setup_ms": results[-1]["stats"]["ms_setup"],
        "energy_ms": results[-1]["stats"]["ms_energy"],
        "pair_kernel_ms": avg_pair_ms,
        "pair_kernel_gpairs_per_s": pairs_mv / (avg_pair_ms * 1e-3) / 1e9,
        "energy_kcal_mol": E,
        "energy_rel_err_vs_kirkwood": abs(E / E_exact - 1) if E_exact else None,
        "roofline": pair_roofline(args.precision, prob.kappa > 0, pairs_mv, avg_pair_ms, wkey),
    }
    # matvec alone (rows a1-a4, device vectors): median of 20 after 3 warm-ups, HIP events
    # on the library's stream around each call
    out["matvec_ms_median"] = matvec_median(pb, stream, 2 * n_sites)
    out["matvec_gpairs_per_s"] = pairs_mv / (out["matvec_ms_median"] * 1e-3) / 1e9
    if sample is not None:
        # the GPU's rows of the same matvec against the oracle's rows of cpu_baseline
        y = pb.matvec(sample[0])
        out["oracle_rows"] = {"rows": int(sample[1].size), "rel_err": rows_rel_err(y, sample),
                              "what": "max |y_gpu - y_oracle| / max |y_oracle| over the cpu_baseline rows, same u"}
    progress("matvec timed")
    if args.field_map > 0:
        out["field"] = field_bench(pb, prob, args.field_map, results[-1], mixed, n_nodes)
        progress("field map done")
    if args.tree_theta > 0:
        # (hobi_field takes the treecode with the higher-order method only: no map otherwise)
        out["tree"] = tree_bench(ctx, stream, prob, args.tree_theta, args.tree_degree, args.tree_leaf,
                                 args.tree_batch, mixed, pb, results[-1], out["matvec_ms_median"], pairs_mv,
                                 grid=0 if lower else args.field_map, lower=lower,
                                 refine=(args.refine_theta, args.refine_degree, args.refine_leaf, args.refine_batch))
        progress("treecode leg done")
        ref = out["tree"].get("refined") or {}
        if "solve_ms" in ref:
            # the time to the dense system's solution at rtol: GMRES on it, and defect correction
            out["time_to_dense_solution_ms"] = {"gmres": out["solve_ms"], "defect_correction": ref["solve_ms"],
                                                "defect_correction_treecode": [ref["theta"], ref["degree"],
                                                                               ref["leaf"], ref["batch"]]}
    if not args.no_compare:
        # the other precision on the same problem (outside the timed region)
        pb.set_precision(hobi.HOBI_FP64 if mixed else hobi.HOBI_MIXED)
        pb.reset_stats()
        other = pb.solve()
        ost = pb.stats()
        o_pair = ost["ms_pair_kernel"] / max(1, ost["pair_launches"])
        fp64_E = other["energy"] if mixed else E
        mixed_E = E if mixed else other["energy"]
        out["compare"] = {
            "other_precision": "fp64" if mixed else "mixed",
            "other_solve_ms": other["stats"]["ms_solve"],
            "other_iterations": other["stats"]["iterations"],
            "other_converged": bool(other["stats"]["converged"]),
            "other_pair_kernel_ms": o_pair,
            "other_roofline": pair_roofline("fp64" if mixed else "mixed", prob.kappa > 0, pairs_mv, o_pair, wkey),
            "mixed_vs_fp64_energy_rel": abs(mixed_E / fp64_E - 1),
            "speedup_mixed_over_fp64_pair_kernel": (o_pair / avg_pair_ms) if mixed else (avg_pair_ms / o_pair),
        }
        if sample is not None:
            out["compare"]["other_oracle_rows_rel_err"] = rows_rel_err(pb.matvec(sample[0]), sample)
        pb.set_precision(hobi.HOBI_MIXED if mixed else hobi.HOBI_FP64)
        progress("comparison solve done")
    if not args.no_l6 and not (args.workload == "kirkwood" and args.level == 6) and not lower:
        out["l6"] = l6_leg(ctx, stream, mixed)
        progress("L6 leg done")
    if args.calibrate_copy:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    if pool_mols is not None:
        out["serving"] = serve_bench(pool_mols, args.serve_requests, 5,
                                     [float(f) for f in args.serve_rate.split(",")],
                                     int(args.serve_budget_gb * (1 << 30)), args.serve_slots, args.serve_checks,
                                     tree_theta=args.serve_tree_theta, fp64_all=args.serve_fp64_all,
                                     tree_degree=args.serve_tree_degree, tree_leaf=args.serve_tree_leaf,
                                     tree_refine=1 if args.serve_tree_refine else 0)
        full = (args.serve_requests >= 512 and args.serve_pool >= 16 and args.serve_max_atoms >= 3000)
        out["serving"]["reduced"] = not full
        if not full:
            out["serving"]["full_stream"] = ("512 requests, 16 molecules of 50-3000 atoms: "
                                             "profiles/serving_stream_512_requests.md")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
