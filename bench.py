"""Benchmark of the HOBI-PB hot path on one MI355X.

One step = one pass of the whole path on resident inputs: device setup (curved elements,
regular nodes, singular coefficients, source terms), restarted GMRES to ||r||/||b|| <= 1e-6
(every iteration one matvec: gather, dense pair kernel, singular correction + diagonal,
then Gram-Schmidt/Givens on the device) and the solvation energy.

Workload (default): the off-centre Kirkwood sphere -- radius 4 A, 8 seeded charges in
r < 2.5 A, eps1 = 1, eps2 = 80, kappa = 0.1257 / A -- on the level-6 icosphere (40962
vertices, 81920 curved triangles, 327680 quadrature nodes, 1.34e10 pairs per matvec),
mixed precision (FP32 pair kernel, FP64 everywhere else).

Prints one JSON line: value = matvec (vertex, node) pairs evaluated per second over the
timed steps (G-pairs/s), with the dominant kernel's roofline and the FP64 oracle's rate on
the host cores beside it.
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
PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}  # published FP32 (packed) and FP64 vector peaks
PEAK_NONPACKED_FP32 = 78.6                    # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
# HBM bytes per launch of the FP32 pair kernel on the default workload (icosphere L6):
# rocprofv3 FETCH_SIZE (x2.000) + WRITE_SIZE (x1.000), each scaled by a 256 MiB copy.
# Only valid for the kernel build it was measured on; null for any other configuration.
PAIR_F32_L6_TRAFFIC_BYTES = (29821.0 * 2.000 + 518569.0 * 1.000) * 1024


def workload(args):
    from paper_1301_5914_amd import inputs
    if args.mesh:
        # a surface saved by a previous run of the same generator (xyz, nrm, tri, qpos, q)
        d = np.load(args.mesh)
        return inputs.Problem(d["xyz"], d["nrm"], d["tri"].astype(np.int32), d["qpos"], d["q"],
                              name=os.path.basename(args.mesh))
    if args.workload == "molecule":
        return inputs.molecule(args.atoms, seed=args.seed)
    return inputs.kirkwood_offcenter(args.level)


def workload_name(args, prob):
    if args.mesh:
        return f"surface loaded from {prob.name} ({args.mesh_label or 'saved surface'}), {prob.nf} triangles"
    if args.workload == "molecule":
        return (f"protein-like surface, {args.atoms} atoms (seed {args.seed}) at protein density, "
                f"Gaussian density marched at 0.5 A, {prob.nf} triangles")
    return f"off-centre Kirkwood sphere R=4 A, 8 charges, icosphere L{args.level}"


def cpu_baseline(prob, seconds: float, workers: int, lower: bool = False):
    """The FP64 oracle's matvec on a bounded sample of rows of the same workload."""
    from paper_1301_5914_amd import inputs

    eps = prob.eps2 / prob.eps1
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
    u = inputs.random_vector(2 * n_sites, 1)
    # per-row cost measured with all workers busy, then a sample sized to ~`seconds`
    probe = np.arange(4 * cores)
    t0 = time.perf_counter()
    rows_fn(u, probe)
    per_row = (time.perf_counter() - t0) / probe.size
    nrows = int(min(n_sites, max(probe.size, seconds / max(per_row, 1e-9))))
    rows = np.arange(nrows)
    t0 = time.perf_counter()
    rows_fn(u, rows)
    dt = time.perf_counter() - t0
    pairs = nrows * n_nodes
    return {"value": pairs / dt / 1e9, "unit": "G-pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{nrows} of {n_sites} matvec rows (x {n_nodes} nodes), {dt:.1f} s"}


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
               grid=0, lower=False):
    """The treecode form of the matvec on the same problem: matvec time (HIP events, median
    of 20), the dense pair count it replaces per second, its error against the dense matvec
    on a random vector, and the solve with it against the dense solve."""
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
            "energy_rel_diff_vs_dense": abs(res[-1]["energy"] / dense_res["energy"] - 1)}


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


def _make_molecule_job(indexed_job):
    k, job = indexed_job
    return k, _make_molecule(*job)


def serve_bench(pool_mols, n_requests, seed, rate_factor, budget_bytes, max_slots, n_check, tree_theta=0.0):
    """Poisson request stream through the continuous-batching server (mixed precision; with
    tree_theta > 0 every request takes the treecode with the default degree, leaf and
    batch, and the energy check is still against the dense FP64 solve)."""
    from paper_1301_5914_amd import hobi

    rng = np.random.default_rng(seed)

    def draw(k):
        out = []
        for _ in range(k):
            m = pool_mols[int(rng.integers(len(pool_mols)))]
            out.append((m, float(rng.choice([1.0, 2.0, 4.0])), float(rng.choice([0.0, 0.1257]))))
        return out

    ctx = hobi.Context(0)
    sv = hobi.Server(ctx, hbm_budget_bytes=budget_bytes, max_slots=max_slots)

    def submit(req):
        m, e1, kap = req
        return sv.submit(m, precision=hobi.HOBI_MIXED, eps1=e1, kappa=kap, max_iter=400, tree_theta=tree_theta)

    # saturated throughput: a burst submitted at once
    burst = draw(min(16, n_requests))
    t0 = time.perf_counter()
    ts = [submit(r) for r in burst]
    left = set(ts)
    while left:
        for t in list(left):
            if sv.poll(t, raise_errors=False) is not None:
                left.discard(t)
        time.sleep(0.0005)
    sat = len(burst) / (time.perf_counter() - t0)
    rate = rate_factor * sat
    reqs = draw(n_requests)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    sub_time, lat, results = {}, [], {}
    i = 0
    start = time.perf_counter()
    while len(results) < n_requests:
        now = time.perf_counter() - start
        while i < n_requests and arrivals[i] <= now:
            t = submit(reqs[i])
            sub_time[t] = (time.perf_counter(), i)
            i += 1
        for t in [t for t in sub_time if t not in results]:
            r = sv.poll(t, raise_errors=False)
            if r is not None:
                results[t] = r
                lat.append(time.perf_counter() - sub_time[t][0])
                if len(results) % 32 == 0:
                    print(f"[bench] served {len(results)}/{n_requests}", file=sys.stderr, flush=True)
        time.sleep(0.0002)
    wall = time.perf_counter() - start
    st = sv.stats()
    sv.close()
    pairs = sum(r["stats"]["pairs_per_matvec"] * r["stats"]["iterations"] for r in results.values())
    ok = sum(1 for r in results.values() if r["status"] == "HOBI_OK")
    # per-request energy error against the single-problem FP64 path (oracle-validated)
    errs, checks = [], []
    for t in list(results)[:n_check]:
        m, e1, kap = reqs[sub_time[t][1]]
        ref = hobi.Problem(ctx, m.xyz, m.nrm, m.tri, m.qpos, m.q, eps1=e1, eps2=m.eps2, kappa=kap,
                           max_iter=400, restart=400).solve(allow_noconv=True)
        errs.append(abs(results[t]["energy"] / ref["energy"] - 1))
        print(f"[bench] check {len(errs)}/{n_check}: {m.nf} triangles, energy error {errs[-1]:.2e}",
              file=sys.stderr, flush=True)
        checks.append({"nf": m.nf, "eps1": e1, "kappa": kap, "err": errs[-1],
                       "its": results[t]["stats"]["iterations"], "its_fp64": ref["stats"]["iterations"],
                       "status": results[t]["status"], "status_fp64": ref["status"],
                       "E": results[t]["energy"], "E_fp64": ref["energy"]})
    lat_ms = np.array(lat) * 1e3
    sizes = [m.nf for m in pool_mols]
    return {
        "requests": n_requests, "tree_theta": tree_theta, "converged": ok, "arrival_rate_per_s": rate,
        "saturated_rate_per_s": sat, "rate_factor": rate_factor,
        "throughput_requests_per_s": n_requests / wall, "throughput_gpairs_per_s": pairs / wall / 1e9,
        "latency_ms_p50": float(np.percentile(lat_ms, 50)), "latency_ms_p99": float(np.percentile(lat_ms, 99)),
        "latency_ms_mean": float(lat_ms.mean()),
        "mean_active_per_tick": st["mean_batch"], "ticks": st["ticks"], "peak_hbm_bytes": st["peak_bytes"],
        "budget_bytes": budget_bytes,
        "pool": {"molecules": len(pool_mols), "triangles_min": int(min(sizes)), "triangles_max": int(max(sizes))},
        "energy_rel_err_vs_fp64_max": float(max(errs)) if errs else None, "energy_checked": len(errs),
        "checks": checks,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["kirkwood", "molecule"], default="kirkwood")
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
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests in the served stream (0: skip the serving measurement)")
    ap.add_argument("--serve-pool", type=int, default=8, help="distinct molecules the stream draws from")
    ap.add_argument("--serve-min-atoms", type=int, default=50)
    ap.add_argument("--serve-max-atoms", type=int, default=1000)
    ap.add_argument("--serve-rate", type=float, default=0.7, help="arrival rate / saturated throughput")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-tree-theta", type=float, default=0.0,
                    help="serve the stream with the treecode at this opening parameter (0: dense)")
    ap.add_argument("--field-map", type=int, default=64,
                    help="potential map of grid^3 points after the timed steps (hobi_field); 0 = off")
    ap.add_argument("--tree-theta", type=float, default=0.7,
                    help="also time the treecode matvec and solve with this opening parameter (0: skip)")
    ap.add_argument("--tree-degree", type=int, default=5)
    ap.add_argument("--tree-leaf", type=int, default=256)
    ap.add_argument("--tree-batch", type=int, default=128)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    prob = workload(args)
    pool_mols = None
    if args.serve_requests > 0:
        pool_mols = build_pool(args.serve_pool, args.serve_min_atoms, args.serve_max_atoms, 5,
                               max(1, min(16, len(os.sched_getaffinity(0)))))
    cpu = None
    if not args.no_cpu_baseline:
        # before any GPU call: the oracle forks worker processes
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
        cpu = cpu_baseline(prob, args.cpu_seconds, workers, lower=args.method == "lower")

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

    def step():
        pb.set_dielectric(prob.eps1, prob.eps2, prob.kappa)
        return pb.solve()

    for _ in range(args.warmup):
        step()
    pb.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kst = pb.stats()

    pairs_mv = n_sites * n_nodes
    matvecs = sum(r["stats"]["iterations"] + 1 for r in results)   # + the true-residual matvec
    value = matvecs * pairs_mv / wall / 1e9
    avg_pair_ms = kst["ms_pair_kernel"] / max(1, kst["pair_launches"])
    flops = FLOPS_PER_PAIR[prob.kappa > 0] * pairs_mv
    achieved = flops / (avg_pair_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    E = results[-1]["energy"]
    E_exact = None
    if args.workload == "kirkwood" and not args.mesh:
        E_exact = KW.solvation_energy(prob.qpos, prob.q, 4.0, prob.eps1, prob.eps2, prob.kappa)
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
                   "nv": prob.nv, "nf": prob.nf, "nodes": n_nodes, "pairs_per_matvec": pairs_mv,
                   "method": args.method,
                   "kappa": prob.kappa, "eps1": prob.eps1, "eps2": prob.eps2, "rtol": 1e-6,
                   "precision": args.precision},
        "gmres_iterations": results[-1]["stats"]["iterations"],
        "solve_ms": float(np.mean([r["stats"]["ms_solve"] for r in results])),
        "setup_ms": results[-1]["stats"]["ms_setup"],
        "energy_ms": results[-1]["stats"]["ms_energy"],
        "pair_kernel_ms": avg_pair_ms,
        "pair_kernel_gpairs_per_s": pairs_mv / (avg_pair_ms * 1e-3) / 1e9,
        "energy_kcal_mol": E,
        "energy_rel_err_vs_kirkwood": abs(E / E_exact - 1) if E_exact else None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": (PAIR_F32_L6_TRAFFIC_BYTES
                                 if (mixed and args.workload == "kirkwood" and args.level == 6 and not args.mesh and not lower)
                                 else None),
                     "frac_nonpacked_fp32": achieved / PEAK_NONPACKED_FP32 if mixed else None,
                     "kernel": "pair_f32_kernel" if mixed else "pair_f64_kernel",
                     "flops_per_pair": FLOPS_PER_PAIR[prob.kappa > 0]},
    }
    # matvec alone (rows a1-a4, device vectors): median of 20 after 3 warm-ups, HIP events
    # on the library's stream around each call
    uvec = torch.randn(2 * n_sites, dtype=torch.float64, device="cuda")
    yvec = torch.empty_like(uvec)
    torch.cuda.synchronize()
    mv_ms = []
    for i in range(23):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        pb.matvec(uvec, out=yvec)
        ev1.record(stream)
        ev1.synchronize()
        if i >= 3:
            mv_ms.append(ev0.elapsed_time(ev1))
    out["matvec_ms_median"] = float(np.median(mv_ms))
    out["matvec_gpairs_per_s"] = pairs_mv / (out["matvec_ms_median"] * 1e-3) / 1e9
    if args.field_map > 0:
        out["field"] = field_bench(pb, prob, args.field_map, results[-1], mixed, n_nodes)
    if args.tree_theta > 0:
        # (hobi_field takes the treecode with the higher-order method only: no map otherwise)
        out["tree"] = tree_bench(ctx, stream, prob, args.tree_theta, args.tree_degree, args.tree_leaf,
                                 args.tree_batch, mixed, pb, results[-1], out["matvec_ms_median"], pairs_mv,
                                 grid=0 if lower else args.field_map, lower=lower)
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
            "other_pair_kernel_ms": o_pair,
            "mixed_vs_fp64_energy_rel": abs(mixed_E / fp64_E - 1),
            "speedup_mixed_over_fp64_pair_kernel": (o_pair / avg_pair_ms) if mixed else (avg_pair_ms / o_pair),
        }
    if args.calibrate_copy:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    if pool_mols is not None:
        out["serving"] = serve_bench(pool_mols, args.serve_requests, 5, args.serve_rate,
                                     int(args.serve_budget_gb * (1 << 30)), args.serve_slots, n_check=8,
                                     tree_theta=args.serve_tree_theta)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
