#!/usr/bin/env python3
"""Push/pull sweep benchmark on one MI355X.

One step = the whole hot path over the R-MAT scale-22 graph (edge factor 16,
a,b,c = .57,.19,.19, seed 1, symmetrised, deduplicated, int32 CSR):
  * PageRank, 20 Jacobi steps, pulling form (f = 0.85, FP32)
  * PageRank, 20 Jacobi steps, pushing form
  * BFS from 64 seeded non-isolated roots: top-down (push), bottom-up (pull)
    and direction-switching.
value = traversed edges per second over the step, in GTEPS: a PageRank step
traverses nnz edges; a BFS traverses the undirected edges of the root's
component (sum of reached degrees / 2).  Per-part rates are in "parts".

The roofline object covers one pull step (the sweep's kernels): algorithmic
bytes per step (4*nnz + 20*n: offsets, indices, gathered contributions, 1/d,
the iterate and the next contributions) over the average step time measured
with HIP events around the 20-step pull run, against the published 8 TB/s and
against a measured device-to-device copy.  roofline_bfs_{push,pull,switch} do
the same per BFS run for the level kernels.  "batched" holds the measured
speedups of the batched forms over their sequential counterparts: PPR with
k = 256 sources on R-MAT 20 against 256 single-vector runs, and the 512-graph
launch against the graphs run one by one.  The CPU baseline is the FP64 C
oracle on the host's cores on a bounded sample of the same work.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
F = 0.85
PR_ITERS = 20
N_ROOTS = 64


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--scale", type=int, default=22)
    p.add_argument("--roots", type=int, default=N_ROOTS)
    p.add_argument("--only", default="", help="comma list of parts to run (pr_pull,pr_push,bfs_push,bfs_pull,bfs_switch)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-batched", action="store_true", help="skip the batched-vs-sequential measurements")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 1 GiB read + 1 GiB write elementwise kernel (counter calibration)")
    p.add_argument("--workload", default="rmat22",
                   help="rmat22 (default: the headline step), or a supplementary measurement: "
                        "ppr20, multi512, grid4096, er22, adjoint20, tc16, tc18, bc16, pprgrid")
    p.add_argument("--tuned", default=os.path.join(ROOT, "paper_2010_16012_amd", "tuned.json"),
                   help="autotuner cache to apply (ignored when missing)")
    p.add_argument("--counters-summary", nargs="+", metavar="CSV",
                   help="no GPU work: turn two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, "
                        "WRITE_SIZE) of 'bench.py --only pr_pull --copy-calibration' into the pull kernel's "
                        "HBM traffic per launch, written to profiles/; an optional third file with "
                        "TCC_EA0_RDREQ_{32B,64B,128B}_sum adds the read-request size breakdown")
    return p.parse_args()


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2010_16012_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_src_hash):
    """HBM traffic per pull step from a committed counter summary, if it still
    describes the current kernel source."""
    path = os.path.join(ROOT, "profiles", "pr_pull_rmat22_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_src_hash:
        return None
    return d.get("traffic_bytes_per_launch")


# kernels of one pull step: the sweep (one dispatch per step) and its fix-ups
STEP_SWEEP = ("pp::k_pr_tiled<", "pp::k_pr_pull<")
STEP_AUX = ("pp::k_pr_tiled_combine(", "pp::k_pr_pull_fix(")
CALIB_BYTES = 1 << 30  # the calibration kernel reads 1 GiB and writes 1 GiB


def counters_summary(fetch_csv, write_csv, sizes_csv=None):
    """HBM bytes per pull step from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), summed over the step's kernels and each divided by what the
    same counter reads for the plain 1 GiB-in / 1 GiB-out calibration kernel
    over 1 GiB."""
    import csv

    def per_step(path, counter, scale=1024.0):
        total, sweeps, calib = 0.0, 0, []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"]) * scale
                name = r["Kernel_Name"]
                if any(k in name for k in STEP_SWEEP):
                    total += v
                    sweeps += 1
                elif any(k in name for k in STEP_AUX):
                    total += v
                elif "neg_kernel" in name:
                    calib.append(v)
        if not sweeps or not calib:
            raise SystemExit(f"{path}: expected pull sweeps and a calibration dispatch "
                             f"(got {sweeps} and {len(calib)})")
        return total / sweeps, _median(calib)

    f_step, f_cal = per_step(fetch_csv, "FETCH_SIZE")
    w_step, w_cal = per_step(write_csv, "WRITE_SIZE")
    k_f, k_w = f_cal / CALIB_BYTES, w_cal / CALIB_BYTES
    traffic = f_step / k_f + w_step / k_w
    out = {"kernels": list(STEP_SWEEP + STEP_AUX), "per": "pull step", "workload": "rmat22_ef16_seed1_sym",
           "source_hash": source_hash("pr.hip"),
           "fetch_bytes_per_launch_raw": round(f_step), "write_bytes_per_launch_raw": round(w_step),
           "fetch_calibration_factor": round(k_f, 4), "write_calibration_factor": round(k_w, 4),
           "traffic_bytes_per_launch": round(traffic)}
    if sizes_csv:
        # read requests from L2 to memory by size; bytes = sum(size * count)
        by = {}
        for sz in (32, 64, 128):
            by[sz] = per_step(sizes_csv, f"TCC_EA0_RDREQ_{sz}B_sum", 1.0)
        out["read_requests_per_launch"] = {f"{sz}B": round(by[sz][0]) for sz in by}
        out["read_bytes_per_launch_by_size"] = round(sum(sz * by[sz][0] for sz in by))
        out["calibration_read_bytes_by_size"] = round(sum(sz * by[sz][1] for sz in by))
    path = os.path.join(ROOT, "profiles", "pr_pull_rmat22_counters.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=5):
    """Device-to-device streaming rate (GB/s, bytes read + written) of a plain
    copy and of an elementwise kernel over 1 GiB; the faster of the two."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    best = (0.0, "")
    for kind, fn in (("copy_", lambda: b.copy_(a)), ("neg", lambda: torch.neg(a, out=b))):
        fn()
        ms = _median([_events_ms(fn) for _ in range(reps)])
        gbs = 2 * nbytes / (ms * 1e-3) / 1e9
        if gbs > best[0]:
            best = (gbs, f"{kind} of 1 GiB")
    del a, b
    torch.cuda.empty_cache()
    return best


def bfs_replay_bytes(n, fr, ex, di, dirs):
    """Algorithmic bytes of a BFS run from the oracle's replay of its direction
    schedule: top-down steps 4*E + 8*|F| + 12*|new|; bottom-up steps
    4*E + 8*|unvisited| + 8*|new| + 3*ceil(n/8) (three bitmaps)."""
    tot, visited = 0, 1
    for step in range(len(ex)):
        if dirs[step] == 0:
            tot += 4 * ex[step] + 8 * fr[step] + 12 * di[step]
        else:
            tot += 4 * ex[step] + 8 * (n - visited) + 8 * di[step] + 3 * ((n + 7) // 8)
        visited += di[step]
    return int(tot)


def cpu_leg(args, host, roots, root_edges, runs, policy, alpha, beta, parts):
    """The FP64 oracle timed on the host's cores (a bounded sample of the
    step), plus the oracle's replay of the GPU's BFS direction schedules for
    two roots, which gives the algorithmic bytes of the pull and switch runs."""
    import oracle

    n, nnz = host.n, host.nnz
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass

    def timed(fn):
        t = time.perf_counter()
        r = fn()
        return time.perf_counter() - t, r

    # each call builds its own in-adjacency first: the per-step time is the
    # difference of a 21-step and a 1-step run (median of three each)
    t1 = _median([timed(lambda: oracle.pagerank_threads(host.off, host.idx, F, 1))[0] for _ in range(3)])
    t21s, threads = [], 1
    for _ in range(3):
        dt, (_, threads) = timed(lambda: oracle.pagerank_threads(host.off, host.idx, F, 21))
        t21s.append(dt)
    t_iter_mt = (_median(t21s) - t1) / 20
    if t_iter_mt <= 0:
        raise RuntimeError("CPU baseline: the 21-step run was not slower than the 1-step run")
    s1, _ = timed(lambda: oracle.pagerank(host.off, host.idx, F, 1))
    s3, _ = timed(lambda: oracle.pagerank(host.off, host.idx, F, 3))
    t_iter_st = (s3 - s1) / 2
    if t_iter_st <= 0:
        raise RuntimeError("CPU baseline: the 3-step run was not slower than the 1-step run")
    t_bfs, _ = timed(lambda: [oracle.bfs(host.off, host.idx, int(r)) for r in roots[:2]])
    bfs_edges = float(root_edges[:2].sum())
    cpu = {"value": round(nnz / t_iter_mt / 1e9, 5), "unit": "GTEPS", "cores": threads, "kind": "oracle",
           "sample": f"FP64 pulling PageRank step on the same rmat{args.scale} graph over {threads} threads "
                     f"({t_iter_mt * 1e3:.1f} ms per step: 21-step minus 1-step run, median of 3)",
           "nproc": os.cpu_count(), "cpu_model": model,
           "single_thread_pr_gteps": round(nnz / t_iter_st / 1e9, 5),
           "single_thread_bfs_gteps": round(bfs_edges / t_bfs / 1e9, 5),
           "single_thread_sample": f"one PageRank step ({t_iter_st:.2f} s, 3-step minus 1-step run) and FIFO BFS "
                                   f"from 2 of the {len(roots)} roots ({t_bfs:.2f} s)"}

    out = {}
    for p, name in (("bfs_pull", "pull"), ("bfs_switch", "switch")):
        if p not in parts:
            continue
        tot_bytes, tot_ms = 0, 0.0
        for root in roots[:2]:
            r = runs[p]
            _, dirs, _, _ = r.run_logged(int(root), policy[p], alpha, beta)
            tot_ms += _median([_events_ms(lambda: r.run(int(root), policy[p], alpha, beta)) for _ in range(3)])
            fr, ex, di = oracle.bfs_replay(host.off, host.idx, int(root), dirs)
            tot_bytes += bfs_replay_bytes(n, fr, ex, di, dirs)
        achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
        out[name] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"k_bfs_level+k_bfs_chunks, {name} runs",
                     "algorithmic_bytes_per_run": round(tot_bytes / 2), "run_ms": round(tot_ms / 2, 4),
                     "roots": 2, "bytes_from": "oracle replay of the GPU direction schedule"}
    return cpu, out


def batched_speedups(args, torch, gg, pp, autotune):
    """Measured (not extrapolated) speedups of the batched forms."""
    return {"ppr_rmat20_k256": ppr_speedup(args, torch, gg, pp, autotune),
            "multi512": multi_speedup(args, torch, gg, pp, autotune)}


def ppr_speedup(args, torch, gg, pp, autotune):
    """PPR on R-MAT 20 with k = 256 seeded sources, 30 sweeps, in k-column
    tiles, against the 256 columns run one after another with the
    single-vector sweep (k_tile = 1), pull and push."""
    host = gg.rmat(20, 16, seed=1)
    src = gg.pick_vertices(host, 256, seed=2)
    tuned = autotune.load(args.tuned, host.n, host.nnz)
    autotune.apply(tuned)
    kt = tuned.get("k_tile", 64)
    g = pp.Graph(host)
    work = host.nnz * len(src) * 30
    ppr = {"n": host.n, "nnz": host.nnz, "k": len(src), "iters": 30, "k_tile": kt}
    for d, name in ((pp.PP_PULL, "pull"), (pp.PP_PUSH, "push")):
        pp.ppr(g, src[:kt], iters=2, k_tile=kt, direction=d)
        ms_b = _median([_events_ms(lambda: pp.ppr(g, src, iters=30, k_tile=kt, direction=d)) for _ in range(3)])
        pp.ppr(g, src[:2], iters=2, k_tile=1, direction=d)
        ms_s = _events_ms(lambda: pp.ppr(g, src, iters=30, k_tile=1, direction=d))
        ppr[name] = {"batched_ms": round(ms_b, 2), "batched_gteps": round(work / (ms_b * 1e-3) / 1e9, 2),
                     "sequential_ms": round(ms_s, 2), "sequential_gteps": round(work / (ms_s * 1e-3) / 1e9, 2),
                     "speedup": round(ms_s / ms_b, 2)}
    g.close()
    del g
    torch.cuda.empty_cache()
    return ppr


def multi_speedup(args, torch, gg, pp, autotune):
    """512 R-MAT graphs (scales 8-14) in one launch (PageRank x20 pull, BFS
    switch from vertex 0) against the same work graph by graph.  The launch
    mapping comes from the autotuner's entry for this batch's size class."""
    gs = gg.rmat_batch(512, 8, 14, seed=1)
    tuned = autotune.load_key(args.tuned, autotune.multi_key(len(gs), sum(h.n for h in gs),
                                                                 sum(int(h.nnz) for h in gs)))
    autotune.apply(tuned)
    mg = pp.MultiGraph(gs)
    mg.run(pr_iters=20, pr_dir=pp.PP_PULL, bfs_policy=pp.PP_SWITCH)
    ms_one = _median([_events_ms(lambda: mg.run(pr_iters=20, pr_dir=pp.PP_PULL, bfs_policy=pp.PP_SWITCH))
                      for _ in range(3)])
    graphs = [pp.Graph(h) for h in gs]
    bruns = [pp.BfsRun(gr) for gr in graphs]
    xs = [torch.empty(h.n, dtype=torch.float32, device="cuda") for h in gs]

    def seq():
        for gr, r, x, h in zip(graphs, bruns, xs, gs):
            x.fill_(1.0 / h.n)
            pp.pagerank_into(gr, x, 20, 0.85, pp.PP_PULL)
            r.run(0, pp.PP_SWITCH)
    seq()
    ms_seq = _events_ms(seq)
    out = {"graphs": len(gs), "total_nnz": int(sum(h.nnz for h in gs)), "pr_iters": 20,
           "one_launch_ms": round(ms_one, 3), "graph_by_graph_ms": round(ms_seq, 2),
           "speedup": round(ms_seq / ms_one, 2)}
    for gr in graphs:
        gr.close()
    return out


def main():
    args = parse()
    if args.counters_summary:
        return counters_summary(*args.counters_summary)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the sweep would shard by "
              "vertex ranges across GPUs; the library runs on one GPU)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import scipy.sparse as sp
    import scipy.sparse.csgraph as csg
    import torch

    import graphgen as gg
    import paper_2010_16012_amd as pp

    if args.workload != "rmat22":
        return supplementary(args)
    from paper_2010_16012_amd import autotune

    parts = ["pr_pull", "pr_push", "bfs_push", "bfs_pull", "bfs_switch"]
    if args.only:
        parts = [p for p in parts + ["pr_hybrid"] if p in args.only.split(",")]
    dev = torch.device("cuda:0")
    t_gen = time.time()
    host = gg.rmat(args.scale, 16, seed=1)
    n, nnz = host.n, host.nnz
    roots = gg.pick_vertices(host, args.roots, seed=1)
    print(f"# graph rmat{args.scale}: n={n} nnz={nnz} generated in {time.time() - t_gen:.1f}s", flush=True)
    # edges of each root's component, from the host graph (independent of the GPU path)
    root_edges = np.zeros(len(roots))
    if any(p.startswith("bfs_") for p in parts):
        A = sp.csr_matrix((np.ones(nnz, dtype=np.int8), host.idx, host.off), shape=(n, n))
        ncomp, comp = csg.connected_components(A, directed=False)
        deg = np.diff(host.off)
        comp_edges = np.bincount(comp, weights=deg, minlength=ncomp)
        root_edges = comp_edges[comp[roots]] / 2.0
        del A

    tuned = autotune.load(args.tuned, n, nnz) if os.path.exists(args.tuned) else {}
    autotune.apply(tuned)
    alpha, beta = tuned.get("alpha", 14.0), tuned.get("beta", 24.0)
    t_up = time.time()
    g = pp.Graph(host, device=dev)
    torch.cuda.synchronize()
    print(f"# uploaded and registered in {time.time() - t_up:.1f}s", flush=True)
    x = torch.empty(n, dtype=torch.float32, device=dev)
    runs = {p: pp.BfsRun(g) for p in ("bfs_push", "bfs_pull", "bfs_switch")}
    policy = {"bfs_push": pp.PP_PUSH, "bfs_pull": pp.PP_PULL, "bfs_switch": pp.PP_SWITCH}

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def step(times):
        for p in parts:
            e0 = ev()
            if p.startswith("pr_"):
                x.fill_(1.0 / n)
                e0 = ev()  # the fill is not part of the sweep
                d = {"pr_pull": pp.PP_PULL, "pr_push": pp.PP_PUSH, "pr_hybrid": pp.PP_SWITCH}[p]
                pp.pagerank_into(g, x, PR_ITERS, F, d)
            else:
                # every root in turn on the device, one host wait for all
                runs[p].run_many(roots, policy[p], alpha, beta)
            e1 = ev()
            times.setdefault(p, []).append((e0, e1))

    for _ in range(args.warmup):
        step({})
    torch.cuda.synchronize()
    times = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(times)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps

    part_ms = {p: float(np.mean([a.elapsed_time(b) for a, b in times[p]])) for p in parts}
    part_edges = {"pr_pull": PR_ITERS * nnz, "pr_push": PR_ITERS * nnz, "pr_hybrid": PR_ITERS * nnz}
    for p in ("bfs_push", "bfs_pull", "bfs_switch"):
        part_edges[p] = float(root_edges.sum())
    step_edges = sum(part_edges[p] for p in parts)
    value = step_edges / (ms_step * 1e-3) / 1e9

    out_parts = {}
    for p in parts:
        d = {"ms": round(part_ms[p], 4), "gteps": round(part_edges[p] / (part_ms[p] * 1e-3) / 1e9, 3)}
        if p.startswith("bfs_"):
            ms_root = part_ms[p] / len(roots)
            per_root = root_edges / (ms_root * 1e-3) / 1e9
            d["ms_per_root"] = round(ms_root, 4)
            d["gteps_hmean_roots"] = round(float(len(per_root) / np.sum(1.0 / per_root)), 3)
        else:
            d["us_per_iter"] = round(part_ms[p] * 1e3 / PR_ITERS, 2)
        out_parts[p] = d

    roofline = None
    if "pr_pull" in parts:
        # one pull step reads offsets (4n), indices (4 nnz), the gathered
        # contribution (4n) and 1/d (4n) and writes the iterate (4n) and the
        # next contribution (4n).  The library writes the iterate only after
        # the last step, so 4 nnz + 16n is reported beside it.
        algo = 4 * nnz + 20 * n
        algo_min = 4 * nnz + 16 * n
        t_launch = part_ms["pr_pull"] * 1e-3 / PR_ITERS
        achieved = algo / t_launch / 1e9
        tiled = g.slices()[0] > 0
        copy_gbs, copy_kind = copy_bandwidth(torch, dev)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(source_hash("pr.hip")),
                    "kernel": ("k_pr_tiled+k_pr_tiled_combine+k_pr_pull_fix" if tiled else "k_pr_pull+k_pr_pull_fix"),
                    "per": "pull step", "algorithmic_bytes_per_launch": algo, "launch_us": round(t_launch * 1e6, 2),
                    "frac_without_x_write": round(algo_min / t_launch / 1e9 / HBM_PEAK_GBS, 4),
                    "copy_gbs": round(copy_gbs, 1), "copy_kind": copy_kind,
                    "frac_of_copy": round(achieved / copy_gbs, 4)}

    # The BFS level kernels take much of the step, but their work changes from
    # level to level, so their roofline is stated per run.  A top-down BFS
    # examines every out-edge of every frontier vertex once: per run
    # 4*E (indices) + 8*R (frontier offsets) + 12*(R-1) (level, parent, queue
    # of every new vertex), with E the out-edges of the R reached vertices.
    roofline_bfs = {}
    if "bfs_push" in parts:
        tot = 0
        for root in roots:  # outside the timed region: statistics only
            st = runs["bfs_push"].run(int(root), pp.PP_PUSH, alpha, beta)
            tot += 4 * st.edges_reached + 8 * st.reached + 12 * (st.reached - 1)
        achieved = tot / (part_ms["bfs_push"] * 1e-3) / 1e9
        roofline_bfs["push"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                                "kernel": "k_bfs_level+k_bfs_chunks, top-down runs",
                                "algorithmic_bytes_per_run": round(tot / len(roots)),
                                "run_ms": round(part_ms["bfs_push"] / len(roots), 4), "roots": len(roots)}

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.neg(a, out=b)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b

    batched = None if args.no_batched else batched_speedups(args, torch, gg, pp, autotune)

    cpu = None
    if not args.no_cpu_baseline:
        cpu, replay_rooflines = cpu_leg(args, host, roots, root_edges, runs, policy, alpha, beta, parts)
        roofline_bfs.update(replay_rooflines)

    line = {
        "metric": "GTEPS per PageRank iter & BFS, push vs pull; % of HBM roofline",
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+i32",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_ef16_seed1_sym: PageRank x{PR_ITERS} pull+push, "
                               f"BFS from {len(roots)} roots push/pull/switch",
                   "n": n, "nnz": nnz, "parts": parts, "tuning": tuned or "defaults"},
        "parts": out_parts,
        "roofline": roofline,
        "roofline_bfs": roofline_bfs or None,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def _events_ms(fn):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def supplementary(args):
    """Measurements of the other configurations (one JSON line each)."""
    import numpy as np
    import torch

    import graphgen as gg
    import paper_2010_16012_amd as pp
    from paper_2010_16012_amd import autotune

    w = args.workload
    line = {"workload": w, "n_gpus": 1, "data": "synthetic"}
    if w == "ppr20":
        line.update(ppr_speedup(args, torch, gg, pp, autotune))
    elif w == "multi512":
        line.update(multi_speedup(args, torch, gg, pp, autotune))
    elif w in ("grid4096", "er22"):
        host = gg.workload(w)
        g = pp.Graph(host)
        x = torch.empty(host.n, dtype=torch.float32, device="cuda")
        for d, name in ((pp.PP_PULL, "pr_pull"), (pp.PP_PUSH, "pr_push")):
            x.fill_(1.0 / host.n)
            pp.pagerank_into(g, x, 2, 0.85, d)
            ms = _events_ms(lambda: pp.pagerank_into(g, x, 20, 0.85, d))
            line[name] = {"us_per_iter": round(ms * 1e3 / 20, 1), "gteps": round(host.nnz * 20 / (ms * 1e-3) / 1e9, 2)}
        r = pp.BfsRun(g)
        for pol, name in ((pp.PP_PUSH, "bfs_push"), (pp.PP_PULL, "bfs_pull"), (pp.PP_SWITCH, "bfs_switch")):
            st = r.run(0, pol)
            ms = _events_ms(lambda: r.run(0, pol))
            line[name] = {"ms": round(ms, 2), "levels": st.levels,
                          "gteps": round(st.edges_reached / 2 / (ms * 1e-3) / 1e9, 3)}
        line.update({"n": host.n, "nnz": host.nnz})
    elif w == "adjoint20":
        host = gg.rmat(20, 16, seed=1)
        gg.with_weights(host, seed=5)
        src = gg.pick_vertices(host, 32, seed=3)
        g = pp.Graph(host)
        c = torch.as_tensor(gg.normal(host.n * 32, seed=1).reshape(host.n, 32), device="cuda")
        for fd, ad, name in ((pp.PP_PUSH, pp.PP_PULL, "push_then_pull"), (pp.PP_PULL, pp.PP_PUSH, "pull_then_push")):
            X, it_f = pp.ppr(g, src, iters=300, k_tile=32, direction=fd, tol=1e-6)
            ms_f = _events_ms(lambda: pp.ppr(g, src, iters=it_f, k_tile=32, direction=fd))
            _, _, it_a = pp.ppr_adjoint(g, X, c, iters=300, k_tile=32, direction=ad, tol=1e-6)
            ms_a = _events_ms(lambda: pp.ppr_adjoint(g, X, c, iters=it_a, k_tile=32, direction=ad))
            line[name] = {"forward_sweeps": it_f, "forward_ms": round(ms_f, 2), "adjoint_sweeps": it_a,
                          "adjoint_ms": round(ms_a, 2)}
        line.update({"n": host.n, "nnz": host.nnz, "k": 32})
    elif w in ("tc16", "tc18"):
        # triangle counting, pulling (owner writes) vs pushing (64-bit fetch-and-add)
        host = gg.rmat(int(w[2:]), 16, seed=1)
        g = pp.Graph(host, relabel=False)
        for d, name in ((pp.PP_PULL, "pull"), (pp.PP_PUSH, "push")):
            pp.triangles(g, d)
            ms = _events_ms(lambda: pp.triangles(g, d))
            line[name] = {"ms": round(ms, 3), "gteps": round(host.nnz / (ms * 1e-3) / 1e9, 3)}
        line["triangles"] = int(pp.triangles(g, pp.PP_PULL).sum().item() // 3)
        line.update({"n": host.n, "nnz": host.nnz})
    elif w == "pprgrid":
        # personalised PageRank on a 2048 x 2048 grid (5% of edges removed), k = 32
        # sources, 30 sweeps: Generic-Switch (sparse push from the support, then
        # dense pull) against dense pull sweeps from the start
        host = gg.grid(2048, 2048, 0.05, seed=1)
        src = gg.pick_vertices(host, 32, seed=5)
        g = pp.Graph(host)
        for d, name in ((pp.PP_PULL, "pull"), (pp.PP_SWITCH, "switch")):
            pp.ppr(g, src, iters=2, k_tile=32, direction=d)
            ms = _events_ms(lambda: pp.ppr(g, src, iters=30, k_tile=32, direction=d))
            line[name] = {"ms": round(ms, 2)}
        line["speedup_switch_vs_pull"] = round(line["pull"]["ms"] / line["switch"]["ms"], 2)
        line.update({"n": host.n, "nnz": host.nnz, "k": 32, "iters": 30})
    elif w == "bc16":
        # Brandes BC from 64 seeded sources on R-MAT 16, every phase combination
        host = gg.rmat(16, 16, seed=1)
        src = gg.pick_vertices(host, 64, seed=4)
        g = pp.Graph(host)
        for fd, bd, name in ((pp.PP_PUSH, pp.PP_PUSH, "push_push"), (pp.PP_PULL, pp.PP_PULL, "pull_pull"),
                             (pp.PP_PUSH, pp.PP_PULL, "push_pull"), (pp.PP_PULL, pp.PP_PUSH, "pull_push")):
            pp.betweenness(g, src[:2], fd, bd)
            ms = _events_ms(lambda: pp.betweenness(g, src, fd, bd))
            line[name] = {"ms": round(ms, 2), "ms_per_source": round(ms / len(src), 3)}
        line.update({"n": host.n, "nnz": host.nnz, "sources": len(src)})
    else:
        raise SystemExit(f"unknown workload {w}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
