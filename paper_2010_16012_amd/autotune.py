"""Autotuner for the sweep parameters, cached as JSON.

Searches, per (GPU architecture, graph size class):
  * degree-bin thresholds and the split chunk of the longest rows (both
    sweeps);
  * pull sweep: LDS-staged contributions, workgroup size and how many of the
    heaviest rows take the tiled (source-sliced) sweep;
  * push sweep: LDS-privatised targets and persistent workgroups;
  * BFS direction switch: the alpha/beta constants of the switch rule (on
    roots of their own seed);
  * personalised PageRank: the column tile width for a given k;
  * the many-graph launch: which PageRank rows take a wavefront, a middle
    group or a small group, and the group widths (on a batch of its own
    seed, stored under a key of its own: graph count and size class).
Every candidate is timed with HIP events on the device; the fastest wins.
The cache maps "arch|size class" to the chosen values; ``apply`` installs a
cached entry through the library's tuning entry points.

CLI: python -m paper_2010_16012_amd.autotune --scale 22 --out tuned.json
"""
from __future__ import annotations

import argparse
import json
import math
import os

import numpy as np
import torch

from . import PP_PULL, PP_PUSH, PP_SWITCH, BfsRun, Graph, _lib, pagerank_into, ppr

TUNE_ROOT_SEED = 11  # BFS roots the switch constants are tuned on

DEFAULTS = {"upper": [4, 16, 64, 1024, 4096], "split_chunk": 4096, "hot": 8192, "push_blocks": 1024,
            "pull_hot": 32768, "pull_block": 1024, "slice_rows": 0, "slice_width": 32768, "alpha": 14.0,
            "beta": 24.0, "k_tile": 32, "multi_big": 512, "multi_mid": 64, "multi_pull_group": 2,
            "multi_mid_lanes": 16, "bfs_multi_n": 256, "bfs_multi_m": 1024}

# one-workgroup BFS launch caps (frontier vertices, out-edges per level) the
# switch search tries: the default, smaller, and off
BFS_MULTI_CAPS = ((256, 1024), (64, 256), (0, 0))

TUNE_BATCH_SEED = 11  # many-graph batch the launch mapping is tuned on


def arch() -> str:
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def size_class(n: int, nnz: int) -> str:
    return f"n2^{int(round(math.log2(max(n, 1))))}_m2^{int(round(math.log2(max(nnz, 1))))}"


def key(n: int, nnz: int, gpu_arch: str | None = None) -> str:
    return f"{gpu_arch or arch()}|{size_class(n, nnz)}"


def multi_key(count: int, total_n: int, total_nnz: int, gpu_arch: str | None = None) -> str:
    return f"{gpu_arch or arch()}|multi{count}_{size_class(total_n, total_nnz)}"


def apply(cfg: dict) -> None:
    c = dict(DEFAULTS)
    c.update(cfg or {})
    _lib.pp_set_bin_thresholds(c["upper"], c["split_chunk"])
    _lib.pp_set_push_tuning(c["hot"], c["push_blocks"])
    _lib.pp_set_pull_tuning(c["pull_hot"], c["pull_block"])
    _lib.pp_set_pull_slices(c["slice_rows"], c["slice_width"])
    _lib.pp_set_multi_tuning(c["multi_big"], c["multi_mid"], c["multi_pull_group"], c["multi_mid_lanes"])
    _lib.pp_set_bfs_multi(c["bfs_multi_n"], c["bfs_multi_m"])


def load(path: str, n: int, nnz: int, gpu_arch: str | None = None) -> dict:
    """Cached entry for this GPU (or ``gpu_arch``) and size class (empty when absent)."""
    return load_key(path, key(n, nnz, gpu_arch))


def load_key(path: str, k: str) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh).get(k, {})


def _time(fn, reps=3) -> float:
    fn()  # warm up
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


SLICE_ROWS = (65536, 131072, 196608, 262144, 524288)

BIN_CANDIDATES = (
    ([4, 16, 64, 1024, 4096], 4096),
    ([8, 32, 128, 1024, 4096], 4096),
    ([2, 8, 32, 256, 2048], 2048),
    ([4, 16, 64, 512, 8192], 8192),
)


def tune_bins(host, iters=5, log=print) -> dict:
    """Degree-bin thresholds with the lowest pull + push sweep time."""
    x = torch.empty(host.n, dtype=torch.float32, device="cuda")
    best = None
    for upper, chunk in BIN_CANDIDATES:
        apply({"upper": upper, "split_chunk": chunk})
        g = Graph(host)
        t = 0.0
        for d in (PP_PULL, PP_PUSH):
            def f():
                x.fill_(1.0 / host.n)
                pagerank_into(g, x, iters, 0.85, d)
            t += _time(f)
        g.close()
        log(f"bins upper={upper} chunk={chunk}: {t / iters * 1e3:.1f} us per pull+push step")
        if best is None or t < best[0]:
            best = (t, upper, chunk)
    return {"upper": best[1], "split_chunk": best[2]}


def tune_pagerank(host, iters=5, log=print, base=None) -> dict:
    """Best pull and push settings for this graph."""
    out = dict(base or {})
    x = torch.empty(host.n, dtype=torch.float32, device="cuda")

    def run(g, d):
        def f():
            x.fill_(1.0 / host.n)
            pagerank_into(g, x, iters, 0.85, d)
        return _time(f)

    best = None
    # tiled rows: none, or the heaviest R rows (only for graphs with more
    # rows than one source slice holds)
    slice_rows = [0] + [r for r in SLICE_ROWS if host.n > 2 * 32768 and r < host.n]
    for pull_hot in (32768, 40960):
        for block in (512, 1024):
            for rows in slice_rows:
                apply({**out, "pull_hot": pull_hot, "pull_block": block, "slice_rows": rows, "slice_width": 32768})
                g = Graph(host)
                t = run(g, PP_PULL)
                g.close()
                log(f"pull hot={pull_hot} block={block} slice_rows={rows}: {t / iters * 1e3:.1f} us/iter")
                if best is None or t < best[0]:
                    best = (t, pull_hot, block, rows)
    out["pull_hot"], out["pull_block"], out["slice_rows"], out["slice_width"] = best[1], best[2], best[3], 32768
    best = None
    for hot in (8192, 16384, 32768, 40960):
        for blocks in ((512, 1024, 2048) if hot <= 16384 else (256, 512)):
            apply({**out, "hot": hot, "push_blocks": blocks})
            g = Graph(host)
            t = run(g, PP_PUSH)
            g.close()
            log(f"push hot={hot} blocks={blocks}: {t / iters * 1e3:.1f} us/iter")
            if best is None or t < best[0]:
                best = (t, hot, blocks)
    out["hot"], out["push_blocks"] = best[1], best[2]
    apply(out)
    return out


def tune_bfs_switch(host, roots, log=print) -> dict:
    """alpha/beta of the direction switch, and the one-workgroup launch caps,
    with the least time over the roots, run through the many-roots call as a
    batch of roots is run (one host wait; root-by-root runs also pay a host
    round trip per level batch, which favours other constants).  The caps
    take effect at registration: one graph per setting."""
    roots = [int(x) for x in roots]
    best = None
    for caps in BFS_MULTI_CAPS:
        _lib.pp_set_bfs_multi(*caps)
        g = Graph(host)
        r = BfsRun(g)
        for alpha in (8.0, 14.0, 24.0, 48.0, 96.0, 192.0, 384.0):
            for beta in (24.0, 64.0, 128.0, 256.0, 512.0, 1024.0):
                def f():
                    r.run_many(roots, PP_SWITCH, alpha, beta)
                t = _time(f, reps=3)
                log(f"bfs caps={caps} alpha={alpha} beta={beta}: {t / len(roots):.3f} ms/root")
                if best is None or t < best[0]:
                    best = (t, alpha, beta, caps)
        g.close()
    _lib.pp_set_bfs_multi(*best[3])
    return {"alpha": best[1], "beta": best[2], "bfs_multi_n": best[3][0], "bfs_multi_m": best[3][1]}


def tune_ppr_tile(host, k, iters=3, log=print) -> dict:
    g = Graph(host)
    src = np.arange(k, dtype=np.int32) % host.n
    best = None
    for kt in (8, 16, 32, 64):
        t = _time(lambda: ppr(g, src, iters=iters, k_tile=kt), reps=2)
        log(f"ppr k={k} k_tile={kt}: {t:.2f} ms for {iters} sweeps")
        if best is None or t < best[0]:
            best = (t, kt)
    g.close()
    return {"k_tile": best[1]}


MULTI_GRID = [(big, mid, pg, ml) for big in (256, 512, 1024) for mid in (32, 64, 128) for pg in (1, 2, 4)
              for ml in (8, 16, 32) if mid < big]


def tune_multi(hosts, log=print) -> dict:
    """Many-graph mapping with the lowest PageRank x20 (pull, then push) plus
    switching-BFS launch time over the batch."""
    from . import MultiGraph
    mg = MultiGraph(hosts)
    best = None
    for big, mid, pg, ml in MULTI_GRID:
        _lib.pp_set_multi_tuning(big, mid, pg, ml)
        t = sum(_time(lambda: mg.run(pr_iters=20, pr_dir=d, bfs_policy=PP_SWITCH)) for d in (PP_PULL, PP_PUSH))
        log(f"multi big={big} mid={mid} pull_group={pg} mid_lanes={ml}: {t:.3f} ms pull+push")
        if best is None or t < best[0]:
            best = (t, big, mid, pg, ml)
    out = {"multi_big": best[1], "multi_mid": best[2], "multi_pull_group": best[3], "multi_mid_lanes": best[4]}
    apply(out)
    return out


def main():
    import graphgen as gg

    p = argparse.ArgumentParser()
    p.add_argument("--scale", type=int, default=22)
    p.add_argument("--roots", type=int, default=8)
    p.add_argument("--ppr-k", type=int, default=0)
    p.add_argument("--out", required=True)
    p.add_argument("--only", default="", help="comma list of searches to rerun (pagerank, bfs, ppr); the cached "
                   "entry keeps the other settings, which also apply while searching")
    p.add_argument("--multi", type=int, default=0, metavar="GRAPHS",
                   help="instead: tune the many-graph launch on GRAPHS R-MAT graphs of scales 8-14")
    a = p.parse_args()
    if a.multi:
        cache = {}
        if os.path.exists(a.out):
            with open(a.out) as fh:
                cache = json.load(fh)
        hosts = gg.rmat_batch(a.multi, 8, 14, seed=TUNE_BATCH_SEED)
        k = multi_key(len(hosts), sum(h.n for h in hosts), sum(int(h.nnz) for h in hosts))
        cache[k] = tune_multi(hosts)
        with open(a.out, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        print(json.dumps({k: cache[k]}))
        return
    host = gg.rmat(a.scale, 16, seed=1)
    cache = {}
    if os.path.exists(a.out):
        with open(a.out) as fh:
            cache = json.load(fh)
    k = key(host.n, host.nnz)
    only = set(filter(None, a.only.split(",")))
    cfg = dict(cache.get(k, {})) if only else {}
    if only:
        apply(cfg)
    if not only or "pagerank" in only:
        cfg.update(tune_pagerank(host, base=tune_bins(host)))
    if not only or "bfs" in only:
        # roots drawn with a seed of their own: the benchmark's roots (seed 1)
        # are not the ones the constants are chosen on
        cfg.update(tune_bfs_switch(host, gg.pick_vertices(host, a.roots, seed=TUNE_ROOT_SEED)))
    if a.ppr_k and (not only or "ppr" in only):
        cfg.update(tune_ppr_tile(host, a.ppr_k))
    cache[k] = cfg
    with open(a.out, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    print(json.dumps({key(host.n, host.nnz): cfg}))


if __name__ == "__main__":
    main()
