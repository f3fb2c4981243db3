"""Autotuner for the supernode and tile shapes.

The tunable knobs are options of the symbolic analysis: the largest
nested-dissection leaf (leaf_cols, which sets how small the supernodes at
the bottom of the tree get), the panel width (columns per factor/SelInv
panel, the K-depth of the in-panel products) and the tile height of the
panel products (64 or 128 rows per workgroup).  Shapes are grouped into
buckets by structural features only (matrix size, fill of L, pole count), so
any input -- not just the synthetic lattices -- maps to a bucket.  For each
bucket the tuner times one density matrix per candidate (graph-captured plan,
median of a few replays) and keeps the fastest in a JSON cache.  On top of
the tuned shape, wide nested-dissection separators are cut into several
supernodes when that removes enough stored zeros (a structural rule, no
timing; see with_separator_cut).
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time

import numpy as np

from . import binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned.json")
DEFAULTS = dict(leaf_cols=128, panel_width=64, tile_rows=64)
CANDIDATES = dict(leaf_cols=(64, 128, 256), panel_width=(32, 64), tile_rows=(64, 128))


def bucket(analysis, P):
    """Shape bucket of an analysed pattern and pole count."""
    i = analysis.info
    n = max(1, i["n"])
    fill = max(1.0, i["nnz_L_exact"] / n)
    return f"n{int(round(math.log2(n)))}_f{int(round(math.log2(fill)))}_p{'hi' if P > 50 else 'lo'}"


def load_cache(path=DEFAULT_CACHE):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


# Separators wider than this are cut into supernodes of at most this many
# columns (13 panels of 64) when the cut removes at least CUT_MIN_GAIN of the
# stored entries of L: in 3D the columns of a separator plane reach different
# parts of the ancestors, and one supernode over the plane stores the widest
# structure for all of them (cubic bulk N = 22,464: 2.6% fewer stored entries,
# 22% less factor storage, 3.9% faster; 1,664 columns 2.8% faster, 416
# slower).  In 2D the separators' columns share their structure and a cut
# only adds supernodes (honeycomb N = 26,624: 0.02% fewer entries, 0.3%
# slower), so it is not taken.
SEP_COLS = 832
CUT_MIN_GAIN = 0.01


def tuned_analysis(system, P, cache=None, path=DEFAULT_CACHE):
    """Analysis of the system with the tuned options of its bucket (the
    default analysis when the bucket is untuned or tuned to the defaults),
    with wide separators cut (SEP_COLS) when that removes enough stored
    zeros."""
    cache = load_cache(path) if cache is None else cache
    a = B.Analysis.from_system(system)
    opts = cache.get(bucket(a, P), {}).get("options") if cache else None
    if opts and opts != DEFAULTS:
        a = B.Analysis.from_system(system, **opts)
    return with_separator_cut(system, a)


def with_separator_cut(system, analysis):
    """`analysis`, or the same options with separators cut into pieces of
    SEP_COLS columns when that stores at least CUT_MIN_GAIN fewer entries."""
    if analysis.options.get("sep_cols") or analysis.info["nnz_L"] <= SEP_COLS * SEP_COLS:
        return analysis
    cut = B.Analysis.from_system(system, **{**analysis.options, "sep_cols": SEP_COLS})
    if cut.info["nnz_L"] <= (1.0 - CUT_MIN_GAIN) * analysis.info["nnz_L"]:
        return cut
    return analysis


def fit_to_budget(system, analysis, P, budget_bytes):
    """An analysis whose factor storage and workspace for P complex shifts
    fit budget_bytes of device memory: `analysis` itself when it fits,
    else the same options with the largest SelInv shift chunk (40, 20, 16,
    10, 8, 5, 4, 2 or 1 shifts per pass; the dense Z_CC workspace grows
    with the chunk) that fits.  Raises if none does."""
    def need(a):
        return a.info["bytes_per_shift"] * P + a.workspace_size(P)
    if need(analysis) <= budget_bytes:
        return analysis
    for ch in (40, 20, 16, 10, 8, 5, 4, 2, 1):
        if ch >= P:
            continue
        a2 = B.Analysis.from_system(system, **{**analysis.options, "selinv_chunk": ch})
        if need(a2) <= budget_bytes:
            return a2
    raise B.PxsError("fit_to_budget", B.PXS_ENOMEM,
                     f"{P} shifts need more than {budget_bytes / 2**30:.1f} GiB even one at a time")


def options_for(system, P, cache=None, path=DEFAULT_CACHE):
    """Tuned analysis options for this system's bucket (defaults if the
    bucket has not been tuned)."""
    cache = load_cache(path) if cache is None else cache
    if not cache:
        return dict(DEFAULTS)
    a = B.Analysis.from_system(system)
    return dict(cache.get(bucket(a, P), {}).get("options", DEFAULTS))


def time_candidate(system, P, opts, reps=3, device="cuda"):
    import torch
    a = B.Analysis.from_system(system, **opts).bind(device)
    H = torch.from_numpy(system.hval).to(device)
    S = torch.from_numpy(system.sval).to(device)
    plan = B.Plan(a, H, S, P, nsets=2)
    sh, wt = B.poles(B_BETA(), 1.0, 0.0, P, 2)
    plan.run(sh, wt)                      # warm-up (also checks pivots)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.run(sh, wt)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    del plan
    return float(np.median(ts)), a


def B_BETA():
    from .lattice import BETA_300K
    return BETA_300K


def tune_system(system, P, cache, candidates=CANDIDATES, reps=3, log=sys.stderr):
    """Tunes the bucket of one system (skips buckets already in the cache)."""
    a0 = B.Analysis.from_system(system)
    key = bucket(a0, P)
    if key in cache:
        return key, cache[key]
    best = None
    trials = []
    names = sorted(candidates)
    for vals in itertools.product(*(candidates[k] for k in names)):
        opts = dict(zip(names, vals))
        t, _ = time_candidate(system, P, opts, reps=reps)
        trials.append(dict(options=opts, seconds=round(t, 6)))
        if best is None or t < best[0]:
            best = (t, opts)
        print(f"# tune {key} {opts}: {t * 1e3:.2f} ms", file=log, flush=True)
    d0 = next(tr["seconds"] for tr in trials if tr["options"] == DEFAULTS) if any(
        tr["options"] == DEFAULTS for tr in trials) else None
    cache[key] = dict(options=best[1], seconds=round(best[0], 6), default_seconds=d0,
                      example=dict(kind=system.kind, n=system.n, poles=P), trials=trials)
    return key, cache[key]


def main():
    ap = argparse.ArgumentParser(description="autotune supernode/tile shapes on the GPU")
    ap.add_argument("--workload", default="batch", choices=("batch", "honeycomb", "serve"))
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--max-systems", type=int, default=64)
    args = ap.parse_args()
    from . import lattice
    cache = load_cache(args.out)
    if args.workload == "honeycomb":
        items = [(lattice.config_system(1), 60)]
    elif args.workload == "batch":
        items = lattice.batch_systems()
    else:
        items = [(r["system"], 40) for r in lattice.serving_requests(64, kmax=16) if not r["repeat"]]
    for s, P in items[: args.max_systems]:
        key, ent = tune_system(s, P, cache)
        print(f"# {key}: {ent['options']} {ent['seconds'] * 1e3:.2f} ms (default {ent['default_seconds']})",
              file=sys.stderr, flush=True)
        with open(args.out, "w") as f:      # saved after every bucket
            json.dump(cache, f, indent=1, sort_keys=True)
    print(json.dumps({k: v["options"] for k, v in cache.items()}))


if __name__ == "__main__":
    main()
