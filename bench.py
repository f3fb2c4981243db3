#!/usr/bin/env python3
"""Benchmark of the PEXSI hot path on one MI355X.

Workload (default): the periodic honeycomb sheet of 32 x 32 cells x 2 atoms
x 13 orbitals (N = 26,624; 24 neighbours within 3 nearest-neighbour
distances), 60 poles at 300 K, all 60 shifts in one batch.  One step is one
density-matrix evaluation with the symbolic analysis resident: pole table,
assembly of the 60 shifted matrices, supernodal LDL^T, selected inversion
and the pole sums of Gamma and Gamma^E with their traces.

Prints one JSON line.  value = pole-solves per second (one pole-solve = the
LDL^T and selected inversion of one shift, assembly and pole sum included in
the wall time).  roofline: the selected-inversion off-diagonal product
kernel (the largest share of kernel time), timed with HIP events inside the
library over the timed region.  cpu_baseline: the CPU oracle (dense LU
inverse per shift) on a bounded sample, scaled to this workload.
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E

MULTI = {
    "batch": "64 uneven systems (chain / honeycomb / cubic, kind = s mod 3), N log-uniform in "
             "[500, 8000], 40-80 poles each, 250 GiB budget",
    "serve": "Poisson request stream: sizes Zipf(1.2) over k*1000 basis functions, chain / honeycomb / "
             "cubic, 40 poles, 30% SCF-style repeats of a resident pattern, 16-shift inertia counts on "
             "new patterns, 250 GiB admission budget, 4 streams",
    "hermitian": "complex Hermitian honeycomb pencil (same lattice and pattern as the honeycomb workload, "
                 "imaginary parts 0.5 N(0,1) |Re| on off-diagonal entries), N=26624, 60 poles, one batch: "
                 "L D U, two-sided selected inversion, Gamma = (M - M^H)/2i and Gamma^E with traces",
    "dos": "honeycomb N=26624: DOS on 200 bins over [-1.05, 1.05] Ha from 201 inertia counts "
           "(batched real LDL^T, 32 shifts per batch) and the LDOS matrix at 4 energies (eta = 1e-3 Ha, "
           "one batched complex factorization + SelInv + pole sums)",
}

WORKLOADS = {
    "honeycomb": dict(cfg=1, desc="periodic honeycomb 32x32 cells x 2 atoms x 13 orbitals, "
                      "cutoff 3 NN distances, N=26624, 60 poles, one batch"),
    "cubic": dict(cfg=2, desc="periodic simple cubic 12^3 atoms x 13 orbitals, cutoff 2 spacings, "
                  "N=22464, 80 poles, one batch"),
    "chain": dict(cfg=0, desc="open 1D chain 64 atoms x 4 orbitals, neighbours within 2 sites, "
                  "N=256, 40 poles, one batch"),
}


SOURCES_HASHED = ("numeric.hip", "batch.inc", "symbolic.cpp")


def kernel_source_hash(text=None):
    """Hash of the code that sets a kernel's memory traffic (the kernels and
    the symbolic layout of the factor storage): comments and layout do not
    count, so a counter summary stays valid across edits of comments only."""
    if text is None:
        text = ""
        for name in SOURCES_HASHED:
            with open(os.path.join(ROOT, "paper_1405_0194_amd", "csrc", name)) as f:
                text += f.read()
    code = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    code = re.sub(r"//[^\n]*", " ", code)
    code = " ".join(code.split())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none for this kernel/workload or the kernel source has
    changed since it was taken."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def _counter_rows(d):
    import csv
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        return list(csv.DictReader(f))


def _kernel_is(name, kernel):
    """rocprofv3 kernel names carry the namespace and template arguments."""
    base = name.split("<")[0].split("(")[0].strip()
    return base.split("::")[-1] == "k_" + kernel


def traffic_from_counters(kernel, workload, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, commands):
    """Writes the HBM bytes per launch of one kernel from four rocprofv3
    --pmc runs (FETCH_SIZE, WRITE_SIZE of the workload; the same two counters
    over a plain device copy of 1 GiB, which scale the counters to bytes)."""
    def values(d, name_pred):
        return [float(r["Counter_Value"]) for r in _counter_rows(d) if name_pred(r["Kernel_Name"])]

    gib = float(2**30)
    def ours(n):
        return _kernel_is(n, kernel)

    fk = values(fetch_dir, ours)
    wk = values(write_dir, ours)
    fc = values(copy_fetch_dir, lambda n: "copyBuffer" in n or "copy" in n.lower())
    wc = values(copy_write_dir, lambda n: "copyBuffer" in n or "copy" in n.lower())
    if not fk or len(fk) != len(wk) or not fc or not wc:
        raise SystemExit("counter files do not match the kernel or hold no copy launch")
    f_scale = gib / (1024.0 * sum(fc) / len(fc))   # bytes per counted KiB
    w_scale = gib / (1024.0 * sum(wc) / len(wc))
    fetch = 1024.0 * f_scale * sum(fk) / len(fk)
    write = 1024.0 * w_scale * sum(wk) / len(wk)
    out = {"kernel": kernel, "workload": workload, "launches": len(fk),
           "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
           "hbm_bytes_per_launch": round(fetch + write),
           "fetch_counter_scale": round(f_scale, 4), "write_counter_scale": round(w_scale, 4),
           "source_hash": kernel_source_hash(), "commands": commands}
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    with open(p, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
    return out


def mfma_from_counters(workload, counter_dir, command):
    """Per kernel, from one rocprofv3 --pmc run of SQ_INSTS_VALU_MFMA_MOPS_F64
    (FP64 matrix operations / 512), SQ_VALU_MFMA_BUSY_CYCLES, SQ_BUSY_CYCLES
    and GRBM_GUI_ACTIVE: the FP64 MFMA flops the hardware executed per launch
    (padding of partial tiles included), their rate over the launch duration,
    and the fraction of SIMD cycles in which the matrix cores were busy.
    GRBM_GUI_ACTIVE sums the busy clocks of the 8 XCDs and the MFMA busy
    cycles sum over the 1,024 SIMDs (256 CUs x 4).  Writes
    profiles/mfma_<workload>.json."""
    n_xcd, n_simd = 8, 1024
    per = {}
    for r in _counter_rows(counter_dir):
        base = r["Kernel_Name"].split("<")[0].split("(")[0].strip().split("::")[-1]
        if not base.startswith("k_"):
            continue
        k = per.setdefault(base, {"dur": {}})
        k.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        k["dur"][r["Dispatch_Id"]] = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9
    out = {"workload": workload, "command": command, "kernels": {}}
    for base, c in sorted(per.items()):
        mops = c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", [])
        busy = c.get("SQ_VALU_MFMA_BUSY_CYCLES", [])
        gui = c.get("GRBM_GUI_ACTIVE", [])
        n = len(mops)
        if not n:
            continue
        flops = 512.0 * sum(mops) / n
        dur = sum(c["dur"].values()) / len(c["dur"])
        e = {"launches": n, "mfma_flops_per_launch": flops, "avg_launch_ms": round(dur * 1e3, 4),
             "mfma_tflops": round(flops / dur / 1e12, 2) if dur > 0 else None}
        if busy and gui and sum(gui) > 0:
            clocks = sum(gui) / len(gui) / n_xcd
            e["mfma_busy_frac"] = round(sum(busy) / len(busy) / (clocks * n_simd), 4)
            e["clock_ghz"] = round(clocks / dur / 1e9, 3) if dur > 0 else None
        out["kernels"][base] = e
    p = os.path.join(ROOT, "profiles", f"mfma_{workload}.json")
    with open(p, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def cpu_baseline(full_n, seconds_target=10.0, cells=18):
    """The oracle as it stands: one pole-solve = dense inverse of H - w S.
    Timed on a honeycomb sample of 18 x 18 cells (N = 8,424) and scaled by
    (N_sample / N)^3."""
    import numpy as np
    from oracle import dense
    from paper_1405_0194_amd import lattice
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    s = lattice.make_system("honeycomb", (cells, cells), 13, 3.0, 7)
    Hd, Sd = s.dense()
    w = 0.01 + 0.003j
    t0 = time.perf_counter()
    reps = 0
    while True:
        dense.shifted_inverse(Hd, Sd, w)
        reps += 1
        el = time.perf_counter() - t0
        if el > seconds_target or reps >= 20:
            break
    per = el / reps
    scale = (s.n / float(full_n)) ** 3
    return {"value": (1.0 / per) * scale, "unit": "pole-solves/s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"{reps} dense complex128 inverses (numpy LAPACK) of H - wS for a honeycomb "
                       f"{cells}x{cells}x2 atoms x 13 orbitals (N={s.n}), {per:.3f} s each, "
                       f"scaled by (N_sample/N)^3 to N={full_n}")}


def cpu_eigh_baseline(full_n, reps=1, cells=18):
    """The dense-diagonalization route the method replaces: the oracle's
    generalized eigendecomposition of (H, S) (one per density matrix, any P),
    timed on a honeycomb sample (N = 8,424) and scaled by (N / N_sample)^3."""
    from oracle import dense
    from paper_1405_0194_amd import lattice
    s = lattice.make_system("honeycomb", (cells, cells), 13, 3.0, 7)
    Hd, Sd = s.dense()
    t0 = time.perf_counter()
    for _ in range(reps):
        dense.gen_eigh(Hd, Sd)
    per = (time.perf_counter() - t0) / reps
    return {"seconds_per_density_matrix": round(per * (float(full_n) / s.n) ** 3, 1), "kind": "oracle",
            "sample": (f"{reps} generalized dense eigendecompositions (scipy eigh) of a honeycomb {cells}x{cells}x2 "
                       f"atoms x 13 orbitals pencil (N={s.n}), {per:.2f} s each, scaled by (N/N_sample)^3 to "
                       f"N={full_n}; the GPU path takes ms_per_step for one density matrix")}


def chain_leg(reps=200):
    """The chain workload (open 1D chain, 64 atoms x 4 orbitals, N = 256, 40
    poles at 300 K): microseconds per density matrix through a replayed graph
    plan (no host synchronisation between replays), through the eager fused
    call and through the allocation-free call (both synchronise per call)."""
    import numpy as np
    import torch
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import lattice
    from paper_1405_0194_amd import tune
    s = lattice.config_system(0)
    P, mu = lattice.CONFIG_POLES[0], 0.0
    dE = 1.0 + abs(mu)
    a = tune.tuned_analysis(s, P).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    plan = B.Plan(a, H, S, P, nsets=2)
    sh, wt = B.poles(lattice.BETA_300K, dE, mu, P, 2)
    L, W = a.buffers(P)

    def timed(fn, n):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return 1e6 * (time.perf_counter() - t) / n

    # the pole table on the device (as the serving loop keeps it): replays
    # queue back to back; from host arrays each replay first copies the
    # table from pageable memory, which waits for the stream
    sh_d = torch.from_numpy(np.ascontiguousarray(sh, dtype=np.complex128)).cuda()
    wt_d = torch.from_numpy(np.ascontiguousarray(wt, dtype=np.complex128).reshape(-1)).cuda()
    plan_us = timed(lambda: plan.run_device(sh_d, wt_d), reps)
    plan_host_us = timed(lambda: plan.run(sh, wt, sync=False), reps)
    eager_us = timed(lambda: B.density_matrix(a, H, S, lattice.BETA_300K, dE, mu, P, nsets=2, L=L, work=W), reps // 4)
    noalloc_us = timed(lambda: B.density_matrix_noalloc(a, H, S, lattice.BETA_300K, dE, mu, P, nsets=2, L=L),
                       reps // 4)
    # the same plan with the subtrees on streams instead of fused lanes
    # (the analysis fuses them by default for this tree of small supernodes);
    # timed last: eager calls right after many replays of a large graph were
    # measured up to 2x slower for a while
    a_st = B.Analysis.from_system(s, **{**a.options, "fused_lanes": -1}).bind()
    plan_st = B.Plan(a_st, H, S, P, nsets=2)
    plan_streams_us = timed(lambda: plan_st.run_device(sh_d, wt_d), reps)
    del plan_st
    return {"workload": WORKLOADS["chain"]["desc"], "graph_plan_us_per_density_matrix": round(plan_us, 1),
            "graph_plan_pole_solves_per_s": round(P / (plan_us * 1e-6), 1),
            "graph_plan_host_table_us_per_density_matrix": round(plan_host_us, 1),
            "fused_lanes": a.info["fused_lanes"],
            "graph_plan_streams_us_per_density_matrix": round(plan_streams_us, 1),
            "eager_us_per_density_matrix": round(eager_us, 1),
            "noalloc_us_per_density_matrix": round(noalloc_us, 1), "replays": reps}


def per_pole_sample(a, H, S, beta, dE, mu, P, nsample):
    """The plain per-pole loop (same kernels, one shift per factorization,
    no batching, no graphs) on the first nsample shifts: seconds per shift."""
    import torch
    from paper_1405_0194_amd import batch
    from paper_1405_0194_amd import binding as B
    sh, wt = B.poles(beta, dE, mu, P, 2)
    batch.per_pole_loop(a, H, S, sh[:1], wt[:, :1])      # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    batch.per_pole_loop(a, H, S, sh[:nsample], wt[:, :nsample])
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / nsample


def pole_groups_leg(a, H, S, beta, dE, mu, P, groups, batched_value, reps=3):
    """The same density matrix with its P poles in `groups` groups, each a
    captured graph plan on a stream of its own (pole table on the device),
    outputs added: the top of the tree of one group overlaps the wide levels
    of the others.  At most 4 groups run at once (4 hardware queues)."""
    import numpy as np
    import torch
    from paper_1405_0194_amd import binding as B
    if P % groups:
        return None
    g = P // groups
    sh, wt = B.poles(beta, dE, mu, P, 2)
    wt = np.asarray(wt).reshape(2, P)
    dev = H.device
    streams = [torch.cuda.Stream(device=dev) for _ in range(groups)]
    plans = [B.Plan(a, H, S, g, nsets=2) for _ in range(groups)]
    shd = [torch.from_numpy(np.ascontiguousarray(sh[i * g:(i + 1) * g])).to(dev) for i in range(groups)]
    wtd = [torch.from_numpy(np.ascontiguousarray(wt[:, i * g:(i + 1) * g]).reshape(-1)).to(dev)
           for i in range(groups)]

    def run():
        for i in range(groups):
            plans[i].run_device(shd[i], wtd[i], stream=streams[i])
        for st in streams:
            st.synchronize()
    torch.cuda.synchronize()
    run()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        run()
        ts.append(time.perf_counter() - t)
    sec = float(np.median(ts))
    out = {"groups": groups, "poles_per_group": g, "ms_per_density_matrix": round(1e3 * sec, 3),
           "pole_solves_per_s": round(P / sec, 4), "vs_one_batch": round(P / sec / batched_value, 4)}
    del plans
    torch.cuda.empty_cache()
    return out


def run_batch(args):
    import torch
    from paper_1405_0194_amd import lattice, tune
    from paper_1405_0194_amd.batch import BatchRunner, Job
    t = time.perf_counter()
    items = lattice.batch_systems()
    print(f"# batch: {len(items)} systems generated in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    tuned = tune.load_cache() or None

    def measure(mode, streams, groups, steps, warmup):
        jobs = [Job(system=s, poles=P, mu=0.0) for s, P in items]
        t_an = time.perf_counter()
        br = BatchRunner(jobs, budget_bytes=250 * 2**30, nstreams=streams, tuned=tuned, mode=mode, groups=groups,
                         alone_share=args.batch_alone_share)
        t_an = time.perf_counter() - t_an
        t_first = br.run()        # creates the plans or the fused graphs
        print(f"# {mode} x{streams}: analyses {t_an:.1f}s, first run {t_first:.2f}s", file=sys.stderr, flush=True)
        for i in range(max(0, warmup - 1)):
            print(f"# {mode} warmup {i}: {br.run():.3f}s", file=sys.stderr, flush=True)
        times = []
        for i in range(steps):
            times.append(br.run())
            waves = getattr(br, "wave_seconds", None)
            print(f"# {mode} step {i}: {times[-1]:.3f}s" + (f" waves {[round(w, 3) for w in waves]}" if waves else ""),
                  file=sys.stderr, flush=True)
        launches = br.fused_launches() if mode == "fused" else None
        out = dict(solves=br.total_solves(), flops=br.total_flops(), times=times, first=t_first,
                   launches=launches, info_ok=all(np.all(j.info == 0) for j in jobs))
        del br, jobs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return out

    main = measure(args.batch_mode, args.batch_streams, args.batch_streams, args.steps, args.warmup)
    alt_mode = "plans" if args.batch_mode == "fused" else "fused"
    alt = measure(alt_mode, 4, 4, max(1, args.steps // 2), args.warmup)
    elapsed = sum(main["times"])
    solves = main["solves"] * args.steps
    flops = main["flops"] * args.steps
    res = dict(value=round(solves / elapsed, 4), ms_per_step=round(1e3 * elapsed / args.steps, 3),
               path_tflops=round(flops / elapsed / 1e12, 3),
               fp64_mfma_pct=round(100.0 * flops / elapsed / 1e12 / PEAK_FP64_TFLOPS, 2),
               latency_s={"p50": round(float(np.percentile(main["times"], 50)), 4),
                          "p99": round(float(np.percentile(main["times"], 99)), 4)},
               first_run_s=round(main["first"], 3), fused_launches=main["launches"],
               all_info_zero=bool(main["info_ok"] and alt["info_ok"]),
               comparison={f"{alt_mode}_4_streams_pole_solves_per_s":
                           round(alt["solves"] * len(alt["times"]) / sum(alt["times"]), 4)},
               config={"workload": MULTI["batch"], "systems": len(items), "mode": args.batch_mode,
                       "streams": args.batch_streams, "pole_solves_per_step": main["solves"],
                       "tflop_per_step": round(main["flops"] / 1e12, 2), "tuned_buckets": len(tuned or {})})
    return res


def run_dos(args):
    import numpy as np
    import torch
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import dos as pdos
    from paper_1405_0194_amd import lattice, tune
    s = lattice.config_system(1)
    a = tune.tuned_analysis(s, 60).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    edges = np.linspace(-1.05, 1.05, 201)
    energies = np.array([-0.2, -0.05, 0.0, 0.1])
    pdos.dos(a, H, S, edges[:33], batch=32)            # warm-up
    torch.cuda.synchronize()
    tds = []
    for _ in range(args.steps):
        t = time.perf_counter()
        centres, g, c = pdos.dos(a, H, S, edges, batch=32)
        torch.cuda.synchronize()
        tds.append(time.perf_counter() - t)
    tls = []
    for _ in range(max(1, args.steps)):
        t = time.perf_counter()
        out, tr, info = pdos.ldos(a, H, S, energies, 1e-3)
        torch.cuda.synchronize()
        tls.append(time.perf_counter() - t)
    td, tl = float(np.median(tds)), float(np.median(tls))
    return {"metric": "inertia counts/s (DOS) and LDOS energies/s", "value": round(len(edges) / td, 3),
            "unit": "inertia-counts/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": round(1e3 * td, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64 (DOS), c128 (LDOS)", "data": "synthetic",
            "config": {"workload": MULTI["dos"], "n": s.n, "bins": len(edges) - 1},
            "dos_s": round(td, 4), "electrons_counted": int(c[-1] - c[0]),
            "ldos": {"energies": len(energies), "seconds": round(tl, 4),
                     "energies_per_s": round(len(energies) / tl, 3),
                     "tr_GS": [round(float(x), 6) for x in tr[:, 0]]}}


def run_hermitian(args):
    import numpy as np
    import torch
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import lattice, tune
    P, beta, mu = 60, lattice.BETA_300K, 0.0
    dE = 1.0 + abs(mu)
    s = lattice.make_hermitian_system("honeycomb", (32, 32), 13, 3.0, lattice.CONFIG_SEED_BASE + 1)
    a = tune.tuned_analysis(s, P).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    lb, wb = B.hermitian_sizes(a, P)
    L = torch.empty(lb, dtype=torch.uint8, device="cuda")
    W = torch.empty(wb, dtype=torch.uint8, device="cuda")
    sh, wt = B.poles(beta, dE, mu, P, 2)

    def step():
        f = B.HermitianFactorization(a, H, S, sh, L=L, work=W)
        f.selinv()
        return f.pole_sum(wt)

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        print(f"# warmup {i}: {time.perf_counter() - t:.3f}s", file=sys.stderr, flush=True)
    B.profile_begin(args.profile_kernel)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        out, tr = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        print(f"# step {i}: {lat[-1]:.3f}s  Tr(GS)={tr[0, 0]:.6f}", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    kms, kl, kw, kb = B.profile_end(with_bytes=True)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    f = B.HermitianFactorization(a, H, S, sh, L=L, work=W)
    e[1].record()
    f.selinv()
    e[2].record()
    f.pole_sum(wt)
    e[3].record()
    torch.cuda.synchronize()
    # L D U does the full Schur complement and SelInv both triangles: twice
    # the complex-symmetric operation count
    flops_shift = 2.0 * (a.info["flops_factor"] + a.info["flops_selinv"])
    solves = P * args.steps
    tfl = flops_shift * solves / elapsed / 1e12
    avg = kms / max(kl, 1)
    ach = (kw / max(kl, 1)) / (avg / 1e3) / 1e12 if kl else 0.0
    return dict(value=round(solves / elapsed, 4), ms_per_step=round(1e3 * elapsed / args.steps, 3),
                path_tflops=round(tfl, 3), fp64_mfma_pct=round(100.0 * tfl / PEAK_FP64_TFLOPS, 2),
                latency_s={"p50": round(float(np.percentile(lat, 50)), 4),
                           "p99": round(float(np.percentile(lat, 99)), 4)},
                phases_ms={"assemble_factor_ms": round(e[0].elapsed_time(e[1]), 2),
                           "selinv_ms": round(e[1].elapsed_time(e[2]), 2),
                           "pole_sum_ms": round(e[2].elapsed_time(e[3]), 2)},
                electrons=round(float(tr[0, 0]), 6),
                roofline={"kernel": args.profile_kernel, "bound": "mfma", "achieved": round(ach, 3),
                          "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                          "avg_launch_ms": round(avg, 4), "launches": kl, "traffic": None,
                          "algorithmic_bytes_per_launch": round(kb / max(kl, 1))},
                config={"workload": MULTI["hermitian"], "n": s.n, "poles": P,
                        "factor_storage_GB": round(lb / 1e9, 1),
                        "tflop_per_shift": round(flops_shift / 1e12, 4)})


def run_serve(args):
    import torch
    from paper_1405_0194_amd import lattice
    from paper_1405_0194_amd.serve import Request, Server, poisson_arrivals
    t = time.perf_counter()
    raw = lattice.serving_requests(args.requests, kmax=args.kmax)
    print(f"# serve: {len(raw)} requests generated in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)

    def make():
        return [Request(system=r["system"], mu=r["mu"], poles=40, eps=r["eps"]) for r in raw]

    def rounded(d):
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    from paper_1405_0194_amd import tune
    srv = Server(budget_bytes=250 * 2**30, nstreams=4, tuned=tune.load_cache() or None)
    out = {}
    lam = args.serve_rate
    if not lam:
        sat = srv.run(make(), realtime=False, log=sys.stderr)   # saturated: everything queued at t = 0
        print(f"# saturated: {sat}", file=sys.stderr, flush=True)
        lam = sat["req_per_s"]
        out["saturated"] = rounded(sat)
    loads = [float(x) for x in args.serve_loads.split(",") if x.strip()]
    runs = {}
    for f in loads:
        reqs = make()
        for q, ta in zip(reqs, poisson_arrivals(len(reqs), f * lam, seed=int(f * 10))):
            q.arrival = float(ta)
        runs[f] = srv.run(reqs, realtime=True, log=sys.stderr)
        print(f"# load {f}: {runs[f]}", file=sys.stderr, flush=True)
        out[f"load_{f}".replace(".", "_")] = rounded(runs[f])
    main = runs[loads[-1]] if loads else out["saturated"]
    res = dict(value=round(main["pole_solves_per_s"], 4), ms_per_step=round(1e3 * main["makespan_s"], 3),
               latency_s={"p50": round(main["p50_s"], 4), "p99": round(main["p99_s"], 4)},
               path_tflops=round(main["path_tflops"], 3),
               fp64_mfma_pct=round(100.0 * main["path_tflops"] / PEAK_FP64_TFLOPS, 2),
               config={"workload": MULTI["serve"], "requests": len(raw), "kmax": args.kmax,
                       "saturated_req_per_s": round(lam, 4), "loads": loads,
                       "largest_n": max(r["system"].n for r in raw)},
               **out)
    srv.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="honeycomb", choices=sorted(WORKLOADS) + sorted(MULTI))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-kernel", default="selinv_off")
    ap.add_argument("--compare-perpole", type=int, default=4,
                    help="also time the plain per-pole loop on this many shifts (0: skip)")
    ap.add_argument("--no-chain", action="store_true", help="skip the chain-workload leg")
    ap.add_argument("--pole-groups", type=int, default=4,
                    help="also time the poles in this many graph-plan groups on separate streams (0: skip)")
    ap.add_argument("--tile-rows", type=int, default=0, help="rows per tile of the panel products (64/128)")
    ap.add_argument("--panel-width", type=int, default=0)
    ap.add_argument("--leaf-cols", type=int, default=0)
    ap.add_argument("--selinv-streams", type=int, default=0)
    ap.add_argument("--selinv-chunk", type=int, default=0)
    ap.add_argument("--fused-lanes", type=int, default=None,
                    help="1: subtree lanes fused on one stream, -1: one stream per subtree, "
                         "0: by structure (default: the analysis' own choice)")
    ap.add_argument("--sep-cols", type=int, default=-1,
                    help="max columns of a separator supernode (0: no cut; default: the tuned value)")
    ap.add_argument("--hbm-budget-gib", type=float, default=270.0,
                    help="device memory for factors + workspace; SelInv chunks its shifts beyond it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling the HBM byte counters)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write profiles/<kernel>_<workload>_traffic.json from four rocprofv3 --pmc "
                         "output folders and exit (no GPU use)")
    ap.add_argument("--traffic-kernels", default="",
                    help="with --traffic-from: comma list of kernel classes (default: --profile-kernel)")
    ap.add_argument("--mfma-from", metavar="DIR",
                    help="write profiles/mfma_<workload>.json from one rocprofv3 --pmc output folder and exit")
    ap.add_argument("--only-steps", action="store_true",
                    help="time the steps and print the line, nothing else (for counter runs)")
    ap.add_argument("--batch-mode", default="plans", choices=("fused", "plans"),
                    help="batch: one graph plan per system, or fused multi-system launches")
    ap.add_argument("--batch-streams", type=int, default=4,
                    help="batch: streams (fused: groups of systems per wave)")
    ap.add_argument("--batch-alone-share", type=float, default=0.04,
                    help="batch, fused: systems with at least this share of a wave's work run alone")
    ap.add_argument("--requests", type=int, default=64, help="serve: number of requests")
    ap.add_argument("--kmax", type=int, default=16, help="serve: largest size class (k * 1000)")
    ap.add_argument("--serve-loads", default="0.5,0.8",
                    help="serve: Poisson arrival rates as fractions of the saturated rate (comma list)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="serve: the saturated request rate (req/s) if known; skips the saturated run")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} (world size {world}) "
              "is not supported (multi-GPU pole sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    if args.traffic_from:
        f, w, cf, cw = args.traffic_from
        kernels = [k for k in args.traffic_kernels.split(",") if k] or [args.profile_kernel]
        regex = "|".join("k_" + k for k in kernels)
        run = (f"python3 bench.py --steps 1 --warmup 0 --only-steps --selinv-streams 1 "
               f"--workload {args.workload}")
        cmds = [f"rocprofv3 --pmc {c} --kernel-include-regex '{regex}' -T -f csv -d <dir> -o run "
                f"-- {run}" for c in ("FETCH_SIZE", "WRITE_SIZE")]
        cmds += [f"rocprofv3 --pmc {c} -T -f csv -d <dir> -o run -- python3 bench.py --copy-calibration"
                 for c in ("FETCH_SIZE", "WRITE_SIZE")]
        for k in kernels:
            traffic_from_counters(k, args.workload, f, w, cf, cw, cmds)
        return
    if args.mfma_from:
        cmd = ("rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CYCLES "
               "GRBM_GUI_ACTIVE -T -f csv -d <dir> -o run -- python3 bench.py --steps 1 --warmup 0 "
               f"--only-steps --selinv-streams 1 --workload {args.workload}")
        mfma_from_counters(args.workload, args.mfma_from, cmd)
        return

    import numpy as np
    import torch
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import lattice
    globals()["np"] = np

    if args.copy_calibration:
        # a plain copy kernel of known size: 1 GiB read and 1 GiB written per launch
        x = torch.ones(2**27, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 2**30, "copy_bytes_written_per_launch": 2**30,
                          "launches": 3}), flush=True)
        return

    if args.workload in MULTI:
        torch.cuda.set_device(0)
        res = {"batch": run_batch, "serve": run_serve, "dos": run_dos,
               "hermitian": run_hermitian}[args.workload](args)
        if args.workload == "dos":      # its own metric and unit
            print(json.dumps(res), flush=True)
            return
        steps = args.steps if args.workload in ("batch", "hermitian") else 1
        warm = args.warmup if args.workload in ("batch", "hermitian") else 0
        line = {"metric": "pole-solves/sec (LDL^T+SelInv), FP64 MFMA %, p50/p99 request latency",
                "value": res.pop("value"), "unit": "pole-solves/s", "n_gpus": 1, "steps": steps,
                "warmup": warm, "ms_per_step": res.pop("ms_per_step"), "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
                "config": res.pop("config")}
        line.update(res)
        print(json.dumps(line), flush=True)
        return

    wl = WORKLOADS[args.workload]
    cfg = wl["cfg"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    s = lattice.config_system(cfg)
    t_gen = time.perf_counter() - t_gen
    P = lattice.CONFIG_POLES[cfg]
    mu = 0.0
    dE = 1.0 + abs(mu)
    beta = lattice.BETA_300K
    t_an = time.perf_counter()
    if args.tile_rows or args.panel_width or args.leaf_cols or args.selinv_streams or args.selinv_chunk \
            or args.sep_cols >= 0:
        a = B.Analysis.from_system(s, tile_rows=args.tile_rows, panel_width=args.panel_width,
                                   leaf_cols=args.leaf_cols, selinv_streams=args.selinv_streams,
                                   selinv_chunk=args.selinv_chunk, sep_cols=max(args.sep_cols, 0))
    else:
        from paper_1405_0194_amd import tune
        a = tune.tuned_analysis(s, lattice.CONFIG_POLES[cfg])
    if args.fused_lanes is not None and a.options.get("fused_lanes", 0) != args.fused_lanes:
        a = B.Analysis.from_system(s, **{**a.options, "fused_lanes": args.fused_lanes})
    # SelInv works on shift chunks when the whole batch's workspace would not
    # fit beside the factors (the cubic bulk: 201 GB of factors for 80 shifts)
    if not args.selinv_chunk:
        from paper_1405_0194_amd import tune
        a = tune.fit_to_budget(s, a, P, int(args.hbm_budget_gib * 2**30))
        if a.options["selinv_chunk"]:
            print(f"# SelInv chunk {a.options['selinv_chunk']} shifts to fit {args.hbm_budget_gib} GiB",
                  file=sys.stderr, flush=True)
    t_an = time.perf_counter() - t_an
    t_bind = time.perf_counter()
    a.bind()
    torch.cuda.synchronize()
    t_bind = time.perf_counter() - t_bind
    H = torch.from_numpy(s.hval).to(dev)
    S = torch.from_numpy(s.sval).to(dev)
    L, W = a.buffers(P)
    torch.cuda.synchronize()
    print(f"# workload {args.workload}: N={s.n} nnz_lower={s.nnz_lower} P={P} nsuper={a.info['nsuper']} "
          f"npanel={a.info['npanel']} L={L.numel() / 1e9:.1f} GB; generate {t_gen:.1f}s analyze {t_an:.2f}s",
          file=sys.stderr, flush=True)

    def step():
        return B.density_matrix(a, H, S, beta, dE, mu, P, nsets=2, L=L, work=W)

    first_step = None
    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        first_step = dt if first_step is None else first_step
        print(f"# warmup {i}: {dt:.3f}s", file=sys.stderr, flush=True)

    B.profile_begin(args.profile_kernel)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        out, tr, info, sh, wt = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        print(f"# step {i}: {lat[-1]:.3f}s  Tr(GS)={tr[0, 0]:.6f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms, klaunch, kwork, kbytes, kstored = B.profile_end(with_bytes=True, with_stored=True)
    if args.only_steps:
        avg_ms = kms / max(klaunch, 1)
        print(json.dumps({"metric": "pole-solves/sec (LDL^T+SelInv), FP64 MFMA %, p50/p99 request latency",
                          "value": round(P * args.steps / elapsed, 4), "unit": "pole-solves/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
                          "config": {"workload": wl["desc"]},
                          "roofline": {"kernel": args.profile_kernel, "avg_launch_ms": round(avg_ms, 4),
                                       "launches": klaunch,
                                       "flops_per_launch": round(kwork / max(klaunch, 1))}}), flush=True)
        return

    # phase breakdown on one extra (untimed) step
    phases = {}
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    sh, wt = B.poles(beta, dE, mu, P, 2)
    e[0].record()
    f = B.Factorization(a, H, S, sh, L=L, work=W)
    e[1].record()
    f.selinv()
    e[2].record()
    f.pole_sum(wt)
    e[3].record()
    torch.cuda.synchronize()
    phases = {"assemble_factor_ms": e[0].elapsed_time(e[1]), "selinv_ms": e[1].elapsed_time(e[2]),
              "pole_sum_ms": e[2].elapsed_time(e[3])}

    # the dominant kernel once more with every launch alone on the device
    # (SelInv on one stream): launch durations not stretched by concurrency
    iso = None
    if args.profile_kernel in ("selinv_off", "selinv_diag", "lhat", "gather"):
        a1 = B.Analysis.from_system(s, **{**a.options, "selinv_streams": 1}).bind()
        W1 = W if a1.workspace_size(P) <= W.numel() else None
        L1, W1 = (L, W1) if W1 is not None else a1.buffers(P)
        B.profile_begin(args.profile_kernel)
        B.density_matrix(a1, H, S, beta, dE, mu, P, nsets=2, L=L1, work=W1)
        ims, il, iw, ist = B.profile_end(with_stored=True)
        if il:
            iavg = ims / il
            iach = (iw / il) / (iavg / 1e3) / 1e12
            iso = {"achieved": round(iach, 3), "frac": round(iach / PEAK_FP64_TFLOPS, 4),
                   "avg_launch_ms": round(iavg, 4), "launches": il,
                   "stored_achieved": round((ist / il) / (iavg / 1e3) / 1e12, 3)}
        del a1

    # achieved HBM rate of the memory-bound kernels (assembly, pole sum, Z_CC
    # gather), one untimed step each
    hbm = {}
    for kname in ("assemble", "pole_sum", "gather"):
        B.profile_begin(kname)
        step()
        hms, hl, hw = B.profile_end()
        hbm[kname + "_GBps"] = round(hw / (hms / 1e3) / 1e9, 1) if hms > 0 else None

    solves = P * args.steps
    value = solves / elapsed
    flops_shift = a.info["flops_factor"] + a.info["flops_selinv"]
    path_tflops = flops_shift * solves / elapsed / 1e12
    avg_ms = kms / max(klaunch, 1)
    achieved = (kwork / max(klaunch, 1)) / (avg_ms / 1e3) / 1e12 if klaunch else 0.0
    traffic = measured_traffic(args.profile_kernel, args.workload)
    # device-level rate of each phase: its exact flops over its wall time in
    # the phase-breakdown step (independent of how the launches overlap)
    phase_rates = {}
    for name, fl, key in (("factor", a.info["flops_factor"], "assemble_factor_ms"),
                          ("selinv", a.info["flops_selinv"], "selinv_ms")):
        if phases.get(key):
            t = fl * P / (phases[key] / 1e3) / 1e12
            phase_rates[name] = {"tflops": round(t, 3), "frac": round(t / PEAK_FP64_TFLOPS, 4)}
    lat_sorted = sorted(lat)
    res = {
        "metric": "pole-solves/sec (LDL^T+SelInv), FP64 MFMA %, p50/p99 request latency",
        "value": round(value, 4),
        "unit": "pole-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": s.n, "nnz_H": 2 * s.nnz_lower - s.n, "poles": P,
                   "nnz_L_exact": a.info["nnz_L_exact"], "nsuper": a.info["nsuper"],
                   "tflop_per_shift": round(flops_shift / 1e12, 4), "mu": mu, "beta": beta},
        "fp64_mfma_pct": round(100.0 * path_tflops / PEAK_FP64_TFLOPS, 2),
        "path_tflops": round(path_tflops, 3),
        "latency_s": {"p50": round(float(np.percentile(lat_sorted, 50)), 4),
                      "p99": round(float(np.percentile(lat_sorted, 99)), 4)},
        "phases_ms": {k: round(v, 2) for k, v in phases.items()},
        "phase_rates": phase_rates,
        "hbm_GBps": hbm,
        "cold_s": {"analyze": round(t_an, 3), "bind": round(t_bind, 3),
                   "first_density_matrix": round(first_step, 3) if first_step is not None else None},
        "roofline": {"kernel": args.profile_kernel, "bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "avg_launch_ms": round(avg_ms, 4), "launches": klaunch,
                     "flops_per_launch": round(kwork / max(klaunch, 1)),
                     "stored_flops_per_launch": round(kstored / max(klaunch, 1)),
                     "stored_achieved": round((kstored / max(klaunch, 1)) / (avg_ms / 1e3) / 1e12, 3)
                     if klaunch else 0.0,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": round(kbytes / max(klaunch, 1)),
                     "isolated": iso},
    }
    if args.profile_kernel in ("assemble", "pole_sum"):
        gbs = (kwork / max(klaunch, 1)) / (avg_ms / 1e3) / 1e9 if klaunch else 0.0
        res["roofline"].update({"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                                "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)})
    if not args.no_chain:
        res["chain"] = chain_leg()
    if args.pole_groups > 1:
        res["pole_groups"] = pole_groups_leg(a, H, S, beta, dE, mu, P, args.pole_groups, value)
    if args.compare_perpole:
        del f
        sec = per_pole_sample(a, H, S, beta, dE, mu, P, args.compare_perpole)
        res["per_pole_loop"] = {"pole_solves_per_s": round(1.0 / sec, 4), "shifts_timed": args.compare_perpole,
                                "speedup_of_batched": round(value * sec, 3)}
    if not args.no_cpu_baseline:
        del L, W
        torch.cuda.empty_cache()
        res["cpu_baseline"] = cpu_baseline(s.n)
        res["cpu_eigh"] = cpu_eigh_baseline(s.n)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
