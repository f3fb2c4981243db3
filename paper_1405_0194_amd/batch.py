"""Batched execution of many uneven systems on one GPU.

Every system keeps its own symbolic analysis and device maps; all of its
shifts run as one graph-captured plan (pxs_plan_create / pxs_plan_run), i.e.
as the batch dimension of every launch.  Systems are admitted in decreasing
order of work while their device footprint fits the memory budget, and are
spread over several HIP streams so that small systems overlap with large
ones (the paper's pole-level and system-level independence, Sec. II.B, taken
to one device).  Complex Hermitian systems (k-points of a periodic system)
run the L D U plan; those sharing a pattern may share one analysis.
Host-side orchestration only: every numeric step runs in the
library's kernels.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Optional

import numpy as np

from . import binding as B
from .api import pencil_dE
from .lattice import BETA_300K


def job_dE(system, mu):
    """Delta E of a job's pole table: the Gershgorin bound of its pencil
    plus |mu| (raises when S is not diagonally dominant)."""
    return pencil_dE(system.colptr, system.rowind, system.hval, system.sval, mu)


@dataclasses.dataclass
class Job:
    system: object
    poles: int
    mu: float = 0.0
    beta: float = BETA_300K
    nsets: int = 2
    dE: Optional[float] = None  # bound on max |eps - mu|; None: Gershgorin bound + |mu|
    analysis: object = None
    footprint: int = 0          # device bytes while running (factor + workspace + output)
    flops: float = 0.0
    # results
    out: object = None          # device tensor (nsets, nnz) when keep_outputs
    traces: object = None
    info: object = None
    t_submit: float = 0.0
    t_done: float = 0.0


def footprint(analysis, P, nsets=2, hermitian=False):
    i = analysis.info
    if hermitian:
        lb, wb = B.hermitian_sizes(analysis, P)
        return lb + wb + 16 * nsets * i["nnz_lower"]
    return P * i["bytes_per_shift"] + analysis.workspace_size(P) + 8 * nsets * i["nnz_lower"]


def _hermitian(job):
    return np.iscomplexobj(job.system.hval)


def _buffers(job, device):
    import torch
    if _hermitian(job):
        lb, wb = B.hermitian_sizes(job.analysis, job.poles)
        return (torch.empty(lb, dtype=torch.uint8, device=device),
                torch.empty(wb, dtype=torch.uint8, device=device))
    return job.analysis.buffers(job.poles, device=device)


class BatchRunner:
    """Runs density matrices of a list of jobs.  Analyses are made once per
    job (symbolic analysis once per pattern, as in an SCF cycle).

    mode "plans": one graph-captured plan per system (kept across runs when
    all of them fit the budget together, else created in every run), the
    systems spread over `nstreams` HIP streams, largest first.
    mode "fused": the real systems are split into `groups` sets of about
    equal work; each set runs as one fused batch (pxs_batch_*: every launch
    holds the next panel operation of all its systems that use the same
    kernel), the sets side by side on their own streams.  Complex Hermitian
    jobs always run on plans."""

    def __init__(self, jobs, budget_bytes=200 * 2**30, nstreams=4, device="cuda",
                 keep_outputs=False, tuned=None, mode="plans", groups=None, alone_share=0.0):
        import torch
        if mode not in ("plans", "fused"):
            raise ValueError("mode must be 'plans' or 'fused'")
        self.torch = torch
        self.jobs = list(jobs)
        self.budget = int(budget_bytes)
        self.device = device
        self.keep = keep_outputs
        self.mode = mode
        self.groups = groups
        self.alone_share = float(alone_share)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, nstreams))]
        for j in self.jobs:
            if j.dE is None:
                j.dE = job_dE(j.system, j.mu)
            fused_job = mode == "fused" and not _hermitian(j)
            if j.analysis is None:
                if tuned is not None:
                    from .tune import options_for
                    opts = options_for(j.system, j.poles, cache=tuned)
                else:
                    opts = {}
                if fused_job:
                    # one stream: one per-shift workspace region
                    opts = {**opts, "selinv_streams": 1}
                j.analysis = B.Analysis.from_system(j.system, **opts)
            j.analysis.bind(device)
            j.footprint = footprint(j.analysis, j.poles, j.nsets, _hermitian(j))
            # L D U: full Schur complements and both triangles of SelInv
            j.flops = (2.0 if _hermitian(j) else 1.0) * j.poles * (
                j.analysis.info["flops_factor"] + j.analysis.info["flops_selinv"])
            if j.footprint > self.budget:
                raise B.PxsError("BatchRunner", B.PXS_ENOMEM,
                                 f"job of {j.footprint / 2**30:.1f} GiB exceeds the budget")
        self._H = {}
        self._S = {}
        # plans (with their buffers) are kept across runs when all of them
        # fit the budget together; otherwise each run creates them again
        self._keep_plans = sum(j.footprint for j in self.jobs) <= self.budget
        self._plans = {}        # id(job) -> (plan, L, W) kept across runs
        self._kept = 0
        self._fused = None      # per wave: list of (FusedBatch, jobs, stream index)
        self._arena = None
        self._stream_arena = None
        if not self._keep_plans and mode == "plans":
            # one arena per stream holds any job: admission needs a free stream only
            need = len(self.streams) * max(footprint(j.analysis, j.poles, j.nsets, _hermitian(j)) for j in self.jobs)
            if need > self.budget:
                raise B.PxsError("BatchRunner", B.PXS_ENOMEM,
                                 f"{len(self.streams)} streams of the largest job need {need / 2**30:.1f} GiB")

    def _values(self, j):
        torch = self.torch
        k = id(j)
        if k not in self._H:
            self._H[k] = torch.from_numpy(j.system.hval).to(self.device)
            self._S[k] = torch.from_numpy(j.system.sval).to(self.device)
        return self._H[k], self._S[k]

    # ------------------------------------------------------------------ fused
    def _build_fused(self):
        """Waves of systems that fit the budget together (largest first);
        each wave's systems split into groups of about equal work, one fused
        batch per group on its own stream.  The factor storage and workspace
        of every wave are views into one arena of the largest wave's size:
        the waves run one after another, so they share it."""
        torch = self.torch
        real = sorted([j for j in self.jobs if not _hermitian(j)], key=lambda j: -j.flops)
        align = lambda b: (b + 255) // 256 * 256

        def need(j):
            return align(j.poles * j.analysis.info["bytes_per_shift"]) + align(j.analysis.workspace_size(j.poles))
        # as few waves as the memory allows, each a mix of large and small
        # systems (largest first into the wave with the least memory in use
        # that still has room), so small systems overlap large ones
        total = sum(need(j) for j in real)
        nw = max(1, -(-total // self.budget))
        while True:
            waves = [[] for _ in range(nw)]
            used = [0] * nw
            fits = True
            for j in real:
                order = sorted(range(nw), key=lambda w: used[w])
                w = next((w for w in order if used[w] + need(j) <= self.budget), None)
                if w is None:
                    fits = False
                    break
                waves[w].append(j)
                used[w] += need(j)
            if fits:
                break
            nw += 1
        waves = [w for w in waves if w]
        arena_bytes = max(sum(need(j) for j in w) for w in waves) if waves else 0
        self._arena = torch.empty(max(256, arena_bytes), dtype=torch.uint8, device=self.device)
        self._fused = []     # per wave: list of (FusedBatch, jobs, stream index)
        for wave in waves:
            ng = max(1, min(self.groups or len(self.streams), len(wave), len(self.streams)))
            # systems with a large share of the wave's work run alone (their
            # own launches are large); the others share lockstep launches, one
            # fused batch per stream; every stream runs its batches in turn
            wave_flops = sum(j.flops for j in wave)
            large = [j for j in wave if j.flops >= self.alone_share * wave_flops] if self.alone_share else []
            small = [j for j in wave if not any(j is q for q in large)]
            batches = [[] for _ in range(ng)]       # per stream: list of job lists
            work = [0.0] * ng
            for j in large:
                g = int(np.argmin(work))
                batches[g].append([j])
                work[g] += j.flops
            groups_small = [[] for _ in range(ng)]
            for j in small:
                g = int(np.argmin(work))
                groups_small[g].append(j)
                work[g] += j.flops
            for g in range(ng):
                if groups_small[g]:
                    batches[g].append(groups_small[g])
            off = 0
            items = []
            for g in range(ng):
                for js in batches[g]:
                    by_sets = {}
                    for j in js:
                        by_sets.setdefault(j.nsets, []).append(j)
                    for nsets, jj in by_sets.items():
                        bufs = []
                        for j in jj:
                            lb = j.poles * j.analysis.info["bytes_per_shift"]
                            wb = j.analysis.workspace_size(j.poles)
                            L = self._arena[off:off + lb]
                            W = self._arena[off + align(lb):off + align(lb) + wb]
                            off += need(j)
                            bufs.append((L, W))
                        with torch.cuda.stream(self.streams[g]):
                            fb = B.FusedBatch([(j.analysis, *self._values(j), j.poles) for j in jj], nsets=nsets,
                                              device=self.device, buffers=bufs)
                        items.append((fb, jj, g))
            self._fused.append(items)

    def _run_fused(self):
        torch = self.torch
        if self._fused is None:
            self._build_fused()
        self.wave_seconds = []
        for wave in self._fused:
            tw = time.perf_counter()
            # the previous wave's results were read (its streams synchronised)
            # before this one overwrites the shared arena
            for fb, jj, g in wave:
                tables = [B.poles(j.beta, j.dE, j.mu, j.poles, j.nsets) for j in jj]
                for j in jj:
                    j.t_submit = time.perf_counter()
                fb.run(tables, stream=self.streams[g])
            for fb, jj, g in wave:
                trs, infos = fb.results(stream=self.streams[g])
                now = time.perf_counter()
                outs = fb.outputs() if self.keep else [None] * len(jj)
                for j, tr, inf, o in zip(jj, trs, infos, outs):
                    j.t_done = now
                    j.traces, j.info = tr, inf
                    if self.keep:
                        with torch.cuda.stream(self.streams[g]):
                            j.out = o.clone()
            self.wave_seconds.append(time.perf_counter() - tw)

    def fused_launches(self):
        """Fused launches per wave and group (after the first run)."""
        return [[fb.launches for fb, _, _ in wave] for wave in (self._fused or [])]

    # ------------------------------------------------------------------ plans
    def _sizes(self, j):
        if _hermitian(j):
            return B.hermitian_sizes(j.analysis, j.poles)
        return j.poles * j.analysis.info["bytes_per_shift"], j.analysis.workspace_size(j.poles)

    def _plan_for(self, j, si):
        hit = self._plans.get(id(j))
        if hit is not None:
            return hit, True
        H, S = self._values(j)
        if self._keep_plans:
            L, W = _buffers(j, self.device)
        else:
            # a stream runs one job at a time: its factor storage and
            # workspace are views into that stream's arena (allocated once,
            # so runs do not churn the allocator)
            if self._stream_arena is None:
                align = lambda b: (b + 255) // 256 * 256
                size = max(align(lb) + wb for lb, wb in (self._sizes(q) for q in self.jobs))
                self._stream_arena = [self.torch.empty(size, dtype=self.torch.uint8, device=self.device)
                                      for _ in self.streams]
            lb, wb = self._sizes(j)
            off = (lb + 255) // 256 * 256
            L = self._stream_arena[si][:lb]
            W = self._stream_arena[si][off:off + wb]
        plan = B.Plan(j.analysis, H, S, j.poles, nsets=j.nsets, L=L, work=W, device=self.device)
        return (plan, L, W), False

    def run(self):
        """Executes every job once; returns wall seconds."""
        torch = self.torch
        t0 = time.perf_counter()
        if self.mode == "fused":
            self._run_fused()
            herm = [j for j in self.jobs if _hermitian(j)]
            if herm:
                self._run_plans(herm)
        else:
            self._run_plans(self.jobs)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def _run_plans(self, jobs):
        torch = self.torch
        order = sorted(jobs, key=lambda j: -j.flops)
        pending = list(order)
        active = []     # (job, stream index, event, plan entry, kept)
        used = self._kept
        free_streams = list(range(len(self.streams)))
        while pending or active:
            launched = False
            while pending and free_streams:
                j = pending[0]
                kept = id(j) in self._plans
                if self._keep_plans and not kept and used + j.footprint > self.budget:
                    break
                pending.pop(0)
                si = free_streams.pop(0)
                st = self.streams[si]
                with torch.cuda.stream(st):
                    entry, kept = self._plan_for(j, si)
                    sh, wt = B.poles(j.beta, j.dE, j.mu, j.poles, j.nsets)
                    j.t_submit = time.perf_counter()
                    entry[0].run(sh, wt, stream=st, sync=False)
                    ev = torch.cuda.Event()
                    ev.record(st)
                if not kept:
                    used += j.footprint
                active.append((j, si, ev, entry, kept))
                launched = True
            if not active:
                if pending and not launched:
                    raise B.PxsError("BatchRunner", B.PXS_ENOMEM, "cannot admit the next job")
                continue
            # the first of the running jobs to complete
            done = None
            while done is None:
                for k, item in enumerate(active):
                    if item[2].query():
                        done = k
                        break
                else:
                    time.sleep(1e-4)
            j, si, ev, entry, kept = active.pop(done)
            j.t_done = time.perf_counter()
            j.traces, j.info = entry[0].results(stream=self.streams[si])
            if self.keep:
                # copied on the job's stream, before its buffers can be reused
                with torch.cuda.stream(self.streams[si]):
                    j.out = entry[0].out.view(j.nsets, -1).clone()
            if not kept:
                if self._keep_plans:
                    # every job's plan fits at once: keep it for the next run
                    self._plans[id(j)] = entry
                    self._kept += j.footprint
                else:
                    used -= j.footprint
            free_streams.append(si)

    def total_flops(self):
        return sum(j.flops for j in self.jobs)

    def total_solves(self):
        return sum(j.poles for j in self.jobs)


def per_pole_loop(analysis, H, S, shifts, weights, device="cuda"):
    """The plain per-pole loop on the same kernels: one shift per
    factorization, no batching and no graphs; returns the pole sums."""
    import torch
    nsets = weights.shape[0]
    nnz = analysis.info["nnz_lower"]
    acc = torch.zeros(nsets, nnz, dtype=torch.float64, device=device)
    L, W = analysis.buffers(1, device=device)
    for l in range(shifts.shape[0]):
        f = B.Factorization(analysis, H, S, shifts[l:l + 1], L=L, work=W)
        f.selinv()
        out, _ = f.pole_sum(weights[:, l:l + 1], traces=False)
        acc += out
    return acc
