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
    """Runs density matrices of a list of jobs.  analyses are cached per job
    (symbolic analysis once per pattern, as in an SCF cycle)."""

    def __init__(self, jobs, budget_bytes=200 * 2**30, nstreams=4, device="cuda",
                 keep_outputs=False, tuned=None):
        import torch
        self.torch = torch
        self.jobs = list(jobs)
        self.budget = int(budget_bytes)
        self.device = device
        self.keep = keep_outputs
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, nstreams))]
        for j in self.jobs:
            if j.dE is None:
                j.dE = job_dE(j.system, j.mu)
            if j.analysis is None:
                if tuned is not None:
                    from .tune import tuned_analysis
                    j.analysis = tuned_analysis(j.system, j.poles, cache=tuned)
                else:
                    j.analysis = B.Analysis.from_system(j.system)
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

    def _values(self, j):
        torch = self.torch
        k = id(j)
        if k not in self._H:
            self._H[k] = torch.from_numpy(j.system.hval).to(self.device)
            self._S[k] = torch.from_numpy(j.system.sval).to(self.device)
        return self._H[k], self._S[k]

    def run(self):
        """Executes every job once; returns wall seconds."""
        torch = self.torch
        order = sorted(self.jobs, key=lambda j: -j.flops)
        pending = list(order)
        active = []     # (job, stream index, event, plan, tensors)
        used = 0
        free_streams = list(range(len(self.streams)))
        busy = {}
        t0 = time.perf_counter()
        while pending or active:
            launched = False
            while pending and free_streams and used + pending[0].footprint <= self.budget:
                j = pending.pop(0)
                si = free_streams.pop(0)
                st = self.streams[si]
                with torch.cuda.stream(st):
                    H, S = self._values(j)
                    L, W = _buffers(j, self.device)
                    plan = B.Plan(j.analysis, H, S, j.poles, nsets=j.nsets, L=L, work=W, device=self.device)
                    sh, wt = B.poles(j.beta, j.dE, j.mu, j.poles, j.nsets)
                    j.t_submit = time.perf_counter()
                    plan.run(sh, wt, stream=st, sync=False)
                    ev = torch.cuda.Event()
                    ev.record(st)
                active.append((j, si, ev, plan, (L, W)))
                used += j.footprint
                launched = True
            if not active:
                if pending and not launched:
                    raise B.PxsError("BatchRunner", B.PXS_ENOMEM, "cannot admit the next job")
                continue
            # wait for the earliest-submitted active job
            j, si, ev, plan, bufs = active.pop(0)
            ev.synchronize()
            j.t_done = time.perf_counter()
            j.traces, j.info = plan.results(stream=self.streams[si])
            if self.keep:
                # copied on the job's stream: the buffers freed below go back
                # to that stream's pool, so a later job on it cannot reuse
                # them before the copy has read them
                with torch.cuda.stream(self.streams[si]):
                    j.out = plan.out.view(j.nsets, -1).clone()
            del plan, bufs
            used -= j.footprint
            free_streams.append(si)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

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
