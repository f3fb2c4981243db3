"""Serving loop: continuous batching of density-matrix requests on one GPU.

A request is (H, S, mu, beta, number of poles[, real shifts for an inertia
count]).  The server
  * keeps one symbolic analysis per sparsity pattern (SCF-style repeats hit
    the cache; the paper performs the symbolic factorization once per SCF
    cycle, Sec. II.B),
  * keeps graph-captured plans with their factor buffers resident on the
    device, so a repeat of a resident pattern only uploads new values and a
    new pole table,
  * admits requests in arrival order while their device footprint fits the
    memory budget (idle resident plans are evicted least-recently-used first;
    a request larger than the budget runs its poles in chunks that add into
    one output),
  * runs admitted requests concurrently on several HIP streams (continuous
    batching: a request arriving while others run starts as soon as a stream
    and memory are free, and overlaps with them on the device),
  * reports latency from arrival to result (p50 / p99) beside throughput.
Host-side orchestration only: every numeric step runs in the library's
kernels.
"""
from __future__ import annotations

import dataclasses
import hashlib
import time
from collections import OrderedDict
from typing import Optional

import numpy as np

from . import binding as B
from .batch import job_dE
from .lattice import BETA_300K


def pattern_key(system) -> str:
    h = hashlib.blake2b(digest_size=16)
    h.update(np.ascontiguousarray(system.colptr).tobytes())
    h.update(np.ascontiguousarray(system.rowind).tobytes())
    if system.blkptr is not None:
        h.update(np.ascontiguousarray(system.blkptr).tobytes())
    return h.hexdigest()


@dataclasses.dataclass
class Request:
    system: object
    mu: float = 0.0
    beta: float = BETA_300K
    poles: int = 40
    eps: Optional[np.ndarray] = None
    arrival: float = 0.0
    nsets: int = 2
    dE: Optional[float] = None   # bound on max |eps - mu|; None: Gershgorin bound + |mu|
    rid: int = -1
    # filled by the server
    traces: object = None
    info: object = None
    neg_counts: object = None
    out: object = None
    t_admit: float = 0.0
    t_done: float = 0.0
    chunks: int = 1
    key: str = ""

    @property
    def latency(self):
        return self.t_done - self.arrival


class Resident:
    """Device state of one (pattern, pole count): values, factor buffers and
    the graph plan(s) over them."""

    def __init__(self, analysis, P, nsets, chunk, device):
        import torch
        self.analysis = analysis
        self.P, self.nsets, self.chunk = P, nsets, chunk
        nnz = analysis.info["nnz_lower"]
        self.H = torch.empty(nnz, dtype=torch.float64, device=device)
        self.S = torch.empty(nnz, dtype=torch.float64, device=device)
        self.L, self.W = analysis.buffers(chunk, device=device)
        self.out = torch.empty(nsets * nnz, dtype=torch.float64, device=device)
        self.plans = {}
        self.busy = False
        self.footprint = resident_bytes(analysis, chunk, nsets)

    def plan(self, nshift, accumulate):
        k = (nshift, accumulate)
        if k not in self.plans:
            self.plans[k] = B.Plan(self.analysis, self.H, self.S, nshift, nsets=self.nsets, L=self.L,
                                   work=self.W, out=self.out, accumulate=accumulate)
        return self.plans[k]


def resident_bytes(analysis, nshift, nsets=2):
    i = analysis.info
    return (nshift * i["bytes_per_shift"] + analysis.workspace_size(nshift) + 8 * (nsets + 2) * i["nnz_lower"])


class Server:
    def __init__(self, budget_bytes=250 * 2**30, nstreams=4, max_patterns=64, device="cuda",
                 keep_outputs=False, tuned=None):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.device = device
        self.keep = keep_outputs
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, nstreams))]
        self.analyses = OrderedDict()       # pattern key -> Analysis (LRU)
        self.max_patterns = max_patterns
        self.tuned = tuned
        self.residents = OrderedDict()      # (key, P) -> Resident (LRU)
        self.used = 0
        self.stats = dict(symbolic_hits=0, symbolic_misses=0, plan_hits=0, plan_misses=0,
                          evictions=0, chunked=0, analyze_s=0.0)

    # ------------------------------------------------------------------ caches
    def analysis(self, system, key=None, poles=40):
        key = key or pattern_key(system)
        a = self.analyses.get(key)
        if a is not None:
            self.analyses.move_to_end(key)
            self.stats["symbolic_hits"] += 1
            return key, a
        t = time.perf_counter()
        if self.tuned:
            from .tune import tuned_analysis
            a = tuned_analysis(system, poles, cache=self.tuned).bind(self.device)
        else:
            a = B.Analysis.from_system(system).bind(self.device)
        self.stats["analyze_s"] += time.perf_counter() - t
        self.stats["symbolic_misses"] += 1
        self.analyses[key] = a
        while len(self.analyses) > self.max_patterns:
            old, _ = self.analyses.popitem(last=False)
            for rk in [k for k in self.residents if k[0] == old and not self.residents[k].busy]:
                self._evict(rk)
        return key, a

    def _evict(self, rk):
        r = self.residents.pop(rk)
        self.used -= r.footprint
        self.stats["evictions"] += 1
        del r

    def _make_room(self, need):
        for rk in list(self.residents.keys()):
            if self.used + need <= self.budget:
                break
            if not self.residents[rk].busy:
                self._evict(rk)
        return self.used + need <= self.budget

    def chunk_for(self, a, P, nsets):
        c = P
        while c > 2 and resident_bytes(a, c, nsets) > self.budget:
            c = max(2, (c // 2) & ~1)
        if resident_bytes(a, c, nsets) > self.budget:
            raise B.PxsError("Server", B.PXS_ENOMEM, "request does not fit the memory budget")
        return c

    def acquire(self, req):
        """Resident state for the request, or None while it cannot run yet.
        The cache counters count each request once."""
        first = not req.key
        if first:
            req.key = pattern_key(req.system)
            key, a = self.analysis(req.system, req.key, req.poles)
        else:
            key, a = req.key, self.analyses.get(req.key)
            if a is None:
                key, a = self.analysis(req.system, req.key, req.poles)
        chunk = self.chunk_for(a, req.poles, req.nsets)
        rk = (key, req.poles, req.nsets, chunk)
        r = self.residents.get(rk)
        if r is not None:
            if r.busy:
                return None
            self.residents.move_to_end(rk)
            self.stats["plan_hits"] += 1
            return r
        need = resident_bytes(a, chunk, req.nsets)
        if not self._make_room(need):
            return None
        import torch
        with torch.cuda.device(self.device):
            r = Resident(a, req.poles, req.nsets, chunk, self.device)
        self.residents[rk] = r
        self.used += r.footprint
        self.stats["plan_misses"] += 1
        return r

    # -------------------------------------------------------------- execution
    def _start(self, req, r, si, now):
        torch = self.torch
        st = self.streams[si]
        r.busy = True
        req.t_admit = now
        with torch.cuda.stream(st):
            r.H.copy_(torch.from_numpy(req.system.hval), non_blocking=False)
            r.S.copy_(torch.from_numpy(req.system.sval), non_blocking=False)
            if req.eps is not None and len(req.eps):
                # the resident buffers hold `chunk` complex shifts, i.e. at
                # least `chunk` real ones
                counts = []
                for q0 in range(0, len(req.eps), r.chunk):
                    neg, _ = B.inertia(r.analysis, r.H, r.S, req.eps[q0:q0 + r.chunk], L=r.L, work=r.W,
                                       stream=st)
                    counts.append(neg)
                req.neg_counts = np.concatenate(counts)
            if req.dE is None:
                req.dE = job_dE(req.system, req.mu)
            sh, wt = B.poles(req.beta, req.dE, req.mu, req.poles, req.nsets)
            req.chunks = (req.poles + r.chunk - 1) // r.chunk
            if req.chunks == 1:
                r.plan(req.poles, False).run(sh, wt, stream=st, sync=False)
            else:
                self.stats["chunked"] += 1
                tr = np.zeros((req.nsets, 2))
                infos = []
                for c0 in range(0, req.poles, r.chunk):
                    c1 = min(req.poles, c0 + r.chunk)
                    p = r.plan(c1 - c0, c0 > 0)
                    _, t, inf = p.run(sh[c0:c1], wt[:, c0:c1], stream=st, sync=True)
                    tr += t
                    infos.append(inf)
                req.traces = tr
                req.info = np.concatenate(infos)
            ev = torch.cuda.Event()
            ev.record(st)
        return ev

    def _finish(self, req, r, si):
        if req.traces is None:
            req.traces, req.info = r.plan(req.poles, False).results(stream=self.streams[si])
        if self.keep:
            # the resident output is rewritten by the next request on this
            # resident, possibly on another stream: copy it on this request's
            # stream and wait for the copy before releasing the resident
            st = self.streams[si]
            with self.torch.cuda.stream(st):
                req.out = r.out.view(req.nsets, -1).clone()
            st.synchronize()
        r.busy = False

    def run(self, requests, realtime=True):
        """Serves the requests (arrival times in seconds from the start);
        returns a summary dict.  realtime=False ignores arrival times
        (saturated throughput)."""
        torch = self.torch
        reqs = sorted(requests, key=lambda q: q.arrival)
        for i, q in enumerate(reqs):
            if q.rid < 0:
                q.rid = i
        waiting = []
        active = []   # (req, resident, stream index, event)
        free = list(range(len(self.streams)))
        nxt = 0
        t0 = time.perf_counter()
        while nxt < len(reqs) or waiting or active:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= now):
                if not realtime:
                    reqs[nxt].arrival = 0.0
                waiting.append(reqs[nxt])
                nxt += 1
            # completions
            still = []
            for item in active:
                req, r, si, ev = item
                if ev.query():
                    req.t_done = time.perf_counter() - t0
                    self._finish(req, r, si)
                    free.append(si)
                else:
                    still.append(item)
            active = still
            # admissions (arrival order; a request that does not fit waits)
            while waiting and free:
                r = self.acquire(waiting[0])
                if r is None:
                    break
                req = waiting.pop(0)
                si = free.pop(0)
                ev = self._start(req, r, si, time.perf_counter() - t0)
                active.append((req, r, si, ev))
            if not active and waiting and not free:
                raise RuntimeError("scheduler stalled")
            if active and (not waiting or not free):
                # nothing to admit: wait for the oldest request or the next arrival
                if nxt < len(reqs) and realtime:
                    time.sleep(min(0.001, max(0.0, reqs[nxt].arrival - (time.perf_counter() - t0))))
                else:
                    active[0][3].synchronize()
            elif not active and nxt < len(reqs):
                time.sleep(max(0.0, min(0.01, reqs[nxt].arrival - (time.perf_counter() - t0))))
        torch.cuda.synchronize()
        makespan = time.perf_counter() - t0
        lat = np.array([q.latency for q in reqs])
        solves = sum(q.poles for q in reqs)
        return dict(requests=len(reqs), makespan_s=makespan, req_per_s=len(reqs) / makespan,
                    pole_solves_per_s=solves / makespan,
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    mean_s=float(lat.mean()), **self.stats)


def poisson_arrivals(n, rate, seed=0):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
