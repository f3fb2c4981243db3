"""Serving loop: continuous batching of density-matrix requests on one GPU.

A request is (H, S, mu, beta, number of poles[, real shifts for an inertia
count]).  The server
  * keeps one symbolic analysis per sparsity pattern (SCF-style repeats hit
    the cache; the paper performs the symbolic factorization once per SCF
    cycle, Sec. II.B); the analysis of a new pattern and the pinned host
    staging of a request's values run on host worker threads as soon as the
    request arrives, overlapping the device work of the requests running,
  * keeps graph-captured plans with their factor buffers resident on the
    device, so a repeat of a resident pattern only uploads new values and a
    new pole table,
  * admits waiting requests whose analysis is ready while their device
    footprint fits the memory budget (idle resident plans are evicted
    least-recently-used first; a request larger than the budget runs its
    poles in chunks that add into one output),
  * runs admitted requests concurrently on several HIP streams: everything
    a request needs (value uploads from pinned memory, the inertia counts of
    Sec. II.C, every pole chunk, the copies of its traces and pivot flags)
    is enqueued on its stream without waiting for the device, and the loop
    polls the completion events of all running requests, so a request that
    finishes early frees its stream and memory at once and a new arrival is
    admitted while others run (continuous batching),
  * reports latency from arrival to result (p50 / p99) beside throughput.
Host-side orchestration only: every numeric step runs in the library's
kernels.
"""
from __future__ import annotations

import concurrent.futures
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
    flops: float = 0.0            # algorithmic flops of the request (pole solves + inertia counts)
    key: str = ""
    _staged: object = None        # future of the pinned host copies of H and S values
    _dev: object = None           # device tensors alive until completion

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


def _pinned(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


class Server:
    def __init__(self, budget_bytes=250 * 2**30, nstreams=4, max_patterns=64, device="cuda",
                 keep_outputs=False, tuned=None, host_workers=2, max_request_share=0.5):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        # no request holds more than this share of the budget: a larger one
        # runs its poles in chunks, leaving room for others to run beside it
        self.request_cap = int(max(0.0, min(1.0, max_request_share)) * self.budget)
        self.device = device
        self.keep = keep_outputs
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, nstreams))]
        self.analyses = OrderedDict()       # pattern key -> bound Analysis (LRU)
        self.pending = {}                   # pattern key -> future of its (unbound) Analysis
        self.max_patterns = max_patterns
        self.tuned = tuned
        self.residents = OrderedDict()      # (key, P, nsets, chunk) -> Resident (LRU)
        self.used = 0
        self.workers = concurrent.futures.ThreadPoolExecutor(max_workers=max(1, host_workers))
        self.stats = dict(symbolic_hits=0, symbolic_misses=0, plan_hits=0, plan_misses=0,
                          evictions=0, chunked=0, analyze_s=0.0, inertia_retries=0, alloc_retries=0,
                          deep_cleans=0)

    # ------------------------------------------------------------------ host side
    def _analyse(self, system, poles):
        """Symbolic analysis on a worker thread (host only; binding the maps
        to the device happens on the serving thread)."""
        t = time.perf_counter()
        if self.tuned:
            from .tune import tuned_analysis
            a = tuned_analysis(system, poles, cache=self.tuned)
        else:
            a = B.Analysis.from_system(system)
        return a, time.perf_counter() - t

    def _arrive(self, req):
        """Starts the host work of a request as it arrives: the analysis of
        a new pattern and the pinned copies of its values."""
        req.key = pattern_key(req.system)
        if req.key in self.analyses or req.key in self.pending:
            self.stats["symbolic_hits"] += 1
        else:
            self.stats["symbolic_misses"] += 1
            self.pending[req.key] = self.workers.submit(self._analyse, req.system, req.poles)
        req._staged = self.workers.submit(lambda s: (_pinned(s.hval), _pinned(s.sval)), req.system)

    def analysis(self, req):
        """The bound analysis of the request's pattern, or None while it is
        computed."""
        key = req.key
        a = self.analyses.get(key)
        if a is not None:
            self.analyses.move_to_end(key)
            return a
        fut = self.pending.get(key)
        if fut is None:
            # dropped from the cache since the request arrived: analyse again
            self.pending[key] = self.workers.submit(self._analyse, req.system, req.poles)
            return None
        if not fut.done():
            return None
        a, secs = fut.result()
        del self.pending[key]
        self.stats["analyze_s"] += secs
        a.bind(self.device)
        self.analyses[key] = a
        self.used += a.info["map_bytes"]       # the bound maps live on the device
        while len(self.analyses) > self.max_patterns:
            old = next(iter(self.analyses))
            self._drop_analysis(old)
        return a

    def _drop_analysis(self, key):
        """Forgets a pattern's analysis (its maps) and its idle residents;
        busy residents keep their own reference until they are evicted."""
        a = self.analyses.pop(key)
        self.used -= a.info["map_bytes"]
        for rk in [k for k in self.residents if k[0] == key and not self.residents[k].busy]:
            self._evict(rk)

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
        """Shifts per pole chunk: all P when the request fits the per-request
        cap, else the largest even chunk (halving) that does.  The pattern's
        bound maps stay on the device while the request runs, so the resident
        must fit beside them."""
        room = self.budget - a.info["map_bytes"]
        cap = max(min(self.request_cap, room), 1)
        c = P
        while c > 2 and resident_bytes(a, c, nsets) > cap:
            c = max(2, (c // 2) & ~1)
        if resident_bytes(a, c, nsets) > room:
            raise B.PxsError("Server", B.PXS_ENOMEM, "request does not fit the memory budget")
        return c

    def acquire(self, req):
        """Resident state for the request, or None while it cannot run yet
        (analysis or staging not ready, resident busy, no memory)."""
        a = self.analysis(req)
        if a is None or not req._staged.done():
            return None
        chunk = self.chunk_for(a, req.poles, req.nsets)
        rk = (req.key, req.poles, req.nsets, chunk)
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
        r = self._new_resident(a, req, chunk, need)
        if r is None:
            return None
        self.residents[rk] = r
        self.used += r.footprint
        self.stats["plan_misses"] += 1
        return r

    def _new_resident(self, a, req, chunk, need):
        """Allocates a resident; None if the memory is not there yet."""
        torch = self.torch
        try:
            with torch.cuda.device(self.device):
                return Resident(a, req.poles, req.nsets, chunk, self.device)
        except torch.OutOfMemoryError:
            pass
        # within the budget, but the allocator's free memory is split into
        # blocks too small: drop the idle residents, return the allocator's
        # cached blocks to the device and try once more; else wait for
        # running requests to end
        self.stats["alloc_retries"] += 1
        for idle in [k for k in self.residents if not self.residents[k].busy]:
            self._evict(idle)
        torch.cuda.empty_cache()
        if not self._make_room(need):
            return None
        try:
            with torch.cuda.device(self.device):
                return Resident(a, req.poles, req.nsets, chunk, self.device)
        except torch.OutOfMemoryError:
            return None

    # -------------------------------------------------------------- execution
    def _start(self, req, r, si, now):
        """Enqueues all of the request's work on its stream; returns the
        completion event.  Nothing here waits for the device."""
        torch = self.torch
        st = self.streams[si]
        dev = self.device
        r.busy = True
        req.t_admit = now
        hp, sp = req._staged.result()
        if req.dE is None:
            req.dE = job_dE(req.system, req.mu)
        sh, wt = B.poles(req.beta, req.dE, req.mu, req.poles, req.nsets)
        req.chunks = (req.poles + r.chunk - 1) // r.chunk
        if req.chunks > 1:
            self.stats["chunked"] += 1
        info = r.analysis.info
        # complex shifts: factor + SelInv; real inertia shifts: a real
        # factorization (2 flops per multiply-add instead of 8)
        req.flops = req.poles * (info["flops_factor"] + info["flops_selinv"])
        if req.eps is not None:
            req.flops += len(req.eps) * info["flops_factor"] / 4.0
        d = {"pinned": (hp, sp)}
        with torch.cuda.stream(st):
            r.H.copy_(hp, non_blocking=True)
            r.S.copy_(sp, non_blocking=True)
            if req.eps is not None and len(req.eps):
                # the resident buffers hold `chunk` complex shifts, i.e. at
                # least `chunk` real ones with their workspace
                nq = len(req.eps)
                eps_h = _pinned(np.asarray(req.eps, dtype=np.float64))
                d["eps"] = eps_h.to(dev, non_blocking=True)
                d["neg"] = torch.empty(nq, dtype=torch.int64, device=dev)
                d["ninfo"] = torch.empty(nq, dtype=torch.int64, device=dev)
                for q0 in range(0, nq, r.chunk):
                    q1 = min(nq, q0 + r.chunk)
                    B.inertia_async(r.analysis, r.H, r.S, d["eps"][q0:q1], d["neg"][q0:q1], d["ninfo"][q0:q1],
                                    L=r.L, work=r.W, stream=st)
            tab = np.concatenate([sh, wt.reshape(-1)])
            d["table"] = _pinned(tab.view(np.float64)).to(dev, non_blocking=True).view(torch.complex128)
            d["traces"] = torch.empty((req.chunks, 2 * req.nsets), dtype=torch.float64, device=dev)
            d["info"] = torch.empty(req.poles, dtype=torch.int64, device=dev)
            P = req.poles
            for c, c0 in enumerate(range(0, P, r.chunk)):
                c1 = min(P, c0 + r.chunk)
                p = r.plan(c1 - c0, c0 > 0)
                # the chunk's shifts and its columns of every weight set
                wsl = torch.stack([d["table"][P + g * P + c0:P + g * P + c1] for g in range(req.nsets)])
                p.run_device(d["table"][c0:c1], wsl.reshape(-1), stream=st)
                p.copy_results(d["traces"][c], d["info"][c0:c1], stream=st)
                d.setdefault("weights", []).append(wsl)
            if self.keep:
                # on this stream, before the resident is released to others
                req.out = r.out.view(req.nsets, -1).clone()
            ev = torch.cuda.Event()
            ev.record(st)
        req._dev = d
        return ev

    def _finish(self, req, r, si):
        """Collects the results of a completed request (its event has
        fired, so these reads do not wait)."""
        d = req._dev
        with self.torch.cuda.stream(self.streams[si]):
            req.traces = d["traces"].cpu().numpy().reshape(req.chunks, req.nsets, 2).sum(axis=0)
            req.info = d["info"].cpu().numpy()
            if "neg" in d:
                neg = d["neg"].cpu().numpy()
                ninfo = d["ninfo"].cpu().numpy()
        if "neg" in d:
            bad = np.nonzero(ninfo)[0]
            if len(bad):
                # a tiny pivot makes a count unreliable: shift those eps and
                # count again (the count is piecewise constant in eps)
                from .chempot import inertia_counts
                self.stats["inertia_retries"] += len(bad)
                eps = np.array(req.eps, dtype=np.float64)[bad]
                eps += 1e-9 * max(1.0, float(np.abs(eps).max()))
                with self.torch.cuda.stream(self.streams[si]):
                    neg[bad] = inertia_counts(r.analysis, r.H, r.S, eps, L=r.L, work=r.W,
                                              stream=self.streams[si])
            req.neg_counts = neg
        req._dev = None
        req._staged = None
        r.busy = False

    def run(self, requests, realtime=True, poll_s=2e-4, log=None, log_every_s=10.0):
        """Serves the requests (arrival times in seconds from the start);
        returns a summary dict (its counters cover this call only; caches
        and residents carry over between calls).  realtime=False ignores
        arrival times (saturated throughput).  log: a text stream for a
        progress line every log_every_s seconds."""
        torch = self.torch
        reqs = sorted(requests, key=lambda q: q.arrival)
        for i, q in enumerate(reqs):
            if q.rid < 0:
                q.rid = i
        waiting = []
        active = []   # (req, resident, stream index, event)
        free = list(range(len(self.streams)))
        nxt = 0
        ndone = 0
        cleaned = False
        stats0 = dict(self.stats)   # the summary counts this run only
        t0 = time.perf_counter()
        t_log = t0
        while nxt < len(reqs) or waiting or active:
            now = time.perf_counter() - t0
            if log is not None and time.perf_counter() - t_log >= log_every_s:
                t_log = time.perf_counter()
                print(f"# serve: {now:.0f}s, {ndone}/{len(reqs)} done, {len(active)} running, "
                      f"{len(waiting)} waiting", file=log, flush=True)
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= now):
                if not realtime:
                    reqs[nxt].arrival = 0.0
                self._arrive(reqs[nxt])
                waiting.append(reqs[nxt])
                nxt += 1
            # completions: every running request, in any order
            progressed = False
            still = []
            for item in active:
                req, r, si, ev = item
                if ev.query():
                    req.t_done = time.perf_counter() - t0
                    self._finish(req, r, si)
                    free.append(si)
                    progressed = True
                    ndone += 1
                else:
                    still.append(item)
            active = still
            # admissions: in arrival order, skipping requests whose analysis,
            # staging, resident or memory is not ready yet
            i = 0
            while i < len(waiting) and free:
                r = self.acquire(waiting[i])
                if r is None:
                    i += 1
                    continue
                req = waiting.pop(i)
                si = free.pop(0)
                ev = self._start(req, r, si, time.perf_counter() - t0)
                active.append((req, r, si, ev))
                progressed = True
            if (not progressed and not active and waiting and not self.pending
                    and all(q._staged.done() for q in waiting)):
                # nothing runs and nothing is being prepared, yet no waiting
                # request could start: free everything idle (residents, the
                # analyses no waiting request needs, the allocator's cached
                # blocks) and try again; if that was done already, none ever will
                if cleaned:
                    raise RuntimeError("scheduler stalled: a waiting request can never be admitted")
                keep = {q.key for q in waiting}
                for rk in [k for k in self.residents if not self.residents[k].busy]:
                    self._evict(rk)
                for key in [k for k in self.analyses if k not in keep]:
                    self._drop_analysis(key)
                torch.cuda.empty_cache()
                self.stats["deep_cleans"] += 1
                cleaned = True
                continue
            if progressed:
                cleaned = False
            if not progressed:
                time.sleep(poll_s)
        torch.cuda.synchronize()
        makespan = time.perf_counter() - t0
        lat = np.array([q.latency for q in reqs])
        solves = sum(q.poles for q in reqs)
        flops = sum(q.flops for q in reqs)
        return dict(requests=len(reqs), makespan_s=makespan, req_per_s=len(reqs) / makespan,
                    pole_solves_per_s=solves / makespan, path_tflops=flops / makespan / 1e12,
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    mean_s=float(lat.mean()), **{k: v - stats0[k] for k, v in self.stats.items()})

    def close(self):
        self.workers.shutdown(wait=True)


def poisson_arrivals(n, rate, seed=0):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
