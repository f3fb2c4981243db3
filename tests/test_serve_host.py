"""Host-side bookkeeping of the serving loop (no GPU): residents are filed
under the request's own key, also after an allocation retry, and the pole
chunk respects the per-request share of the memory budget."""
import contextlib
import types
from collections import OrderedDict

import numpy as np
import pytest

from paper_1405_0194_amd import serve


class _FakeAnalysis:
    def __init__(self, nnz, bps, wps):
        self.info = {"nnz_lower": nnz, "bytes_per_shift": bps, "map_bytes": 4096}
        self._wps = wps

    def workspace_size(self, nshift, real=False):
        return 1024 + nshift * self._wps


class _Done:
    def done(self):
        return True


class _NoDevice:
    """Stands in for torch.cuda on the host: device scopes do nothing."""
    @staticmethod
    def device(d):
        return contextlib.nullcontext()

    @staticmethod
    def empty_cache():
        pass


def _server(budget, share=1.0):
    import torch
    srv = object.__new__(serve.Server)
    srv.torch = types.SimpleNamespace(cuda=_NoDevice, OutOfMemoryError=torch.OutOfMemoryError)
    srv.budget = budget
    srv.request_cap = int(share * budget)
    srv.device = "cpu"
    srv.analyses = OrderedDict()
    srv.pending = {}
    srv.max_patterns = 64
    srv.residents = OrderedDict()
    srv.used = 0
    srv.stats = dict(symbolic_hits=0, symbolic_misses=0, plan_hits=0, plan_misses=0, evictions=0, chunked=0,
                     analyze_s=0.0, inertia_retries=0, alloc_retries=0, deep_cleans=0)
    return srv


def _request(key, P=40):
    q = serve.Request(system=None, poles=P)
    q.key = key
    q._staged = _Done()
    return q


def test_resident_keyed_by_request_after_allocation_retry(monkeypatch):
    import torch
    made = []

    class FakeResident:
        fail_next = True

        def __init__(self, analysis, P, nsets, chunk, device):
            if FakeResident.fail_next:
                FakeResident.fail_next = False
                raise torch.OutOfMemoryError("fragmented")
            self.analysis, self.P, self.chunk = analysis, P, chunk
            self.busy = False
            self.footprint = serve.resident_bytes(analysis, chunk, nsets)
            made.append(self)

    monkeypatch.setattr(serve, "Resident", FakeResident)
    srv = _server(budget=10**12)
    small, big = _FakeAnalysis(150033, 10**6, 10**5), _FakeAnalysis(2464969, 10**8, 10**7)
    srv.analyses["big"] = big
    srv.analyses["small"] = small
    FakeResident.fail_next = False
    rb = srv.acquire(_request("big"))          # an idle resident of another pattern
    assert rb is not None and ("big", 40, 2, 40) in srv.residents
    FakeResident.fail_next = True              # the next allocation fails once
    rs = srv.acquire(_request("small"))
    assert rs is not None and rs.analysis is small
    assert srv.stats["alloc_retries"] == 1
    # filed under the small request's key; the idle big resident was dropped
    assert list(srv.residents.keys()) == [("small", 40, 2, 40)]
    assert srv.residents[("small", 40, 2, 40)] is rs
    # a later request of the big pattern gets a resident of its own size
    rb2 = srv.acquire(_request("big"))
    assert rb2.analysis is big


def test_pole_chunk_respects_request_share():
    a = _FakeAnalysis(1000, 10**9, 10**8)
    full = serve.resident_bytes(a, 40, 2)
    srv = _server(budget=full + 10, share=0.5)
    c = srv.chunk_for(a, 40, 2)
    assert c < 40 and c % 2 == 0
    assert serve.resident_bytes(a, c, 2) <= srv.request_cap
    srv = _server(budget=full + a.info["map_bytes"] + 10, share=1.0)
    assert srv.chunk_for(a, 40, 2) == 40
    # the pattern's maps stay on the device beside the resident
    srv = _server(budget=full + 10, share=1.0)
    c = srv.chunk_for(a, 40, 2)
    assert c < 40 and serve.resident_bytes(a, c, 2) + a.info["map_bytes"] <= srv.budget
    with pytest.raises(Exception):
        _server(budget=10, share=1.0).chunk_for(a, 40, 2)
