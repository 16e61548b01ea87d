"""Host logic of the serving engine (no GPU): the least-recently-used
eviction of the device tier, the admission refusal while hierarchies are in
use, the choice of the next batch, and the request stream's shape."""
import pytest

pytest.importorskip("torch")

from ldg_inputs import serving_requests
from paper_2412_12506_amd.serving import (Entry, Pending, ServingEngine, batch_workspace_bytes,
                                          problem_key, summarize, Result)


class _Stub:
    def __init__(self):
        self.unloaded = 0

    def unload(self):
        self.unloaded += 1


def _engine(budget, **kw):
    return ServingEngine(hbm_budget=budget, workers=2, **kw)


def _resident(eng, key, nbytes, busy=False):
    e = eng._entry(key)
    e.solver, e.resident, e.bytes, e.busy = _Stub(), True, nbytes, busy
    eng.used += nbytes
    return e


def test_reserve_evicts_least_recently_used_idle():
    eng = _engine(100)
    a = _resident(eng, "a", 40)
    b = _resident(eng, "b", 30, busy=True)
    c = _resident(eng, "c", 20)
    eng.entries.move_to_end("a")            # a used most recently: c is now the LRU idle one
    d = eng._entry("d")
    assert eng._reserve(d, 30)              # 90 + 30 > 100: evict c (LRU, idle)
    assert not c.resident and c.solver.unloaded == 1 and a.resident and b.resident
    assert eng.used == 40 + 30 + 30 and d.bytes == 30
    assert [k for k, _ in eng.evictions] == ["c"]
    e = eng._entry("e")
    assert eng._reserve(e, 30)              # evicts a (idle); b is busy and stays
    assert not a.resident and b.resident
    assert eng.used == 30 + 30 + 30
    assert eng.peak_used <= eng.budget


def test_reserve_refuses_when_all_in_use():
    eng = _engine(100)
    _resident(eng, "a", 60, busy=True)
    f = eng._entry("f")
    assert not eng._reserve(f, 50)
    assert eng.used == 60 and not eng.evictions


def test_pick_oldest_idle_key_and_batch_cap():
    from collections import deque
    eng = _engine(100, max_batch=3)
    eng.waiting = {
        "x": deque(Pending(i, 0.5 + i, i) for i in range(5)),
        "y": deque(Pending(10 + i, 0.1 + i, i) for i in range(2)),
    }
    _resident(eng, "y", 10, busy=True)      # y's requests are older but its hierarchy is in use
    key, batch = eng._pick()
    assert key == "x" and [r.rid for r in batch] == [0, 1, 2]
    eng.entries["y"].busy = False
    key, batch = eng._pick()
    assert key == "y" and [r.rid for r in batch] == [10, 11]
    key, batch = eng._pick()
    assert key == "x" and [r.rid for r in batch] == [3, 4]
    assert eng._pick() == (None, [])


def test_workspace_matches_the_batched_allocation():
    # 4 vectors x 8 right-hand sides per level (levels halve per dimension) + 5 fine
    n = 8 ** 3 * 27
    levels = sum(n // 8 ** l for l in range(3))          # 8^3 -> 4^3 -> 2^3
    exact = (4 * levels + 5 * n) * 8 * 8
    est = batch_workspace_bytes(n, 3)
    assert exact <= est <= exact * 1.01 + 4096


def test_request_stream_shape():
    reqs = serving_requests()
    assert len(reqs) == 512
    arr = [r.arrival for r in reqs]
    assert arr == sorted(arr) and arr[0] > 0
    for r in reqs:
        assert r.p in (1, 2, 3)
        assert (r.dim == 2 and r.n in (32, 64, 128, 256)) or (r.dim == 3 and r.n in (16, 24, 32, 48))
        assert 1.0 <= r.contrast <= 1e4
        assert (r.kind == "poisson") == (r.contrast == 1.0)
    assert len({problem_key(r) for r in reqs}) > 50
    # mean inter-arrival 1/rate (rate 100/s), within sampling error
    assert 0.008 < arr[-1] / len(reqs) < 0.012


def test_summarize():
    rs = [Result(i, (2, 16, 1, 1.0), 0.0, 0.0, 0.001 * (i + 1), 10, True, 1e-11, 2) for i in range(100)]
    s = summarize(rs)
    assert s["requests"] == 100 and s["converged"] == 100 and s["rejected"] == 0
    assert abs(s["p50_ms"] - 50.5) < 1e-9 and abs(s["p99_ms"] - 99.01) < 1e-9
    assert s["mean_batch"] == 2 and s["dofs_solved"] == 100 * 16 ** 2 * 4
