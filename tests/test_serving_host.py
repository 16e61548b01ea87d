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


class _StubSolver:
    """Host-tier stand-in that checks the engine's ownership rules: a key is
    solved by one worker at a time and never unloaded while it is solved."""

    def __init__(self, key, log):
        self.key, self.log = key, log
        self.solving = 0
        self.closed = False

    def upload(self, stream=None):
        assert self.solving == 0, "upload while solving"

    def unload(self):
        if self.solving:
            self.log.append(f"unload of {self.key} while solving")

    def close(self):
        self.closed = True

    def resmoothed(self, **kw):
        raise RuntimeError("rebuild failed")


def _stub_engine(budget, workers, log, need=40, solve_s=0.002, fail_keys=()):
    import threading
    import time as _t
    eng = ServingEngine(hbm_budget=budget, workers=workers, max_batch=2)
    eng._new_stream = lambda: None
    lock = threading.Lock()

    def build(key):
        with eng.cv:
            e = eng._entry(key)
            e.solver, e.building = _StubSolver(key, log), False
            eng.cv.notify_all()
        return 0.0

    def solve(e, batch, stream, setup_s, upload_s):
        sv = e.solver
        with lock:
            if sv.solving:
                log.append(f"concurrent solves of {e.key}")
            sv.solving += 1
        if not e.busy:
            log.append(f"{e.key} solved while not marked busy")
        _t.sleep(solve_s)
        with lock:
            sv.solving -= 1
        failed = [r for r in batch if e.key in fail_keys and e.smoother == "sai"]
        with eng.cv:
            for r in batch:
                if r not in failed:
                    eng.results.append(Result(r.rid, e.key, r.arrival, 0.0, eng._now(), 1, True, 0.0,
                                              len(batch), smoother=e.smoother))
        return failed

    eng._build_host = build
    eng._need_bytes = lambda key: need
    eng._solve_batch = solve
    return eng


def test_memory_wait_keeps_ownership():
    """Keys that wait for memory are handed back and taken by other workers
    meanwhile: no key is solved by two workers at once, none is unloaded or
    evicted while it is solved, and every request is served exactly once."""
    from types import SimpleNamespace
    log = []
    eng = _stub_engine(budget=100, workers=4, log=log, need=40)
    reqs = [SimpleNamespace(rid=i, arrival=0.0005 * i, dim=2, n=8 + 2 * (i % 6), p=1, contrast=1.0,
                            seed=i) for i in range(240)]
    res = eng.run(reqs)
    assert not log, log[:5]
    assert sorted(r.rid for r in res) == list(range(240))
    assert all(not r.error for r in res)
    assert eng.evictions                      # the budget forced evictions along the way
    assert eng.peak_used <= eng.budget


def test_failed_rebuild_requeues_without_double_reports():
    """A key whose SAI batch fails and whose GS rebuild raises: its requests
    are queued again (not reported twice), the entry drops its host tier and
    keeps the GS label, and the next batch (built from scratch with GS) serves
    them."""
    from types import SimpleNamespace
    log = []
    eng = _stub_engine(budget=1000, workers=2, log=log, fail_keys=((2, 8, 1, 10.0),))
    reqs = [SimpleNamespace(rid=i, arrival=0.0, dim=2, n=8, p=1, contrast=10.0, seed=i) for i in range(3)]
    res = eng.run(reqs)
    assert not log
    assert sorted(r.rid for r in res) == [0, 1, 2]
    assert all(r.converged and r.smoother == "gs" and not r.error for r in res)
    e = eng.entries[(2, 8, 1, 10.0)]
    assert e.smoother == "gs" and e.fallbacks == 1
    assert any("GS rebuild failed" in m for m in eng.errors)
