"""Continuous-batching solve service on one GPU, above the C-ABI.

Requests (one Poisson or elliptic-interface problem each: dim, n, p, viscosity
contrast, right-hand-side seed) arrive over time.  Each request is solved to
the same relative residual by CG preconditioned with one V-cycle (FP32
operator blocks, BF16 SAI blocks by default, FP64 vectors and Krylov), exactly
as a lone ldgmg_solve would.

Hierarchy cache, two tiers, keyed by the problem:
  * host tier: the hierarchy built by ldgmg_setup_host (block pools, indices,
    bottom pseudo-inverse).  Built once per key; it is compact because every
    distinct block is stored once.
  * device tier (HBM): hierarchies uploaded with ldgmg_upload.  A hierarchy is
    admitted only while the device bytes of all resident hierarchies stay
    within the budget (ldgmg_upload_bytes of the built host tier plus the
    batched-solve workspace, the measured ldgmg_device_bytes once it is larger);
    idle ones are
    evicted least recently used with ldgmg_unload, keeping their host tier.
    Requests whose hierarchy does not fit wait until a running batch ends.

Robustness: when a batch's CG solves with the SAI V-cycle do not converge (the
engine enables the library's CG guard, which stops CG at once when the
preconditioner shows it is not positive definite), the hierarchy of that
problem is rebuilt with the coloured Gauss-Seidel smoother (the paper's
second-ranked smoother; ldgmg_rebuild_smoother keeps the operators and the
bottom) and the affected requests are queued again at the front; later
requests of the key use it.

Scheduling: several workers, each with its own HIP stream, take the key whose
oldest waiting request is oldest among the keys not in use (ties: the most
work first) and serve it with continuous batching (ldgmg_solve_stream): up to
max_batch CG recurrences of that key run together, every matrix block streamed
once per V-cycle stage for all of them, and a slot freed by a converged
request is refilled at the next stage with a request of the same key that is
waiting by then, including requests that arrived while the batch ran.  Batches
of different hierarchies run on the device at the same time.  A request's
latency is completion minus arrival.

Interface requests put the request's viscosity contrast inside the box
(1/4, 3/4)^d (the multiphase geometry of Section 2.4.3).
"""
from __future__ import annotations

import os
import threading
import time
from collections import OrderedDict, deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from . import ldgmg as L


def problem_key(req) -> tuple:
    return (req.dim, req.n, req.p, float(req.contrast))


def problem_kwargs(key, precision="fp32", smoother="sai", setup_device=False):
    from ldg_inputs import mu_box
    dim, n, p, contrast = key
    mu = None if contrast == 1.0 else mu_box(dim, n, contrast)
    if smoother != "sai" and precision == "bf16s":     # BF16 storage is for the SAI matrices
        precision = "fp32"
    return dict(dim=dim, n=n, p=p, mu=mu, smoother=smoother, sai_level=1, order="OI",
                precision=precision, setup_device=setup_device)


def batch_workspace_bytes(ndofs_fine: int, dim: int, max_batch: int = 8) -> int:
    """Device bytes of the batched-solve workspace: 4 level vectors on every
    level (geometric sum over the hierarchy) and 5 fine Krylov vectors, each
    holding 8 right-hand sides in FP64 (16 when more than 8 share a batch)."""
    nrhs = 8 if max_batch <= 8 else 16
    levels = ndofs_fine * nrhs * 8 * 4 / (1.0 - 0.5 ** dim)
    return int(levels + ndofs_fine * nrhs * 8 * 5) + 4096


@dataclass
class Pending:
    rid: int
    arrival: float     # seconds after the start of the run
    seed: int


@dataclass
class Entry:
    key: tuple
    smoother: str = "sai"
    solver: Optional["L.Solver"] = None      # host tier (None until built)
    building: bool = False
    resident: bool = False                   # device tier
    bytes: int = 0
    busy: bool = False
    uploads: int = 0
    fallbacks: int = 0


@dataclass
class Result:
    rid: int
    key: tuple
    arrival: float
    start: float
    end: float
    iters: int
    converged: bool
    rel_res_true: float
    batch: int
    setup_s: float = 0.0
    upload_s: float = 0.0
    x: Optional[np.ndarray] = None
    error: str = ""
    smoother: str = "sai"

    @property
    def latency(self):
        return self.end - self.arrival


class ServingEngine:
    def __init__(self, hbm_budget: int, workers: int = 4, max_batch: int = 8, precision: str = "bf16s",
                 smoother: str = "sai", rtol: float = 1e-10, maxit: int = 200, keep_solutions: bool = False,
                 setup_threads: int = 0, allocator: str = "torch", setup_device: bool = False):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget)
        self.workers = workers
        self.max_batch = max(1, min(max_batch, L.MAX_BATCH))
        self.precision, self.smoother = precision, smoother
        self.rtol, self.maxit = rtol, maxit
        self.keep = keep_solutions
        # "torch": hierarchies live in torch's caching allocator (counted by it;
        # eviction hands memory back without a device-wide synchronisation);
        # "hip": the library's own hipMalloc / hipFree
        self.allocator = allocator
        # cache misses solve their SAI least-squares problems on the GPU (setup_device)
        self.setup_device = setup_device
        # host setup threads per worker: the host's share of cores split over the workers
        self.setup_threads = setup_threads or max(1, min(16, os.cpu_count() or 1) // workers)
        self.entries: "OrderedDict[tuple, Entry]" = OrderedDict()   # LRU order of use
        self.used = 0
        self.peak_used = 0
        self.cv = threading.Condition()
        self.waiting: Dict[tuple, deque] = {}
        self.results: List[Result] = []
        self.errors: List[str] = []
        self.evictions: List[tuple] = []     # (key, time)
        self.admissions: List[tuple] = []    # (key, time)
        self.fallback_keys: List[tuple] = []
        self.t0 = time.perf_counter()

    def _now(self):
        return time.perf_counter() - self.t0

    # -- host tier -------------------------------------------------------------
    def _entry(self, key) -> Entry:
        e = self.entries.get(key)
        if e is None:
            e = self.entries[key] = Entry(key, smoother=self.smoother)
        return e

    def _build_host(self, key) -> float:
        """Host setup of `key` (outside the lock); returns seconds."""
        ts = time.perf_counter()
        with self.cv:
            smoother = self._entry(key).smoother
        kw = problem_kwargs(key, self.precision, smoother, self.setup_device)
        solver = L.Solver(host_only=True, nthreads=self.setup_threads, allocator=self._new_allocator(), **kw)
        L.ldgmg_cg_guard(solver.handle, True)     # fail fast when the V-cycle is not SPD
        with self.cv:
            e = self._entry(key)
            e.solver, e.building = solver, False
            self.cv.notify_all()
        return time.perf_counter() - ts

    def prebuild(self, keys, threads: int = 4) -> float:
        """Build the host tier of `keys` ahead of the requests; returns seconds."""
        keys = [k for k in dict.fromkeys(keys) if self._entry(k).solver is None]
        per = max(1, min(16, os.cpu_count() or 1) // max(1, threads))
        saved, self.setup_threads = self.setup_threads, per
        ts = time.perf_counter()
        # largest first so that the pool finishes together
        keys.sort(key=lambda k: -(k[1] ** k[0]) * (k[2] + 1) ** (2 * k[0]))
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(self._build_host, keys))
        self.setup_threads = saved
        return time.perf_counter() - ts

    # -- device tier -------------------------------------------------------------
    def _need_bytes(self, key) -> int:
        """Device bytes of the key's hierarchy with the batch workspace: exact
        from the host tier when it is built, else the expanded-storage bound."""
        dim, n, p, _c = key
        ndofs = n ** dim * (p + 1) ** dim
        e = self.entries.get(key)
        if e is not None and e.solver is not None:
            return e.solver.upload_bytes + batch_workspace_bytes(ndofs, dim, self.max_batch)
        pr, _ = L.make_problem(**problem_kwargs(key, self.precision, self.smoother))
        return L.ldgmg_estimate_bytes(pr) + batch_workspace_bytes(ndofs, dim, self.max_batch)

    def _reserve(self, e: Entry, need: int) -> bool:
        """Under the lock: make room for `need` bytes (need <= budget) by
        evicting idle resident hierarchies, least recently used first.  False
        when the hierarchies in use leave too little room."""
        while self.used + need > self.budget:
            victim = next((v for v in self.entries.values()
                           if v.resident and not v.busy and v is not e), None)
            if victim is None:
                return False
            victim.solver.unload()
            victim.resident = False
            self.used -= victim.bytes
            victim.bytes = 0
            self.evictions.append((victim.key, self._now()))
        self.used += need
        e.bytes = need
        self.peak_used = max(self.peak_used, self.used)
        return True

    def _reject(self, key, batch, why):
        now = self._now()
        self.errors.append(f"{key}: {why}")
        for r in batch:
            self.results.append(Result(r.rid, key, r.arrival, now, now, 0, False, float("nan"), 0,
                                       error=why))

    # -- scheduling ----------------------------------------------------------------
    def _pick(self):
        """Under the lock: the key (not in use, not being built) with the oldest
        waiting request (among equally old ones, the most work: unknowns times
        waiting requests), and up to max_batch of its requests."""
        def rank(key, q):
            size = key[1] ** key[0] * (key[2] + 1) ** key[0] if isinstance(key, tuple) and len(key) == 4 else 1
            return (q[0].arrival, -size * min(len(q), self.max_batch))
        best, best_rank = None, None
        for key, q in self.waiting.items():
            if not q:
                continue
            e = self.entries.get(key)
            if e is not None and (e.busy or e.building):
                continue
            r = rank(key, q)
            if best is None or r < best_rank:
                best, best_rank = key, r
        if best is None:
            return None, []
        q = self.waiting[best]
        return best, [q.popleft() for _ in range(min(self.max_batch, len(q)))]

    def _new_allocator(self):
        # allocations follow the calling thread's current stream: uploads run
        # under the worker's stream, which the hierarchy's kernels then use
        return L.TorchAllocator() if self.allocator == "torch" else None

    def _new_stream(self):
        return self.torch.cuda.Stream()

    def _worker(self, stop):
        stream = self._new_stream()
        while True:
            with self.cv:
                key, batch = self._pick()
                while key is None:
                    if stop.is_set() and not any(self.waiting.values()):
                        return
                    self.cv.wait(timeout=0.005)
                    key, batch = self._pick()
                e = self._entry(key)
                self.entries.move_to_end(key)
                e.busy = True
                owned = True                 # this worker holds the key until it clears `owned`
                if e.solver is None:
                    e.building = True
            setup_s = upload_s = 0.0
            try:
                if e.solver is None:
                    setup_s = self._build_host(key)
                if not e.resident:
                    with self.cv:
                        need = self._need_bytes(key)
                        if need > self.budget:
                            self._reject(key, batch, f"needs {need} bytes, budget {self.budget}")
                            continue
                        if not self._reserve(e, need):        # wait for memory: hand the key back
                            self.waiting[key].extendleft(reversed(batch))
                            e.busy = False
                            owned = False                     # another worker may take it meanwhile
                            self.cv.notify_all()
                            self.cv.wait(timeout=0.005)
                            continue
                        self.admissions.append((key, self._now()))
                    tu = time.perf_counter()
                    try:
                        if stream is not None:
                            with self.torch.cuda.stream(stream):
                                e.solver.upload(stream)
                        else:
                            e.solver.upload(stream)
                    except Exception:
                        with self.cv:
                            self.used -= e.bytes
                            e.bytes = 0
                        raise
                    upload_s = time.perf_counter() - tu
                    e.resident = True
                    e.uploads += 1
                failed = self._solve_batch(e, batch, stream, setup_s, upload_s)
                if failed:                         # SAI did not converge: switch the key to GS
                    self._fallback(e, key, failed)
            except Exception as ex:  # keep serving; report the failure
                with self.cv:
                    # requests already recorded by _solve_batch are not reported twice
                    done_ids = {r.rid for r in self.results}
                    self._reject(key, [r for r in batch if r.rid not in done_ids], str(ex))
            finally:
                with self.cv:
                    if owned:
                        e.busy = False
                        e.building = False
                    self.cv.notify_all()

    def _fallback(self, e: Entry, key, failed):
        """Rebuild e's hierarchy with the coloured Gauss-Seidel smoother (same
        operators and bottom) and queue `failed` again at the front.  The key
        stays busy meanwhile.  If the rebuild fails, the entry is reset to no
        host tier with the GS label, so that its next batch builds the GS
        hierarchy from scratch; `failed` is queued again either way."""
        with self.cv:
            old = e.solver
            old.unload()
            e.resident = False
            self.used -= e.bytes
            e.bytes = 0
            e.smoother = "gs"
            e.fallbacks += 1
            self.fallback_keys.append(key)
        try:
            new = old.resmoothed(nthreads=self.setup_threads, allocator=self._new_allocator(),
                                 **problem_kwargs(key, self.precision, "gs", self.setup_device))
            L.ldgmg_cg_guard(new.handle, True)
        except Exception as ex:
            with self.cv:
                e.solver = None
                self.errors.append(f"{key}: GS rebuild failed ({ex}); rebuilding from scratch")
                self.waiting[key].extendleft(reversed(failed))
            old.close()
            return
        old.close()
        with self.cv:
            e.solver = new
            self.waiting[key].extendleft(reversed(failed))

    def _other_key_waiting(self, key) -> bool:
        """Under the lock: another idle key has waiting requests."""
        for k, q in self.waiting.items():
            if k != key and q:
                o = self.entries.get(k)
                if o is None or not (o.busy or o.building):
                    return True
        return False

    def _solve_batch(self, e: Entry, batch, stream, setup_s, upload_s):
        """Solve `batch`, and the requests of the same key that arrive while it
        runs, with continuous batching (ldgmg_solve_stream: up to max_batch CG
        recurrences in flight; a slot freed by a converged request is refilled
        at the next V-cycle stage).  Records the results; returns the requests
        to retry (not converged with the SAI smoother).  Admission stops after
        4 x max_batch requests when another key is waiting, so that a busy key
        does not hold a worker forever."""
        from ldg_inputs import rhs_normal_device
        torch = self.torch
        n = e.solver.ndofs
        first = deque(batch)
        inflight = {}
        failed = []
        admitted = [0]

        def next_rhs():
            with self.cv:
                if failed:                    # the SAI V-cycle fails on this key: stop feeding it
                    return None
                if first:
                    r = first.popleft()
                else:
                    q = self.waiting.get(e.key)
                    if not q or (admitted[0] >= 4 * self.max_batch and self._other_key_waiting(e.key)):
                        return None
                    r = q.popleft()
                admitted[0] += 1
            with torch.cuda.stream(stream):        # the request's right-hand side, resident on the device
                b = rhs_normal_device(n, r.seed)
                x = torch.empty_like(b)
            inflight[r.rid] = (r, self._now(), len(inflight) + 1, x)
            return b, x, r.rid

        def on_done(tag, info):
            r, start, width, x = inflight.pop(tag)
            if not info["converged"] and e.smoother == "sai":
                failed.append(r)
                return
            xs = x.cpu().numpy() if self.keep else None
            with self.cv:
                self.results.append(Result(r.rid, e.key, r.arrival, start, self._now(), info["iters"],
                                           info["converged"], info["rel_res_true"], width, setup_s, upload_s,
                                           xs, smoother=e.smoother))

        L.ldgmg_solve_stream(e.solver.handle, self.max_batch, next_rhs, on_done, self.rtol, self.maxit,
                             stream=stream)
        with self.cv:
            first_left = list(first)
            if first_left:                    # not admitted (the key failed first): back to the queue
                self.waiting[e.key].extendleft(reversed(first_left))
            actual = e.solver.device_bytes
            if actual > e.bytes:           # measured bytes replace the estimate
                self.used += actual - e.bytes
                e.bytes = actual
                self.peak_used = max(self.peak_used, self.used)
        return failed

    def run(self, requests, time_scale: float = 1.0) -> List[Result]:
        """Replay `requests` (objects with rid, arrival in seconds, dim, n, p,
        contrast, seed) in real time scaled by time_scale; returns one Result
        per request, ordered by rid."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        stop = threading.Event()
        self.t0 = time.perf_counter()
        threads = [threading.Thread(target=self._worker, args=(stop,), daemon=True)
                   for _ in range(self.workers)]
        for th in threads:
            th.start()
        for r in reqs:
            due = r.arrival * time_scale
            delay = due - self._now()
            if delay > 0:
                time.sleep(delay)
            with self.cv:
                self.waiting.setdefault(problem_key(r), deque()).append(Pending(r.rid, due, r.seed))
                self.cv.notify_all()
        stop.set()
        with self.cv:
            self.cv.notify_all()
        for th in threads:
            th.join()
        return sorted(self.results, key=lambda x: x.rid)

    def close(self):
        self.torch.cuda.synchronize()
        for e in self.entries.values():
            if e.solver is not None:
                e.solver.close()
        self.entries.clear()
        self.used = 0


def summarize(results: List[Result]) -> dict:
    ok = [r for r in results if not r.error]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    wall = (max(r.end for r in results) - min(r.arrival for r in results)) if results else 0.0
    return {"requests": len(results), "converged": int(sum(r.converged for r in results)),
            "rejected": len(results) - len(ok),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_batch": float(np.mean([r.batch for r in ok])) if ok else 0.0,
            "solves_per_s": len(ok) / wall if wall > 0 else 0.0, "wall_s": wall,
            "dofs_solved": int(sum(r.key[1] ** r.key[0] * (r.key[2] + 1) ** r.key[0] for r in ok)),
            "max_rel_res_true": float(max((r.rel_res_true for r in ok), default=float("nan")))}
