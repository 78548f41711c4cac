"""Continuous-batching solve server for Helmholtz requests on one GPU.

Requests (a problem: mesh, order, wave number, medium, source) arrive over
time.  The server keeps several solves on the device at once and admits new
work as slots and HBM free up:

* **slots**: S worker threads, each driving the library on its own HIP stream
  (default priority), so setups and solves of different requests overlap on
  the device;
* **admission by HBM footprint**: a job is started only if its device bytes
  (the library's own plan: `hps_setup_bytes` for the tables, medium and
  blocks, `hps_solve_bytes` for the solver workspaces) fit in the budget next
  to everything already resident; idle cached contexts are evicted (LRU) to
  make room; the queue is served oldest first, with backfill of smaller jobs
  while the oldest one waits for memory (bounded, so it cannot starve);
* **resident operators**: the context of an operator (its dense blocks) stays
  cached after a solve, so later requests on the same scatterer skip setup;
* **batching**: queued requests on the same operator (same mesh, order, wave
  number and medium; different sources) are solved together as one lock-step
  multi-right-hand-side solve, where the preconditioner's block product is a
  GEMM on the matrix cores.

Latency of a request = completion (solution copied to the host) - arrival.
`Scheduler` is the policy and has no GPU dependency; `Server` executes it.
"""
from __future__ import annotations

import collections
import hashlib
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import problems as P


def operator_key(prob: P.Problem) -> str:
    """Identity of the discrete operator A (and J^-1): mesh, order, kappa, eta, box, medium."""
    h = hashlib.sha1()
    h.update(repr((tuple(prob.n_elem), prob.p, float(prob.kappa), float(prob.eta),
                   tuple(prob.lo), tuple(prob.hi), float(prob.bump_width),
                   prob.plane_dir is not None)).encode())
    h.update(np.ascontiguousarray(prob.bump_centres, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(prob.bump_amps, dtype=np.complex128).tobytes())
    return h.hexdigest()[:16]


@dataclass
class Job:
    key: str
    requests: list
    need_bytes: int
    needs_setup: bool


@dataclass
class Scheduler:
    """Admission and batching policy (host logic only).

    size_fn(key, prob, nrhs, resident) -> device bytes the job needs *in
    addition* to what is resident (blocks are counted only if not resident).
    """
    budget: int
    size_fn: Callable
    max_batch: int = 64
    starve_s: float = 2.0
    pending: list = field(default_factory=list)

    def submit(self, req, now: float):
        req.t_queued = now
        self.pending.append(req)

    def next_job(self, busy_keys, resident_keys, used_bytes: int, now: float,
                 evictable_bytes: int = 0) -> Optional[Job]:
        """Pick the next job or None.  used_bytes: bytes held now (resident
        contexts + running jobs); evictable_bytes: of those, what idle cached
        contexts could release."""
        head_waits = bool(self.pending) and (now - self.pending[0].t_queued) > self.starve_s
        seen = set()
        for i, req in enumerate(self.pending):
            key = req.key
            if key in seen or key in busy_keys:
                seen.add(key)
                continue
            seen.add(key)
            batch = [r for r in self.pending if r.key == key][: self.max_batch]
            resident = key in resident_keys
            need = int(self.size_fn(key, req.prob, len(batch), resident))
            fits = used_bytes + need <= self.budget
            fits_after_evict = used_bytes - evictable_bytes + need <= self.budget
            if fits or fits_after_evict:
                ids = {id(r) for r in batch}
                self.pending = [r for r in self.pending if id(r) not in ids]
                return Job(key, batch, need, not resident)
            if i == 0 and head_waits:
                return None   # the oldest request has waited long enough: no backfill
        return None


@dataclass
class ServeConfig:
    slots: int = 4
    hbm_fraction: float = 0.85       # of the free device memory at start
    block_prec: str = "fp64"
    precond_prec: str = "fp64"
    restart: int = 50
    tol: float = 1e-8
    solver: str = "gmres"            # single right-hand side: "gmres" (left, FP64 J^-1) or "fgmres"
    max_batch: int = 64
    keep_solution_on_host: bool = True


@dataclass
class Result:
    rid: int
    key: str
    arrival: float
    start: float
    finish: float
    iters: int
    batch: int
    setup: bool
    converged: bool
    true_rel_res: float
    n_unknowns: int = 0
    u: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class Server:
    """Executes the Scheduler on the GPU with S slots (threads + HIP streams)."""

    def __init__(self, cfg: ServeConfig = ServeConfig()):
        import torch
        from . import hps
        self.torch = torch
        self.hps = hps
        self.cfg = cfg
        free, _total = torch.cuda.mem_get_info()
        self.budget = int(free * cfg.hbm_fraction)
        self.lock = threading.Condition()
        self.cache: "collections.OrderedDict[str, object]" = collections.OrderedDict()
        self.cache_bytes: Dict[str, int] = {}
        self.busy: set = set()
        self.running_bytes = 0
        self.results: List[Result] = []
        self.sched = Scheduler(self.budget, self._size, cfg.max_batch)
        self.streams = [torch.cuda.Stream() for _ in range(cfg.slots)]
        self.free_slots = list(range(cfg.slots))
        self.errors: list = []

    # ---------------------------------------------------------------- sizing
    def _blocks(self):
        return (self.cfg.block_prec,) if self.cfg.block_prec == self.cfg.precond_prec else \
            (self.cfg.block_prec, self.cfg.precond_prec)

    def _size(self, key, prob, nrhs, resident) -> int:
        setup, transient = self.hps.setup_bytes(prob.n_elem, prob.p, self._blocks(),
                                                complex_medium=bool(np.any(np.imag(prob.bump_amps))))
        n = prob.n_unknowns
        k = min(nrhs, 64)
        flexible = self.cfg.precond_prec != "fp64" or self.cfg.solver == "fgmres"
        m = self.cfg.restart
        vec = 16 * n * k
        solve = vec * ((m + 1) + (m if flexible else 0) + 1) + 16 * n * nrhs + \
            (224 * 1024 * 16 + 660_000) * k + 16 * k * prob.n_leaves * 6 * (prob.p - 2) ** 2
        if k >= 4:
            solve += k * prob.n_leaves * 6 * (prob.p - 2) ** 2 * 32
        io = 3 * 16 * n * nrhs   # s, t, u tensors
        return (0 if resident else setup + transient) + solve + io

    def _used(self) -> int:
        return sum(self.cache_bytes.values()) + self.running_bytes

    def _evictable(self) -> int:
        return sum(b for k, b in self.cache_bytes.items() if k not in self.busy)

    def _evict_for(self, need: int):
        for key in list(self.cache.keys()):
            if self._used() + need <= self.budget:
                return
            if key in self.busy:
                continue
            ctx = self.cache.pop(key)
            self.cache_bytes.pop(key, None)
            ctx.free()

    # ------------------------------------------------------------- execution
    def _run_job(self, slot: int, job: Job):
        torch = self.torch
        cfg = self.cfg
        stream = self.streams[slot]
        t_start = time.perf_counter()
        try:
            with torch.cuda.stream(stream):
                prob0 = job.requests[0].prob
                ctx = None
                with self.lock:
                    if job.key in self.cache:
                        ctx = self.cache[job.key]
                        self.cache.move_to_end(job.key)
                setup = ctx is None
                if setup:
                    ctx = self.hps.Context.from_problem(prob0, block_precs=self._blocks())
                xyz = ctx.nodes()
                k = len(job.requests)
                S = np.concatenate([P.rhs_data(r.prob, xyz, 0)[0] for r in job.requests])
                T = np.concatenate([P.rhs_data(r.prob, xyz, 0)[1] for r in job.requests])
                s = torch.from_numpy(S).to("cuda", non_blocking=False)
                t = torch.from_numpy(T).to("cuda", non_blocking=False)
                single = cfg.solver if cfg.precond_prec == "fp64" else "fgmres"
                solver = "batched" if k > 1 else single
                u, st, ok = ctx.gmres(s, t, tol=cfg.tol, restart=cfg.restart, solver=solver,
                                      precond_prec=cfg.precond_prec)
                uh = u.cpu().numpy() if cfg.keep_solution_on_host else None
                stream.synchronize()
                del s, t, u
            t_fin = time.perf_counter()
            with self.lock:
                if setup:
                    self.cache[job.key] = ctx
                    self.cache_bytes[job.key] = ctx.device_bytes()
                else:
                    self.cache_bytes[job.key] = ctx.device_bytes()
                for i, r in enumerate(job.requests):
                    self.results.append(Result(
                        r.rid, job.key, r.t_arrival, t_start, t_fin, st["iters"], k, setup, ok,
                        st["true_rel_res"], ctx.N,
                        uh[i * ctx.N:(i + 1) * ctx.N].copy() if uh is not None else None))
        except Exception as e:  # reported after the run
            with self.lock:
                self.errors.append((job.key, repr(e)))
        finally:
            with self.lock:
                self.busy.discard(job.key)
                self.running_bytes -= job.need_bytes
                self.free_slots.append(slot)
                self.lock.notify_all()

    def run(self, requests: List[P.Request], time_scale: float = 1.0,
            closed_loop: bool = False) -> List[Result]:
        """Serve a request stream.  Arrivals are replayed in real time (scaled by
        time_scale), or all at once if closed_loop.  Returns the results."""
        t0 = time.perf_counter()
        order = sorted(requests, key=lambda r: r.arrival)
        for r in order:
            r.key = operator_key(r.prob)
        arrivals = [(0.0 if closed_loop else r.arrival * time_scale, r) for r in order]
        ai = 0
        workers = []
        with self.lock:
            while True:
                now = time.perf_counter() - t0
                while ai < len(arrivals) and arrivals[ai][0] <= now:
                    r = arrivals[ai][1]
                    r.t_arrival = t0 + arrivals[ai][0]
                    self.sched.submit(r, now)
                    ai += 1
                started = False
                if self.free_slots and self.sched.pending:
                    job = self.sched.next_job(self.busy, set(self.cache.keys()), self._used(), now,
                                              self._evictable())
                    if job is not None:
                        self._evict_for(job.need_bytes)
                        slot = self.free_slots.pop()
                        self.busy.add(job.key)
                        self.running_bytes += job.need_bytes
                        th = threading.Thread(target=self._run_job, args=(slot, job), daemon=True)
                        th.start()
                        workers.append(th)
                        started = True
                if ai >= len(arrivals) and not self.sched.pending and \
                        len(self.free_slots) == self.cfg.slots:
                    break
                if not started:
                    wait = 0.05
                    if ai < len(arrivals):
                        wait = max(0.0, min(wait, arrivals[ai][0] - (time.perf_counter() - t0)))
                    self.lock.wait(timeout=wait if wait > 0 else 0.001)
        for th in workers:
            th.join()
        if self.errors:
            raise RuntimeError(f"{len(self.errors)} jobs failed, first: {self.errors[0]}")
        return sorted(self.results, key=lambda r: r.rid)

    def close(self):
        for ctx in self.cache.values():
            ctx.free()
        self.cache.clear()
        self.cache_bytes.clear()


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    t_first = min(r.arrival for r in results)
    t_last = max(r.finish for r in results)
    return {"requests": len(results), "solves_per_s": len(results) / (t_last - t_first),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_batch": max(r.batch for r in results),
            "jobs": len({(r.key, r.start) for r in results}),
            "setups": len({(r.key, r.start) for r in results if r.setup}),
            "all_converged": all(r.converged for r in results),
            "operator_applies_munknowns_per_s":
                float(sum(r.n_unknowns * r.iters for r in results) / (t_last - t_first) / 1e6)}
