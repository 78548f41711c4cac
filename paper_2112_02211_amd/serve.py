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
  cached after a job, so later requests on the same scatterer skip setup;
* **continuous batching by ticks**: a job owns one operator (same mesh, order,
  wave number and medium; different sources) and advances all its active
  requests together, one restart cycle per tick, as one lock-step
  multi-right-hand-side solve (J^-1's block product becomes a GEMM on the
  matrix cores).  After every tick each converged request is returned and
  leaves the batch, and queued requests on the same operator join it (as far
  as the HBM budget allows).  Restarted GMRES starts every cycle from the
  current iterate, so a request sees the same iteration whether it runs in
  one call or tick by tick, alone or in a batch.

* **operator groups** (optional): requests that are alone on their operator
  but share a mesh (leaf grid, order, box) with other queued requests are
  solved as one operator group: one context holds all their operators and
  every launch of the solve covers all of them.

Latency of a request = completion (solution copied to the host) - arrival.
`Scheduler` is the policy and has no GPU dependency; `Server` executes it.
"""
from __future__ import annotations

import collections
import hashlib
import sys
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


def shape_key(prob: P.Problem) -> tuple:
    """Problems with equal shape keys share a mesh and can form an operator group."""
    return (tuple(prob.n_elem), prob.p, tuple(prob.lo), tuple(prob.hi))


@dataclass
class Job:
    key: str
    requests: list
    need_bytes: int
    needs_setup: bool
    group: bool = False      # an operator group: one request per operator, one shared mesh


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
    group_ops: int = 0       # > 1: requests alone on their operator are grouped by mesh, up to this many
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
            if self.group_ops > 1 and len(batch) == 1 and not resident:
                grp = self._group_for(req, busy_keys, resident_keys)
                if len(grp) > 1:
                    need = sum(int(self.size_fn(r.key, r.prob, 1, False)) for r in grp)
                    if used_bytes + need <= self.budget or used_bytes - evictable_bytes + need <= self.budget:
                        ids = {id(r) for r in grp}
                        self.pending = [r for r in self.pending if id(r) not in ids]
                        gkey = "group:" + "+".join(r.key for r in grp)
                        return Job(gkey, grp, need, True, group=True)
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

    def _group_for(self, head, busy_keys, resident_keys) -> list:
        """head and the oldest pending requests on other operators of the same
        mesh that are alone on their operator, neither running nor cached."""
        shape = shape_key(head.prob)
        count = collections.Counter(r.key for r in self.pending)
        grp, keys = [head], {head.key}
        for r in self.pending:
            if len(grp) >= self.group_ops:
                break
            if r.key in keys or r.key in busy_keys or r.key in resident_keys or count[r.key] > 1:
                continue
            if shape_key(r.prob) == shape:
                grp.append(r)
                keys.add(r.key)
        return grp

    def take(self, key: str, n: int) -> list:
        """Up to n pending requests on operator `key` (oldest first), removed from
        the queue: they join the running job of that operator at its next tick."""
        if n <= 0:
            return []
        got = [r for r in self.pending if r.key == key][:n]
        ids = {id(r) for r in got}
        self.pending = [r for r in self.pending if id(r) not in ids]
        return got


@dataclass
class ServeConfig:
    slots: int = 4
    hbm_fraction: float = 0.85       # of the free device memory at start
    block_prec: str = "fp64"         # "separable": the FP64 J^-1 without stored blocks
    precond_prec: str = "fp64"
    restart: int = 10                # Krylov dimension of a cycle = one tick (10: the fastest
                                     # of 10/20/50 on the mixed stream, 67 vs 60 vs 41 solves/s;
                                     # BF16 blocks need about 50: at 10 some requests stalled)
    tol: float = 1e-8
    solver: str = "gmres"            # single right-hand side: "gmres" (left, FP64 J^-1), "fgmres",
                                     # or "ir" (iterative refinement with FP32 inner solves; needs
                                     # block_prec "separable"; a tick is one inner cycle)
    max_batch: int = 64
    max_iters: int = 20000           # per request; beyond it the request is returned unconverged
    keep_solution_on_host: bool = True
    lambda_bucket: float = 0.0       # > 0: operators share blocks on a lambda grid of this * kappa^2
    group_ops: int = 0               # > 1: requests alone on their operator run in operator groups
                                     # of up to this many on the same mesh (one launch for all)


@dataclass
class Result:
    rid: int
    key: str
    arrival: float
    start: float                     # the request entered a running batch
    finish: float
    iters: int                       # Arnoldi steps of the ticks it took part in
    batch: int                       # largest batch it ran in
    setup: bool                      # its job built the operator
    converged: bool
    true_rel_res: float              # in the norm of the stopping test
    n_unknowns: int = 0
    u: Optional[np.ndarray] = None
    job: int = 0
    ticks: int = 0

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


@dataclass
class _Active:
    req: object
    s: object
    t: object
    u: object
    start: float
    iters: int = 0
    ticks: int = 0
    batch: int = 1


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
        self.sched = Scheduler(self.budget, self._size, cfg.max_batch, group_ops=cfg.group_ops)
        self.streams = [torch.cuda.Stream() for _ in range(cfg.slots)]
        self.free_slots = list(range(cfg.slots))
        self.errors: list = []
        self.n_jobs = 0

    # ---------------------------------------------------------------- sizing
    def _fp64_pc(self) -> bool:
        """J^-1 in FP64 (stored FP64 blocks or the separable form): left GMRES applies."""
        return self.cfg.precond_prec in ("fp64", "separable")

    def _blocks(self):
        bp, pp = self.cfg.block_prec, self.cfg.precond_prec
        if bp == "separable" and pp in ("fp64", "separable"):
            return ("separable",)
        return (bp,) if bp == pp else (bp, pp)

    def _size(self, key, prob, nrhs, resident) -> int:
        setup, transient = self.hps.setup_bytes(prob.n_elem, prob.p, self._blocks(),
                                                complex_medium=bool(np.any(np.imag(prob.bump_amps))))
        n = prob.n_unknowns
        k = min(nrhs, 64)
        flexible = not self._fp64_pc() or self.cfg.solver == "fgmres"
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
    def _activate(self, r, xyz, now: float) -> _Active:
        torch = self.torch
        sv, tv = P.rhs_data(r.prob, xyz, 0)
        s = torch.from_numpy(sv).to("cuda", non_blocking=False)
        t = torch.from_numpy(tv).to("cuda", non_blocking=False)
        return _Active(r, s, t, torch.zeros_like(s), now)

    def _grow(self, job: Job, prob, n_old: int, n_new: int) -> bool:
        """Reserve the extra solver bytes of a larger batch (lock held)."""
        extra = max(0, self._size(job.key, prob, n_new, True) - self._size(job.key, prob, n_old, True))
        if self._used() + extra > self.budget:
            return False
        self.running_bytes += extra
        job.need_bytes += extra
        return True

    def _run_group(self, stream, job: Job, job_id: int):
        """An operator group: one context for all operators of the job (same
        mesh), their requests advanced in lock step one restart cycle per tick;
        each request is returned when it converges (it keeps riding along, as
        a no-op, until the whole group has)."""
        torch = self.torch
        cfg = self.cfg
        ctx = self.hps.Context.group([r.prob for r in job.requests], block_precs=self._blocks())
        try:
            xyz = ctx.nodes()
            N = ctx.N
            t_now = time.perf_counter()
            act = [self._activate(r, xyz, t_now) for r in job.requests]
            k = len(act)
            S = torch.cat([a.s for a in act])
            T = torch.cat([a.t for a in act])
            U = torch.zeros_like(S)
            single = cfg.solver if self._fp64_pc() else "fgmres"
            left = set(range(k))
            while left:
                _, st, _ = ctx.gmres(S, T, tol=cfg.tol, restart=cfg.restart, u=U, solver=single,
                                     precond_prec=cfg.precond_prec, max_iters=cfg.restart, use_x0=True)
                res = st["rhs_rel_res"]
                done = []
                for i in sorted(left):
                    a = act[i]
                    a.iters += st["iters"]
                    a.ticks += 1
                    a.batch = k
                    if res[i] <= cfg.tol or a.iters >= cfg.max_iters:
                        done.append(i)
                if done:
                    uh = [U[i * N:(i + 1) * N].cpu().numpy() if cfg.keep_solution_on_host else None
                          for i in done]
                    stream.synchronize()
                    t_fin = time.perf_counter()
                    with self.lock:
                        for i, u_i in zip(done, uh):
                            a = act[i]
                            self.results.append(Result(
                                a.req.rid, a.req.key, a.req.t_arrival, a.start, t_fin, a.iters, k, True,
                                bool(res[i] <= cfg.tol), float(res[i]), N, u_i, job_id, a.ticks))
                    left -= set(done)
            stream.synchronize()
        finally:
            ctx.free()

    def _run_job(self, slot: int, job: Job, job_id: int):
        torch = self.torch
        cfg = self.cfg
        stream = self.streams[slot]
        if job.group:
            try:
                with torch.cuda.stream(stream):
                    self._run_group(stream, job, job_id)
            except Exception as e:  # reported after the run
                with self.lock:
                    self.errors.append((job.key, repr(e)))
            finally:
                with self.lock:
                    self.busy.discard(job.key)
                    self.running_bytes -= job.need_bytes
                    self.free_slots.append(slot)
                    self.lock.notify_all()
            return
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
                    ctx = self.hps.Context.from_problem(prob0, block_precs=self._blocks(),
                                                        lambda_bucket=cfg.lambda_bucket)
                xyz = ctx.nodes()
                N = ctx.N
                t_now = time.perf_counter()
                active = [self._activate(r, xyz, t_now) for r in job.requests]
                single = cfg.solver if self._fp64_pc() else "fgmres"
                while active:
                    k = len(active)
                    S = torch.cat([a.s for a in active]) if k > 1 else active[0].s
                    T = torch.cat([a.t for a in active]) if k > 1 else active[0].t
                    U = torch.cat([a.u for a in active]) if k > 1 else active[0].u
                    # flexible GMRES runs a batch in lock step itself (true-residual stops
                    # for every request); left GMRES batches as "batched"
                    solver = single if single == "fgmres" or k == 1 else "batched"
                    _, st, _ = ctx.gmres(S, T, tol=cfg.tol, restart=cfg.restart, u=U, solver=solver,
                                         precond_prec=cfg.precond_prec, max_iters=cfg.restart,
                                         use_x0=True)
                    res = st["rhs_rel_res"]
                    done, keep = [], []
                    for i, a in enumerate(active):
                        a.u = U[i * N:(i + 1) * N]
                        a.iters += st["iters"]
                        a.ticks += 1
                        a.batch = max(a.batch, k)
                        if res[i] <= cfg.tol or a.iters >= cfg.max_iters:
                            done.append((a, res[i]))
                        else:
                            keep.append(a)
                    if done:
                        uh = [a.u.cpu().numpy() if cfg.keep_solution_on_host else None for a, _ in done]
                        stream.synchronize()
                        t_fin = time.perf_counter()
                        with self.lock:
                            for (a, r_i), u_i in zip(done, uh):
                                self.results.append(Result(
                                    a.req.rid, job.key, a.req.t_arrival, a.start, t_fin, a.iters, a.batch,
                                    setup, bool(r_i <= cfg.tol), float(r_i), N, u_i, job_id, a.ticks))
                    active = keep
                    # queued requests on this operator join the batch for the next tick
                    with self.lock:
                        joined = []
                        while len(active) + len(joined) < cfg.max_batch:
                            nxt = self.sched.take(job.key, 1)
                            if not nxt:
                                break
                            if not self._grow(job, prob0, len(active) + len(joined),
                                              len(active) + len(joined) + 1):
                                self.sched.pending.insert(0, nxt[0])   # back to the head of the queue
                                break
                            joined += nxt
                    if joined:
                        t_now = time.perf_counter()
                        active += [self._activate(r, xyz, t_now) for r in joined]
                stream.synchronize()
            with self.lock:
                self.cache[job.key] = ctx
                self.cache.move_to_end(job.key)
                self.cache_bytes[job.key] = ctx.device_bytes()
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
            closed_loop: bool = False, progress_every: int = 0) -> List[Result]:
        """Serve a request stream.  Arrivals are replayed in real time (scaled by
        time_scale), or all at once if closed_loop.  Returns the results.  With
        progress_every > 0, a line goes to stderr each time that many more
        requests have finished."""
        t0 = time.perf_counter()
        reported = 0
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
                        self.n_jobs += 1
                        th = threading.Thread(target=self._run_job, args=(slot, job, self.n_jobs),
                                              daemon=True)
                        th.start()
                        workers.append(th)
                        started = True
                if progress_every > 0 and len(self.results) >= reported + progress_every:
                    reported = len(self.results) - len(self.results) % progress_every
                    print(f"served {len(self.results)}/{len(arrivals)} requests "
                          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
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
            "jobs": len({r.job for r in results}),
            "setups": len({r.job for r in results if r.setup}),
            "mean_ticks": float(np.mean([r.ticks for r in results])),
            "all_converged": all(r.converged for r in results),
            "operator_applies_munknowns_per_s":
                float(sum(r.n_unknowns * r.iters for r in results) / (t_last - t_first) / 1e6)}
