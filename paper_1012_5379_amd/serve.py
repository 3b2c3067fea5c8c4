"""Continuous-batching serving loop over libcsg.

Requests (a problem: grid, phi, beta, ...; 1..max RHS) arrive over time.  The
engine admits a request as soon as its exact workspace (csg_workspace_bytes)
fits the HBM budget and a stream slot is free; the hierarchy is built on a
worker thread (ctypes releases the GIL) and stays resident until the solve
retires.  Admitted solves advance one FGMRES iteration at a time through the
non-blocking csg_solve_step / csg_solve_poll pair, each on its own HIP stream,
so the iterations of different requests overlap on the device; the right-hand
sides of one request run batched in the same launches.  Latency is arrival ->
last RHS done (queueing and setup included); setup is also reported apart.
A retired request's hierarchy is kept in an LRU cache keyed by a hash of its
parameters and phi, so a repeated problem skips setup; cached hierarchies are
evicted, oldest first, when an admission needs their memory.

Requests of one size class (same grid shape, levels, cycle, tolerance) that
are queued together are batched into one operator (csg_batch_create): their
hierarchies sit side by side in one workspace and every V-cycle and FGMRES
iteration of all of them runs in the same launches; each request's answer is
bit-identical to its solve alone.

Every arithmetic step runs in libcsg's kernels; this module only schedules.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import time
from collections import OrderedDict
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import binding as B


@dataclass
class Request:
    rid: int
    params: dict             # csg_params fields (dim, n, h, layers, gamma, beta, levels, s, nu1, nu2, cycle_prec)
    phi: np.ndarray          # real FP64 on the finest unknowns
    chi: np.ndarray          # complex128 (nrhs, *grid)
    tol: float = 1e-6
    restart: int = 30
    maxit: int = 3000
    arrival: float = 0.0     # seconds after the start of the run
    # filled by the engine
    t_admit: float = float("nan")
    t_ready: float = float("nan")
    t_done: float = float("nan")
    status: Optional[int] = None
    infos: list = field(default_factory=list)
    u: Optional[np.ndarray] = None

    @property
    def nrhs(self) -> int:
        return int(self.chi.shape[0])

    def csg_params(self, graphs: int = -1):
        return B.make_params(**dict(self.params, max_rhs=self.nrhs, restart=self.restart, graphs=graphs))

    def workspace_bytes(self) -> int:
        """Device bytes the request holds while admitted: the library's
        workspace plus the complex128 chi and u vectors of every RHS."""
        return B.csg_workspace_bytes(self.csg_params()) + 2 * self.chi.nbytes

    def class_key(self) -> tuple:
        """Requests with equal keys can share a batched operator."""
        p = self.params
        keep = ("dim", "n", "layer_lo", "layer_hi", "levels", "s", "nu1", "nu2", "cycle_prec")
        return tuple((k, tuple(p[k]) if isinstance(p[k], (list, tuple)) else p[k]) for k in keep) + \
            (("restart", self.restart), ("tol", self.tol), ("maxit", self.maxit))

    def key(self) -> str:
        h = hashlib.sha1(repr(sorted(self.params.items())).encode())
        h.update(repr((self.nrhs, self.restart)).encode())
        h.update(np.ascontiguousarray(self.phi, dtype=np.float64).tobytes())
        return h.hexdigest()


class _Active:
    """One operator on the device: a single request, or a batch of requests of
    one size class (members[q] owns RHS q*R .. q*R + nrhs - 1)."""

    def __init__(self, members, R, slot, ws, op, chi, u, stream):
        self.members, self.R = members, R
        self.req = members[0]
        self.slot, self.ws, self.op, self.chi, self.u, self.stream = slot, ws, op, chi, u, stream
        self.sv = None
        self.nbytes = 0
        self.key = None

    @property
    def nrhs(self) -> int:
        return self.R * len(self.members)


class Engine:
    """Admit by HBM budget, overlap solves on `streams` HIP streams."""

    def __init__(self, hbm_budget: Optional[int] = None, streams: int = 4, device: str = "cuda",
                 keep_solutions: bool = True, cache: bool = True, batch: int = 4, graphs: bool = False):
        import torch
        self.torch = torch
        # FGMRES iterations replayed from captured HIP graphs (capture on an
        # operator's first solve) or launched one kernel at a time
        self.graphs = 1 if graphs else -1
        self.device = torch.device(device)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self.used = 0
        self.high_water = 0
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.free_slots = list(range(streams))
        self.queue: list = []
        self.active: list = []
        self.pending: list = []        # (future, request, slot, bytes)
        self.done: list = []
        self.keep = keep_solutions
        self.pool = cf.ThreadPoolExecutor(max_workers=1)
        self.use_cache = cache
        self.cache: "OrderedDict[str, tuple]" = OrderedDict()   # key -> (ws tensor, op, bytes)
        self.cache_hits = 0
        self.max_batch = max(1, int(batch))
        self.batches = 0          # batched operators built
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        nb = req.workspace_bytes()
        if nb > self.budget:
            raise ValueError(f"request {req.rid} needs {nb} bytes, more than the HBM budget {self.budget}")
        self.queue.append(req)

    # -- admission -------------------------------------------------------------
    def _batch_params(self, members, R):
        return [B.make_params(**dict(m.params, max_rhs=R, restart=m.restart, graphs=self.graphs)) for m in members]

    def _batch_bytes(self, members) -> int:
        R = max(m.nrhs for m in members)
        ps = self._batch_params(members, R)
        grid = int(np.prod(members[0].chi.shape[1:]))
        return B.csg_batch_workspace_bytes(ps[0], len(members)) + 2 * len(members) * R * grid * 16

    def _setup(self, req: Request, slot: int, cached=None):
        torch = self.torch
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            chi = torch.from_numpy(np.ascontiguousarray(req.chi)).to(self.device, non_blocking=False)
            u = torch.empty_like(chi)
        if cached is not None:
            ws, op, _ = cached
            return _Active([req], req.nrhs, slot, ws, op, chi, u, stream)
        p = req.csg_params(self.graphs)
        nb = B.csg_workspace_bytes(p)   # the library's share of req.workspace_bytes()
        with torch.cuda.stream(stream):
            ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        phi = np.ascontiguousarray(req.phi, dtype=np.float64)
        op = B.csg_operator_create(p, phi.ctypes.data, ws.data_ptr(), nb, stream.cuda_stream)
        return _Active([req], req.nrhs, slot, ws, op, chi, u, stream)

    def _setup_batch(self, members, slot: int):
        """One operator for several same-class requests: RHS of member q at
        q*R .. q*R + nrhs - 1, the rest zero sources (they stop at once)."""
        torch = self.torch
        stream = self.streams[slot]
        R = max(m.nrhs for m in members)
        shape = members[0].chi.shape[1:]
        host = np.zeros((len(members) * R,) + tuple(shape), dtype=np.complex128)
        for q, m in enumerate(members):
            host[q * R:q * R + m.nrhs] = m.chi
        ps = self._batch_params(members, R)
        nb = B.csg_batch_workspace_bytes(ps[0], len(members))
        phis = [np.ascontiguousarray(m.phi, dtype=np.float64) for m in members]
        with torch.cuda.stream(stream):
            chi = torch.from_numpy(host).to(self.device, non_blocking=False)
            u = torch.empty_like(chi)
            ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        op = B.csg_batch_create(ps, [f.ctypes.data for f in phis], ws.data_ptr(), nb, stream.cuda_stream)
        return _Active(list(members), R, slot, ws, op, chi, u, stream)

    def _take_batch(self):
        """The head of the queue and the queued requests of its size class
        (at most max_batch problems and CSG_MAX_RHS right-hand sides), shrunk
        until its bytes fit the budget; None if not even the head fits."""
        head = self.queue[0]
        members = [head]
        if self.max_batch > 1:
            cls = head.class_key()
            for r in self.queue[1:]:
                if len(members) >= self.max_batch:
                    break
                if r.class_key() == cls and (len(members) + 1) * max(r.nrhs, max(m.nrhs for m in members)) \
                        <= B.CSG_MAX_RHS:
                    members.append(r)
        while len(members) > 1 and self.used + self._batch_bytes(members) > self.budget:
            members.pop()
        return members

    def _evict_one(self) -> bool:
        if not self.cache:
            return False
        _, (ws, op, nb) = self.cache.popitem(last=False)
        B.csg_operator_destroy(op)
        self.used -= nb
        return True

    def _admit(self) -> None:
        while self.queue and self.free_slots:
            members = self._take_batch()
            if len(members) > 1:
                nb = self._batch_bytes(members)
                self.used += nb
                self.high_water = max(self.high_water, self.used)
                for m in members:
                    self.queue.remove(m)
                slot = self.free_slots.pop(0)
                now = self.now()
                for m in members:
                    m.t_admit = now
                self.batches += 1
                self.pending.append((self.pool.submit(self._setup_batch, members, slot), members[0], slot, nb, None))
                continue
            req = self.queue[0]
            key = req.key() if self.use_cache else None
            cached = self.cache.pop(key, None) if key is not None else None
            if cached is not None:
                nb = cached[2]
                self.cache_hits += 1
            else:
                nb = req.workspace_bytes()
                while self.used + nb > self.budget and self._evict_one():
                    pass
                if self.used + nb > self.budget:
                    break
                self.used += nb
                self.high_water = max(self.high_water, self.used)
            self.queue.pop(0)
            slot = self.free_slots.pop(0)
            req.t_admit = self.now()
            self.pending.append((self.pool.submit(self._setup, req, slot, cached), req, slot, nb, key))

    def _start_ready(self) -> None:
        still = []
        for fut, req, slot, nb, key in self.pending:
            if not fut.done():
                still.append((fut, req, slot, nb, key))
                continue
            a = fut.result()
            a.nbytes, a.key = nb, key
            now = self.now()
            for m in a.members:
                m.t_ready = now
            a.sv = B.csg_solve_begin(a.op, a.chi.data_ptr(), a.u.data_ptr(), a.nrhs, req.tol, req.restart,
                                     req.maxit, 0, a.stream.cuda_stream)
            self.active.append(a)
        self.pending = still

    # -- stepping --------------------------------------------------------------
    def _retire(self, a: _Active) -> None:
        rc, infos = B.csg_solve_end(a.sv, a.nrhs)
        now = self.now()
        u = a.u.cpu().numpy() if self.keep else None
        for q, m in enumerate(a.members):
            lo = q * a.R
            m.infos = infos[lo:lo + m.nrhs]
            if len(a.members) == 1:
                m.status = rc
            else:
                m.status = 0 if all(i["converged"] for i in m.infos) else B.CSG_ENOCONV
            m.t_done = now
            if self.keep:
                m.u = u[lo:lo + m.nrhs]
            if m is not a.req:
                self.done.append(m)
        if a.key is not None:
            self.cache[a.key] = (a.ws, a.op, a.nbytes)
        else:
            B.csg_operator_destroy(a.op)
            self.used -= a.nbytes
        a.op = None
        a.ws = None
        self.free_slots.append(a.slot)
        self.done.append(a.req)

    def step(self) -> bool:
        """Admit what fits, advance every solve whose last iteration landed.
        Returns True while work remains."""
        self._admit()
        self._start_ready()
        keep = []
        for a in self.active:
            r, done = B.csg_solve_poll(a.sv)
            if done:
                self._retire(a)
                continue
            if r == 1:
                B.csg_solve_step(a.sv)
            keep.append(a)
        self.active = keep
        return bool(self.queue or self.pending or self.active)

    def run(self, requests, realtime: bool = True) -> list:
        """Serve `requests` (arrival times in seconds from now when realtime)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        i = 0
        while True:
            t = self.now()
            while i < len(reqs) and (not realtime or reqs[i].arrival <= t):
                if not realtime:
                    reqs[i].arrival = t
                self.submit(reqs[i])
                i += 1
            busy = self.step()
            if i >= len(reqs) and not busy:
                break
        return self.done

    def close(self) -> None:
        self.pool.shutdown(wait=True)
        while self._evict_one():
            pass


def report(done: list, t_total: float) -> dict:
    lat = np.array([r.t_done - r.arrival for r in done]) * 1e3
    setup = np.array([r.t_ready - r.t_admit for r in done]) * 1e3
    solves = sum(r.nrhs for r in done)
    ok = all(r.status == 0 for r in done)
    return {
        "requests": len(done),
        "solves": solves,
        "seconds": t_total,
        "requests_per_s": len(done) / t_total if t_total > 0 else 0.0,
        "solves_per_s": solves / t_total if t_total > 0 else 0.0,
        "p50_latency_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_latency_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "p50_setup_ms": float(np.percentile(setup, 50)) if len(setup) else None,
        "all_converged": ok,
    }


def request_from_workload(w, rid: int, arrival: float = 0.0) -> Request:
    """Wrap a seeded workload (synth.workloads.Workload) as a request."""
    params = dict(w.params(), cycle_prec=w.cycle_prec)
    return Request(rid=rid, params=params, phi=w.phi, chi=w.chi, tol=w.tol, restart=w.restart,
                   maxit=w.maxit, arrival=arrival)
