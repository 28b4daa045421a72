"""Request loop serving many OkMC replicas on one device (continuous batching).

A replica is one defect population on its own periodic grid (its own size and
defect count) with a resident state on the device: owner map, footprints,
half spectrum, FP64 stress and energies.  Requests arrive over time and either
move one defect of a replica by a whole-voxel hop (the incremental update of
App. B, most requests) or re-solve the replica's current defect list.  Every
request ends with the replica's interaction energies in host memory.

The loop
  * keeps one FIFO per replica and runs a replica's requests one after the
    other (an OkMC replica needs the energies of its last event before it can
    pick the next one);
  * admits a replica's state against the context's HBM budget; when the budget
    is full it evicts the least recently used idle replica, whose state is
    rebuilt by a solve of its current defect list when it runs again;
  * runs up to ``slots`` requests (or batches) of different replicas at the
    same time, each on a stream of its own, so their kernels overlap on the
    device, and hands a slot to the next ready work as soon as its work
    completes (a slot is refilled immediately; requests are not drained in
    rounds);
  * merges ready whole-voxel hops of replicas of one shape (grid size and
    precision) into one batch, up to ``batch`` of them and ``batch_voxels``
    grid voxels in all, which ``ec_update_batch`` runs as one launch per pass,
    replayed from a HIP graph captured once per (shape, batch size, slot);
  * times every request from its arrival to the completion of the copy of its
    energies to host memory, using device events, and splits that latency at
    the request's dispatch (the wait for a slot or for its replica's previous
    request, then the service on the device).

All device work goes through the C ABI in ``libec.so``; this module only
schedules it.  ``run_plain`` is the reference it is compared with: the same
requests one at a time through the synchronous calls, nothing overlapped.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import ec, inputs


@dataclasses.dataclass
class Request:
    rid: int
    replica: int
    t: float  # arrival time, seconds after the start of the trace
    op: str  # "update" or "solve"
    idx: int = -1  # moved defect (updates)
    hop: tuple = (0, 0, 0)  # whole-voxel displacement (updates)


def serving_requests(replicas, nreq: int, rate_per_s: float = 2000.0, update_frac: float = 0.9):
    """Poisson request trace over ``replicas`` (list of (problem, defects))."""
    t, rep, is_update, draw, hop = inputs.serving_trace(len(replicas), nreq, rate_per_s, update_frac)
    out = []
    for k in range(nreq):
        r = int(rep[k])
        ndef = len(replicas[r][1])
        if is_update[k]:
            out.append(Request(k, r, float(t[k]), "update", int(draw[k] * ndef), tuple(int(v) for v in inputs.HOPS111[hop[k]])))
        else:
            out.append(Request(k, r, float(t[k]), "solve"))
    return out


def moved_defect(defs: np.ndarray, req: Request, h: float) -> np.ndarray:
    """The defect record of ``req`` after its hop (centre shifted by hop * h)."""
    d = defs[req.idx].copy()
    d["c"] = d["c"] + np.asarray(req.hop, dtype=np.float64) * h
    return d


class _Replica:
    def __init__(self, torch, k: int, problem, defects):
        self.k = k
        self.problem = problem
        self.defs = ec.as_defects(defects).copy()
        self.state = None
        self.solved = False
        self.queue = collections.deque()
        self.busy = False
        self.last_used = -1.0
        self.E_dev = None
        self.energies_ok = False
        self.E_host = torch.empty(max(1, len(self.defs)), dtype=torch.float64, pin_memory=True)

    @property
    def shape(self):
        return (self.problem.n, self.problem.prec)


class _Slot:
    def __init__(self, torch):
        self.stream = torch.cuda.Stream()
        self.done = torch.cuda.Event(enable_timing=True)
        self.reqs = []


@dataclasses.dataclass
class ServeStats:
    completed: int
    wall_s: float
    throughput: float  # requests per second
    p50_ms: float
    p99_ms: float
    mean_ms: float
    admissions: int
    evictions: int
    latency_ms: np.ndarray
    results: dict  # rid -> energies (when kept)
    batches: int = 0  # launches that carried two or more hops
    wait_ms: np.ndarray = None  # arrival -> dispatch on the host, per request (arrival order)
    grid: np.ndarray = None  # grid size of each request's replica (arrival order)

    def by_grid(self):
        """Latency percentiles per replica grid size: {n: {requests, p50_ms,
        p99_ms, wait_p99_ms, service_p50_ms}} (service = latency - wait)."""
        out = {}
        for n in sorted(set(self.grid.tolist())):
            m = self.grid == n
            lat, wait = self.latency_ms[m], self.wait_ms[m]
            out[int(n)] = {"requests": int(m.sum()), "p50_ms": round(float(np.median(lat)), 4),
                           "p99_ms": round(float(np.quantile(lat, 0.99)), 4),
                           "wait_p99_ms": round(float(np.quantile(wait, 0.99)), 4),
                           "service_p50_ms": round(float(np.median(lat - wait)), 4)}
        return out


class Server:
    """Continuous-batching request loop over replicas sharing one context."""

    def __init__(self, ctx: ec.Context, replicas, slots: int = 4, keep_results: bool = False, batch: int = 8,
                 batch_voxels: int = 8_000_000, graphs: bool = True):
        import torch

        self.torch = torch
        self.ctx = ctx
        self.reps = [_Replica(torch, k, p, d) for k, (p, d) in enumerate(replicas)]
        self.keep = keep_results
        self.slots = [_Slot(torch) for _ in range(max(1, slots))]
        self.batch = max(1, min(batch, 16))
        self.batch_voxels = batch_voxels
        self.graphs = graphs
        self.admissions = 0
        self.evictions = 0
        self.batches = 0  # batched launches (two or more hops)

    # -------------------------------------------------------------- admission
    def _evict_one(self, keep: _Replica) -> bool:
        """Release the least recently used idle replica other than ``keep``."""
        idle = [r for r in self.reps if r.state is not None and not r.busy and r is not keep]
        if not idle:
            return False
        victim = min(idle, key=lambda r: r.last_used)
        victim.state.close()
        victim.state = None
        victim.solved = False
        victim.E_dev = None
        self.evictions += 1
        return True

    def _admit(self, rep: _Replica, clock: float) -> bool:
        """Create ``rep``'s state, evicting idle replicas while the budget is
        short.  False if nothing can be evicted now (retry later)."""
        while True:
            try:
                rep.state = ec.State(self.ctx, rep.problem)
            except ec.EcError as e:
                if e.status != ec.EC_ERR_ADMIT or not self._evict_one(rep):
                    if e.status != ec.EC_ERR_ADMIT:
                        raise
                    return False
                continue
            rep.E_dev = self.torch.empty(len(rep.defs), dtype=self.torch.float64, device="cuda")
            rep.solved = False
            self.admissions += 1
            return True

    def warm(self):
        """Admit and solve every replica once (builds the Green windows)."""
        for rep in self.reps:
            if rep.state is None and not self._admit(rep, 0.0):
                continue
            rep.state.solve(rep.defs)
            rep.state.energies()
            rep.solved = rep.energies_ok = True
        self.torch.cuda.synchronize()

    # --------------------------------------------------------------- dispatch
    def _enqueue_work(self, rep: _Replica, req: Request, s):
        st = rep.state
        if not rep.solved:  # rebuilt after admission: fields, then self terms
            st.solve(rep.defs, stream=s)
            rep.solved = True
            rep.energies_ok = False
        if not rep.energies_ok:  # before a move, so that a refusal cannot come after it
            st.energies(stream=s, out=rep.E_dev)
            rep.energies_ok = True
        if req.op == "update":
            d = moved_defect(rep.defs, req, rep.problem.h)
            st.update(req.idx, d, stream=s, out=rep.E_dev)
            rep.defs[req.idx] = d
        else:
            st.solve(rep.defs, stream=s)
            st.energies(stream=s, out=rep.E_dev)

    def _dispatch(self, slot: _Slot, rep: _Replica, req: Request) -> bool:
        """Enqueue ``req`` on ``slot``.  A call refused by the budget leaves the
        state as it was; idle replicas are then evicted and the request is
        enqueued again.  False if the budget cannot be met now."""
        torch = self.torch
        s = slot.stream
        while True:
            try:
                self._enqueue_work(rep, req, s)
                break
            except ec.EcError as e:
                if e.status != ec.EC_ERR_ADMIT:
                    raise
                if not self._evict_one(rep):
                    return False
        with torch.cuda.stream(s):
            rep.E_host[: len(rep.defs)].copy_(rep.E_dev, non_blocking=True)
        slot.done.record(s)
        slot.reqs = [req]
        rep.busy = True
        return True

    def _hop_ready(self, rep: _Replica) -> bool:
        """Whether ``rep``'s head request can join a batch of hops."""
        return (rep.queue and rep.queue[0].op == "update" and rep.state is not None and rep.solved
                and rep.energies_ok and not rep.busy)

    def _dispatch_batch(self, slot: _Slot, group) -> None:
        """Enqueue the head hops of the replicas in ``group`` (one shape) as one
        batch on ``slot`` (ec_update_batch: one launch per pass, from a HIP
        graph)."""
        torch = self.torch
        s = slot.stream
        reqs = [rep.queue[0] for rep in group]
        moved = [moved_defect(rep.defs, rq, rep.problem.h) for rep, rq in zip(group, reqs)]
        ec.update_batch([rep.state for rep in group], [rq.idx for rq in reqs],
                        np.concatenate([m.reshape(1) for m in moved]), stream=s,
                        outs=[rep.E_dev for rep in group], use_graph=self.graphs)
        with torch.cuda.stream(s):
            for rep, rq, m in zip(group, reqs, moved):
                rep.defs[rq.idx] = m
                rep.E_host[: len(rep.defs)].copy_(rep.E_dev, non_blocking=True)
        slot.done.record(s)
        slot.reqs = reqs
        for rep in group:
            rep.queue.popleft()
            rep.busy = True
        if len(group) > 1:
            self.batches += 1

    @staticmethod
    def _stalled(busy, rep: _Replica):
        """A replica that does not fit even with every other one evicted and
        nothing running would wait forever."""
        if not busy:
            raise ec.EcError(ec.EC_ERR_ADMIT, f"replica {rep.k} does not fit in the HBM budget on its own")

    # -------------------------------------------------------------------- run
    def run(self, requests, realtime: bool = True) -> ServeStats:
        """Serve ``requests`` (sorted by arrival).  ``realtime``: requests become
        visible at their arrival times; otherwise all are queued at once."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r.t)
        n = len(reqs)
        ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ref.record()
        ref.synchronize()
        t0 = time.perf_counter()
        arrive = np.array([r.t if realtime else 0.0 for r in reqs])
        done_t = np.zeros(n)
        disp_t = np.zeros(n)
        results = {}
        order = {r.rid: i for i, r in enumerate(reqs)}
        ptr = 0
        completed = 0
        free = list(self.slots)
        busy = []
        waiting = collections.deque()  # replicas with queued work, in order of their head request
        batches0 = self.batches
        while completed < n:
            now = time.perf_counter() - t0
            while ptr < n and arrive[ptr] <= now:
                rq = reqs[ptr]
                rep = self.reps[rq.replica]
                if not rep.queue and not rep.busy:
                    waiting.append(rep)
                rep.queue.append(rq)
                ptr += 1
            # fill free slots with the oldest ready requests; a ready hop takes
            # the ready hops of other replicas of its shape along in one batch
            if free and waiting:
                for _ in range(len(waiting)):
                    if not free or not waiting:  # a batch may take several waiting replicas
                        break
                    rep = waiting.popleft()
                    if rep.busy or not rep.queue:
                        continue
                    if self.batch > 1 and self._hop_ready(rep):
                        group, vox = [rep], rep.problem.n ** 3
                        for other in list(waiting):
                            if len(group) >= self.batch:
                                break
                            if (other is not rep and other.shape == rep.shape and self._hop_ready(other)
                                    and vox + other.problem.n ** 3 <= self.batch_voxels):
                                group.append(other)
                                vox += other.problem.n ** 3
                        for other in group[1:]:
                            waiting.remove(other)
                        slot = free.pop()
                        for g in group:
                            g.last_used = now
                            disp_t[order[g.queue[0].rid]] = now
                        self._dispatch_batch(slot, group)
                        busy.append(slot)
                        continue
                    if rep.state is None and not self._admit(rep, now):
                        self._stalled(busy, rep)
                        waiting.append(rep)
                        continue
                    slot = free.pop()
                    rep.last_used = now
                    if self._dispatch(slot, rep, rep.queue[0]):
                        disp_t[order[rep.queue[0].rid]] = now
                        rep.queue.popleft()
                        busy.append(slot)
                    else:  # over budget until running requests finish
                        self._stalled(busy, rep)
                        free.append(slot)
                        waiting.append(rep)
            # retire finished requests
            still = []
            for slot in busy:
                if slot.done.query():
                    t_done = ref.elapsed_time(slot.done) * 1e-3
                    for rq in slot.reqs:
                        rep = self.reps[rq.replica]
                        done_t[order[rq.rid]] = t_done
                        if self.keep:
                            results[rq.rid] = rep.E_host[: len(rep.defs)].numpy().copy()
                        rep.busy = False
                        rep.last_used = now
                        if rep.queue:
                            waiting.append(rep)
                        completed += 1
                    slot.reqs = []
                    free.append(slot)
                else:
                    still.append(slot)
            busy = still
        wall = max(done_t.max(), 1e-9) if n else 0.0
        lat = (done_t - arrive) * 1e3
        return ServeStats(
            completed=n,
            wall_s=wall,
            throughput=n / wall if n else 0.0,
            p50_ms=float(np.median(lat)) if n else 0.0,
            p99_ms=float(np.quantile(lat, 0.99)) if n else 0.0,
            mean_ms=float(lat.mean()) if n else 0.0,
            admissions=self.admissions,
            evictions=self.evictions,
            latency_ms=lat,
            results=results,
            batches=self.batches - batches0,
            wait_ms=np.maximum(disp_t - arrive, 0.0) * 1e3,
            grid=np.array([self.reps[r.replica].problem.n for r in reqs]),
        )

    def close(self):
        for rep in self.reps:
            if rep.state is not None:
                rep.state.close()
                rep.state = None


def run_plain(ctx: ec.Context, replicas, requests, keep_results: bool = False):
    """The same requests one at a time through the synchronous calls (host
    energies after each), with every replica resident: (requests/s, per-request
    service times in ms, results)."""
    reps = [(p, ec.as_defects(d).copy()) for p, d in replicas]
    states = []
    for p, d in reps:
        st = ec.State(ctx, p)
        st.solve(d)
        st.energies()
        states.append(st)
    svc = []
    results = {}
    t_start = time.perf_counter()
    for rq in requests:
        t = time.perf_counter()
        p, defs = reps[rq.replica]
        st = states[rq.replica]
        if rq.op == "update":
            d = moved_defect(defs, rq, p.h)
            E = st.update(rq.idx, d)
            defs[rq.idx] = d
        else:
            st.solve(defs)
            E = st.energies()
        svc.append((time.perf_counter() - t) * 1e3)
        if keep_results:
            results[rq.rid] = E.copy()
    wall = time.perf_counter() - t_start
    for st in states:
        st.close()
    return len(requests) / wall, np.array(svc), results
