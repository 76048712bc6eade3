"""Batched serving of simulation requests on one GPU.

A request is a network specification and a biological duration.  Requests
arrive over time into one queue.  A pool of workers takes them: a free worker
packs the queued requests of the oldest request's model family that fit the
memory left in the budget (by the estimate below) and binned delivery's
resident capacity as independent instances of one network
(``snn_begin_instance``) and advances them together in the same kernels, on
the network's own stream; the workers' batches overlap on the device, so a
request that arrives while others run is admitted as soon as a worker and
memory are free.  Each request completes, with its own raster, when its batch
reaches its duration.  Instances draw exactly what they would draw alone, so
a request's result does not depend on what it was batched with.  With one
worker and ``max_batch=1`` the same loop serves the requests one at a time in
arrival order (the FIFO baseline).

Only host-side scheduling lives here: every simulation step runs in the
library's kernels through the C ABI.
"""
from __future__ import annotations

import hashlib
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import snn as S
from . import workloads as W

RECORD_SLOTS = 64  # selection records per neuron (Dmax + 1 at the largest Dmax)
# neuron-ports of one batch: 512 tiles of 4096 int64 sums, so that the tile
# blocks and the delivery blocks of a binned step are resident at once (three
# 53 KB blocks per CU); a larger batch runs its tile blocks in several rounds,
# each bounded by the ~100-substep RK45 spike steps of AdEx neurons
TILE_LIMIT = 512 * 4096


@dataclass
class Request:
    rid: int
    arrival_s: float
    family: str          # "microcircuit" or "adex": the model family a batch is formed from
    spec: dict
    steps: int
    est_bytes: int


@dataclass
class Result:
    rid: int
    arrival_s: float
    start_s: float       # when the batch holding it started (build included)
    finish_s: float
    batch_size: int
    spikes: int
    digest: str          # sha256 of the request's own raster (step, local gid, multiplicity)


@dataclass
class ServeReport:
    results: list = field(default_factory=list)
    batches: int = 0
    events: int = 0
    makespan_s: float = 0.0

    def latencies(self) -> np.ndarray:
        return np.array([r.finish_s - r.arrival_s for r in self.results])


def estimate_bytes(spec: dict) -> int:
    """Device memory of one instance: synapse words, neuron state, selection
    records, raster ring at one spike per neuron and step, input buffers,
    with a factor 2 of headroom."""
    n = W.total_neurons(spec)
    syn = W.count_synapses(spec)
    ports = max(p["ports"] for p in spec["populations"])
    per_neuron = 64 + 16 * RECORD_SLOTS + 4 * 1301 + 2 * 8 * ports
    return 2 * (4 * syn + n * per_neuron)


def request_trace(n: int, rate_hz: float = 20.0, key: int = 4) -> list:
    """Seeded arrival trace: exponential inter-arrival times at `rate_hz`
    (Philox key `key`), requests alternately a microcircuit stand-in at scale
    s ~ U[0.1, 1] (fixed connection probabilities) and a balanced AdEx network
    of N ~ U[10k, 200k] neurons with in-degree 1000, each for U[0.1, 2] s of
    biological time, request i seeded 1000 + i."""
    g = np.random.Generator(np.random.Philox(key=[key, 0]))
    t = 0.0
    out = []
    for i in range(n):
        t += float(g.exponential(1.0 / rate_hz))
        if i % 2 == 0:
            s = float(g.uniform(0.1, 1.0))
            spec = W.microcircuit(scale=s, seed=1000 + i)
            family = "microcircuit"
        else:
            nn = int(round(g.uniform(10_000, 200_000) / 5.0)) * 5
            spec = W.adex_balanced(n=nn, k=1000, seed=1000 + i)
            family = "adex"
        dur_ms = float(g.uniform(100.0, 2000.0))
        steps = W.steps_for(dur_ms, spec["dt"])
        out.append(Request(i, t, family, spec, steps, estimate_bytes(spec)))
    return out


_REC = np.dtype([("step", "<i8"), ("gid", "<i8"), ("mult", "<i8")])


def raster_records(step: np.ndarray, gid: np.ndarray, mult: np.ndarray) -> bytes:
    """(step, local gid, multiplicity) records of a raster in (step, gid) order,
    the bytes its digest is taken over (consecutive pieces hash as the whole)."""
    r = np.empty(len(step), dtype=_REC)
    r["step"], r["gid"], r["mult"] = step, gid, mult
    return r.tobytes()


def run_alone(req: Request) -> str:
    """Digest of the request's raster simulated as the only network."""
    net = S.Net(req.spec)
    net.simulate(req.steps)
    st, gid, m = net.spikes(0, req.steps)
    net.close()
    return hashlib.sha256(raster_records(st, gid, m)).hexdigest()


def neuron_ports(spec: dict) -> int:
    """Neurons times the port count rounded up to a power of two: the LDS
    accumulators the network takes in binned delivery."""
    ports = max(p["ports"] for p in spec["populations"])
    p2 = 1
    while p2 < ports:
        p2 *= 2
    return W.total_neurons(spec) * p2


class Server:
    """Batching scheduler over the C ABI.  `budget_bytes` bounds the estimated
    device memory of the batches in flight, `workers` how many run at once,
    `max_batch` the instances of one batch; a batch also stays within what
    binned delivery holds resident."""

    def __init__(self, budget_bytes: int = 200 << 30, max_batch: int = 64, workers: int = 4, log=None,
                 digest_ids=None):
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.workers = workers
        self.log = log
        self.digest_ids = digest_ids  # requests whose raster digest is taken (None: all)
        self.lock = threading.Lock()

    def _take_batch(self, queue: list, budget: int | None = None) -> list:
        budget = self.budget if budget is None else budget
        family = queue[0].family
        batch, used, nports = [], 0, 0
        for r in list(queue):
            if r.family != family:
                continue
            npr = neuron_ports(r.spec) if r.spec else 0
            if batch and (len(batch) >= self.max_batch or used + r.est_bytes > budget or nports + npr > TILE_LIMIT):
                break
            batch.append(r)
            used += r.est_bytes
            nports += npr
        for r in batch:
            queue.remove(r)
        return batch

    def _serve_batch(self, batch: list, t0: float, rep: ServeReport):
        start = time.perf_counter() - t0
        net = S.Net([r.spec for r in batch])
        firsts = np.array([inst["first"] for inst in net.instances], dtype=np.int64)
        pending = sorted(range(len(batch)), key=lambda j: batch[j].steps)
        digest = {j: hashlib.sha256() for j in range(len(batch))}
        count = {j: 0 for j in range(len(batch))}
        done = 0
        t_sim = t_ras = 0.0
        while pending:
            target = batch[pending[0]].steps
            ta = time.perf_counter()
            net.simulate(target - done)
            tb = time.perf_counter()
            t_sim += tb - ta
            # the segment's raster, grouped by instance (stable: (step, gid) order kept)
            st, gid, m = net.spikes(done, target)
            who = (np.searchsorted(firsts, gid.astype(np.int64), side="right") - 1).astype(np.int16)
            order = np.argsort(who, kind="stable")
            bounds = np.concatenate([[0], np.cumsum(np.bincount(who, minlength=len(batch)))])
            for j in pending:
                idx = order[bounds[j]:bounds[j + 1]]
                count[j] += int(idx.size)
                if self.digest_ids is None or batch[j].rid in self.digest_ids:
                    digest[j].update(raster_records(st[idx], gid[idx].astype(np.int64) - firsts[j], m[idx]))
            done = target
            t_ras += time.perf_counter() - tb
            now = time.perf_counter() - t0
            while pending and batch[pending[0]].steps == done:
                j = pending.pop(0)
                r = batch[j]
                res = Result(r.rid, r.arrival_s, start, now, len(batch), count[j], digest[j].hexdigest())
                with self.lock:
                    rep.results.append(res)
        ev = net.counters()["events"]
        net.close()
        with self.lock:
            rep.events += ev
            rep.batches += 1
        if self.log:
            self.log(f"batch of {len(batch)} {batch[0].family} requests done at {time.perf_counter() - t0:.2f} s "
                     f"(started {start:.2f} s; {done} steps simulated in {t_sim:.2f} s, rasters {t_ras:.2f} s)")

    def serve(self, trace: list) -> ServeReport:
        """Serve the trace in real time (arrivals released at their times)."""
        rep = ServeReport()
        errors: list = []
        state = {"next": 0, "queue": [], "in_flight": 0, "taken": 0}
        cv = threading.Condition(self.lock)
        t0 = time.perf_counter()

        def release(now):  # with the lock held: arrivals up to `now` into the queue
            while state["next"] < len(trace) and trace[state["next"]].arrival_s <= now:
                state["queue"].append(trace[state["next"]])
                state["next"] += 1

        def worker():
            try:
                while True:
                    with cv:
                        while True:
                            if errors or state["taken"] == len(trace):
                                return
                            now = time.perf_counter() - t0
                            release(now)
                            free = self.budget - state["in_flight"]
                            q = state["queue"]
                            if q and (q[0].est_bytes <= free or state["in_flight"] == 0):
                                batch = self._take_batch(q, max(free, 0))
                                used = sum(r.est_bytes for r in batch)
                                state["in_flight"] += used
                                state["taken"] += len(batch)
                                break
                            wait = (trace[state["next"]].arrival_s - now) if state["next"] < len(trace) else 0.05
                            cv.wait(timeout=min(max(wait, 0.0005), 0.05))
                    try:
                        self._serve_batch(batch, t0, rep)
                    finally:
                        with cv:
                            state["in_flight"] -= used
                            cv.notify_all()
            except Exception as e:  # reported by serve()
                with cv:
                    errors.append(e)
                    cv.notify_all()

        threads = [threading.Thread(target=worker) for _ in range(max(1, self.workers))]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        if errors:
            raise errors[0]
        rep.makespan_s = max(r.finish_s for r in rep.results) - min(r.arrival_s for r in trace)
        rep.results.sort(key=lambda r: r.rid)
        return rep
