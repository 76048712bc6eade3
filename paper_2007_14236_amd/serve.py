"""Serving simulation requests on one GPU through the library's request
server (the snn_server_* calls of include/snn.h).

A request is a network specification and a biological duration.  Requests
arrive over time; each is defined as a network (not built) and submitted at
its arrival time.  The server queues them in submission order and its
`slots` worker threads each take the first queued request whose memory need
fits what is left of the device-memory budget, build it, simulate it on the
network's own stream and release its memory the moment it is done, so
requests arriving while others run are admitted as slots and memory free up
and their work overlaps on the device.  Every device allocation of a served
network passes through the server, which holds the budget exactly.  Each
network runs the kernels it would run alone, so its raster does not depend
on what it was served with.  With one slot the same server serves the
requests one at a time in arrival order (the FIFO baseline).

Only the arrival clock, the trace and the report live here: admission,
building, stepping and release happen in the library.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import time
from dataclasses import dataclass, field

import numpy as np

from . import snn as S
from . import workloads as W


@dataclass
class Request:
    rid: int
    arrival_s: float
    family: str          # "microcircuit" or "adex"
    spec: dict
    steps: int


@dataclass
class Result:
    rid: int
    arrival_s: float
    start_s: float       # first taken by a slot (build included from here)
    finish_s: float
    status: int          # 0, or the snn_status of a failed request
    attempts: int        # builds tried (more than one after budget refusals)
    spikes: int
    events: int
    device_bytes: int    # most device memory the request held
    digest: str          # sha256 of the request's raster (step, gid, multiplicity)


@dataclass
class ServeReport:
    results: list = field(default_factory=list)
    makespan_s: float = 0.0
    peak_bytes: int = 0
    budget_bytes: int = 0

    def latencies(self) -> np.ndarray:
        return np.array([r.finish_s - r.arrival_s for r in self.results if r.status == 0])

    @property
    def events(self) -> int:
        return sum(r.events for r in self.results)


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
        out.append(Request(i, t, family, spec, W.steps_for(dur_ms, spec["dt"])))
    return out


_REC = np.dtype([("step", "<i8"), ("gid", "<i8"), ("mult", "<i8")])


def raster_records(step: np.ndarray, gid: np.ndarray, mult: np.ndarray) -> bytes:
    """(step, gid, multiplicity) records of a raster in (step, gid) order, the
    bytes its digest is taken over."""
    r = np.empty(len(step), dtype=_REC)
    r["step"], r["gid"], r["mult"] = step, gid, mult
    return r.tobytes()


def digest_of(net: "S.Net", steps: int) -> tuple:
    st, gid, m = net.spikes(0, steps)
    return len(st), hashlib.sha256(raster_records(st, gid, m)).hexdigest()


def run_alone(req: Request, **net_kw) -> str:
    """Digest of the request's raster simulated as the only network."""
    net = S.Net(req.spec, **net_kw)
    try:
        net.simulate(req.steps)
        return digest_of(net, req.steps)[1]
    finally:
        net.close()


class Server:
    """Arrival clock over the library's request server: `budget_bytes` of
    device memory, `slots` requests in flight at most."""

    def __init__(self, budget_bytes: int = 200 << 30, slots: int = 4, log=None, digest_ids=None,
                 keep_nets: bool = False, net_kw: dict | None = None):
        self.net_kw = dict(net_kw or {})  # configuration of every served network (e.g. delivery_blocks)
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.log = log
        self.digest_ids = digest_ids  # requests whose raster digest is taken (None: all)
        self.keep_nets = keep_nets    # hand the finished networks to the caller (report.nets)

    def serve(self, trace: list) -> ServeReport:
        """Submit each request at its arrival time (seconds after the start),
        collect the results as they finish."""
        L = S.lib()
        h = C.c_void_p()
        rc = L.snn_server_create(self.budget, self.slots, C.byref(h))
        if rc != 0:
            raise S.SnnError(f"server: {S.ERRORS.get(rc, rc)}")
        rep = ServeReport(budget_bytes=self.budget)
        rep.nets = {}
        pending = {}
        t0 = time.perf_counter()  # CLOCK_MONOTONIC, the clock of the server's job times
        i = 0
        try:
            while i < len(trace) or pending:
                now = time.perf_counter() - t0
                while i < len(trace) and trace[i].arrival_s <= now:
                    r = trace[i]
                    net = S.Net(r.spec, build=False, **self.net_kw)
                    ticket = C.c_uint64()
                    rc = L.snn_server_submit(h, net.h, r.steps, C.byref(ticket))
                    if rc != 0:
                        rep.results.append(Result(r.rid, r.arrival_s, now, now, rc, 0, 0, 0, 0, ""))
                        net.close()
                    else:
                        pending[ticket.value] = (r, net)
                    i += 1
                done = []
                for t in pending:
                    state = C.c_int32()
                    if L.snn_server_poll(h, t, C.byref(state)) == 0 and state.value in (S.JOB_DONE, S.JOB_FAILED):
                        done.append(t)
                for t in done:
                    r, net = pending.pop(t)
                    out = C.c_void_p()
                    info = S.JobInfo()
                    rc = L.snn_server_result(h, t, C.byref(out), C.byref(info))
                    spikes = events = 0
                    dg = ""
                    if rc == 0:
                        c = net.counters()
                        events = c["events"]
                        if self.digest_ids is None or r.rid in self.digest_ids:
                            spikes, dg = digest_of(net, r.steps)
                        else:
                            spikes = c["spikes"]
                    elif self.log:
                        self.log(f"request {r.rid} failed: {S.ERRORS.get(rc, rc)} {info.error.decode()}")
                    rep.results.append(Result(r.rid, r.arrival_s, info.t_start - t0, info.t_done - t0, rc,
                                              info.attempts, spikes, events, info.device_bytes_peak, dg))
                    if self.keep_nets and rc == 0:
                        rep.nets[r.rid] = net
                    else:
                        net.close()
                    if self.log:
                        self.log(f"request {r.rid} ({r.family}) done at {info.t_done - t0:.2f} s "
                                 f"(arrived {r.arrival_s:.2f} s, started {info.t_start - t0:.2f} s)")
                if i < len(trace):
                    wait = trace[i].arrival_s - (time.perf_counter() - t0)
                    time.sleep(min(max(wait, 0.0), 0.002))
                else:
                    time.sleep(0.001)
            st = S.ServerStats()
            L.snn_server_get_stats(h, C.byref(st))
            rep.peak_bytes = st.peak
        finally:
            L.snn_server_destroy(h)
            for r, net in pending.values():  # never finished: back to us with the server gone
                net.close()
        rep.results.sort(key=lambda x: x.rid)
        ok = [x for x in rep.results if x.status == 0]
        rep.makespan_s = (max(x.finish_s for x in ok) - min(x.arrival_s for x in trace)) if ok else 0.0
        return rep
