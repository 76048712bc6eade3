"""Autotuner of the step kernel's shapes for one network.

The shapes that do not change results (every sum is over integers) but do
change speed are chosen by timing: direct or binned delivery, the tile size of
binned delivery (neurons per tile block, which is also the work-queue size of
the RK45 update) and the number of blocks that deliver the delays >= 2.  Each
candidate is built as a fresh copy of the network, run for a warm-up and then
timed over a short window; the fastest wins.  Results are kept per network
signature for the life of the process (and in a JSON file if one is given).
"""
from __future__ import annotations

import json
import os
import time

from . import snn as S
from . import workloads as W


def signature(spec) -> str:
    specs = list(spec) if isinstance(spec, (list, tuple)) else [spec]
    n = sum(W.total_neurons(sp) for sp in specs)
    syn = sum(W.count_synapses(sp) for sp in specs)
    models = sorted({p["model"] for sp in specs for p in sp["populations"]})
    ports = max(p["ports"] for sp in specs for p in sp["populations"])
    return f"n={n};syn={syn};ports={ports};models={','.join(models)};instances={len(specs)}"


def candidates(spec) -> list:
    """Configurations to try: direct delivery at three delivery-grid sizes,
    binned delivery at every tile size the port count allows (at most 1024
    tiles) and, for the library's tile size, three grid sizes."""
    specs = list(spec) if isinstance(spec, (list, tuple)) else [spec]
    n = sum(W.total_neurons(sp) for sp in specs)
    ports = max(p["ports"] for sp in specs for p in sp["populations"])
    p2 = 1
    while p2 < ports:
        p2 *= 2
    tmax = 4096 // p2
    out = [dict(delivery="direct", delivery_blocks=b) for b in (0, 128, 512)]
    t = 256
    while t <= tmax:
        if (n + t - 1) // t <= 1024:
            out.append(dict(delivery="binned", tile_neurons=t))
        t *= 2
    if (n + tmax - 1) // tmax <= 1024:
        out += [dict(delivery="binned", tile_neurons=tmax, delivery_blocks=b) for b in (128, 512)]
    return out


_cache: dict = {}


def tune(spec, steps: int = 300, warmup: int = 200, cache_path: str | None = None, log=None):
    """Best configuration for `spec` (a specification or a list of them) and
    the table of timings (microseconds per step, per candidate)."""
    import torch
    key = signature(spec)
    if cache_path and os.path.exists(cache_path):
        _cache.update(json.load(open(cache_path)))
    if key in _cache:
        return _cache[key]["best"], _cache[key]["table"]
    table = []
    for cfg in candidates(spec):
        try:
            net = S.Net(spec, record=False, **cfg)
        except S.SnnError:
            continue
        net.simulate(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.simulate(steps)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) / steps * 1e6
        c = net.counters()
        net.close()
        table.append(dict(cfg, us_per_step=round(us, 3), tile=c["tile_neurons"], blocks=c["delivery_blocks"]))
        if log:
            log(f"autotune {cfg}: {us:.2f} us per step")
    best = min(table, key=lambda r: r["us_per_step"])
    best_cfg = {k: best[k] for k in ("delivery", "tile_neurons", "delivery_blocks") if k in best}
    _cache[key] = {"best": best_cfg, "table": table}
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(_cache, f, indent=1)
    return best_cfg, table
