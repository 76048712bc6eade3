"""Write the fp64 oracle's long-run statistics that the GPU statistics test
compares against (Sec. 3.1 protocol: rates and ISI coefficients of variation
per population, the first second discarded):

  mc_n10_stats.json     microcircuit stand-in at N/10 with the full in-degrees
                        and drive, 10 s of biological time
  adex_1e4_stats.json   balanced AdEx network of the C2 shape at 10^4
                        neurons (in-degree 1000, exponential conductances on
                        two ports, delays U[1, 2) ms), 5 s

Only the oracle (all host cores, same results as one thread) and the
seeded specification generators run here:

    python tests/golden/make_stats.py [mc|adex ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2007_14236_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SKIP_S = 1.0


def cases():
    return {
        "mc": ("mc_n10_stats.json", W.microcircuit(scale=0.1, k_scale=1.0), 10.0),
        "adex": ("adex_1e4_stats.json", W.adex_balanced(n=10_000, k=1000), 5.0),
    }


def population_stats(st, gid, ranges, dt_ms, steps, skip_steps):
    """Per population: rate (Hz) over [skip, steps), mean over neurons with at
    least 3 spikes there of the ISI coefficient of variation, spike count."""
    out = {}
    for name, (first, n) in ranges.items():
        sel = (gid >= first) & (gid < first + n) & (st >= skip_steps)
        s, g = st[sel].astype(np.int64), gid[sel].astype(np.int64)
        rate = s.size / (n * (steps - skip_steps) * dt_ms * 1e-3)
        order = np.lexsort((s, g))
        s, g = s[order], g[order]
        cvs = []
        for seg in np.split(s, np.flatnonzero(np.diff(g)) + 1):
            if seg.size >= 3:
                isi = np.diff(seg).astype(np.float64)
                cvs.append(isi.std() / isi.mean())
        out[name] = {"rate_hz": rate, "cv": float(np.mean(cvs)) if cvs else None, "spikes": int(s.size),
                     "neurons_with_cv": len(cvs)}
    return out


def run(key):
    fname, spec, t_s = cases()[key]
    steps = int(round(t_s * 1e3 / spec["dt"]))
    skip = int(round(SKIP_S * 1e3 / spec["dt"]))
    t0 = time.time()
    o = O.OracleNet(spec, O.FP64, openmp=True)
    o.simulate(steps)
    st, gid, _ = o.spikes()
    stats = population_stats(st, gid, W.population_ranges(spec), spec["dt"], steps, skip)
    rec = {"spec": spec["name"], "neurons": W.total_neurons(spec), "synapses": W.count_synapses(spec),
           "steps": steps, "skip_steps": skip, "dt_ms": spec["dt"], "mode": "fp64 oracle", "events": o.events,
           "populations": stats}
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"{fname}: {time.time() - t0:.0f} s, {len(st)} spikes", flush=True)


if __name__ == "__main__":
    for k in (sys.argv[1:] or list(cases())):
        run(k)
