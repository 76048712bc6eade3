"""Long-run statistics of the GPU path (fp32) against the fp64 oracle (the
Sec. 3.1 protocol: rates and ISI coefficients of variation per population,
the first second discarded).  After seconds of biological time the two
simulations have long left the same trajectory (fp32 against fp64), so the
statistics are compared: every population with at least 500 spikes in the
window must have its rate within 2 % and its mean ISI CV within 5 % of the
oracle's; quieter populations are held to 0.05 Hz.

Cases: the active Brunel net and a small microcircuit (oracle run here,
10 s); the microcircuit stand-in at N/10 with the full in-degrees and drive
(the per-neuron input statistics of the full network, 10 s) and a
C2-shaped balanced AdEx network of 10^4 neurons with in-degree 1000 (5 s),
whose oracle statistics were written by tests/golden/make_stats.py."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14236_amd import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_stats import population_stats  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MIN_SPIKES = 500


@pytest.fixture(scope="module")
def snn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_14236_amd import snn as S
    S.lib()
    return S


def compare(a, b):
    checked = 0
    for pop in b:
        ga, oa = a[pop], b[pop]
        if min(ga["spikes"], oa["spikes"]) >= MIN_SPIKES:
            assert abs(ga["rate_hz"] - oa["rate_hz"]) <= 0.02 * oa["rate_hz"], (pop, ga, oa)
            assert abs(ga["cv"] - oa["cv"]) <= 0.05 * oa["cv"], (pop, ga, oa)
            checked += 1
        else:
            assert abs(ga["rate_hz"] - oa["rate_hz"]) <= 0.05, (pop, ga, oa)
    return checked


def gpu_stats(S, spec, steps, skip):
    g = S.Net(spec)
    g.simulate(steps)
    st, gid, _ = g.spikes()
    g.close()
    return population_stats(st, gid, W.population_ranges(spec), spec["dt"], steps, skip)


@pytest.mark.parametrize("name", ["c0a", "mc_small"])
def test_rates_and_cv_small_networks(snn, name):
    print(f"\n[gpu-case] statistics {name}", flush=True)
    spec = {"c0a": lambda: W.c0(True),
            "mc_small": lambda: W.microcircuit(scale=0.05, k_scale=0.25, k_ext=3500, seed=3)}[name]()
    steps, skip = 100_000, 10_000
    a = gpu_stats(snn, spec, steps, skip)
    o = O.OracleNet(spec, O.FP64, openmp=True)
    o.simulate(steps)
    st, gid, _ = o.spikes()
    b = population_stats(st, gid, W.population_ranges(spec), spec["dt"], steps, skip)
    assert compare(a, b) >= 1


@pytest.mark.parametrize("name,make,expect", [
    ("mc_n10_stats.json", lambda: W.microcircuit(scale=0.1, k_scale=1.0), 6),
    ("adex_1e4_stats.json", lambda: W.adex_balanced(n=10_000, k=1000), 2)])
def test_rates_and_cv_representative_networks(snn, name, make, expect):
    print(f"\n[gpu-case] statistics {name}", flush=True)
    ref = json.load(open(os.path.join(GOLDEN, name)))
    spec = make()
    assert ref["spec"] == spec["name"] and ref["neurons"] == W.total_neurons(spec)
    a = gpu_stats(snn, spec, ref["steps"], ref["skip_steps"])
    assert compare(a, ref["populations"]) >= expect
