"""Pins of the oracle's devices (Sec. 2.1: spike generators and parrot
neurons): a generator's raster is its list of times on the step grid
(computed here independently, duplicates as multiplicity), a parrot repeats
exactly the spikes that reach it -- from generators through one-to-one
connections of a fixed delay, and from a Poisson drive of weight 1 (the
drawn counts) -- and the invalid set-ups are refused (no GPU)."""
import numpy as np
import pytest

from oracle import oracle as O

DT = 0.1


def device_spec(times, delay_ms=0.7, poisson_rate=0.0):
    n = len(times)
    pops = [dict(name="G", model="spike_generator", n=n, ports=1, params={}, spike_times=times),
            dict(name="R", model="parrot_neuron", n=n, ports=1, params={}),
            dict(name="Q", model="parrot_neuron", n=5, ports=1, params={})]
    projs = [dict(src="G", tgt="R", rule="one_to_one", weight=1.0, delay=("const", delay_ms, 0.0), port=0)]
    pois = [dict(tgt="Q", rate=poisson_rate, n_inputs=10, weight=1.0, port=0)] if poisson_rate else []
    return dict(name="devices", dt=DT, seed=3, dmax=20, populations=pops, projections=projs, poisson=pois)


def grid_steps(times):
    """step of each time: t/dt rounded half up, minus one (reported at t)"""
    return [int(np.floor(t / DT + 0.5)) - 1 for t in times]


def raster_of(net, first, n):
    st, gid, m = net.spikes()
    sel = (gid >= first) & (gid < first + n)
    return {(int(s), int(g) - first): int(k) for s, g, k in zip(st[sel], gid[sel], m[sel])}


def test_generator_emits_its_times():
    rng = np.random.default_rng(2)
    times = [np.round(rng.uniform(0.1, 30.0, size=rng.integers(0, 12)), 2).tolist() for _ in range(8)]
    times[0] = [0.1, 0.1, 0.1, 5.0, 5.04, 4.96]   # three in one step; rounding to the same step
    times[1] = []
    o = O.OracleNet(device_spec(times))
    o.simulate(400)
    got = raster_of(o, 0, len(times))
    expect = {}
    for g, ts in enumerate(times):
        for s in grid_steps(ts):
            expect[(s, g)] = expect.get((s, g), 0) + 1
    assert got == expect
    assert got[(0, 0)] == 3 and got[(49, 0)] == 3


def test_parrot_repeats_generator_spikes_after_the_delay():
    rng = np.random.default_rng(3)
    times = [np.round(rng.uniform(0.1, 20.0, size=6), 1).tolist() for _ in range(10)]
    o = O.OracleNet(device_spec(times, delay_ms=0.7))
    o.simulate(300)
    gen = raster_of(o, 0, 10)
    par = raster_of(o, 10, 10)
    assert par == {(s + 7, g): m for (s, g), m in gen.items()}


def test_parrot_repeats_poisson_counts():
    o = O.OracleNet(device_spec([[1.0]], poisson_rate=800.0))
    o.simulate(200)
    par = raster_of(o, 2, 5)
    expect = {}
    for n in range(200):
        for j in range(5):
            k = o.poisson_count(2 + j, n)
            if k:
                expect[(n, j)] = k
    assert par == expect and len(par) > 50


def test_device_errors():
    spec = device_spec([[1.0]])
    spec["projections"][0]["weight"] = 0.5
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
    spec = device_spec([[0.04]])  # rounds to step -1
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
    spec = device_spec([[1.0]])
    spec["populations"][1]["spike_times"] = [[2.0]]  # times on a parrot
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
