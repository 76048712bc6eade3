"""Pins of the oracle's nearest-neighbour STDP (Sec. 2.1, after Morrison et
al. 2008; the reading of its timing and fixed-point weight rule is stated in
oracle/snn_oracle.c at the plasticity step):

- one pre/post pair at a known time difference, both orders: the weight
  change is lambda W e^{-dt/tau_+} (potentiation) or alpha lambda W
  e^{-dt/tau_-} (depression), in fixed point, additive and multiplicative;
- nearest-neighbour pairing on three-spike patterns (only the nearest spike
  pairs; every post spike pairs with the latest arrival);
- an arrival and a post spike in the same step (the arrival comes first),
  and a post spike one step before an arrival;
- weights stay in [0, w_max]; a spike of multiplicity m pairs m times;
- dense brute force on a tiny recurrent network: replaying the oracle's own
  raster through the rule, event by event in plain Python, gives every
  delivered input and every final weight.
The pre and post neurons of the pair tests are spike generators (their
spike times are set; the plastic synapse onto a generator changes nothing
else).  Expected values come from the closed forms computed here with
Python's math.exp.  No GPU."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14236_amd import workloads as W

DT = 0.1


def pair_spec(pre, post, delay_ms=0.3, w0=50.0, **stdp):
    sd = dict(tau_plus=20.0, tau_minus=15.0, lambda_=0.05, alpha=0.8, mu_plus=0, mu_minus=0, w_max=100.0)
    sd.update(stdp)
    sd["lambda"] = sd.pop("lambda_")
    return dict(name="stdp_pair", dt=DT, seed=1, dmax=8, poisson=[],
                populations=[dict(name="PRE", model="spike_generator", n=1, ports=1, params={}, spike_times=[pre]),
                             dict(name="POST", model="spike_generator", n=1, ports=1, params={},
                                  spike_times=[post])],
                projections=[dict(src="PRE", tgt="POST", rule="one_to_one", weight=w0, delay=("const", delay_ms, 0.0),
                                  port=0, stdp=sd)]), sd


def run_pair(pre, post, steps=120, **kw):
    spec, sd = pair_spec(pre, post, **kw)
    o = O.OracleNet(spec)
    S = o.shift_of(1, 0)
    w0 = int(o.synapses()["wq"][0])
    o.simulate(steps)
    return int(o.synapses()["wq"][0]), w0, S, sd


def frac(scale, tau, d):
    """round(scale e^{-d dt / tau} 2^32), the rule's fixed-point factor"""
    return int(round(math.ldexp(scale * math.exp(-(d * DT) / tau), 32)))


def step_of(t):
    """emission step of a generator time"""
    return int(math.floor(t / DT + 0.5)) - 1


@pytest.mark.parametrize("mu", [0, 1])
def test_single_pair_potentiation(mu):
    pre, post = [1.0], [2.5]
    w, w0, S, sd = run_pair(pre, post, mu_plus=mu)
    a, k = step_of(1.0) + 3, step_of(2.5)
    assert k - a == 12
    Wq = int(round(math.ldexp(sd["w_max"], S)))
    B = Wq - w0 if mu else Wq
    assert w - w0 == (B * frac(sd["lambda"], sd["tau_plus"], k - a)) >> 32
    # the physical size of the change
    expect = sd["lambda"] * (sd["w_max"] - 50.0 if mu else sd["w_max"]) * math.exp(-(k - a) * DT / sd["tau_plus"])
    assert abs(math.ldexp(w - w0, -S) - expect) <= 2.0 ** -S + 1e-9 * expect


@pytest.mark.parametrize("mu", [0, 1])
def test_single_pair_depression(mu):
    pre, post = [2.0], [1.0]
    w, w0, S, sd = run_pair(pre, post, mu_minus=mu)
    a, k = step_of(2.0) + 3, step_of(1.0)
    assert a - k == 13
    Wq = int(round(math.ldexp(sd["w_max"], S)))
    B = w0 if mu else Wq
    assert w0 - w == (B * frac(sd["alpha"] * sd["lambda"], sd["tau_minus"], a - k)) >> 32
    expect = sd["alpha"] * sd["lambda"] * (50.0 if mu else sd["w_max"]) * math.exp(-(a - k) * DT / sd["tau_minus"])
    assert abs(math.ldexp(w0 - w, -S) - expect) <= 2.0 ** -S + 1e-9 * expect


def test_nearest_neighbour_pairing():
    # two arrivals before one post spike: only the nearest arrival pairs
    w, w0, S, sd = run_pair([1.0, 1.5], [3.0])
    Wq = int(round(math.ldexp(sd["w_max"], S)))
    a2, k = step_of(1.5) + 3, step_of(3.0)
    assert w - w0 == (Wq * frac(sd["lambda"], sd["tau_plus"], k - a2)) >> 32
    # two post spikes before one arrival: only the nearest post spike pairs
    w, w0, S, sd = run_pair([3.0], [1.0, 1.5])
    a, k2 = step_of(3.0) + 3, step_of(1.5)
    assert w0 - w == (Wq * frac(sd["alpha"] * sd["lambda"], sd["tau_minus"], a - k2)) >> 32
    # one arrival, two post spikes: each post spike pairs with that arrival (multiplicative)
    w, w0, S, sd = run_pair([1.0], [2.0, 3.0], mu_plus=1)
    a, k1, k2 = step_of(1.0) + 3, step_of(2.0), step_of(3.0)
    w1 = w0 + (((Wq - w0) * frac(sd["lambda"], sd["tau_plus"], k1 - a)) >> 32)
    w2 = w1 + (((Wq - w1) * frac(sd["lambda"], sd["tau_plus"], k2 - a)) >> 32)
    assert w == w2


def test_same_step_and_adjacent_steps():
    # the arrival comes first in its step: a post spike in that step pairs with it (difference 0)
    a = step_of(1.0) + 3
    w, w0, S, sd = run_pair([1.0], [(a + 1) * DT])
    Wq = int(round(math.ldexp(sd["w_max"], S)))
    assert w - w0 == (Wq * frac(sd["lambda"], sd["tau_plus"], 0)) >> 32
    # a post spike one step before the arrival depresses with difference 1
    w, w0, S, sd = run_pair([1.0], [a * DT])
    assert w0 - w == (Wq * frac(sd["alpha"] * sd["lambda"], sd["tau_minus"], 1)) >> 32


def test_bounds_and_multiplicity():
    # lambda = 1: an arrival with a post spike in the same step takes the weight to w_max
    w, w0, S, sd = run_pair([1.0], [1.3], lambda_=1.0, alpha=1.0)
    assert w == int(round(math.ldexp(sd["w_max"], S)))
    # ... and a post spike one step before an arrival takes it to 0
    w, w0, S, sd = run_pair([1.0], [1.2], lambda_=1.0, alpha=1.0)
    assert w == 0
    # an arrival of multiplicity 3 depresses three times (multiplicative)
    w, w0, S, sd = run_pair([2.0, 2.0, 2.0], [1.0], mu_minus=1)
    a, k = step_of(2.0) + 3, step_of(1.0)
    F = frac(sd["alpha"] * sd["lambda"], sd["tau_minus"], a - k)
    x = w0
    for _ in range(3):
        x -= (x * F) >> 32
    assert w == x


def test_dense_brute_force_tiny_network():
    """A tiny recurrent LIF network with plastic all-to-all E->E synapses and
    static ones onto it: the rule replayed in plain Python over the oracle's
    own raster, step by step (deliver with the current weights, potentiate for
    the post spikes of the step, depress for the arrivals of the next step),
    gives every recorded input and every final weight."""
    spec = W.brunel_lif(n=10, k=4, nu_ext=1000.0, seed=21, delay=("uniform", 0.1, 0.45), dmax=8)
    spec["projections"].append(dict(src="E", tgt="E", rule="all_to_all", weight=0.4, port=0,
                                    delay=("uniform", 0.1, 0.45),
                                    stdp=dict(tau_plus=5.0, tau_minus=7.0, alpha=1.1, mu_plus=1, mu_minus=0,
                                              w_max=2.0, **{"lambda": 0.2})))
    steps = 600
    o = O.OracleNet(spec)
    syn0 = o.synapses()
    rec = o.record_input(steps + 1)
    o.simulate(steps)
    st, gid, mult = o.spikes()
    syn1 = o.synapses()
    sd = dict(spec["projections"][-1]["stdp"])
    # which synapses are plastic: the last projection's (E -> E, all-to-all); in
    # the canonical order they follow the static synapses with equal keys, so
    # mark them by sorting each (src, delay, tgt, port, w0) tie static first
    ne = spec["populations"][0]["n"]
    S = o.shift_of(0, 0)
    w_static = int(round(math.ldexp(0.1, S)))  # E weight of the Brunel projections
    pl = np.zeros(len(syn0["src"]), bool)
    keys = {}
    for j in range(len(pl)):
        key = (syn0["src"][j], syn0["delay"][j], syn0["tgt"][j], syn0["wq"][j])
        keys.setdefault(key, []).append(j)
    w0p = int(round(math.ldexp(0.4, S)))
    n_all = ne * ne
    for key, js in keys.items():
        if key[3] == w0p and key[0] < ne and key[2] < ne:
            for j in js:
                pl[j] = True
    assert pl.sum() == n_all and w_static != w0p
    Wq = int(round(math.ldexp(sd["w_max"], S)))
    w = syn0["wq"].astype(np.int64).copy()
    last_pre = np.full(len(w), -1, np.int64)
    last_post = np.full(o.N, -1, np.int64)
    spikes = {}
    for s_, g_, m_ in zip(st.tolist(), gid.tolist(), mult.tolist()):
        spikes.setdefault(s_, []).append((g_, m_))
    by_src = {}
    for j in range(len(w)):
        by_src.setdefault(int(syn0["src"][j]), []).append(j)
    for n in range(steps):
        # delivery of the input of step n + 1 with the current weights
        inp = np.zeros(o.N, np.int64)
        arr = {}
        for j_src, js in by_src.items():
            for j in js:
                d = int(syn0["delay"][j])
                if n + 1 - d < 0:
                    continue
                for (g_, m_) in spikes.get(n + 1 - d, []):
                    if g_ == j_src:
                        inp[int(syn0["tgt"][j])] += m_ * int(w[j])
                        if pl[j]:
                            arr[j] = m_
        assert np.array_equal(inp, rec[n + 1][:, 0]), n
        for (t, m_) in spikes.get(n, []):  # potentiation
            for j in np.flatnonzero(pl & (syn0["tgt"] == t)):
                if last_pre[j] >= 0:
                    F = frac(sd["lambda"], sd["tau_plus"], n - last_pre[j])
                    for _ in range(m_):
                        w[j] = min(Wq, w[j] + (((Wq - w[j]) * F) >> 32))
            last_post[t] = n
        for j, m_ in arr.items():  # depression
            k = last_post[int(syn0["tgt"][j])]
            if k >= 0:
                F = frac(sd["alpha"] * sd["lambda"], sd["tau_minus"], n + 1 - k)
                for _ in range(m_):
                    w[j] = max(0, w[j] - ((Wq * F) >> 32))
            last_pre[j] = n + 1
    assert len(st) > 100
    assert np.array_equal(w, syn1["wq"])
    changed = np.flatnonzero(pl & (w != syn0["wq"]))
    assert len(changed) > 0.8 * n_all  # the rule acted on nearly every plastic synapse
    assert np.array_equal(w[~pl], syn0["wq"][~pl])  # static synapses unchanged


def test_bad_parameters_refused():
    for bad in (dict(lambda_=1.5), dict(alpha=2.0, lambda_=0.9), dict(w_max=-1.0), dict(mu_plus=2),
                dict(w_max=10.0)):  # w0 = 50 above w_max
        spec, _ = pair_spec([1.0], [2.0], **bad)
        with pytest.raises(RuntimeError):
            O.OracleNet(spec)
