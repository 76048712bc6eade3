"""Pins of the oracle's spike delivery: brute force with a dense
(target, port, source, delay) weight tensor on tiny nets, the delivered-events
invariant, and agreement of the simulator's own per-step input with the
plain replay definition (no GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14236_amd import workloads as W


def tiny_net(seed=3, n=48, k=9, dmax=8, delay=("uniform", 0.1, 0.8)):
    spec = W.brunel_lif(n=n, k=k, seed=seed, delay=delay, dmax=dmax, nu_ext=400.0, c_ext=80)
    return spec, O.OracleNet(spec, O.FP64)


def dense_tensor(net, dmax):
    syn = net.synapses()
    Wt = np.zeros((net.N, net.P, net.N, dmax + 1), dtype=np.int64)
    np.add.at(Wt, (syn["tgt"], syn["port"], syn["src"], syn["delay"]), syn["wq"])
    return Wt


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_replay_equals_dense_brute_force(seed):
    dmax = 8
    spec, net = tiny_net(seed=seed, dmax=dmax)
    Wt = dense_tensor(net, dmax)
    rng = np.random.default_rng(seed)
    steps = 30
    # random spike history with multiplicities 1..3
    S = (rng.random((steps, net.N)) < 0.2) * rng.integers(1, 4, size=(steps, net.N))
    st, gid = np.nonzero(S)
    mult = S[st, gid]
    for target in range(0, steps + dmax):
        got = net.replay_input(st, gid, mult, target)
        ref = np.zeros((net.N, net.P), dtype=np.int64)
        for d in range(1, dmax + 1):
            nf = target - d
            if 0 <= nf < steps:
                ref += np.einsum("tpsd,s->tp", Wt[:, :, :, d:d + 1], S[nf].astype(np.int64))
        assert np.array_equal(got, ref), target


def test_events_invariant():
    """With one weight everywhere, the summed input equals the weight times the
    number of delivered events, i.e. the summed out-degree of each matured
    (source, delay) pair times the spike multiplicity."""
    dmax = 8
    spec = W.brunel_lif(n=60, k=12, seed=5, g=-1.0, delay=("uniform", 0.1, 0.8), dmax=dmax)
    net = O.OracleNet(spec)
    syn = net.synapses()
    wq = int(syn["wq"][0])
    assert np.all(syn["wq"] == wq)
    outdeg = np.zeros((net.N, dmax + 1), dtype=np.int64)
    np.add.at(outdeg, (syn["src"], syn["delay"]), 1)
    rng = np.random.default_rng(0)
    S = (rng.random((20, net.N)) < 0.3) * rng.integers(1, 3, size=(20, net.N))
    st, gid = np.nonzero(S)
    mult = S[st, gid]
    total = 0
    for target in range(1, 20 + dmax):
        got = net.replay_input(st, gid, mult, target)
        events = sum(int(S[target - d] @ outdeg[:, d]) for d in range(1, dmax + 1) if 0 <= target - d < 20)
        assert got.sum() == wq * events
        total += events
    # over the whole window every spike reaches every one of its synapses once
    assert total == int(S.sum(axis=0) @ outdeg.sum(axis=1))


@pytest.mark.parametrize("mode", [O.FP64, O.FP32SO])
def test_simulation_input_equals_replay_of_own_raster(mode):
    spec = W.c0(active=True)
    net = O.OracleNet(spec, mode)
    steps = 300
    rec = net.record_input(steps)
    net.simulate(steps)
    st, gid, m = net.spikes()
    assert len(st) > 100
    for n in list(range(0, steps, 17)) + [steps - 1]:
        assert np.array_equal(rec[n], net.replay_input(st, gid, m, n)), n


def test_raster_sorted_and_refractory_respected():
    spec = W.c0(active=True)
    net = O.OracleNet(spec, O.FP32SO)
    net.simulate(1000)
    st, gid, m = net.spikes()
    key = st.astype(np.int64) * 10**6 + gid
    assert np.all(np.diff(key) > 0)
    assert np.all(m == 1)
    # no neuron fires twice within t_ref + dt (2 ms = 20 steps -> ISI >= 21)
    order = np.lexsort((st, gid))
    g2, s2 = gid[order], st[order].astype(np.int64)
    same = g2[1:] == g2[:-1]
    assert np.all(np.diff(s2)[same] >= 21)


def test_c0_literal_is_subthreshold_and_c0a_active():
    """With 20 Hz x 80 inputs of 0.1 mV the mean drive is 3.2 mV against a
    20 mV threshold: the literal C0 network stays silent; at 250 Hz it fires."""
    n0 = O.OracleNet(W.c0(False), O.FP32SO)
    n0.simulate(1000)
    assert len(n0.spikes()[0]) == 0
    n1 = O.OracleNet(W.c0(True), O.FP32SO)
    n1.simulate(1000)
    rate = len(n1.spikes()[0]) / 1000 / 0.1
    assert 20.0 < rate < 200.0


def test_openmp_build_gives_the_same_results():
    """The oracle built with OpenMP (the all-core CPU baseline) simulates
    exactly what the plain build simulates: rasters, potentials and event
    counts of a small microcircuit and an AdEx net."""
    from paper_2007_14236_amd import workloads as W
    for spec, steps in ((W.c0(active=True), 300), (W.microcircuit(scale=0.05, k_scale=0.5), 300), (W.adex_balanced(n=400, k=40), 600)):
        a = O.OracleNet(spec, O.FP64)
        b = O.OracleNet(spec, O.FP64, openmp=True)
        a.simulate(steps)
        b.simulate(steps)
        for x, y in zip(a.spikes(), b.spikes()):
            assert np.array_equal(x, y)
        assert len(a.spikes()[0]) > 0
        assert np.array_equal(a.get_state("V_m"), b.get_state("V_m"))
        assert a.events == b.events
