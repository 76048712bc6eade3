"""GPU parity of the two ways a step's events are summed (direct device
atomics; bins per target tile summed in LDS), across tile sizes and with bins
too small for the traffic so that events spill into the atomic path: every
configuration gives the oracle's rasters and per-step integer inputs
exactly (the sum is over integers, so neither order nor route may change it).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14236_amd import workloads as W

pytestmark = pytest.mark.gpu

SPECS = {
    "c0a": lambda: W.c0(True),
    "brunel_ragged": lambda: W.brunel_lif(n=333, k=17, seed=7, delay=("uniform", 0.1, 2.0), dmax=25, nu_ext=300.0),
    "brunel_k1_const": lambda: W.brunel_lif(n=50, k=1, seed=2, delay=("const", 0.1, 0.0), dmax=1, nu_ext=300.0),
    "brunel_normal": lambda: W.brunel_lif(n=700, k=60, seed=11, delay=("normal", 1.5, 0.75), dmax=63, nu_ext=250.0),
    "mc_small": lambda: W.microcircuit(scale=0.05, k_scale=0.25, k_ext=3500, seed=3),
}

# (delivery, tile_neurons, bin_capacity); capacity 24 makes busy tiles spill
MODES = {
    "direct": ("direct", 0, 0),
    "binned_auto": ("binned", 0, 0),
    "binned_t256": ("binned", 256, 0),
    "binned_t512_spill": ("binned", 512, 24),
}

STEPS = 600
_oracle_cache = {}


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def snn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_14236_amd import snn as S
    S.lib()
    return S


def oracle_raster(name):
    if name not in _oracle_cache:
        o = O.OracleNet(SPECS[name](), O.FP32SO)
        o.simulate(STEPS)
        _oracle_cache[name] = (o.spikes(), o.get_state("V_m").astype(np.float32))
    return _oracle_cache[name]


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("name", list(SPECS))
def test_raster_bit_exact_every_mode(snn, name, mode):
    delivery, tile, cap = MODES[mode]
    g = snn.Net(SPECS[name](), delivery=delivery, tile_neurons=tile, bin_capacity=cap)
    g.simulate(STEPS)
    (os_, og, om), oV = oracle_raster(name)
    gs, gg, gm = g.spikes()
    assert np.array_equal(gs, os_) and np.array_equal(gg, og) and np.array_equal(gm, om)
    assert np.array_equal(g.get_state("V_m").astype(np.float32), oV)
    c = g.counters()
    assert c["delivery"] == (1 if delivery == "direct" else 2)
    if delivery == "binned":
        assert c["tile_neurons"] == (tile or c["tile_neurons"]) and c["tile_neurons"] >= 256
    assert c["overflow"] == 0


def test_spill_path_is_taken_and_exact(snn):
    """Tiny bins: most events spill; input per step still equals the oracle's."""
    spec = W.c0(True)
    steps = 80
    o = O.OracleNet(spec, O.FP32SO)
    rec = o.record_input(steps + 1)
    o.simulate(steps + 1)
    g = snn.Net(spec, delivery="binned", tile_neurons=256, bin_capacity=4)
    for n in range(steps):
        g.simulate(1)
        assert np.array_equal(g.get_input(0), rec[n + 1][:, 0]), n
    c = g.counters()
    assert c["spill_events"] > 0 and c["events"] > c["spill_events"]


@pytest.mark.parametrize("mode", ["direct", "binned_t256", "binned_t512_spill"])
def test_adex_replay_every_mode(snn, mode):
    """Two-port AdEx: the delivered input of both ports equals the oracle's
    replay of the GPU's own spikes, in every mode."""
    delivery, tile, cap = MODES[mode]
    spec = W.adex_balanced(n=2000, k=200, seed=5)
    g = snn.Net(spec, delivery=delivery, tile_neurons=tile, bin_capacity=cap)
    o = O.OracleNet(spec)
    steps = 150
    for n in range(steps):
        g.simulate(1)
        if n % 15 == 14:
            st, gid, m = g.spikes()
            ref = o.replay_input(st, gid, m, n + 1)
            for port in (0, 1):
                assert np.array_equal(g.get_input(port), ref[:, port]), (n, port)
    assert len(g.spikes()[0]) > 0


def test_modes_count_the_same_events(snn):
    spec = W.microcircuit(scale=0.05, k_scale=0.25, k_ext=3500, seed=3)
    a = snn.Net(spec, delivery="direct")
    b = snn.Net(spec, delivery="binned", tile_neurons=256)
    a.simulate(400)
    b.simulate(400)
    ca, cb = a.counters(), b.counters()
    for k in ("spikes", "events", "pairs"):
        assert ca[k] == cb[k], k
    assert ca["events"] > 0


def test_binned_tile_too_large_for_ports_is_rejected(snn):
    spec = W.adex_balanced(n=2000, k=200, seed=5)  # two ports: tiles of at most 2048 neurons
    with pytest.raises(snn.SnnError):
        snn.Net(spec, delivery="binned", tile_neurons=4096)


def _queue_batch():
    """Ten small Brunel instances of uneven size (a batch of at least 8
    instances of at most 32 tiles each: the delivery blocks share the items
    through the queue), delays up to 2 ms, strong drive."""
    return [W.brunel_lif(n=300 + 137 * i, k=10 + 3 * i, seed=40 + i, delay=("uniform", 0.1, 2.0), dmax=25,
                         nu_ext=250.0 + 10 * i) for i in range(10)]


@pytest.mark.parametrize("cap", [0, 24])
def test_batch_delivery_queue_bit_exact(snn, cap):
    """Binned delivery through the queue (and, with tiny bins, its spill path):
    every instance's raster and per-step input equal the oracle's."""
    g = _batch_parity(snn, _queue_batch(), 256, cap)
    assert g.counters()["delivery_queue"] == 1
    if cap:
        assert g.counters()["spill_events"] > 0


@pytest.mark.parametrize("tile,window", [(256, 1), (4096, 0)])
def test_batch_population_window(snn, tile, window):
    """LIF-only batch: where every tile overlaps at most 8 populations, the
    step kernels read the population tables from an LDS window; 4096-neuron
    tiles overlap up to 13 of the batch's 20 populations, and the network
    runs the kernel built for AdEx as well.  Both bit-exact."""
    g = _batch_parity(snn, _queue_batch(), tile, 0)
    assert g.counters()["tile_window"] == window


def _batch_parity(snn, specs, tile, cap):
    """Every instance's raster and its per-step input at two probe steps
    equal the oracle's; returns the network after 300 steps."""
    steps = 300
    g = snn.Net(specs, delivery="binned", tile_neurons=tile, bin_capacity=cap)
    probe = (99, 200)
    recs = []
    for sp in specs:
        o = O.OracleNet(sp, O.FP32SO)
        rec = o.record_input(steps + 1)
        o.simulate(steps + 1)
        st, gid, m = o.spikes()
        keep = st < steps
        recs.append(((st[keep], gid[keep], m[keep]), rec))
    done = 0
    for n in probe:  # the input of step n + 1 after n + 1 steps
        g.simulate(n + 1 - done)
        done = n + 1
        inp = g.get_input(0)
        for inst, (_, rec) in zip(g.instances, recs):
            assert np.array_equal(inp[inst["first"]:inst["first"] + inst["n"]], rec[n + 1][:, 0]), n
    g.simulate(steps - done)
    gs, gg, gm = g.spikes()
    total = 0
    for inst, ((os_, og, om), _) in zip(g.instances, recs):
        sel = (gg >= inst["first"]) & (gg < inst["first"] + inst["n"])
        assert np.array_equal(gs[sel], os_) and np.array_equal(gg[sel] - inst["first"], og)
        assert np.array_equal(gm[sel], om)
        total += len(os_)
    assert total > 1000
    assert g.counters()["overflow"] == 0
    return g


def test_single_network_keeps_the_strided_share(snn):
    g = snn.Net(W.brunel_lif(n=3000, k=100, seed=3, nu_ext=250.0), delivery="binned", tile_neurons=256)
    assert g.counters()["delivery_queue"] == 0


def _runs_net():
    """LIF-delta network whose groups are long (one delay, ~300 synapses per
    source) over few tiles: the binned delivery counts per tile run."""
    return W.brunel_lif(n=2500, k=300, seed=21, delay=("const", 0.8, 0.0), dmax=25, nu_ext=200.0)


@pytest.mark.parametrize("cap", [0, 16])
def test_tile_runs_bit_exact(snn, cap):
    """Delivery whose count pass reads the groups' tile runs (and, with tiny
    bins, its spill path): raster and per-step input equal the oracle's."""
    spec = _runs_net()
    steps = 200
    o = O.OracleNet(spec, O.FP32SO)
    rec = o.record_input(steps + 1)
    o.simulate(steps + 1)
    g = snn.Net(spec, delivery="binned", tile_neurons=256, bin_capacity=cap)
    assert g.counters()["tile_runs"] == 1
    for n in range(steps):
        g.simulate(1)
        if n % 20 == 19:
            assert np.array_equal(g.get_input(0), rec[n + 1][:, 0]), n
    gs, gg, gm = g.spikes()
    os_, og, om = o.spikes()
    keep = os_ < steps
    assert np.array_equal(gs, os_[keep]) and np.array_equal(gg, og[keep]) and np.array_equal(gm, om[keep])
    assert len(gs) > 500
    c = g.counters()
    assert c["overflow"] == 0
    if cap:
        assert c["spill_events"] > 0


def test_tile_runs_only_where_they_pay(snn):
    """Short runs (random targets over many tiles), AdEx neurons or direct
    delivery: no run index."""
    a = snn.Net(W.brunel_lif(n=3000, k=100, seed=3, delay=("uniform", 0.1, 2.0), nu_ext=250.0), delivery="binned",
                tile_neurons=256)
    b = snn.Net(W.adex_balanced(n=2000, k=200, seed=5), delivery="binned", tile_neurons=256)
    c = snn.Net(_runs_net(), delivery="direct")
    assert [x.counters()["tile_runs"] for x in (a, b, c)] == [0, 0, 0]
