"""GPU parity of the connection rules (fixed in-degree, fixed out-degree,
all-to-all, one-to-one, fixed total number) through the C ABI: the device-
built CSR equals the oracle's canonical table bit for bit (alone, inside a
batch of instances, and at 20,000 neurons), and a network using every rule
gives the oracle's raster bit for bit in both delivery modes."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

from test_oracle_rules import rules_spec

pytestmark = pytest.mark.gpu


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


def canonical(syn, offset=0):
    return {k: (syn[k].astype(np.int64) - (offset if k in ("src", "tgt") else 0)) for k in
            ("src", "delay", "tgt", "port", "wq")}


def assert_same(a, b):
    for k in ("src", "delay", "tgt", "port", "wq"):
        assert a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k]), k


def driven(spec):
    for p in spec["populations"]:
        p["I_e"] = 600.0
        p["V0"] = np.linspace(0.0, 19.0, p["n"])
    return spec


@pytest.mark.parametrize("delivery", ["direct", "binned"])
def test_rules_csr_bit_exact(snn, delivery):
    spec = rules_spec()
    g = snn.Net(spec, delivery=delivery, tile_neurons=256 if delivery == "binned" else 0)
    assert_same(canonical(g.synapses()), canonical(O.OracleNet(spec).synapses()))


def test_rules_csr_bit_exact_20k(snn):
    spec = rules_spec(seed=9, sizes=(8000, 6000, 6000), total=400_000, outdeg=30)
    # all-to-all from a 50-neuron population (B -> C would be 3.6e7 synapses)
    spec["populations"].append(dict(name="D", model="lif_delta", n=50, ports=1,
                                    params=dict(spec["populations"][0]["params"]), V0=None, I_e=0.0))
    spec["projections"][2]["src"] = "D"
    g = snn.Net(spec)
    o = O.OracleNet(spec)
    assert_same(canonical(g.synapses()), canonical(o.synapses()))
    assert g.counters()["n_synapses"] == o.synapses()["src"].size


def test_rules_inside_a_batch(snn):
    specs = [rules_spec(seed=5), rules_spec(seed=6, sizes=(30, 20, 20), total=90, outdeg=4)]
    g = snn.Net(specs)
    syn = g.synapses()
    first = 0
    for sp in specs:
        n = sum(p["n"] for p in sp["populations"])
        sel = (syn["src"] >= first) & (syn["src"] < first + n)
        part = {k: v[sel] for k, v in syn.items()}
        assert_same(canonical(part, first), canonical(O.OracleNet(sp).synapses()))
        first += n


@pytest.mark.parametrize("delivery", ["direct", "binned"])
def test_rules_raster_bit_exact(snn, delivery):
    spec = driven(rules_spec())
    steps = 400
    g = snn.Net(spec, delivery=delivery, tile_neurons=256 if delivery == "binned" else 0)
    g.simulate(steps)
    o = O.OracleNet(spec, O.FP32SO)
    o.simulate(steps)
    a, b = g.spikes(), o.spikes()
    assert len(b[0]) > 100
    for x, y in zip(a, b):
        assert np.array_equal(x.astype(np.int64), y.astype(np.int64))
    assert np.array_equal(g.get_state("V_m").astype(np.float32), o.get_state("V_m").astype(np.float32))


def test_rule_errors(snn):
    spec = rules_spec()
    spec["projections"][3]["src"] = "A"  # one-to-one with unequal sizes
    with pytest.raises(snn.SnnError):
        snn.Net(spec)
    spec = rules_spec()
    spec["projections"][0]["rule"] = "fixed_indegree"
    spec["projections"][0]["K"] = 2**33
    with pytest.raises(snn.SnnError):
        snn.Net(spec)


def with_list(spec, seed=12, count=700):
    rng = np.random.default_rng(seed)
    n = sum(p["n"] for p in spec["populations"])
    spec["projections"].append(dict(rule="list", src_gids=rng.integers(0, n, size=count).tolist(),
                                    tgt_gids=rng.integers(0, n, size=count).tolist(),
                                    delays_ms=np.round(rng.uniform(0.05, 1.9, size=count), 3).tolist(),
                                    weight=0.25, port=0))
    return spec


@pytest.mark.parametrize("delivery", ["direct", "binned"])
def test_list_csr_and_raster_bit_exact(snn, delivery):
    spec = driven(with_list(rules_spec()))
    tile = 256 if delivery == "binned" else 0
    g = snn.Net(spec, delivery=delivery, tile_neurons=tile)
    o = O.OracleNet(spec, O.FP32SO)
    assert_same(canonical(g.synapses()), canonical(o.synapses()))
    g.simulate(300)
    o.simulate(300)
    for x, y in zip(g.spikes(), o.spikes()):
        assert np.array_equal(x.astype(np.int64), y.astype(np.int64))


def test_list_inside_a_batch(snn):
    specs = [with_list(rules_spec(seed=5), seed=1), with_list(rules_spec(seed=6), seed=2, count=300)]
    g = snn.Net(specs)
    syn = g.synapses()
    first = 0
    for sp in specs:
        n = sum(p["n"] for p in sp["populations"])
        sel = (syn["src"] >= first) & (syn["src"] < first + n)
        assert_same(canonical({k: v[sel] for k, v in syn.items()}, first), canonical(O.OracleNet(sp).synapses()))
        first += n


def test_list_errors(snn):
    spec = rules_spec()
    spec["projections"].append(dict(rule="list", src_gids=[0], tgt_gids=[1], delays_ms=[2.5], weight=1.0, port=0))
    with pytest.raises(snn.SnnError):  # 25 steps above Dmax = 20
        snn.Net(spec)
