"""GPU parity of connection weights from distributions and per-connection
list weights (Sec. 2.1) through the C ABI: the device-built CSR, with each
synapse's drawn weight level, equals the oracle's canonical table bit for bit
(every drawing rule, alone, in a batch of instances, and at 20,000 neurons
with 256 levels), rasters and potentials are bit-exact in both delivery modes,
and the invalid set-ups are refused."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

from test_gpu_rules import assert_same, canonical, driven
from test_oracle_rules import rules_spec
from test_oracle_weights import spec_with_weights

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


def with_list_weights(spec, seed=12, count=700):
    rng = np.random.default_rng(seed)
    n = sum(p["n"] for p in spec["populations"])
    spec["projections"].append(dict(rule="list", src_gids=rng.integers(0, n, size=count).tolist(),
                                    tgt_gids=rng.integers(0, n, size=count).tolist(),
                                    delays_ms=np.round(rng.uniform(0.05, 1.9, size=count), 3).tolist(),
                                    weights=np.round(rng.uniform(-0.6, 0.6, size=count), 2).tolist(),
                                    weight=0.0, port=0))
    return spec


def all_weight_kinds(seed=5):
    spec = spec_with_weights(seed=seed)
    spec["projections"][2]["weight_dist"] = dict(kind="uniform", low=-0.2, high=0.0, levels=5)  # all-to-all
    spec["projections"][3]["weight_dist"] = dict(kind="normal", mean=0.5, sd=0.2, low=0.3, high=0.9, levels=7)
    return with_list_weights(spec)


@pytest.mark.parametrize("delivery", ["direct", "binned"])
def test_weight_levels_csr_bit_exact(snn, delivery):
    spec = all_weight_kinds()
    g = snn.Net(spec, delivery=delivery, tile_neurons=256 if delivery == "binned" else 0)
    o = O.OracleNet(spec)
    assert_same(canonical(g.synapses()), canonical(o.synapses()))
    assert np.unique(o.synapses()["wq"]).size > 60


@pytest.mark.parametrize("delivery", ["direct", "binned"])
def test_weight_levels_raster_bit_exact(snn, delivery):
    spec = driven(all_weight_kinds())
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


def test_weight_levels_inside_a_batch(snn):
    specs = [all_weight_kinds(seed=5), with_list_weights(spec_with_weights(seed=6), seed=3, count=200)]
    g = snn.Net(specs)
    syn = g.synapses()
    first = 0
    for sp in specs:
        n = sum(p["n"] for p in sp["populations"])
        sel = (syn["src"] >= first) & (syn["src"] < first + n)
        assert_same(canonical({k: v[sel] for k, v in syn.items()}, first), canonical(O.OracleNet(sp).synapses()))
        first += n


def test_weight_levels_20k_bit_exact(snn):
    spec = rules_spec(seed=9, sizes=(8000, 6000, 6000), total=400_000, outdeg=30)
    spec["projections"] = [p for p in spec["projections"] if p["rule"] != "all_to_all"]
    spec["projections"][0]["weight_dist"] = dict(kind="normal", mean=0.2, sd=0.05, levels=256)
    spec["projections"][3]["weight_dist"] = dict(kind="uniform", low=-0.5, high=-0.1, levels=100)
    g = snn.Net(spec)
    o = O.OracleNet(spec)
    assert_same(canonical(g.synapses()), canonical(o.synapses()))


def test_weight_errors(snn):
    from paper_2007_14236_amd import workloads as W
    sp = dict(name="adex", dt=0.1, seed=1, dmax=20, poisson=[],
              populations=[dict(name="A", model="aeif_cond_exp", n=20, ports=2, params=dict(W.ADEX_T2))],
              projections=[dict(src="A", tgt="A", rule="fixed_indegree", K=5, weight=0.0, port=0,
                                delay=("uniform", 1.0, 2.0), weight_dist=dict(kind="normal", mean=0.1, sd=0.1))])
    with pytest.raises(snn.SnnError):  # negative conductance levels
        snn.Net(sp)
    sp["projections"][0]["weight_dist"]["low"] = 0.0
    snn.Net(sp).close()
    spec = spec_with_weights()
    spec["projections"][0]["weight_dist"]["levels"] = 0
    with pytest.raises(snn.SnnError):
        snn.Net(spec)
    spec = spec_with_weights()
    spec["projections"][0]["weight_dist"] = dict(kind="normal", mean=0.0, sd=1.0, low=50.0, high=60.0)
    with pytest.raises(snn.SnnError):
        snn.Net(spec)
    spec = with_list_weights(rules_spec())
    spec["projections"][-1]["weights"] = spec["projections"][-1]["weights"][:-1]  # one short
    with pytest.raises(snn.SnnError):
        snn.Net(spec)


@pytest.mark.parametrize("delivery", ["direct", "binned"])
def test_microcircuit_normal_weights_raster_bit_exact(snn, delivery):
    """the microcircuit stand-in with every weight normal (10 % deviation,
    32 levels): rasters and potentials bit-exact for 1000 steps"""
    from paper_2007_14236_amd import workloads as W
    spec = W.microcircuit(scale=0.05, k_scale=0.25, k_ext=3500, seed=3, weight_sd=0.1)
    g = snn.Net(spec, delivery=delivery, tile_neurons=512 if delivery == "binned" else 0)
    g.simulate(1000)
    o = O.OracleNet(spec, O.FP32SO)
    o.simulate(1000)
    a, b = g.spikes(), o.spikes()
    assert len(b[0]) > 100
    for x, y in zip(a, b):
        assert np.array_equal(x.astype(np.int64), y.astype(np.int64))
    assert np.array_equal(g.get_state("V_m").astype(np.float32), o.get_state("V_m").astype(np.float32))


def lif_state_spec(n=2000, seed=3):
    from paper_2007_14236_amd import workloads as W
    spec = W.brunel_lif(n=n, k=40, seed=seed, nu_ext=100.0)
    for p in spec["populations"]:
        p["state_dists"] = {"V_m": dict(kind="uniform", low=0.0, high=20.0, levels=4096),
                            "I_e": dict(kind="normal", mean=100.0, sd=30.0, low=0.0, high=250.0, levels=500)}
    return spec


@pytest.mark.parametrize("delivery", ["direct", "binned"])
def test_state_distributions_bit_exact(snn, delivery):
    """drawn potentials and currents equal the oracle's at build, and the
    raster and potentials after 300 steps"""
    spec = lif_state_spec()
    g = snn.Net(spec, delivery=delivery, tile_neurons=512 if delivery == "binned" else 0)
    o = O.OracleNet(spec, O.FP32SO)
    for var in ("V_m", "I_e"):
        assert np.array_equal(g.get_state(var).astype(np.float32), o.get_state(var).astype(np.float32)), var
    g.simulate(300)
    o.simulate(300)
    a, b = g.spikes(), o.spikes()
    assert len(b[0]) > 100
    for x, y in zip(a, b):
        assert np.array_equal(x.astype(np.int64), y.astype(np.int64))
    assert np.array_equal(g.get_state("V_m").astype(np.float32), o.get_state("V_m").astype(np.float32))


def test_state_distributions_per_instance_and_adex(snn):
    from paper_2007_14236_amd import workloads as W
    ad = W.adex_balanced(n=500, k=50, seed=9)
    for p in ad["populations"]:
        p["state_dists"] = {"V_m": dict(kind="normal", mean=-65.0, sd=4.0, levels=2000),
                            "w": dict(kind="uniform", low=0.0, high=50.0, levels=100)}
    specs = [lif_state_spec(n=300, seed=4), ad, lif_state_spec(n=700, seed=5)]
    g = snn.Net(specs)
    first = 0
    for sp in specs:
        n = sum(p["n"] for p in sp["populations"])
        o = O.OracleNet(sp, O.FP32SO, build=False)
        for var in ("V_m", "I_e") + (("w",) if sp is ad else ()):
            assert np.array_equal(g.get_state(var, first, n).astype(np.float32),
                                  o.get_state(var).astype(np.float32)), (sp["name"], var)
        first += n
