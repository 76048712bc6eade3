"""The oracle on degenerate and boundary networks (no GPU): no synapses,
a silent network, one neuron with an autapse at the largest delay, empty
projections.  Each is checked against what it must do by construction."""
import numpy as np

from oracle import oracle as O

from edge_specs import edge_specs

DT = 0.1


def test_no_synapses_only_poisson():
    o = O.OracleNet(edge_specs()["no_synapses"], O.FP32SO)
    assert o.synapses()["src"].size == 0
    o.simulate(300)
    assert len(o.spikes()[0]) > 0 and o.events == 0


def test_silent_network_decays_exactly():
    spec = edge_specs()["silent"]
    o = O.OracleNet(spec)
    v0 = o.get_state("V_m").copy()
    o.simulate(500)
    assert len(o.spikes()[0]) == 0 and o.events == 0
    # free decay of V (E_L = 0): V(t) = V0 exp(-t / tau_m)
    assert np.allclose(o.get_state("V_m"), v0 * np.exp(-500 * DT / 20.0), rtol=1e-12, atol=1e-12)


def test_one_neuron_autapse_at_the_largest_delay():
    spec = edge_specs()["one_neuron_max_delay"]
    o = O.OracleNet(spec, O.FP32SO)
    syn = o.synapses()
    assert syn["src"].size == 3 and np.all(syn["delay"] == 63)
    rec = o.record_input(400)
    o.simulate(400)
    st = o.spikes()[0].astype(np.int64)
    assert len(st) >= 3
    # each spike of step s arrives three times (three synapses) at step s + 63
    S = o.shift_of(0, 0)
    for n in range(400):
        k = int(np.sum(st == n - 63))
        assert rec[n][0, 0] == k * 3 * int(np.rint(np.ldexp(2.0, S)))


def test_empty_projections():
    spec = edge_specs()["empty_projections_257"]
    o = O.OracleNet(spec, O.FP32SO)
    full = O.OracleNet(dict(spec, projections=spec["projections"][:4]), O.FP32SO)
    assert o.synapses()["src"].size == full.synapses()["src"].size == 257 * 25
    o.simulate(200)
    full.simulate(200)
    for a, b in zip(o.spikes(), full.spikes()):
        assert np.array_equal(a, b)
