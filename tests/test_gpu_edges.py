"""GPU parity on degenerate and boundary networks through the C ABI: no
synapses (Poisson drive only), a silent network, one neuron with an autapse
at the largest delay (Dmax = 63), empty projections beside a real one on 257
neurons -- rasters, potentials and delivered-event counts equal the oracle's
in both delivery modes."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

from edge_specs import edge_specs

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


@pytest.mark.parametrize("delivery", ["direct", "binned"])
@pytest.mark.parametrize("name", list(edge_specs()))
def test_edge_network_bit_exact(snn, name, delivery):
    spec = edge_specs()[name]
    steps = 400
    g = snn.Net(spec, delivery=delivery, tile_neurons=256 if delivery == "binned" else 0)
    o = O.OracleNet(spec, O.FP32SO)
    syn_g, syn_o = g.synapses(), o.synapses()
    assert syn_g["src"].size == syn_o["src"].size
    g.simulate(steps)
    o.simulate(steps)
    for x, y in zip(g.spikes(), o.spikes()):
        assert np.array_equal(x.astype(np.int64), y.astype(np.int64))
    assert np.array_equal(g.get_state("V_m").astype(np.float32), o.get_state("V_m").astype(np.float32))
    c = g.counters()
    assert c["events"] == o.events and c["overflow"] == 0
    if name == "silent":
        assert c["spikes"] == 0 and c["events"] == 0
