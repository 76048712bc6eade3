"""The allocation-free input readback (snn_get_input_noalloc) against the
allocating one (snn_get_input), through the C ABI: binned delivery stages its
sum in the library's fixed device workspace, direct delivery copies the
accumulators.  Two calls in a row on one network, the second over a smaller
range, so that the second reads a workspace holding the first call's values;
then the same on a second network of another size; and the size limit."""
import sys

import numpy as np
import pytest

from paper_2007_14236_amd import workloads as W

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


def _compare(net, port, first, n):
    ref = net.get_input(port=port, first=first, n=n)
    got = net.get_input_noalloc(port=port, first=first, n=n)
    assert got.dtype == np.int64 and got.shape == (n,)
    assert np.array_equal(got, ref), (port, first, n)
    return ref


def two_port_lif(n=3000, k=200, seed=5):
    """LIF neurons with exponential PSCs on two ports (excitatory input on
    port 0, inhibitory on port 1), driven hard enough to fire from the start."""
    ne = n * 4 // 5
    params = dict(tau_m=10.0, C_m=250.0, E_L=-65.0, V_th=-50.0, V_reset=-65.0, t_ref=2.0, tau_syn=[0.5, 1.0])
    pops = [dict(name="E", model="lif_exp", n=ne, ports=2, params=dict(params),
                 V0=W.initial_v(seed, ne, -65.0, -50.0, stream=7), I_e=0.0),
            dict(name="I", model="lif_exp", n=n - ne, ports=2, params=dict(params),
                 V0=W.initial_v(seed, n - ne, -65.0, -50.0, stream=8), I_e=0.0)]
    projs = [dict(src=s, tgt=t, K=k * 4 // 5 if s == "E" else k // 5, weight=80.0 if s == "E" else -300.0,
                  delay=("uniform", 0.1, 2.0), port=0 if s == "E" else 1) for s in ("E", "I") for t in ("E", "I")]
    pois = [dict(tgt=t, rate=8.0, n_inputs=3000, weight=80.0, port=0) for t in ("E", "I")]
    return dict(name="two_port_lif", dt=0.1, seed=seed, dmax=25, populations=pops, projections=projs, poisson=pois)


@pytest.mark.parametrize("delivery,tile,cap", [("binned", 256, 0), ("binned", 512, 24), ("direct", 0, 0)])
def test_noalloc_readback_equals_allocating_readback(snn, delivery, tile, cap):
    # two ports, so both ports (and with capacity 24 the spill path) are read
    spec = two_port_lif()
    net = snn.Net(spec, delivery=delivery, tile_neurons=tile, bin_capacity=cap)
    try:
        for steps in (40, 7):
            net.simulate(steps)
            nonzero = 0
            for port in (0, 1):
                a = _compare(net, port, 0, net.N)           # the whole network
                b = _compare(net, port, 1000, 517)          # then a smaller, unaligned range
                assert np.array_equal(b, a[1000:1517])
                nonzero += int(np.count_nonzero(a))
            assert nonzero > 0, "no pending input to compare"
        if cap:
            assert net.counters()["spill_events"] > 0, "the spill path was not exercised"
    finally:
        net.close()


def test_noalloc_readback_second_network_and_limit(snn):
    big = snn.Net(W.brunel_lif(n=5000, k=400, seed=3, delay=("uniform", 0.1, 2.0), dmax=25, nu_ext=300.0),
                  delivery="binned", tile_neurons=512)
    small = snn.Net(W.brunel_lif(n=700, k=60, seed=9, delay=("uniform", 0.1, 2.0), dmax=25, nu_ext=300.0),
                    delivery="binned", tile_neurons=256)
    try:
        big.simulate(60)
        small.simulate(60)
        a = _compare(big, 0, 0, big.N)
        b = _compare(small, 0, 0, small.N)   # smaller input: the workspace still holds big's values beyond it
        assert np.count_nonzero(a) > 0 and np.count_nonzero(b) > 0
        _compare(small, 0, 3, 5)
        _compare(big, 0, big.N - 1, 1)
        assert big.get_input_noalloc(first=10, n=0).shape == (0,)
        with pytest.raises(snn.SnnError):
            big.get_input_noalloc(first=0, n=big.N + 1)      # beyond the network
    finally:
        big.close()
        small.close()


def test_noalloc_readback_refuses_more_than_the_workspace(snn):
    n = (1 << 18) + 256
    spec = W.brunel_lif(n=n, k=2, seed=1, delay=("const", 0.1, 0.0), dmax=1, nu_ext=100.0)
    net = snn.Net(spec, delivery="binned", tile_neurons=4096)
    try:
        net.simulate(3)
        with pytest.raises(snn.SnnError, match="INVALID"):
            net.get_input_noalloc(first=0, n=n)
        half = _compare(net, 0, 0, 1 << 18)                  # exactly the limit is accepted
        assert half.shape == (1 << 18,)
    finally:
        net.close()
