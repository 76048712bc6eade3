"""GPU parity of per-neuron model parameters (Sec. 2.1: neuron parameters
from fixed values, arrays or probability distributions), through the C ABI:

- LIF networks whose neurons carry their own membrane time constant,
  capacitance, resting potential, threshold, reset and refractory time (from
  arrays and from distributions, beside populations that keep their
  constants) give the fp32 same-order oracle's rasters and potentials bit for
  bit, in both delivery modes and as members of a batch;
- uncoupled AdEx neurons with their own leak, slope, threshold and adaptation
  constants follow the fp64 oracle within 1e-4 with the same spike steps;
- a neuron whose potential was never set starts at its own E_L;
- bad calls are refused.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
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


def hetero_mc(seed=3):
    """Small microcircuit stand-in: L2/3E with per-neuron arrays of all six LIF
    parameters, L4E with V_th and tau_m drawn from distributions, L5E with
    one parameter set per neuron to its population's value (no own
    constants needed), the others unchanged."""
    spec = W.microcircuit(scale=0.05, k_scale=0.25, k_ext=3500, seed=seed)
    g = np.random.Generator(np.random.Philox(key=[seed, 77]))
    pops = {p["name"]: p for p in spec["populations"]}
    a = pops["L23E"]
    n = a["n"]
    E_L = g.uniform(-68.0, -62.0, n)
    a["params"].update(tau_m=g.uniform(7.0, 14.0, n), C_m=g.uniform(200.0, 300.0, n), E_L=E_L,
                       V_th=E_L + g.uniform(12.0, 18.0, n), V_reset=E_L + g.uniform(-3.0, 1.0, n),
                       t_ref=g.choice([0.0, 1.0, 2.0, 2.5], n))
    a["V0"] = None  # starts at each neuron's own E_L
    pops["L4E"]["param_dists"] = {"V_th": dict(kind="normal", mean=-50.0, sd=1.0, levels=512),
                                  "tau_m": dict(kind="uniform", low=8.0, high=12.0)}
    pops["L5E"]["params"]["V_th"] = np.full(pops["L5E"]["n"], -50.0)
    return spec


def hetero_brunel(seed=5):
    spec = W.brunel_lif(n=600, k=60, seed=seed, delay=("uniform", 0.1, 2.0), dmax=25, nu_ext=260.0)
    e = spec["populations"][0]
    e["param_dists"] = {"V_th": dict(kind="uniform", low=18.0, high=22.0, levels=64),
                        "t_ref": dict(kind="uniform", low=1.0, high=3.0, levels=5)}
    return spec


SPECS = {"mc": hetero_mc, "brunel": hetero_brunel}
STEPS = 800


def oracle_run(spec, steps=STEPS):
    o = O.OracleNet(spec, O.FP32SO)
    o.simulate(steps)
    return o.spikes(), o.get_state("V_m").astype(np.float32)


@pytest.mark.parametrize("name", sorted(SPECS))
@pytest.mark.parametrize("delivery", ["direct", "binned"])
def test_lif_per_neuron_parameters_bit_exact(snn, name, delivery):
    spec = SPECS[name]()
    (os_, og, om), ov = oracle_run(spec)
    g = snn.Net(spec, delivery=delivery)
    try:
        g.simulate(STEPS)
        gs, gg, gm = g.spikes()
        assert len(os_) > 100
        assert np.array_equal(gs, os_) and np.array_equal(gg, og) and np.array_equal(gm, om)
        assert np.array_equal(g.get_state("V_m").astype(np.float32), ov)
    finally:
        g.close()


def test_lif_per_neuron_parameters_matter(snn):
    """The same network with its populations' constants fires differently,
    so the rasters above test the neurons' own constants."""
    het, hom = hetero_brunel(), W.brunel_lif(n=600, k=60, seed=5, delay=("uniform", 0.1, 2.0), dmax=25,
                                              nu_ext=260.0)
    a, b = snn.Net(het), snn.Net(hom)
    try:
        a.simulate(400)
        b.simulate(400)
        sa, sb = a.spikes(), b.spikes()
        assert len(sa[0]) != len(sb[0]) or not np.array_equal(sa[1], sb[1])
    finally:
        a.close()
        b.close()


def test_per_neuron_parameters_in_a_batch(snn):
    specs = [hetero_brunel(seed=5), hetero_mc(seed=4), hetero_brunel(seed=6)]
    for sp in specs:
        sp["dmax"] = 63
    g = snn.Net(specs, delivery="binned")
    try:
        g.simulate(500)
        st, gid, mult = g.spikes()
        for k, sp in enumerate(specs):
            inst = g.instances[k]
            lo, n = inst["first"], inst["n"]
            sel = (gid >= lo) & (gid < lo + n)
            (os_, og, om), ov = oracle_run(sp, 500)
            assert np.array_equal(st[sel], os_) and np.array_equal(gid[sel] - lo, og), k
            assert np.array_equal(g.get_state("V_m", lo, n).astype(np.float32), ov), k
    finally:
        g.close()


def test_resting_potential_per_neuron(snn):
    spec = dict(name="rest", dt=0.1, seed=1, dmax=2, projections=[], poisson=[],
                populations=[dict(name="A", model="lif_exp", n=5, ports=1,
                                  params=dict(E_L=np.array([-70.0, -65.0, -60.0, -72.5, -68.0]), V_th=-40.0,
                                              tau_syn=[0.5]),
                                  I_e=0.0)])
    g = snn.Net(spec, build=False)
    try:
        assert np.allclose(g.get_state("V_m"), spec["populations"][0]["params"]["E_L"])
        g.build()
        g.simulate(50)  # at rest without input: stays at its own E_L
        assert np.array_equal(g.get_state("V_m"), spec["populations"][0]["params"]["E_L"])
    finally:
        g.close()


def hetero_adex(n=12):
    g = np.random.Generator(np.random.Philox(key=[9, 1]))
    prm = dict(W.ADEX_T2)
    prm.update(g_L=g.uniform(20.0, 40.0, n), E_L=g.uniform(-72.0, -68.0, n), a=g.uniform(0.0, 8.0, n),
               b=g.uniform(40.0, 120.0, n), tau_w=g.uniform(80.0, 250.0, n), V_T=g.uniform(-52.0, -49.0, n),
               Delta_T=g.uniform(1.5, 2.5, n), C_m=g.uniform(200.0, 320.0, n))
    I_e = np.concatenate([np.linspace(600.0, 1500.0, n // 2), np.linspace(0.0, 150.0, n - n // 2)])
    return dict(name="adex_het", dt=0.1, seed=1, dmax=2, projections=[], poisson=[],
                populations=[dict(name="A", model="aeif_cond_exp", n=n, ports=2, params=prm, V0=None,
                                  I_e=I_e)])


def test_adex_per_neuron_parameters_within_tolerance(snn):
    spec = hetero_adex()
    n = spec["populations"][0]["n"]
    g = snn.Net(spec)
    o = O.OracleNet(spec)
    steps = 3000
    vg, vo, wg, wo = [], [], [], []
    try:
        for _ in range(steps // 10):
            g.simulate(10)
            o.simulate(10)
            vg.append(g.get_state("V_m")); vo.append(o.get_state("V_m"))
            wg.append(g.get_state("w")); wo.append(o.get_state("w"))
        vg, vo, wg, wo = map(np.array, (vg, vo, wg, wo))
        gs, gg, _ = g.spikes()
        os_, og, _ = o.spikes()
        spiking = 0
        for i in range(n):
            a, b = gs[gg == i], os_[og == i]
            k = 0
            while k < min(len(a), len(b)) and a[k] == b[k]:
                k += 1
            if len(b):
                spiking += 1
                assert k >= min(3, len(b)), (i, a[:5], b[:5])
            upto = (int(b[k]) if k < len(b) else steps) // 10  # samples before the first divergence
            ok = np.ones(upto, dtype=bool)
            for sp in b:  # exclude the upswing: the last ms before each spike, and the sample after it
                ok[max(0, int(sp) // 10 - 1):int(sp) // 10 + 2] = False
            ok = ok[:upto]
            assert np.max(np.abs(vg[:upto, i] - vo[:upto, i])[ok] / np.abs(vo[:upto, i])[ok], initial=0.0) < 1e-4, i
            # w relative to the larger of |w| and the neuron's spike-triggered step b: near rest w is
            # a (V - E_L) with V - E_L a few 1e-5 mV, below what the fp32 integrator (error scale
            # |V| + |h dV/dt| + 1 at eps 1e-6, i.e. ~7e-5 mV on V) resolves
            b_i = spec["populations"][0]["params"]["b"][i]
            assert np.max(np.abs(wg[:upto, i] - wo[:upto, i])[ok] / np.maximum(np.abs(wo[:upto, i])[ok], b_i),
                          initial=0.0) < 1e-4, i
        assert spiking >= 4
    finally:
        g.close()


def test_bad_parameter_calls_are_refused(snn):
    import ctypes as C
    spec = hetero_brunel()
    g = snn.Net(spec, build=False)
    try:
        v = np.ones(3)
        p = v.ctypes.data_as(C.POINTER(C.c_double))
        with pytest.raises(snn.SnnError, match="INVALID"):
            g._check(g.L.snn_set_param(g.h, 0, 5, snn.PARAMS["V_th"], p, 3))  # nv neither 1 nor n
        with pytest.raises(snn.SnnError, match="INVALID"):
            g._check(g.L.snn_set_param(g.h, 0, 5, 99, p, 1))  # unknown parameter
        with pytest.raises(snn.SnnError, match="INVALID"):
            g._check(g.L.snn_set_param(g.h, g.N - 1, 5, snn.PARAMS["V_th"], p, 1))  # beyond the network
        bad = np.array([-1.0])
        g._check(g.L.snn_set_param(g.h, 3, 1, snn.PARAMS["tau_m"], bad.ctypes.data_as(C.POINTER(C.c_double)), 1))
        with pytest.raises(snn.SnnError, match="INVALID"):
            g.build()  # tau_m <= 0 of neuron 3
    finally:
        g.close()
