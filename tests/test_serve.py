"""Serving through the library's request server (snn_server_*): the trace
generator (host logic, CPU); and on the GPU, requests of both families
arriving while others run, under a budget that makes them queue, each
result equal to the same request alone and, for the LIF requests, to the
fp32 same-order oracle; a request larger than the budget is refused."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2007_14236_amd import serve as V
from paper_2007_14236_amd import workloads as W


def test_trace_is_seeded_and_alternates_families():
    a = V.request_trace(12)
    b = V.request_trace(12)
    assert [r.arrival_s for r in a] == [r.arrival_s for r in b]
    assert [r.steps for r in a] == [r.steps for r in b]
    assert all(x < y for x, y in zip([r.arrival_s for r in a], [r.arrival_s for r in a][1:]))
    assert [r.family for r in a] == ["microcircuit", "adex"] * 6
    for r in a:
        assert 1000 <= r.steps <= 20000
        n = W.total_neurons(r.spec)
        if r.family == "adex":
            assert 10_000 <= n <= 200_000 and r.spec["projections"][0]["K"] in (800, 200)
        else:
            assert 0.09 * 77169 <= n <= 1.01 * 77169
    # mean inter-arrival near 1/20 s
    assert 0.01 < a[-1].arrival_s / 12 < 0.2


def small_trace():
    """Staggered arrivals mixing LIF networks (checked against the oracle) and
    AdEx networks (checked against themselves alone)."""
    reqs = []
    t = 0.0
    for i in range(8):
        if i % 2 == 0:
            spec = W.brunel_lif(n=600 + 150 * i, k=60, seed=300 + i, delay=("uniform", 0.1, 2.0), dmax=25,
                                nu_ext=260.0)
            fam = "lif"
        else:
            spec = W.adex_balanced(n=2000 + 500 * i, k=200, seed=300 + i)
            fam = "adex"
        reqs.append(V.Request(i, t, fam, spec, 400 + 100 * (i % 3)))
        t += 0.02
    return reqs


def _lif_oracle(req):
    from oracle import oracle as O
    o = O.OracleNet(req.spec, O.FP32SO)
    o.simulate(req.steps)
    return o.spikes()


@pytest.mark.gpu
def test_served_results_equal_alone_and_the_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[gpu-case] serve mix", flush=True)
    sys.stdout.flush()
    trace = small_trace()
    # a budget of about two requests: the others wait for memory, then run
    big = max(W.count_synapses(r.spec) for r in trace)
    budget = 2 * (60 * big + (64 << 20))
    rep = V.Server(budget_bytes=budget, slots=3, keep_nets=True).serve(trace)
    assert [r.status for r in rep.results] == [0] * len(trace)
    assert rep.peak_bytes <= budget
    # overlap: some request started before another finished, and one was admitted
    # only after another had finished (it waited for a slot or for memory)
    res = rep.results
    assert any(a.start_s < b.finish_s and b.start_s < a.finish_s for a in res for b in res if a.rid < b.rid)
    assert any(a.start_s >= min(b.finish_s for b in res if b.rid != a.rid) for a in res)
    for r, req in zip(res, trace):
        net = rep.nets[req.rid]
        st, gid, m = net.spikes(0, req.steps)
        assert len(st) > 0
        if req.family == "lif":
            os_, og, om = _lif_oracle(req)
            assert np.array_equal(st, os_) and np.array_equal(gid, og) and np.array_equal(m, om), req.rid
        assert r.digest == V.run_alone(req), req.rid
        net.close()


@pytest.mark.gpu
def test_request_larger_than_the_budget_is_refused():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[gpu-case] serve budget", flush=True)
    from paper_2007_14236_amd import snn as S
    L = S.lib()
    small = W.brunel_lif(n=400, k=40, seed=1, delay=("uniform", 0.1, 2.0), dmax=25, nu_ext=260.0)
    big = W.brunel_lif(n=4000, k=400, seed=2, delay=("uniform", 0.1, 2.0), dmax=25, nu_ext=260.0)
    h = C.c_void_p()
    assert L.snn_server_create(8 << 20, 2, C.byref(h)) == 0
    try:
        # synapse words alone above the budget: refused at submission
        huge = S.Net(W.brunel_lif(n=40000, k=100, seed=3), build=False)
        t = C.c_uint64()
        assert L.snn_server_submit(h, huge.h, 10, C.byref(t)) == -6
        huge.close()
        # fits by its synapses, not by everything it allocates: refused at build, nothing else running
        nb = S.Net(big, build=False)
        tb = C.c_uint64()
        assert L.snn_server_submit(h, nb.h, 50, C.byref(tb)) == 0
        ns = S.Net(small, build=False)
        ts = C.c_uint64()
        assert L.snn_server_submit(h, ns.h, 50, C.byref(ts)) == 0
        for tk in (tb, ts):
            assert L.snn_server_wait(h, tk.value, 60.0) == 0
        out = C.c_void_p()
        info = S.JobInfo()
        assert L.snn_server_result(h, tb.value, C.byref(out), C.byref(info)) == -6
        assert info.status == -6 and b"budget" in info.error
        assert L.snn_server_result(h, ts.value, C.byref(out), C.byref(info)) == 0
        assert info.device_bytes_peak <= (8 << 20)
        assert len(ns.spikes(0, 50)[0]) > 0
        st = S.ServerStats()
        assert L.snn_server_get_stats(h, C.byref(st)) == 0
        assert st.in_use == 0 and st.peak <= (8 << 20) and st.done == 1 and st.failed == 1
        nb.close()
        ns.close()
    finally:
        L.snn_server_destroy(h)
