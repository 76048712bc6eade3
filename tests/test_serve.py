"""Serving scheduler: the trace generator and the batching policy (host logic,
CPU), and served results against the same requests alone (GPU)."""
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
        assert r.est_bytes > 4 * W.count_synapses(r.spec)
    # mean inter-arrival near 1/20 s
    assert 0.01 < a[-1].arrival_s / 12 < 0.2


def _req(rid, family, nbytes):
    return V.Request(rid, 0.01 * rid, family, {}, 100, nbytes)


def test_pool_serves_every_request_once_within_budget(monkeypatch):
    """Host logic of the worker pool, the device replaced by a recorder: every
    request is served once, no more than `workers` batches run at once, and the
    estimated bytes in flight stay within the budget."""
    import threading
    import time
    active, peak, bytes_peak, seen = [0], [0], [0], []
    lock = threading.Lock()

    def fake_batch(self, batch, t0, rep):
        with lock:
            active[0] += 1
            peak[0] = max(peak[0], active[0])
            seen.extend(r.rid for r in batch)
            bytes_peak[0] = max(bytes_peak[0], sum(r.est_bytes for r in batch))
        time.sleep(0.01)
        for r in batch:
            rep.results.append(V.Result(r.rid, r.arrival_s, 0.0, time.perf_counter() - t0, len(batch), 0, ""))
        with lock:
            active[0] -= 1

    monkeypatch.setattr(V.Server, "_serve_batch", fake_batch)
    reqs = [V.Request(i, 0.002 * i, "ab"[i % 2], {}, 10, 40) for i in range(40)]
    rep = V.Server(budget_bytes=200, max_batch=8, workers=3).serve(reqs)
    assert sorted(seen) == list(range(40)) and len(rep.results) == 40
    assert peak[0] <= 3 and bytes_peak[0] <= 200


def test_batches_take_the_oldest_family_in_order_within_budget():
    srv = V.Server(budget_bytes=100, max_batch=3)
    q = [_req(0, "a", 30), _req(1, "b", 10), _req(2, "a", 30), _req(3, "a", 30), _req(4, "a", 30)]
    b = srv._take_batch(q)
    assert [r.rid for r in b] == [0, 2, 3]          # family of the oldest, arrival order, max 3
    assert [r.rid for r in q] == [1, 4]
    b = srv._take_batch(q)
    assert [r.rid for r in b] == [1]
    srv = V.Server(budget_bytes=50, max_batch=8)
    q = [_req(0, "a", 30), _req(1, "a", 30)]
    assert [r.rid for r in srv._take_batch(q)] == [0]  # budget: the second does not fit
    q = [_req(0, "a", 500)]
    assert [r.rid for r in srv._take_batch(q)] == [0]  # a request alone is always admitted


def test_batches_stay_within_binned_capacity():
    big = W.adex_balanced(n=700_000, k=10)
    srv = V.Server(max_batch=8)
    q = [V.Request(0, 0.0, "adex", big, 10, 1), V.Request(1, 0.1, "adex", big, 10, 1)]
    assert V.neuron_ports(big) == 1_400_000
    assert [r.rid for r in srv._take_batch(q)] == [0]  # two would exceed 512 tiles of 4096 sums


@pytest.mark.gpu
def test_served_results_equal_requests_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[gpu-case] serve small trace", flush=True)
    sys.stdout.flush()
    reqs = []
    for i in range(6):
        spec = W.brunel_lif(n=300 + 50 * i, k=30, g=5.0, nu_ext=300.0, delay=("uniform", 0.1, 3.0), seed=500 + i)
        reqs.append(V.Request(i, 0.0, "lif", spec, 200 + 37 * i, V.estimate_bytes(spec)))
    rep = V.Server(max_batch=4, workers=2).serve(reqs)
    assert rep.batches == 2 and len(rep.results) == 6
    assert sorted(r.batch_size for r in rep.results) == [2, 2, 4, 4, 4, 4]
    for r in rep.results:
        assert r.spikes > 0
        assert r.digest == V.run_alone(reqs[r.rid]), r.rid
