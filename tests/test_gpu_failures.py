"""Failure paths through the C ABI, each forced from the host so that every
kernel still ends normally (no device fault, only status codes):

- the device allocator refuses memory part-way through a build: SNN_E_NOMEM,
  the handle stays usable, and a later build with memory gives the oracle's
  raster;
- an AdEx neuron driven far beyond its range resets more often in one step
  than a spike record holds: the count is clamped and the call reports
  SNN_E_OVERFLOW;
- a released network keeps its raster and counters, frees its device memory
  and refuses device calls with SNN_E_STATE.
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


def test_allocator_refusal_gives_nomem_and_a_usable_handle(snn):
    spec = W.c0(active=True)

    class Refusing(snn.TorchAllocator):
        def __init__(self, allow):
            super().__init__()
            self.allow, self.calls = allow, 0

        def _a(self, nbytes, user):
            self.calls += 1
            if self.calls > self.allow:
                return None
            return super()._a(nbytes, user)

    for allow in (0, 3, 12):
        al = Refusing(allow)
        g = snn.Net(spec, allocator=al, build=False)
        try:
            with pytest.raises(snn.SnnError, match="NOMEM"):
                g.build()
            assert g.counters()["device_bytes"] == 0   # what the failed build had is released
            assert not al.live                          # every block went back to the allocator
            al.allow = 10 ** 9                          # memory is available again: the same handle builds
            g.build()
            g.simulate(300)
            o = O.OracleNet(spec, O.FP32SO)
            o.simulate(300)
            gs, gg, _ = g.spikes()
            os_, og, _ = o.spikes()
            assert len(os_) > 0 and np.array_equal(gs, os_) and np.array_equal(gg, og), allow
        finally:
            g.close()


def test_device_range_flags_are_reported(snn):
    """An AdEx neuron driven by 10^8 pA crosses V_peak hundreds of times in one
    0.1 ms step: more resets than a spike record holds (31) and, at ~100
    substeps per reset, up to the per-step substep cap.  The step still ends
    (the count is clamped, the integration stops at the cap) and the call
    reports SNN_E_OVERFLOW with the flags in the counters."""
    spec = dict(name="flags", dt=0.1, seed=1, dmax=2, projections=[], poisson=[],
                populations=[dict(name="A", model="aeif_cond_exp", n=2, ports=2, params=dict(W.ADEX_T2),
                                  V0=None, I_e=np.array([1e8, 0.0]))])
    g = snn.Net(spec)
    try:
        with pytest.raises(snn.SnnError, match="OVERFLOW"):
            g.simulate(1)
        c = g.counters()
        assert c["overflow"] & 1  # multiplicity above 31
        st, gid, mult = g.spikes()
        assert list(gid) == [0] and list(mult) == [31]  # clamped
        assert np.all(np.isfinite(g.get_state("V_m")))
    finally:
        g.close()


def test_release_keeps_results_and_frees_memory(snn):
    spec = W.c0(active=True)
    g = snn.Net(spec)
    try:
        g.simulate(250)
        before = g.counters()
        sp_before = g.spikes()
        assert before["device_bytes"] > 0
        g._check(g.L.snn_release(g.h))
        after = g.counters()
        assert after["device_bytes"] == 0 and after["steps"] == 250 and after["spikes"] == before["spikes"]
        assert all(np.array_equal(a, b) for a, b in zip(g.spikes(), sp_before))
        with pytest.raises(snn.SnnError, match="STATE"):
            g.simulate(1)
        with pytest.raises(snn.SnnError, match="STATE"):
            g._check(g.L.snn_release(g.h))
        with pytest.raises(snn.SnnError, match="STATE"):
            g.build()
    finally:
        g.close()
