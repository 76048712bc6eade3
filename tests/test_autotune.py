"""Autotuner: the candidate set (CPU) and a tuning run whose choice gives the
same raster as the library's default configuration (GPU)."""
import sys

import numpy as np
import pytest

from paper_2007_14236_amd import autotune as A
from paper_2007_14236_amd import workloads as W


def test_candidates_respect_port_and_tile_limits():
    c1 = A.candidates(W.microcircuit(1.0))          # one port: tiles up to 4096
    tiles = sorted({c["tile_neurons"] for c in c1 if c["delivery"] == "binned"})
    assert tiles == [256, 512, 1024, 2048, 4096]
    c2 = A.candidates(W.adex_balanced(n=1_000_000))  # two ports: at most 2048, at most 1024 tiles
    tiles = sorted({c["tile_neurons"] for c in c2 if c["delivery"] == "binned"})
    assert tiles == [1024, 2048]
    assert any(c["delivery"] == "direct" for c in c2)
    big = [W.brunel_sweep_instance(i) for i in range(128)]  # 3.0e6 neurons: only 4096-neuron tiles fit
    tiles = sorted({c["tile_neurons"] for c in A.candidates(big) if c["delivery"] == "binned"})
    assert tiles == [4096]
    assert A.signature(big).endswith("instances=128")


@pytest.mark.gpu
def test_tuned_configuration_gives_the_default_raster():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[gpu-case] autotune c0a", flush=True)
    sys.stdout.flush()
    from paper_2007_14236_amd import snn as S
    spec = W.c0(True)
    best, table = A.tune(spec, steps=100, warmup=50)
    assert len(table) == len(A.candidates(spec)) and all(r["us_per_step"] > 0 for r in table)
    assert min(r["us_per_step"] for r in table) == [r for r in table if all(r.get(k) == v for k, v in best.items())][0]["us_per_step"]
    a = S.Net(spec, **best)
    b = S.Net(spec)
    a.simulate(500)
    b.simulate(500)
    for x, y in zip(a.spikes(), b.spikes()):
        assert np.array_equal(x, y)
