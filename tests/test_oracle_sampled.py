"""Pins of the oracle's sampled checks (used where a network's synapse table
is too large to build on the CPU): the synapses onto one target drawn one by
one equal that target's synapses in the built table (itself pinned against
an independent Philox), and the sampled input of targets equals the full
delivery definition's replay, on networks small enough for both (no GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2007_14236_amd import workloads as W


def specs():
    return {
        "brunel_normal": W.brunel_lif(n=700, k=60, seed=11, delay=("normal", 1.5, 0.75), dmax=63, nu_ext=250.0),
        "mc_small": W.microcircuit(scale=0.05, k_scale=0.25, k_ext=3500, seed=3),
        "alpha_small": W.adex_balanced_alpha(n=500, k=50, seed=2),
    }


@pytest.mark.parametrize("name", list(specs()))
def test_target_synapses_equal_built_table(name):
    spec = specs()[name]
    full = O.OracleNet(spec)
    lazy = O.OracleNet(spec, build=False)
    syn = full.synapses()
    rng = np.random.default_rng(0)
    for t in rng.choice(full.N, size=25, replace=False):
        sel = syn["tgt"] == t
        a = sorted(zip(syn["src"][sel].tolist(), syn["delay"][sel].tolist(), syn["port"][sel].tolist(),
                       syn["wq"][sel].tolist()))
        s, d, p, w = lazy.target_synapses(int(t))
        b = sorted(zip(s.tolist(), d.tolist(), p.tolist(), w.tolist()))
        assert a == b, t
    for g in (0, full.N - 1):
        for port in range(full.P):
            assert lazy.shift_of(g, port) == full.shift_of(g, port)


@pytest.mark.parametrize("name", list(specs()))
def test_sampled_input_equals_replay(name):
    spec = specs()[name]
    o = O.OracleNet(spec)
    o.simulate(200)
    st, gid, m = o.spikes()
    assert len(st) > 20
    lazy = O.OracleNet(spec, build=False)
    rng = np.random.default_rng(1)
    targets = rng.choice(o.N, size=min(o.N, 200), replace=False)
    nonzero = 0
    for target_step in (60, 100, 150, 200):
        ref = o.replay_input(st, gid, m, target_step)
        got = lazy.sampled_input(targets, st, gid, m, target_step)
        assert np.array_equal(got, ref[targets]), target_step
        nonzero += int(np.count_nonzero(got))
    assert nonzero > 0


def test_sampled_input_rejects_unsorted_spikes():
    spec = specs()["brunel_normal"]
    lazy = O.OracleNet(spec, build=False)
    with pytest.raises(RuntimeError):
        lazy.sampled_input([0], np.array([5, 4]), np.array([1, 1]), np.array([1, 1]), 10)
