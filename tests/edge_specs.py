"""Degenerate and boundary networks shared by the oracle's and the GPU's
edge-case tests: specifications only (no arithmetic of the method)."""
import numpy as np

from paper_2007_14236_amd import workloads as W


def edge_specs() -> dict:
    out = {}
    # no synapses at all: Poisson drive only (empty connection table)
    sp = W.brunel_lif(n=300, k=10, seed=4, nu_ext=400.0)
    sp["projections"] = []
    out["no_synapses"] = sp
    # silent: no drive, every neuron below threshold (no spike, no event)
    sp = W.brunel_lif(n=200, k=20, seed=5)
    sp["poisson"] = []
    for p in sp["populations"]:
        p["V0"] = np.linspace(0.0, 19.0, p["n"])
    out["silent"] = sp
    # one neuron onto itself (autapse), driven over threshold, every delay at Dmax = 63
    lif = dict(tau_m=20.0, C_m=250.0, E_L=0.0, V_th=20.0, V_reset=10.0, t_ref=2.0)
    out["one_neuron_max_delay"] = dict(
        name="one", dt=0.1, seed=3, dmax=63,
        populations=[dict(name="A", model="lif_delta", n=1, ports=1, params=dict(lif), V0=[5.0], I_e=400.0)],
        projections=[dict(src="A", tgt="A", rule="fixed_indegree", K=3, weight=2.0, delay=("const", 6.3, 0.0),
                          port=0)],
        poisson=[])
    # empty pieces: in-degree 0, an empty list, a fixed total of 0, beside one real projection;
    # 257 neurons (one past a full 256-neuron block)
    sp = W.brunel_lif(n=257, k=25, seed=6, nu_ext=300.0)
    sp["projections"] += [dict(src="E", tgt="I", K=0, weight=0.3, delay=("const", 1.0, 0.0), port=0),
                          dict(rule="list", src_gids=[], tgt_gids=[], delays_ms=[], weight=0.2, port=0),
                          dict(src="I", tgt="E", rule="fixed_total_number", K=0, weight=-0.2,
                               delay=("uniform", 0.1, 1.0), port=0)]
    out["empty_projections_257"] = sp
    return out
