"""Pins of the oracle's connection rules (Sec. 2.1: fixed in-degree, fixed
out-degree, all-to-all, one-to-one, fixed total number): every synapse
recomputed from numpy's independent Philox by the stated counter layout,
the exact structural property of each rule, and uniformity of the drawn
indices (no GPU)."""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

from test_oracle_rng_tables import numpy_block

DT = 0.1
LIF = dict(tau_m=20.0, C_m=250.0, E_L=0.0, V_th=20.0, V_reset=10.0, t_ref=2.0)


def rules_spec(seed=5, sizes=(60, 45, 45), total=700, outdeg=9):
    pops = [dict(name=nm, model="lif_delta", n=n, ports=1, params=dict(LIF), V0=None, I_e=0.0)
            for nm, n in zip("ABC", sizes)]
    projs = [
        dict(src="A", tgt="B", rule="fixed_indegree", K=7, weight=0.2, delay=("uniform", 0.1, 1.0), port=0),
        dict(src="A", tgt="C", rule="fixed_outdegree", K=outdeg, weight=0.3, delay=("normal", 0.5, 0.2), port=0),
        dict(src="B", tgt="C", rule="all_to_all", weight=-0.1, delay=("uniform", 0.1, 2.0), port=0),
        dict(src="B", tgt="C", rule="one_to_one", weight=0.5, delay=("const", 0.3, 0.0), port=0),
        dict(src="C", tgt="A", rule="fixed_total_number", K=total, weight=-0.4, delay=("uniform", 0.2, 1.5), port=0),
    ]
    return dict(name="rules", dt=DT, seed=seed, dmax=20, populations=pops, projections=projs, poisson=[])


def ranges(spec):
    out, f = {}, 0
    for p in spec["populations"]:
        out[p["name"]] = (f, p["n"])
        f += p["n"]
    return out


def delay_of(thr, u32, dmax):
    return next(j for j in range(1, dmax + 1) if u32 < int(thr[j]))


def expected_synapses(spec):
    """(src, delay, tgt) of every synapse, from numpy's Philox and the
    counter layout of each rule."""
    rg = ranges(spec)
    key = [spec["seed"], 0]
    out = []
    for p, pr in enumerate(spec["projections"]):
        s0, sn = rg[pr["src"]]
        t0, tn = rg[pr["tgt"]]
        kind, a, b = pr["delay"]
        thr = O.delay_table(kind, a, b, DT, spec["dmax"])
        rule = pr["rule"]
        if rule in ("fixed_indegree", "fixed_outdegree", "all_to_all"):
            ents = range(t0, t0 + tn) if rule != "fixed_outdegree" else range(s0, s0 + sn)
            kn = sn if rule == "all_to_all" else pr["K"]
            for e in ents:
                for k in range(kn):
                    blk = numpy_block([e, (p << 40) | (k >> 1), 1, 0], key)
                    u, ud = int(blk[2 * (k & 1)]), int(blk[2 * (k & 1) + 1])
                    d = delay_of(thr, ud >> 32, spec["dmax"])
                    if rule == "fixed_indegree":
                        out.append((s0 + ((u * sn) >> 64), d, e))
                    elif rule == "fixed_outdegree":
                        out.append((e, d, t0 + ((u * tn) >> 64)))
                    else:
                        out.append((s0 + k, d, e))
        elif rule == "one_to_one":
            for i in range(tn):
                blk = numpy_block([t0 + i, p << 40, 1, 0], key)
                out.append((s0 + i, delay_of(thr, int(blk[1]) >> 32, spec["dmax"]), t0 + i))
        else:
            for j in range(pr["K"]):
                blk = numpy_block([j, p << 40, 1, 0], key)
                out.append((s0 + ((int(blk[0]) * sn) >> 64), delay_of(thr, int(blk[2]) >> 32, spec["dmax"]),
                            t0 + ((int(blk[1]) * tn) >> 64)))
    return sorted(out)


def test_every_rule_matches_numpy_philox_recomputation():
    spec = rules_spec()
    net = O.OracleNet(spec)
    syn = net.synapses()
    got = sorted(zip(syn["src"].tolist(), syn["delay"].tolist(), syn["tgt"].tolist()))
    assert got == expected_synapses(spec)


def test_rule_structure():
    spec = rules_spec(sizes=(300, 200, 200), total=20000, outdeg=40)
    net = O.OracleNet(spec)
    syn = net.synapses()
    rg = ranges(spec)
    src, tgt, w = syn["src"].astype(np.int64), syn["tgt"].astype(np.int64), syn["wq"]
    a0, an = rg["A"]
    b0, bn = rg["B"]
    c0, cn = rg["C"]

    def proj(sfirst, sn, tfirst, tn, sign):
        return (src >= sfirst) & (src < sfirst + sn) & (tgt >= tfirst) & (tgt < tfirst + tn) & (np.sign(w) == sign)

    # fixed in-degree A -> B: every target exactly 7
    m = proj(a0, an, b0, bn, 1)
    assert np.all(np.bincount(tgt[m] - b0, minlength=bn) == 7)
    # fixed out-degree A -> C: every source exactly 40, targets uniform
    m = proj(a0, an, c0, cn, 1) & (w == w[proj(a0, an, c0, cn, 1)].max())
    assert np.all(np.bincount(src[m] - a0, minlength=an) == 40)
    assert stats.chisquare(np.bincount(tgt[m] - c0, minlength=cn)).pvalue > 1e-4
    # all-to-all B -> C: every pair exactly once (weight -0.1)
    m = proj(b0, bn, c0, cn, -1) & (w == w[proj(b0, bn, c0, cn, -1)].max())
    pairs = np.unique((src[m] - b0) * cn + (tgt[m] - c0), return_counts=True)
    assert len(pairs[0]) == bn * cn and np.all(pairs[1] == 1)
    # one-to-one B -> C (weight 0.5, the largest positive one onto C)
    m = proj(b0, bn, c0, cn, 1) & (w == w[proj(b0, bn, c0, cn, 1)].max())
    assert np.array_equal(np.sort(src[m] - b0), np.arange(bn)) and np.all(src[m] - b0 == tgt[m] - c0)
    # fixed total number C -> A: exactly 20000, both ends uniform
    m = proj(c0, cn, a0, an, -1)
    assert m.sum() == 20000
    assert stats.chisquare(np.bincount(src[m] - c0, minlength=cn)).pvalue > 1e-4
    assert stats.chisquare(np.bincount(tgt[m] - a0, minlength=an)).pvalue > 1e-4
    assert len(src) == 200 * 7 + 300 * 40 + 200 * 200 + 200 + 20000


def test_delivery_with_every_rule_equals_replay():
    """The simulation's per-step input equals the plain replay of its own
    raster on a network using every rule (delivery is rule-independent)."""
    spec = rules_spec()
    for p in spec["populations"]:
        p["I_e"] = 600.0
        p["V0"] = np.linspace(0.0, 19.0, p["n"])
    o = O.OracleNet(spec, O.FP32SO)
    rec = o.record_input(121)
    o.simulate(121)
    st, gid, m = o.spikes()
    assert len(st) > 20
    for n in (30, 77, 120):
        assert np.array_equal(o.replay_input(st, gid, m, n)[:, 0], rec[n][:, 0])


def test_sampled_checks_refuse_rules_not_drawn_per_target():
    spec = rules_spec()
    lazy = O.OracleNet(spec, build=False)
    first_c = ranges(spec)["C"][0]
    with pytest.raises(RuntimeError):
        lazy.target_synapses(first_c)
    s, d, p, w = lazy.target_synapses(ranges(spec)["B"][0])  # only fixed in-degree onto B
    assert len(s) == 7


def test_bad_rules_rejected():
    spec = rules_spec()
    spec["projections"][3]["src"] = "A"  # one-to-one between populations of different sizes
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)


def list_projection(rng, n_total, count, dmax_ms):
    src = rng.integers(0, n_total, size=count)
    tgt = rng.integers(0, n_total, size=count)
    delays = np.round(rng.uniform(0.05, dmax_ms, size=count), 3)
    return dict(rule="list", src_gids=src.tolist(), tgt_gids=tgt.tolist(), delays_ms=delays.tolist(),
                weight=0.25, port=0)


def test_list_connections_are_the_listed_synapses():
    spec = rules_spec()
    rng = np.random.default_rng(12)
    n = sum(p["n"] for p in spec["populations"])
    lp = list_projection(rng, n, 500, 1.9)
    spec["projections"].append(lp)
    base = O.OracleNet(rules_spec()).synapses()
    syn = O.OracleNet(spec).synapses()
    triples = lambda t: sorted(zip(t["src"].tolist(), t["delay"].tolist(), t["tgt"].tolist()))
    steps = [max(1, int(np.floor(d / DT + 0.5))) for d in lp["delays_ms"]]
    listed = list(zip(lp["src_gids"], steps, lp["tgt_gids"]))
    assert triples(syn) == sorted(triples(base) + listed)


def test_list_errors():
    spec = rules_spec()
    spec["projections"].append(dict(rule="list", src_gids=[0], tgt_gids=[1], delays_ms=[2.5], weight=1.0, port=0))
    with pytest.raises(RuntimeError):  # 25 steps > Dmax 20
        O.OracleNet(spec)
    spec = rules_spec()
    spec["projections"].append(dict(rule="list", src_gids=[0], tgt_gids=[10**6], delays_ms=[0.5], weight=1.0, port=0))
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
