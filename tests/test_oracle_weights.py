"""Pins of the oracle's weight distributions and per-connection weights
(Sec. 2.1: weights fixed, from arrays, or from probability distributions).
Every drawn weight is recomputed from numpy's independent Philox by the
stated counter layout, with the bin probabilities from scipy's normal
distribution; the drawn levels follow the distribution (chi-square), stay in
the truncation range and average to the truncated-normal mean; listed
weights arrive as listed; delivery with them equals the plain replay; the
invalid set-ups are refused (no GPU)."""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

from test_oracle_rng_tables import numpy_block
from test_oracle_rules import ranges, rules_spec

DT = 0.1


def thresholds(kind, a, b, lo, hi, L):
    """bin edges' probabilities under the distribution restricted to
    [lo, hi], from scipy, as 32-bit thresholds"""
    if kind == "uniform":
        lo, hi = a, b
        cdf = lambda x: (x - a) / (b - a)
    else:
        cdf = lambda x: stats.norm.cdf(x, loc=a, scale=b)
    edges = lo + (hi - lo) * (np.arange(1, L) / L)
    q = (cdf(edges) - cdf(lo)) / (cdf(hi) - cdf(lo))
    return np.append(np.floor(q * 2.0**32), 2.0**32), lo, hi


def spec_with_weights(seed=5, L_normal=32, L_uniform=8, low=None):
    spec = rules_spec(seed=seed)
    wd = dict(kind="normal", mean=0.2, sd=0.05, levels=L_normal)
    if low is not None:
        wd["low"] = low
    spec["projections"][0]["weight_dist"] = wd                                  # fixed in-degree A -> B
    spec["projections"][1]["weight_dist"] = dict(kind="uniform", low=0.1, high=0.5, levels=L_uniform)  # out-degree
    spec["projections"][4]["weight_dist"] = dict(kind="normal", mean=-0.4, sd=0.1, levels=16)  # fixed total C -> A
    return spec


def expected_weights(spec, net):
    """(src, delay, tgt, w_q) of every synapse of the projections with a
    weight distribution, recomputed from numpy's Philox"""
    rg = ranges(spec)
    key = [spec["seed"], 0]
    out = []
    for p, pr in enumerate(spec["projections"]):
        wd = pr.get("weight_dist")
        if wd is None:
            continue
        L = wd["levels"]
        if wd["kind"] == "uniform":
            thr, lo, hi = thresholds("uniform", wd["low"], wd["high"], 0, 0, L)
        else:
            m, sd = wd["mean"], wd["sd"]
            thr, lo, hi = thresholds("normal", m, sd, wd.get("low", m - 4 * sd), wd.get("high", m + 4 * sd), L)
        levels = lo + (hi - lo) * ((np.arange(L) + 0.5) / L)
        s0, sn = rg[pr["src"]]
        t0, tn = rg[pr["tgt"]]
        dthr = O.delay_table(*pr["delay"], DT, spec["dmax"])
        delay = lambda u32: next(j for j in range(1, spec["dmax"] + 1) if u32 < int(dthr[j]))

        def level(e, k):
            blk = numpy_block([e, (p << 40) | (k >> 2), 3, 0], key)
            u = int(blk[k & 3]) >> 32
            return int(np.argmax(u < thr))

        if pr["rule"] in ("fixed_indegree", "fixed_outdegree"):
            ents = range(t0, t0 + tn) if pr["rule"] == "fixed_indegree" else range(s0, s0 + sn)
            for e in ents:
                for k in range(pr["K"]):
                    c = numpy_block([e, (p << 40) | (k >> 1), 1, 0], key)
                    u, d = int(c[2 * (k & 1)]), delay(int(c[2 * (k & 1) + 1]) >> 32)
                    if pr["rule"] == "fixed_indegree":
                        s, t = s0 + ((u * sn) >> 64), e
                    else:
                        s, t = e, t0 + ((u * tn) >> 64)
                    out.append((s, d, t, int(np.rint(np.ldexp(levels[level(e, k)], net.shift_of(t, pr["port"]))))))
        else:  # fixed total number
            for j in range(pr["K"]):
                c = numpy_block([j, p << 40, 1, 0], key)
                s, t = s0 + ((int(c[0]) * sn) >> 64), t0 + ((int(c[1]) * tn) >> 64)
                d = delay(int(c[2]) >> 32)
                out.append((s, d, t, int(np.rint(np.ldexp(levels[level(j, 0)], net.shift_of(t, pr["port"]))))))
    return sorted(out)


def table(net):
    syn = net.synapses()
    return syn["src"].astype(np.int64), syn["delay"].astype(np.int64), syn["tgt"].astype(np.int64), syn["wq"]


def test_drawn_weights_match_numpy_philox_and_scipy_bins():
    spec = spec_with_weights()
    net = O.OracleNet(spec)
    src, d, tgt, wq = table(net)
    # the distributed projections: weights other than the fixed ones
    fixed = {int(np.rint(np.ldexp(pr["weight"], net.shift_of(ranges(spec)[pr["tgt"]][0], 0))))
             for pr in spec["projections"] if "weight_dist" not in pr}
    exp = expected_weights(spec, net)
    got = sorted((int(a), int(b), int(c), int(w)) for a, b, c, w in zip(src, d, tgt, wq))
    # every expected synapse is in the table, and the rest carry fixed weights
    from collections import Counter
    rest = Counter(got) - Counter(exp)
    assert sum((Counter(exp) - Counter(got)).values()) == 0
    assert all(w in fixed for (_, _, _, w) in rest.elements())
    assert sum(rest.values()) == len(got) - len(exp)


def levels_of(net, spec, p):
    """weights (in the spec's units) of projection p's synapses"""
    rg = ranges(spec)
    pr = spec["projections"][p]
    src, d, tgt, wq = table(net)
    s0, sn = rg[pr["src"]]
    t0, tn = rg[pr["tgt"]]
    S = net.shift_of(t0, pr["port"])
    m = (src >= s0) & (src < s0 + sn) & (tgt >= t0) & (tgt < t0 + tn)
    return wq[m] / 2.0**S, m


def test_level_frequencies_follow_the_distribution():
    spec = rules_spec(sizes=(400, 300, 300))
    spec["projections"] = [dict(src="A", tgt="B", rule="fixed_indegree", K=200, weight=0.0, port=0,
                                delay=("uniform", 0.1, 1.0),
                                weight_dist=dict(kind="normal", mean=0.2, sd=0.05, low=0.1, high=0.35, levels=20)),
                           dict(src="A", tgt="C", rule="fixed_indegree", K=200, weight=0.0, port=0,
                                delay=("uniform", 0.1, 1.0),
                                weight_dist=dict(kind="uniform", low=-0.3, high=0.5, levels=16))]
    net = O.OracleNet(spec)
    # normal truncated to [0.1, 0.35]: 20 bins of 0.0125, midpoints
    w, _ = levels_of(net, spec, 0)
    assert w.size == 300 * 200
    assert w.min() >= 0.1 and w.max() <= 0.35
    edges = 0.1 + 0.0125 * np.arange(21)
    j = np.clip(np.floor((w - 0.1) / 0.0125).astype(int), 0, 19)
    assert np.allclose(w, 0.1 + 0.0125 * (j + 0.5), atol=1e-6)
    tn = stats.truncnorm((0.1 - 0.2) / 0.05, (0.35 - 0.2) / 0.05, loc=0.2, scale=0.05)
    p = np.diff(tn.cdf(edges))
    assert stats.chisquare(np.bincount(j, minlength=20), p * w.size).pvalue > 1e-4
    # mean within sampling error plus the binning's shift of the mean
    assert abs(w.mean() - tn.mean()) < 5 * tn.std() / np.sqrt(w.size) + 0.0125 ** 2
    # uniform on [-0.3, 0.5): 16 equally likely midpoints, signs preserved
    w, _ = levels_of(net, spec, 1)
    j = np.rint((w + 0.3) / 0.05 - 0.5).astype(int)
    assert np.allclose(w, -0.3 + 0.05 * (j + 0.5), atol=1e-6)
    assert stats.chisquare(np.bincount(j, minlength=16)).pvalue > 1e-4
    assert (w < 0).any() and (w > 0).any()


def test_listed_weights_arrive_as_listed():
    spec = rules_spec()
    rng = np.random.default_rng(7)
    n = sum(p["n"] for p in spec["populations"])
    cnt = 400
    lw = np.round(rng.choice([-0.5, 0.125, 0.3, 0.75, 1.1], size=cnt), 3)
    spec["projections"] = [dict(rule="list", src_gids=rng.integers(0, n, cnt).tolist(),
                                tgt_gids=rng.integers(0, n, cnt).tolist(),
                                delays_ms=np.round(rng.uniform(0.05, 1.9, cnt), 3).tolist(),
                                weights=lw.tolist(), weight=0.0, port=0)]
    net = O.OracleNet(spec)
    src, d, tgt, wq = table(net)
    steps = [max(1, int(np.floor(x / DT + 0.5))) for x in spec["projections"][0]["delays_ms"]]
    exp = sorted((s, dd, t, int(np.rint(np.ldexp(w, net.shift_of(t, 0)))))
                 for s, dd, t, w in zip(spec["projections"][0]["src_gids"], steps,
                                        spec["projections"][0]["tgt_gids"], lw))
    got = sorted((int(a), int(b), int(c), int(w)) for a, b, c, w in zip(src, d, tgt, wq))
    assert got == exp
    # the largest listed magnitude sets the fixed-point exponent: 1.1 2^S < 2^30
    S = net.shift_of(0, 0)
    assert 1.1 * 2.0**S < 2**30 <= 1.1 * 2.0**(S + 1)


def test_delivery_with_distributed_weights_equals_replay():
    spec = spec_with_weights()
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


def test_sampled_target_synapses_carry_the_drawn_weights():
    spec = spec_with_weights()
    spec["projections"] = spec["projections"][:1]  # fixed in-degree A -> B with normal weights
    net = O.OracleNet(spec)
    src, d, tgt, wq = table(net)
    lazy = O.OracleNet(spec, build=False)
    for t in range(60, 105, 11):
        s, dd, p, w = lazy.target_synapses(t)
        m = tgt == t
        assert sorted(zip(s.tolist(), dd.tolist(), w.tolist())) == \
            sorted(zip(src[m].tolist(), d[m].tolist(), wq[m].tolist()))


def test_weight_distribution_errors():
    spec = spec_with_weights()
    spec["projections"][0]["weight_dist"]["levels"] = 0
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
    spec = spec_with_weights()
    spec["projections"][0]["weight_dist"]["levels"] = 2000
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
    spec = spec_with_weights()
    spec["projections"][1]["weight_dist"] = dict(kind="uniform", low=0.5, high=0.5)
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
    spec = spec_with_weights()
    spec["projections"][0]["weight_dist"] = dict(kind="normal", mean=0.0, sd=1.0, low=50.0, high=60.0)
    with pytest.raises(RuntimeError):  # no probability in [lo, hi] at double precision
        O.OracleNet(spec)
    # conductances cannot take negative levels
    from paper_2007_14236_amd import workloads as W
    sp = dict(name="adex", dt=0.1, seed=1, dmax=20, poisson=[],
              populations=[dict(name="A", model="aeif_cond_exp", n=20, ports=2, params=dict(W.ADEX_T2))],
              projections=[dict(src="A", tgt="A", rule="fixed_indegree", K=5, weight=0.0, port=0,
                                delay=("uniform", 1.0, 2.0), weight_dist=dict(kind="normal", mean=0.1, sd=0.1))])
    with pytest.raises(RuntimeError):
        O.OracleNet(sp)
    sp["projections"][0]["weight_dist"]["low"] = 0.0
    w, _ = levels_of(O.OracleNet(sp), sp, 0)
    assert w.min() > 0


def state_spec():
    from paper_2007_14236_amd import workloads as W
    spec = W.brunel_lif(n=2000, k=20, seed=3)
    for p in spec["populations"]:
        p["state_dists"] = {"V_m": dict(kind="uniform", low=0.0, high=20.0, levels=4096),
                            "I_e": dict(kind="normal", mean=100.0, sd=30.0, low=0.0, high=250.0, levels=500)}
    return spec


def test_state_distributions_match_numpy_philox_and_scipy_bins():
    spec = state_spec()
    o = O.OracleNet(spec)
    key = [spec["seed"], 0]
    for var, vid in (("V_m", 0), ("I_e", 1)):
        wd = spec["populations"][0]["state_dists"][var]
        L = wd["levels"]
        if wd["kind"] == "uniform":
            thr, lo, hi = thresholds("uniform", wd["low"], wd["high"], 0, 0, L)
        else:
            thr, lo, hi = thresholds("normal", wd["mean"], wd["sd"], wd["low"], wd["high"], L)
        levels = lo + (hi - lo) * ((np.arange(L) + 0.5) / L)
        got = o.get_state(var)
        for i in range(0, 2000, 7):
            u = int(numpy_block([i, vid << 8, 4, 0], key)[0]) >> 32
            assert got[i] == levels[int(np.argmax(u < thr))], (var, i)
    # frequencies: V uniform over 4096 bins in 16 groups; I_e against scipy's truncated normal
    v = o.get_state("V_m")
    assert stats.chisquare(np.bincount(np.floor(v / 1.25).astype(int), minlength=16)).pvalue > 1e-4
    ie = o.get_state("I_e")
    tn = stats.truncnorm(-100.0 / 30.0, 150.0 / 30.0, loc=100.0, scale=30.0)
    assert abs(ie.mean() - tn.mean()) < 5 * tn.std() / np.sqrt(ie.size) + 0.5 ** 2
    assert ie.min() >= 0.0 and ie.max() <= 250.0


def test_state_distribution_overrides_arrays_and_errors():
    spec = state_spec()
    o = O.OracleNet(spec)
    base = state_spec()
    for p in base["populations"]:
        p.pop("state_dists")
    ob = O.OracleNet(base)
    assert not np.array_equal(o.get_state("V_m"), ob.get_state("V_m"))  # drawn values replaced V0
    spec = state_spec()
    spec["populations"][0]["state_dists"]["V_m"]["levels"] = 0
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
