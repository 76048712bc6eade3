"""Pins of the oracle's counter-based generator, distribution tables,
fixed-point exponent and connectivity builder against numpy / scipy and
statistics (no GPU)."""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2007_14236_amd import workloads as W

TWO32 = 2**32


def numpy_block(ctr, key):
    """Philox4x64-10 block at counter `ctr` from numpy's independent
    implementation.  numpy advances its 256-bit counter by one before each
    block, so start from ctr - 1."""
    c = [int(x) for x in ctr]
    v = c[0] | (c[1] << 64) | (c[2] << 128) | (c[3] << 192)
    v = (v - 1) % (1 << 256)
    start = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=start, key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


def test_philox_known_answer():
    # numpy's documented default: key=1, counter=0 -> first block is counter (1,0,0,0)
    ref = np.random.Philox(key=1, counter=0).random_raw(4)
    got = O.philox4x64_10([1, 0, 0, 0], [1, 0])
    assert np.array_equal(ref, got)


def test_philox_matches_numpy_random_counters():
    rng = np.random.default_rng(5)
    for _ in range(200):
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        ctr[0] |= np.uint64(1)
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        assert np.array_equal(numpy_block(ctr, key), O.philox4x64_10(ctr, key))


@pytest.mark.parametrize("d0", [0.05, 0.1, 0.14, 0.16, 1.5, 2.0, 6.3, 9.0])
def test_const_delay_table(d0):
    dt, dmax = 0.1, 63
    thr = O.delay_table("const", d0, 0.0, dt, dmax)
    steps = max(1, min(dmax, int(np.floor(d0 / dt + 0.5))))
    for k in range(1, dmax + 1):
        assert thr[k] == (TWO32 if k >= steps else 0)


@pytest.mark.parametrize("kind,a,b", [("uniform", 1.0, 2.0), ("uniform", 0.1, 3.0),
                                      ("normal", 1.5, 0.75), ("normal", 0.75, 0.375)])
def test_delay_table_vs_scipy_cdf(kind, a, b):
    dt, dmax = 0.1, 63
    thr = O.delay_table(kind, a, b, dt, dmax)
    dist = stats.uniform(loc=a, scale=b - a) if kind == "uniform" else stats.norm(loc=a, scale=b)
    assert thr[dmax] == TWO32
    assert np.all(np.diff(thr[1:].astype(np.int64)) >= 0)
    for k in range(1, dmax):
        ref = dist.cdf((k + 0.5) * dt) * TWO32
        assert abs(float(thr[k]) - ref) <= 2.0, (k, thr[k], ref)


@pytest.mark.parametrize("lam", [0.0, 0.016, 0.16, 2.0, 9.6, 40.0])
def test_poisson_table_vs_scipy(lam):
    thr = O.poisson_table(lam)
    assert thr[-1] == TWO32
    for k in range(len(thr) - 1):
        ref = min(stats.poisson(lam).cdf(k) * TWO32, TWO32) if lam > 0 else TWO32
        assert abs(float(thr[k]) - ref) <= 2.0, (k, thr[k], ref)


@pytest.mark.parametrize("w", [0.1, 0.5, 1.0, 0.37, 87.8, 351.2, 2.0**-40, 3e5])
def test_fixed_point_shift_is_largest(w):
    s = O.fixed_point_shift(w)
    # brute force with exact rational arithmetic on the double value
    from fractions import Fraction
    fw = Fraction(w)
    assert fw * Fraction(2) ** s < 2**30
    assert not (fw * Fraction(2) ** (s + 1) < 2**30)


def tiny_spec(n=40, k=7, seed=3, delay=("uniform", 0.1, 0.8), dmax=8, ports=1):
    spec = W.brunel_lif(n=n, k=k, seed=seed, delay=delay, dmax=dmax)
    return spec


def test_connectivity_matches_numpy_philox_recomputation():
    """Every synapse (target t, projection p, draw k) recomputed with numpy's
    Philox: source = first + floor(u * n_src / 2^64), delay by the table."""
    spec = W.brunel_lif(n=100, k=13, seed=9, delay=("normal", 0.4, 0.2), dmax=8)
    net = O.OracleNet(spec)
    syn = net.synapses()
    got = sorted(zip(syn["src"].tolist(), syn["delay"].tolist(), syn["tgt"].tolist()))
    rng = W.population_ranges(spec)
    expect = []
    for p, pr in enumerate(spec["projections"]):
        s0, sn = rng[pr["src"]]
        t0, tn = rng[pr["tgt"]]
        kind, a, b = pr["delay"]
        thr = O.delay_table(kind, a, b, spec["dt"], spec["dmax"])
        for t in range(t0, t0 + tn):
            for k in range(pr["K"]):
                blk = numpy_block([t, (p << 40) | (k >> 1), 1, 0], [spec["seed"], 0])
                us, ud = int(blk[2 * (k & 1)]), int(blk[2 * (k & 1) + 1])
                s = s0 + ((us * sn) >> 64)
                u32 = ud >> 32
                d = next(j for j in range(1, spec["dmax"] + 1) if u32 < int(thr[j]))
                expect.append((s, d, t))
    assert got == sorted(expect)


def test_connectivity_invariants_and_statistics():
    spec = W.brunel_lif(n=2000, k=200, seed=4, delay=("uniform", 0.1, 3.0), dmax=63)
    net = O.OracleNet(spec)
    syn = net.synapses()
    rng = W.population_ranges(spec)
    # canonical order
    key = (syn["src"].astype(np.int64) << 40) | (syn["delay"].astype(np.int64) << 32) | syn["tgt"]
    assert np.all(np.diff(key) >= 0)
    # exact in-degree per (projection source population, target)
    e0, en = rng["E"]
    from_e = (syn["src"] >= e0) & (syn["src"] < e0 + en)
    indeg_e = np.bincount(syn["tgt"][from_e], minlength=2000)
    indeg_i = np.bincount(syn["tgt"][~from_e], minlength=2000)
    assert np.all(indeg_e == 160) and np.all(indeg_i == 40)
    # source uniformity within E (chi-square)
    cnt = np.bincount(syn["src"][from_e] - e0, minlength=en)
    chi = stats.chisquare(cnt)
    assert chi.pvalue > 1e-4
    # delay histogram vs the table's probabilities
    thr = O.delay_table("uniform", 0.1, 3.0, 0.1, 63).astype(np.float64)
    pmf = np.diff(thr) / TWO32
    hist = np.bincount(syn["delay"], minlength=64)[1:]
    keep = pmf > 0
    assert hist[~keep].sum() == 0
    chi = stats.chisquare(hist[keep], pmf[keep] * hist.sum())
    assert chi.pvalue > 1e-4
    # quantised weights
    s = net.shift_of(0)
    wq_e = int(np.rint(0.1 * 2.0**s))
    assert set(np.unique(syn["wq"][from_e]).tolist()) == {wq_e}


def test_poisson_counts_statistics():
    spec = W.brunel_lif(n=200, k=10, seed=2, nu_ext=250.0, c_ext=80)
    net = O.OracleNet(spec)
    lam = 80 * 250.0 * 0.1e-3
    ks = np.array([net.poisson_count(g, n) for g in range(0, 200, 7) for n in range(300)])
    vals, cnt = np.unique(ks, return_counts=True)
    kmax = 12
    obs = np.array([np.sum(ks == k) for k in range(kmax)] + [np.sum(ks >= kmax)])
    pm = np.array([stats.poisson(lam).pmf(k) for k in range(kmax)] + [stats.poisson(lam).sf(kmax - 1)])
    assert stats.chisquare(obs, pm * len(ks)).pvalue > 1e-4
    # the count is a pure function of (seed, gid, step)
    assert net.poisson_count(5, 17) == net.poisson_count(5, 17)
