"""Pins of the oracle's per-neuron model parameters (Sec. 2.1: neuron
parameters set from arrays or drawn from probability distributions):

- LIF neurons with their own membrane time constant, capacitance,
  threshold, reset and refractory time, driven by their own constant
  current, each fire at the closed-form constant-current inter-spike
  interval of their own parameters (fp64 and fp32 modes);
- AdEx neurons with their own leak, adaptation and reversal parameters each
  settle at the fixed point brentq finds for their own parameters;
- drawn parameters equal numpy's independent Philox recomputation through
  scipy's bin thresholds, and a neuron with drawn parameters behaves exactly
  as one given those values as an array.
No GPU."""
import numpy as np
import pytest
from scipy import optimize

from oracle import oracle as O
from test_oracle_rng_tables import numpy_block
from test_oracle_weights import thresholds

DT = 0.1


def lif_spec(model, n, params, I_e, seed=3):
    return dict(name="het", dt=DT, seed=seed, dmax=4, projections=[], poisson=[],
                populations=[dict(name="A", model=model, n=n, ports=1, params=params, I_e=I_e)])


def grid_isi(tau_m, C, I_e, theta, y_r, n_ref):
    """Relaxation from y_r towards tau_m I_e / C crosses theta after
    T = tau_m ln((y_inf - y_r)/(y_inf - theta)); on the grid the neuron fires
    at the first whole step at or after T, then stays n_ref steps at reset."""
    y_inf = tau_m * I_e / C
    T = tau_m * np.log((y_inf - y_r) / (y_inf - theta))
    return n_ref + int(np.ceil(T / DT)), T / DT


@pytest.mark.parametrize("model", ["lif_exp", "lif_delta"])
@pytest.mark.parametrize("mode", [O.FP64, O.FP32SO])
def test_lif_per_neuron_isi_closed_form(model, mode):
    rng = np.random.default_rng(11)
    n = 24
    tau_m = rng.uniform(5.0, 25.0, n)
    C = rng.uniform(100.0, 400.0, n)
    E_L = rng.uniform(-75.0, -60.0, n)
    V_th = E_L + rng.uniform(10.0, 20.0, n)
    V_reset = E_L + rng.uniform(-5.0, 2.0, n)
    t_ref = rng.choice([0.0, 0.5, 2.0, 3.3], n)
    y_inf = V_th - E_L + rng.uniform(2.0, 30.0, n)  # above threshold: repetitive firing
    I_e = y_inf * C / tau_m
    params = dict(tau_m=tau_m, C_m=C, E_L=E_L, V_th=V_th, V_reset=V_reset, t_ref=t_ref, tau_syn=[0.5])
    spec = lif_spec(model, n, params, I_e)
    spec["populations"][0]["V0"] = V_reset  # start at reset, not refractory
    o = O.OracleNet(spec, mode)
    o.simulate(3000)
    st, gid, _ = o.spikes()
    checked = 0
    for i in range(n):
        n_ref = int(np.floor(t_ref[i] / DT + 0.5))
        steps, frac = grid_isi(tau_m[i], C[i], I_e[i], V_th[i] - E_L[i], V_reset[i] - E_L[i], n_ref)
        if abs(frac - round(frac)) < 1e-3:
            continue  # crossing too close to a grid point for the rounding of either mode
        s = st[gid == i].astype(np.int64)
        assert len(s) >= 3
        assert s[0] + 1 == steps - n_ref, i  # from reset without a refractory period in front
        assert np.all(np.diff(s) == steps), i
        checked += 1
    assert checked >= n - 3


def test_adex_per_neuron_fixed_points_brentq():
    T2 = dict(C_m=281.0, g_L=30.0, E_L=-70.6, V_T=-50.4, Delta_T=2.0, tau_w=144.0, a=4.0, b=80.5,
              V_r=-60.0, V_peak=0.0, t_ref=0.0, rk_eps=1e-6, tau_syn=[1.0, 1.0], E_rev=[0.0, -85.0])
    n = 6
    g_L = np.array([20.0, 25.0, 30.0, 35.0, 40.0, 30.0])
    E_L = np.array([-72.0, -70.6, -68.0, -71.0, -69.5, -65.0])
    a = np.array([2.0, 4.0, 6.0, 1.0, 8.0, 0.0])
    tau_w = np.array([100.0, 144.0, 200.0, 80.0, 300.0, 150.0])
    I_e = np.array([100.0, 150.0, 120.0, 80.0, 200.0, 60.0])
    params = dict(T2, g_L=g_L, E_L=E_L, a=a, tau_w=tau_w)
    spec = dict(name="adex_het", dt=DT, seed=1, dmax=4, projections=[], poisson=[],
                populations=[dict(name="A", model="aeif_cond_exp", n=n, ports=2, params=params, I_e=I_e)])
    o = O.OracleNet(spec, O.FP64)
    o.simulate(40000)  # 4 s, many adaptation time constants
    assert len(o.spikes()[0]) == 0
    V, w = o.get_state("V_m"), o.get_state("w")
    for i in range(n):
        f = lambda v: (-g_L[i] * (v - E_L[i]) + g_L[i] * T2["Delta_T"] * np.exp((v - T2["V_T"]) / T2["Delta_T"])
                       - a[i] * (v - E_L[i]) + I_e[i])
        Vs = optimize.brentq(f, E_L[i] - 20.0, T2["V_T"])
        assert V[i] == pytest.approx(Vs, abs=2e-4), i
        assert w[i] == pytest.approx(a[i] * (Vs - E_L[i]), abs=2e-3), i
    # every neuron at its own rest: the parameters are applied per neuron
    assert len(np.unique(np.round(V, 3))) == n


def test_param_distribution_matches_numpy_philox_and_scipy_bins():
    n = 3000
    spec = lif_spec("lif_delta", n, dict(tau_m=20.0, C_m=250.0, E_L=0.0, V_th=20.0, V_reset=10.0, t_ref=2.0),
                    0.0, seed=9)
    spec["populations"][0]["param_dists"] = {
        "V_th": dict(kind="normal", mean=20.0, sd=1.0, low=18.0, high=22.0, levels=256),
        "tau_m": dict(kind="uniform", low=15.0, high=25.0, levels=64)}
    o = O.OracleNet(spec)
    key = [spec["seed"], 0]
    for name, pid in (("V_th", 3), ("tau_m", 0)):
        wd = spec["populations"][0]["param_dists"][name]
        L = wd["levels"]
        if wd["kind"] == "uniform":
            thr, lo, hi = thresholds("uniform", wd["low"], wd["high"], 0, 0, L)
        else:
            thr, lo, hi = thresholds("normal", wd["mean"], wd["sd"], wd["low"], wd["high"], L)
        levels = lo + (hi - lo) * ((np.arange(L) + 0.5) / L)
        got = o.get_param(name)
        for i in range(0, n, 7):
            u = int(numpy_block([i, pid << 8, 5, 0], key)[0]) >> 32
            assert got[i] == levels[int(np.argmax(u < thr))], (name, i)
        assert lo <= got.min() and got.max() <= hi
    # other parameters keep the population's value
    assert np.all(o.get_param("V_reset") == 10.0) and np.all(o.get_param("C_m") == 250.0)


def test_drawn_parameters_act_like_arrays():
    """A network whose V_th and tau_m are drawn simulates exactly as the same
    network given the drawn values as arrays (Poisson-driven, recurrent)."""
    from paper_2007_14236_amd import workloads as W
    spec = W.brunel_lif(n=300, k=30, nu_ext=250.0, seed=4, delay=("uniform", 0.1, 2.0), dmax=25)
    for p in spec["populations"]:
        p["param_dists"] = {"V_th": dict(kind="uniform", low=19.0, high=21.0, levels=128),
                            "t_ref": dict(kind="uniform", low=1.0, high=3.0, levels=8)}
    a = O.OracleNet(spec, O.FP32SO)
    arr = W.brunel_lif(n=300, k=30, nu_ext=250.0, seed=4, delay=("uniform", 0.1, 2.0), dmax=25)
    for p in arr["populations"]:
        t0, tn = a.ranges[p["name"]]
        p["params"]["V_th"] = a.get_param("V_th", t0, tn)
        p["params"]["t_ref"] = a.get_param("t_ref", t0, tn)
    b = O.OracleNet(arr, O.FP32SO)
    assert len(np.unique(a.get_param("V_th"))) > 50
    a.simulate(500)
    b.simulate(500)
    for x, y in zip(a.spikes(), b.spikes()):
        assert np.array_equal(x, y)
    assert len(a.spikes()[0]) > 100
    assert np.array_equal(a.get_state("V_m"), b.get_state("V_m"))


def test_per_neuron_parameters_after_state_refused():
    import ctypes as C
    spec = lif_spec("lif_delta", 10, dict(tau_m=20.0, C_m=250.0, E_L=0.0, V_th=20.0, V_reset=10.0, t_ref=2.0), 0.0)
    o = O.OracleNet(spec)
    v = np.full(10, 19.0)
    assert o.L.orc_set_param(o.h, 0, 10, 3, v.ctypes.data_as(C.POINTER(C.c_double))) != 0
