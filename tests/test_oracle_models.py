"""Pins of the oracle's neuron updates: LIF propagators against the matrix
exponential, the constant-current inter-spike interval closed form, the
Cash-Karp tableau order conditions, and the AdEx integrator against exact and
library solutions (no GPU)."""
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate, linalg, optimize

from oracle import oracle as O

DT = 0.1


def lif_params(model="lif_exp", tau_m=10.0, C_m=250.0, tau_syn=(0.5,), E_L=-65.0, V_th=-50.0,
               V_reset=-65.0, t_ref=2.0):
    return O.pop_params(model, len(tau_syn), dict(tau_m=tau_m, C_m=C_m, E_L=E_L, V_th=V_th,
                                                  V_reset=V_reset, t_ref=t_ref, tau_syn=list(tau_syn)))


@pytest.mark.parametrize("tau_m,tau_s,C", [(10.0, 0.5, 250.0), (20.0, 2.0, 100.0), (10.0, 10.0, 250.0),
                                           (5.0, 7.0, 40.0)])
def test_lif_propagators_vs_expm(tau_m, tau_s, C):
    """State (y, I, I_e): dy/dt = -y/tau_m + (I + I_e)/C, dI/dt = -I/tau_s,
    dI_e/dt = 0.  expm(A dt) gives every propagator."""
    p = lif_params(tau_m=tau_m, C_m=C, tau_syn=(tau_s,))
    pr = O.lif_propagators(p, DT)
    A = np.array([[-1 / tau_m, 1 / C, 1 / C], [0, -1 / tau_s, 0], [0, 0, 0]])
    M = linalg.expm(A * DT)
    P22, P20, P11, P21 = pr[0], pr[1], pr[2], pr[3]
    assert P22 == pytest.approx(M[0, 0], rel=1e-13)
    assert P21 == pytest.approx(M[0, 1], rel=1e-9)
    assert P20 == pytest.approx(M[0, 2], rel=1e-12)
    assert P11 == pytest.approx(M[1, 1], rel=1e-13)


def grid_isi_steps(tau_m, C, I_e, theta, y_r, n_ref, dt=DT):
    """Closed form: after the refractory steps the membrane relaxes from y_r
    towards y_inf = tau_m I_e / C; the continuous crossing time is
    T = tau_m ln((y_inf - y_r)/(y_inf - theta)), reached on the grid at the
    first whole step j >= T/dt."""
    y_inf = tau_m * I_e / C
    T = tau_m * np.log((y_inf - y_r) / (y_inf - theta))
    return n_ref + int(np.ceil(T / dt)), T / dt


@pytest.mark.parametrize("model", ["lif_exp", "lif_delta"])
@pytest.mark.parametrize("I_e", [400.0, 455.0, 620.0, 1000.0, 3000.0])
@pytest.mark.parametrize("fp32", [False, True])
def test_lif_constant_current_isi(model, I_e, fp32):
    tau_m, C = 10.0, 250.0
    p = lif_params(model=model, tau_m=tau_m, C_m=C, tau_syn=(0.5,))
    theta, y_r, n_ref = 15.0, 0.0, 20
    expect, frac = grid_isi_steps(tau_m, C, I_e, theta, y_r, n_ref)
    if abs(frac - round(frac)) < 1e-3:
        pytest.skip("crossing too close to a grid point")
    import ctypes as Cc
    L = O.lib()
    if fp32:
        y = Cc.c_float(0.0); I = (Cc.c_float * 1)(0.0); x = (Cc.c_float * 1)(0.0)
    else:
        y = Cc.c_double(0.0); I = (Cc.c_double * 1)(0.0); x = (Cc.c_double * 1)(0.0)
    r = Cc.c_int32(0)
    spikes = []
    for n in range(4000):
        if model == "lif_exp":
            f = L.orc_lif_exp_step32 if fp32 else L.orc_lif_exp_step64
            s = f(Cc.byref(p), DT, Cc.byref(y), I, Cc.byref(r), I_e, x)
        else:
            f = L.orc_lif_delta_step32 if fp32 else L.orc_lif_delta_step64
            s = f(Cc.byref(p), DT, Cc.byref(y), Cc.byref(r), I_e, 0.0)
        if s:
            spikes.append(n)
    isis = np.diff(spikes)
    assert len(isis) >= 3
    # first spike from rest has no refractory period in front of it
    assert spikes[0] + 1 == expect - n_ref
    assert np.all(isis == expect)


def test_lif_delta_input_dropped_while_refractory():
    p = lif_params(model="lif_delta", tau_m=20.0, E_L=0.0, V_th=20.0, V_reset=10.0, tau_syn=(1.0,))
    import ctypes as Cc
    L = O.lib()
    y = Cc.c_double(19.99); r = Cc.c_int32(0)
    assert L.orc_lif_delta_step64(Cc.byref(p), DT, Cc.byref(y), Cc.byref(r), 0.0, 5.0) == 1
    assert y.value == 10.0 and r.value == 20
    for _ in range(20):  # held at V_reset and deaf for 20 steps
        assert L.orc_lif_delta_step64(Cc.byref(p), DT, Cc.byref(y), Cc.byref(r), 0.0, 50.0) == 0
        assert y.value == 10.0
    assert r.value == 0
    L.orc_lif_delta_step64(Cc.byref(p), DT, Cc.byref(y), Cc.byref(r), 0.0, 1.0)
    assert y.value == pytest.approx(10.0 * np.exp(-DT / 20.0) + 1.0, rel=1e-15)


# ----------------------------------------------------------------- Cash-Karp
def _frac(v):
    return Fraction(v).limit_denominator(1 << 20)


def order_conditions(A, b, c, order):
    """Butcher rooted-tree conditions up to `order` (1 + 1 + 2 + 4 + 9)."""
    s = len(b)
    ac = [sum(A[i][j] * c[j] for j in range(s)) for i in range(s)]
    ac2 = [sum(A[i][j] * c[j] ** 2 for j in range(s)) for i in range(s)]
    ac3 = [sum(A[i][j] * c[j] ** 3 for j in range(s)) for i in range(s)]
    aac = [sum(A[i][j] * ac[j] for j in range(s)) for i in range(s)]
    cac = [c[i] * ac[i] for i in range(s)]
    acac = [sum(A[i][j] * cac[j] for j in range(s)) for i in range(s)]
    aac2 = [sum(A[i][j] * ac2[j] for j in range(s)) for i in range(s)]
    aaac = [sum(A[i][j] * aac[j] for j in range(s)) for i in range(s)]
    S = lambda v: sum(b[i] * v[i] for i in range(s))
    conds = {1: [(S([1] * s), Fraction(1))],
             2: [(S(c), Fraction(1, 2))],
             3: [(S([x ** 2 for x in c]), Fraction(1, 3)), (S(ac), Fraction(1, 6))],
             4: [(S([x ** 3 for x in c]), Fraction(1, 4)), (S(cac), Fraction(1, 8)),
                 (S(ac2), Fraction(1, 12)), (S(aac), Fraction(1, 24))],
             5: [(S([x ** 4 for x in c]), Fraction(1, 5)), (S([c[i] ** 2 * ac[i] for i in range(s)]), Fraction(1, 10)),
                 (S([c[i] * ac2[i] for i in range(s)]), Fraction(1, 15)),
                 (S([c[i] * aac[i] for i in range(s)]), Fraction(1, 30)),
                 (S([ac[i] ** 2 for i in range(s)]), Fraction(1, 20)), (S(ac3), Fraction(1, 20)),
                 (S(acac), Fraction(1, 40)), (S(aac2), Fraction(1, 60)), (S(aaac), Fraction(1, 120))]}
    out = []
    for q in range(1, order + 1):
        out += conds[q]
    return out


def test_cash_karp_order_conditions():
    c, a, b5, b4 = O.cash_karp_tableau()
    C_ = [_frac(x) for x in c]
    A = [[_frac(a[i, j]) for j in range(6)] for i in range(6)]
    B5 = [_frac(x) for x in b5]
    B4 = [_frac(x) for x in b4]
    for i in range(6):
        assert sum(A[i]) == C_[i]
        assert all(A[i][j] == 0 for j in range(i, 6))
    conds5 = order_conditions(A, B5, C_, 5)
    assert len(conds5) == 17
    for lhs, rhs in conds5:
        assert lhs == rhs
    for lhs, rhs in order_conditions(A, B4, C_, 4):
        assert lhs == rhs
    # the embedded solution is only fourth order
    assert any(lhs != rhs for lhs, rhs in order_conditions(A, B4, C_, 5)[8:])


# ---------------------------------------------------------------------- AdEx
T2 = dict(C_m=281.0, g_L=30.0, E_L=-70.6, V_T=-50.4, Delta_T=2.0, tau_w=144.0, a=4.0, b=80.5,
          V_r=-60.0, V_peak=0.0, t_ref=0.0, rk_eps=1e-6)


def adex(ports=2, E_rev=(0.0, -85.0), tau_syn=(1.0, 1.0), **kw):
    prm = dict(T2)
    prm.update(kw)
    prm["E_rev"] = list(E_rev)
    prm["tau_syn"] = list(tau_syn)
    return O.pop_params("aeif_cond_exp", ports, prm)


def test_adex_linear_special_case_vs_expm():
    """Without the exponential term and with zero conductance the (V, w)
    system is linear: exact solution from the matrix exponential."""
    p = adex(adex_no_exp=1)
    I_e = 300.0
    g_L, E_L, C, a, tw = T2["g_L"], T2["E_L"], T2["C_m"], T2["a"], T2["tau_w"]
    A = np.array([[-g_L / C, -1 / C, (g_L * E_L + I_e) / C],
                  [a / tw, -1 / tw, -a * E_L / tw],
                  [0, 0, 0]])
    y = np.array([-65.0, 10.0, 0.0, 0.0]); h = DT
    z0 = np.array([-65.0, 10.0, 1.0])
    for n in range(1, 2001):
        y, h, m, _, _ = O.adex_step(p, DT, y, h, I_e, [0.0, 0.0])
        if n % 250 == 0:
            ex = linalg.expm(A * n * DT) @ z0
            assert y[0] == pytest.approx(ex[0], rel=2e-6)
            assert y[1] == pytest.approx(ex[1], rel=2e-5, abs=1e-6)


def test_adex_conductance_decay_and_sign():
    p = adex()
    y0 = np.array([-70.6, 0.0, 0.0, 0.0])
    # excitatory conductance jump depolarises, inhibitory one hyperpolarises
    ye, h, _, _, _ = O.adex_step(p, DT, y0, DT, 0.0, [5.0, 0.0])
    yi, h, _, _, _ = O.adex_step(p, DT, y0, DT, 0.0, [0.0, 5.0])
    assert ye[0] > -70.6 > yi[0]
    # conductances decay as exp(-t/tau_syn)
    y = y0.copy(); h = DT
    y, h, _, _, _ = O.adex_step(p, DT, y, h, 0.0, [2.0, 3.0])
    for n in range(2, 30):
        y, h, _, _, _ = O.adex_step(p, DT, y, h, 0.0, [0.0, 0.0])
    assert y[2] == pytest.approx(2.0 * np.exp(-29 * DT / 1.0), rel=2e-6)
    assert y[3] == pytest.approx(3.0 * np.exp(-29 * DT / 1.0), rel=2e-6)


def test_adex_subthreshold_fixed_point_brentq():
    """Steady state: w* = a (V* - E_L) and
    -g_L (V* - E_L) + g_L Delta_T exp((V* - V_T)/Delta_T) - w* + I_e = 0."""
    p = adex()
    I_e = 150.0
    f = lambda V: (-T2["g_L"] * (V - T2["E_L"]) + T2["g_L"] * T2["Delta_T"] *
                   np.exp((V - T2["V_T"]) / T2["Delta_T"]) - T2["a"] * (V - T2["E_L"]) + I_e)
    Vs = optimize.brentq(f, T2["E_L"], T2["V_T"])
    y = np.array([T2["E_L"], 0.0, 0.0, 0.0]); h = DT
    for n in range(40000):  # 4 s >> tau_w
        y, h, m, _, _ = O.adex_step(p, DT, y, h, I_e, [0.0, 0.0])
        assert m == 0
    assert y[0] == pytest.approx(Vs, abs=2e-4)
    assert y[1] == pytest.approx(T2["a"] * (Vs - T2["E_L"]), abs=2e-3)


def _reference_adex(I_e, t_end, y0, jumps=(), ports=2, E_rev=(0.0, -85.0), tau_syn=(1.0, 1.0)):
    """DOP853 (rtol = atol = 1e-12) with an event at V = V_peak and the reset
    applied between integrations; conductance jumps at given times."""
    P = ports

    def rhs(t, y):
        V, w = y[0], y[1]
        Vc = min(V, T2["V_peak"])
        isyn = sum(y[2 + q] * (V - E_rev[q]) for q in range(P))
        dV = (-T2["g_L"] * (V - T2["E_L"]) + T2["g_L"] * T2["Delta_T"] * np.exp((Vc - T2["V_T"]) / T2["Delta_T"])
              - isyn - w + I_e) / T2["C_m"]
        dw = (T2["a"] * (V - T2["E_L"]) - w) / T2["tau_w"]
        return [dV, dw] + [-y[2 + q] / tau_syn[q] for q in range(P)]

    # Approach to the peak in two phases: DOP853 at rtol = atol = 1e-12 up to
    # V = -35 mV (far above V_T, the spike is then certain), then at 1e-9 up to
    # V_peak, where the exponential makes the step size collapse.
    def ev_near(t, y):
        return y[0] + 35.0
    ev_near.terminal = True
    ev_near.direction = 1

    def ev_peak(t, y):
        return y[0] - T2["V_peak"]
    ev_peak.terminal = True
    ev_peak.direction = 1
    jumps = sorted(jumps)
    t, y = 0.0, np.array(y0, dtype=float)
    ts, spikes = [], []
    bounds = [tj for tj, _, _ in jumps] + [t_end]
    ji = 0
    while t < t_end - 1e-12:
        while ji < len(jumps) and jumps[ji][0] <= t + 1e-12:
            y[2 + jumps[ji][1]] += jumps[ji][2]
            ji += 1
        t_stop = min(b for b in bounds if b > t + 1e-12)
        sol = integrate.solve_ivp(rhs, (t, t_stop), y, method="DOP853", rtol=1e-12, atol=1e-12,
                                  events=ev_near, dense_output=True)
        assert sol.status >= 0
        ts.append(sol); t = sol.t[-1]; y = sol.y[:, -1].copy()
        if sol.status == 1:
            s2 = integrate.solve_ivp(rhs, (t, t_end), y, method="DOP853", rtol=1e-9, atol=1e-9,
                                     events=ev_peak, dense_output=True)
            # a stall above -1 mV is within 1e-9 ms of the crossing (dV/dt > 1e9 mV/ms there)
            assert s2.status == 1 or (s2.status == -1 and s2.y[0, -1] > -1.0)
            ts.append(s2); t = s2.t[-1]; y = s2.y[:, -1].copy()
            spikes.append(t)
            y[0] = T2["V_r"]; y[1] += T2["b"]
    return ts, spikes


def _eval(sols, t):
    for s in sols:
        if s.t[0] - 1e-12 <= t <= s.t[-1] + 1e-12:
            return s.sol(t)
    raise ValueError(t)


def test_adex_700pA_vs_dop853():
    """Single AdEx neuron, Table 2 parameters, 700 pA (Fig. 9 setting)."""
    p = adex()
    T = 1000.0
    sols, ref_spikes = _reference_adex(700.0, T, [T2["E_L"], 0.0, 0.0, 0.0])
    y = np.array([T2["E_L"], 0.0, 0.0, 0.0]); h = DT
    spikes, maxrel = [], 0.0
    for n in range(int(T / DT)):
        y, h, m, _, _ = O.adex_step(p, DT, y, h, 700.0, [0.0, 0.0])
        if m:
            spikes.append((n + 1) * DT)
        tt = (n + 1) * DT
        if all(abs(tt - s) > 1.0 for s in ref_spikes):
            r = _eval(sols, tt)
            maxrel = max(maxrel, abs(y[0] - r[0]) / abs(r[0]))
    assert len(spikes) == len(ref_spikes) and len(spikes) >= 4
    # reset is applied at the end of the dt step containing the crossing
    for s, r in zip(spikes, ref_spikes):
        assert r <= s + 1e-9 and s - r < DT + 1e-9
    assert maxrel < 1e-4


def test_adex_three_ports_subthreshold_vs_dop853():
    """Three input spikes on three receptor ports in a subthreshold regime
    (Fig. 10 setting): ports E_rev = (0, 0, -85) mV, tau = (1, 2, 5) ms."""
    E_rev, tau = (0.0, 0.0, -85.0), (1.0, 2.0, 5.0)
    p = adex(ports=3, E_rev=E_rev, tau_syn=tau)
    jumps = [(10.0, 0, 2.0), (20.0, 1, 1.5), (30.0, 2, 3.0)]
    sols, sp = _reference_adex(0.0, 60.0, [T2["E_L"], 0.0, 0.0, 0.0, 0.0], jumps, ports=3, E_rev=E_rev,
                               tau_syn=tau)
    assert not sp
    y = np.array([T2["E_L"], 0.0, 0.0, 0.0, 0.0]); h = DT
    for n in range(600):
        x = [0.0, 0.0, 0.0]
        for tj, q, w in jumps:
            if abs(n * DT - tj) < 1e-9:
                x[q] = w
        y, h, m, _, _ = O.adex_step(p, DT, y, h, 0.0, x)
        r = _eval(sols, (n + 1) * DT)
        assert y[0] == pytest.approx(r[0], rel=1e-6, abs=1e-5)
    assert y[0] == pytest.approx(_eval(sols, 60.0)[0], abs=1e-5)
