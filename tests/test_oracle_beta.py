"""Pins of the oracle's AdEx with beta-function conductances (the receptor
model of the Sec. 2.1 example, with the alpha function of the Sec. 2.4
balanced network as its equal-time-constant case): the conductance of a lone
input against the matrix exponential of its linear system, its peak against
the weight (the normalisation), its charge against the closed-form integral,
and whole-neuron trajectories against DOP853 with the normalisation found
numerically (no GPU)."""
import numpy as np
import pytest
from scipy import integrate, linalg, optimize

from oracle import oracle as O

DT = 0.1
T2 = dict(C_m=281.0, g_L=30.0, E_L=-70.6, V_T=-50.4, Delta_T=2.0, tau_w=144.0, a=4.0, b=80.5,
          V_r=-60.0, V_peak=0.0, t_ref=0.0, rk_eps=1e-6)
PAIRS = [(1.0, 1.0), (0.5, 2.0), (0.2, 1.0), (3.0, 1.5)]  # (tau_rise, tau_decay)


def beta(ports=2, E_rev=(0.0, -85.0), tau_decay=(1.0, 1.0), tau_rise=(1.0, 1.0), **kw):
    prm = dict(T2)
    prm.update(kw)
    prm["E_rev"] = list(E_rev)
    prm["tau_syn"] = list(tau_decay)
    prm["tau_rise"] = list(tau_rise)
    return O.pop_params("aeif_cond_beta", ports, prm)


def peak_of_shape(tr, td):
    """Largest value of the unnormalised response r -> g of a unit r jump,
    found by bounded scalar search on the library-integrated kernel."""
    M = np.array([[-1 / td, 1.0], [0.0, -1 / tr]])

    def neg(s):
        return -(linalg.expm(M * s) @ np.array([0.0, 1.0]))[0]
    res = optimize.minimize_scalar(neg, bounds=(1e-6, 20 * max(tr, td)), method="bounded",
                                   options=dict(xatol=1e-10))
    return -res.fun, res.x


@pytest.mark.parametrize("tr,td", PAIRS)
def test_beta_conductance_vs_expm(tr, td):
    """With V held far from spiking, port 0 after one input of weight w
    follows the linear system (g, r)' = [[-1/td, 1], [0, -1/tr]] (g, r) with
    r(0) = g0 w; g0 is fixed by the peak condition (next test)."""
    p = beta(ports=1, E_rev=(0.0,), tau_decay=(td,), tau_rise=(tr,), adex_no_exp=1)
    w = 2.5
    pk, _ = peak_of_shape(tr, td)
    g0 = 1.0 / pk
    M = np.array([[-1 / td, 1.0], [0.0, -1 / tr]])
    y = np.array([-70.6, 0.0, 0.0, 0.0]); h = DT
    for n in range(200):
        y, h, m, _, _ = O.adex_step(p, DT, y, h, 0.0, [w if n == 0 else 0.0])
        ex = linalg.expm(M * (n + 1) * DT) @ np.array([0.0, g0 * w])
        # the step control's tolerance is 1e-6 of max(|y|, 1) per substep
        assert y[2] == pytest.approx(ex[0], rel=1e-5, abs=1e-6)
        assert y[3] == pytest.approx(ex[1], rel=1e-5, abs=1e-6)


@pytest.mark.parametrize("tr,td", PAIRS)
def test_beta_peak_equals_weight(tr, td):
    """The weight is the peak conductance: sampled on a fine grid, the largest
    g of a lone input is w, reached at the time the search finds."""
    p = beta(ports=1, E_rev=(0.0,), tau_decay=(td,), tau_rise=(tr,), adex_no_exp=1)
    w, dt = 0.37, 0.001
    _, s_star = peak_of_shape(tr, td)
    y = np.array([-70.6, 0.0, 0.0, 0.0]); h = dt
    best, t_best = 0.0, 0.0
    for n in range(int(4 * s_star / dt) + 10):
        y, h, m, _, _ = O.adex_step(p, dt, y, h, 0.0, [w if n == 0 else 0.0])
        if y[2] > best:
            best, t_best = y[2], (n + 1) * dt
    assert best == pytest.approx(w, rel=1e-5)
    assert abs(t_best - s_star) <= dt


def test_alpha_charge_closed_form():
    """Alpha kernel (tau_rise = tau_decay = tau): g = w e s/tau e^{-s/tau}, so
    the charge of one input is int g ds = e w tau; summed over 100 ms of
    trapezoids it must match to the trapezoid error."""
    tau, w = 2.0, 1.3
    p = beta(ports=1, E_rev=(0.0,), tau_decay=(tau,), tau_rise=(tau,), adex_no_exp=1)
    y = np.array([-70.6, 0.0, 0.0, 0.0]); h = DT
    prev, q = 0.0, 0.0
    for n in range(1000):
        y, h, m, _, _ = O.adex_step(p, DT, y, h, 0.0, [w if n == 0 else 0.0])
        q += 0.5 * DT * (prev + y[2])
        prev = y[2]
    assert q == pytest.approx(np.e * w * tau, rel=1e-3)


def test_beta_near_equal_time_constants_continuous():
    """The alpha case is the limit of the beta case: tau_rise within 1e-6 of
    tau_decay gives the same trajectory to 1e-5."""
    pa = beta(ports=1, E_rev=(0.0,), tau_decay=(1.0,), tau_rise=(1.0,))
    pb = beta(ports=1, E_rev=(0.0,), tau_decay=(1.0,), tau_rise=(1.0 + 1e-6,))
    ya = np.array([-70.6, 0.0, 0.0, 0.0]); yb = ya.copy(); ha = hb = DT
    for n in range(100):
        x = [3.0 if n in (0, 20, 21) else 0.0]
        ya, ha, _, _, _ = O.adex_step(pa, DT, ya, ha, 0.0, x)
        yb, hb, _, _, _ = O.adex_step(pb, DT, yb, hb, 0.0, x)
        assert yb[0] == pytest.approx(ya[0], rel=1e-7)
        assert yb[2] == pytest.approx(ya[2], rel=1e-5, abs=1e-9)


def test_beta_sign():
    p = beta()
    y0 = np.array([-70.6, 0.0, 0.0, 0.0, 0.0, 0.0])
    ye, ye_h = y0, DT
    yi, yi_h = y0, DT
    for n in range(20):
        ye, ye_h, _, _, _ = O.adex_step(p, DT, ye, ye_h, 0.0, [5.0 if n == 0 else 0.0, 0.0])
        yi, yi_h, _, _, _ = O.adex_step(p, DT, yi, yi_h, 0.0, [0.0, 5.0 if n == 0 else 0.0])
    assert ye[0] > -70.6 > yi[0]


def _reference_beta(I_e, t_end, y0, jumps, E_rev, tau_decay, tau_rise):
    """DOP853 (rtol = atol = 1e-12) on (V, w, g_p, r_p) with jumps of
    w / peak into r_p at given times, the peak found by the numerical search;
    event at V = V_peak (two-phase approach as for the exponential model) and
    the reset between integrations."""
    P = len(E_rev)
    g0 = [1.0 / peak_of_shape(tau_rise[q], tau_decay[q])[0] for q in range(P)]

    def rhs(t, y):
        V, w = y[0], y[1]
        Vc = min(V, T2["V_peak"])
        isyn = sum(y[2 + q] * (V - E_rev[q]) for q in range(P))
        dV = (-T2["g_L"] * (V - T2["E_L"]) + T2["g_L"] * T2["Delta_T"] * np.exp((Vc - T2["V_T"]) / T2["Delta_T"])
              - isyn - w + I_e) / T2["C_m"]
        dw = (T2["a"] * (V - T2["E_L"]) - w) / T2["tau_w"]
        dg = [y[2 + P + q] - y[2 + q] / tau_decay[q] for q in range(P)]
        dr = [-y[2 + P + q] / tau_rise[q] for q in range(P)]
        return [dV, dw] + dg + dr

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
    sols, spikes = [], []
    bounds = [tj for tj, _, _ in jumps] + [t_end]
    ji = 0
    while t < t_end - 1e-12:
        while ji < len(jumps) and jumps[ji][0] <= t + 1e-12:
            q = jumps[ji][1]
            y[2 + P + q] += g0[q] * jumps[ji][2]
            ji += 1
        t_stop = min(b for b in bounds if b > t + 1e-12)
        sol = integrate.solve_ivp(rhs, (t, t_stop), y, method="DOP853", rtol=1e-12, atol=1e-12,
                                  events=ev_near, dense_output=True)
        assert sol.status >= 0
        sols.append(sol); t = sol.t[-1]; y = sol.y[:, -1].copy()
        if sol.status == 1:
            s2 = integrate.solve_ivp(rhs, (t, t_end), y, method="DOP853", rtol=1e-9, atol=1e-9,
                                     events=ev_peak, dense_output=True)
            assert s2.status == 1 or (s2.status == -1 and s2.y[0, -1] > -1.0)
            sols.append(s2); t = s2.t[-1]; y = s2.y[:, -1].copy()
            spikes.append(t)
            y[0] = T2["V_r"]; y[1] += T2["b"]
    return sols, spikes


def _eval(sols, t):
    for s in sols:
        if s.t[0] - 1e-12 <= t <= s.t[-1] + 1e-12:
            return s.sol(t)
    raise ValueError(t)


def test_beta_three_ports_subthreshold_vs_dop853():
    """Inputs on three beta ports (E_rev 0, 0, -85 mV; rise/decay 0.5/2,
    1/1, 0.3/5 ms) below threshold."""
    E_rev, td, tr = (0.0, 0.0, -85.0), (2.0, 1.0, 5.0), (0.5, 1.0, 0.3)
    p = beta(ports=3, E_rev=E_rev, tau_decay=td, tau_rise=tr)
    jumps = [(10.0, 0, 2.0), (20.0, 1, 1.5), (30.0, 2, 3.0), (30.0, 0, 1.0)]
    y0 = [T2["E_L"], 0.0] + [0.0] * 6
    sols, sp = _reference_beta(0.0, 60.0, y0, jumps, E_rev, td, tr)
    assert not sp
    y = np.array(y0); h = DT
    for n in range(600):
        x = [0.0, 0.0, 0.0]
        for tj, q, w in jumps:
            if abs(n * DT - tj) < 1e-9:
                x[q] += w
        y, h, m, _, _ = O.adex_step(p, DT, y, h, 0.0, x)
        r = _eval(sols, (n + 1) * DT)
        assert y[0] == pytest.approx(r[0], rel=1e-6, abs=1e-5)
        for q in range(3):
            assert y[2 + q] == pytest.approx(r[2 + q], rel=1e-6, abs=1e-8)


def test_alpha_input_driven_spikes_vs_dop853():
    """A train of strong excitatory alpha inputs (Table 1 port layout,
    tau = 1 ms) drives spikes: spike times within one step of DOP853's and
    V within 1e-4 relative away from the spikes."""
    E_rev, td, tr = (0.0, -85.0), (1.0, 1.0), (1.0, 1.0)
    p = beta(ports=2, E_rev=E_rev, tau_decay=td, tau_rise=tr)
    jumps = [(5.0 + 2.0 * k, 0, 40.0) for k in range(20)] + [(30.0, 1, 5.0)]
    y0 = [T2["E_L"], 0.0, 0.0, 0.0, 0.0, 0.0]
    T = 80.0
    sols, ref_spikes = _reference_beta(200.0, T, y0, jumps, E_rev, td, tr)
    assert len(ref_spikes) >= 3
    y = np.array(y0); h = DT
    spikes, maxrel = [], 0.0
    for n in range(int(T / DT)):
        x = [0.0, 0.0]
        for tj, q, w in jumps:
            if abs(n * DT - tj) < 1e-9:
                x[q] += w
        y, h, m, _, _ = O.adex_step(p, DT, y, h, 200.0, x)
        if m:
            spikes.append((n + 1) * DT)
        tt = (n + 1) * DT
        if all(abs(tt - s) > 1.0 for s in ref_spikes):
            maxrel = max(maxrel, abs(y[0] - _eval(sols, tt)[0]) / abs(_eval(sols, tt)[0]))
    assert len(spikes) == len(ref_spikes)
    for s, r in zip(spikes, ref_spikes):
        assert r <= s + 1e-9 and s - r < DT + 1e-9
    assert maxrel < 1e-4


def test_beta_rejects_bad_time_constants():
    spec = dict(dt=DT, seed=1, dmax=4, populations=[
        dict(name="A", model="aeif_cond_beta", n=3, ports=1,
             params=dict(T2, tau_syn=[1.0], tau_rise=[0.0]))], projections=[])
    with pytest.raises(RuntimeError):
        O.OracleNet(spec)
