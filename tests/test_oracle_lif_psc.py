"""Pins of the oracle's exponential-PSC LIF step (Sec. 2.3, LIF and
exponential-PSC equations) by how it applies the synaptic current, not only
by its propagator constants:

- a single PSC of weight w delivered at step n0 gives, at every later step
  n0 + k, V - E_L equal to the closed-form postsynaptic potential
      w tau_m tau_s / (C (tau_s - tau_m)) (e^{-t/tau_s} - e^{-t/tau_m}),
  t = k dt, and nothing at or before n0 (the input enters the current at the
  end of the step it arrives in and the membrane from the next step on);
  its peak falls on the grid step nearest the closed-form peak time, and
  tau_s = tau_m gives the limit w t e^{-t/tau} / C;
- a PSC arriving while the neuron is refractory decays as e^{-k dt/tau_s}
  while V stays at V_reset, and V restarts from the carried current;
- P21 stays accurate when tau_s is within 1e-9 or 1e-12 of tau_m (against
  the matrix exponential).
The expected values are computed here from the closed forms in numpy, not
from the oracle's propagators.  No GPU."""
import ctypes as C

import numpy as np
import pytest
from scipy import linalg

from oracle import oracle as O

DT = 0.1
EPS32 = np.finfo(np.float32).eps


def params(tau_m, tau_s, C_m, E_L=0.0, V_th=1e9, V_reset=0.0, t_ref=2.0):
    return O.pop_params("lif_exp", 1, dict(tau_m=tau_m, C_m=C_m, E_L=E_L, V_th=V_th, V_reset=V_reset,
                                           t_ref=t_ref, tau_syn=[tau_s]))


def psp(t, w, tau_m, tau_s, C_m):
    """Membrane response to a current jump w at t = 0 decaying with tau_s."""
    t = np.asarray(t, dtype=np.float64)
    if tau_s == tau_m:
        return w * t / C_m * np.exp(-t / tau_m)
    return w * tau_m * tau_s / (C_m * (tau_s - tau_m)) * (np.exp(-t / tau_s) - np.exp(-t / tau_m))


def run(p, steps, inputs, y0=0.0, refr0=0, fp32=False):
    """Step the oracle's LIF-exp update: inputs {step: x}.  Returns the
    membrane y, current I and refractory count after every step."""
    L = O.lib()
    if fp32:
        y = C.c_float(y0); I = (C.c_float * 1)(0.0); x = (C.c_float * 1)(0.0); f = L.orc_lif_exp_step32
    else:
        y = C.c_double(y0); I = (C.c_double * 1)(0.0); x = (C.c_double * 1)(0.0); f = L.orc_lif_exp_step64
    r = C.c_int32(refr0)
    ys, Is, rs = np.zeros(steps), np.zeros(steps), np.zeros(steps, dtype=np.int64)
    for n in range(steps):
        x[0] = inputs.get(n, 0.0)
        assert f(C.byref(p), DT, C.byref(y), I, C.byref(r), 0.0, x) == 0
        ys[n], Is[n], rs[n] = y.value, I[0], r.value
    return ys, Is, rs


CASES = [(10.0, 0.5, 250.0, 87.8),   # the microcircuit stand-in's constants and excitatory weight
         (20.0, 2.0, 100.0, -40.0),  # an inhibitory PSC
         (5.0, 7.0, 40.0, 10.0),     # tau_s > tau_m
         (10.0, 10.0, 250.0, 87.8)]  # tau_s = tau_m: the limit


@pytest.mark.parametrize("tau_m,tau_s,C_m,w", CASES)
@pytest.mark.parametrize("fp32", [False, True])
def test_single_psc_closed_form(tau_m, tau_s, C_m, w, fp32):
    n0, steps = 5, 600
    p = params(tau_m, tau_s, C_m)
    ys, Is, _ = run(p, steps, {n0: w}, fp32=fp32)
    # nothing before the current exists: V is untouched up to and including
    # the step the PSC arrives in
    assert np.all(ys[: n0 + 1] == 0.0)
    k = np.arange(n0 + 1, steps) - n0
    expect = psp(k * DT, w, tau_m, tau_s, C_m)
    peak = np.max(np.abs(expect))
    got = ys[n0 + 1:]
    if fp32:
        # each step rounds about four fp32 products and sums and the
        # propagators are fp32 roundings of the exact values: the error grows
        # at most by a few ulp of the peak per step
        bound = 4.0 * EPS32 * peak * k
    else:
        bound = 1e-12 * peak
    assert np.all(np.abs(got - expect) <= bound), np.max(np.abs(got - expect) / peak)
    # the current itself: w e^{-k dt / tau_s} after the arrival step
    rel = 8 * k * EPS32 if fp32 else 1e-13 * np.maximum(k, 1)
    Iexp = w * np.exp(-(k - 1) * DT / tau_s)
    assert np.all(np.abs(Is[n0:-1] - Iexp) <= rel * abs(w))
    # peak time and amplitude
    if tau_s == tau_m:
        t_peak = tau_m
    else:
        t_peak = tau_m * tau_s * np.log(tau_m / tau_s) / (tau_m - tau_s)
    v_peak = psp(t_peak, w, tau_m, tau_s, C_m)
    kmax = int(np.argmax(np.abs(got))) + 1
    assert kmax in (int(np.floor(t_peak / DT)), int(np.ceil(t_peak / DT)))
    assert abs(got[kmax - 1]) <= abs(v_peak) * (1 + 1e-6)
    assert abs(got[kmax - 1]) >= abs(psp(np.array([np.floor(t_peak / DT), np.ceil(t_peak / DT)]) * DT, w, tau_m,
                                         tau_s, C_m)).min() * (1 - 1e-5)


@pytest.mark.parametrize("fp32", [False, True])
def test_psc_during_refractoriness(fp32):
    """The neuron has just fired (held at V_reset for n_ref = 20 steps); a PSC
    arrives at step 3.  The current keeps integrating, V does not move, and
    when the hold ends V relaxes from V_reset under the carried current."""
    tau_m, tau_s, C_m, w = 10.0, 0.5, 250.0, 300.0
    E_L, V_reset = -65.0, -70.0
    y_r = V_reset - E_L
    p = params(tau_m, tau_s, C_m, E_L=E_L, V_reset=V_reset, t_ref=2.0)
    n_ref, j = 20, 3
    ys, Is, rs = run(p, 200, {j: w}, y0=y_r, refr0=n_ref, fp32=fp32)
    # held exactly at V_reset, counting down
    assert np.all(ys[:n_ref] == np.float32(y_r) if fp32 else ys[:n_ref] == y_r)
    assert list(rs[:n_ref]) == list(range(n_ref - 1, -1, -1))
    assert np.all(rs[n_ref:] == 0)
    # the current: w e^{-(s - j) dt / tau_s} after step s >= j, 0 before
    s = np.arange(200)
    Iexp = np.where(s >= j, w * np.exp(-(s - j) * DT / tau_s), 0.0)
    tol = (8 * EPS32 * (s - j + 1) if fp32 else 1e-13 * (s - j + 1)) * w
    assert np.all(np.abs(Is - Iexp) <= np.maximum(tol, 0))
    # from step n_ref on: relaxation from y_r with the current of step n_ref - 1
    I0 = w * np.exp(-(n_ref - 1 - j) * DT / tau_s)
    k = np.arange(n_ref, 200) - (n_ref - 1)
    expect = y_r * np.exp(-k * DT / tau_m) + psp(k * DT, I0, tau_m, tau_s, C_m)
    bound = (4.0 * EPS32 * k if fp32 else 1e-12) * np.max(np.abs(expect))
    assert np.all(np.abs(ys[n_ref:] - expect) <= bound)
    # the current raised V above the pure relaxation from V_reset
    assert ys[n_ref + 5] > y_r * np.exp(-6 * DT / tau_m)


@pytest.mark.parametrize("rel", [1e-9, -1e-9, 1e-12, -1e-12, 1e-6])
@pytest.mark.parametrize("tau_m,C", [(10.0, 250.0), (20.0, 100.0)])
def test_p21_near_equal_time_constants(tau_m, C, rel):
    tau_s = tau_m * (1.0 + rel)
    p = params(tau_m, tau_s, C)
    pr = O.lif_propagators(p, DT)
    A = np.array([[-1 / tau_m, 1 / C, 1 / C], [0, -1 / tau_s, 0], [0, 0, 0]])
    M = linalg.expm(A * DT)
    assert pr[3] == pytest.approx(M[0, 1], rel=1e-12)
    assert pr[2] == pytest.approx(M[1, 1], rel=1e-13)
