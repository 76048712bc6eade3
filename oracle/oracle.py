"""ctypes front end of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It loads liboracle.so (built from snn_oracle.c by
build_oracle()) and turns a network specification dictionary into oracle calls.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# the same source built with OpenMP (the neuron and delivery loops split over
# the host's cores; same results): used only to time the oracle on all cores
LIB_OMP_PATH = os.path.join(HERE, "liboracle_omp.so")

LIF_DELTA, LIF_EXP, AEIF_COND_EXP, AEIF_COND_BETA, SPIKE_GENERATOR, PARROT = 0, 1, 2, 3, 4, 5
FP64, FP32SO = 0, 1
MODEL_IDS = {"lif_delta": LIF_DELTA, "lif_exp": LIF_EXP, "aeif_cond_exp": AEIF_COND_EXP,
             "aeif_cond_beta": AEIF_COND_BETA, "spike_generator": SPIKE_GENERATOR, "parrot_neuron": PARROT}
DELAY_IDS = {"const": 0, "uniform": 1, "normal": 2}
VAR_IDS = {"V_m": 0, "I_e": 1, "w": 2, "g": 3, "I_syn": 4, "refr": 5, "h": 6, "g_rise": 7}
PARAM_IDS = {"tau_m": 0, "C_m": 1, "E_L": 2, "V_th": 3, "V_reset": 4, "t_ref": 5, "g_L": 6, "Delta_T": 7,
             "V_T": 8, "tau_w": 9, "a": 10, "b": 11, "V_peak": 12, "V_r": 13, "rk_eps": 14, "rk_hmin": 15}
# connection rules; a projection's "K" is the in-degree, the out-degree or the
# number of synapses (unused for all_to_all and one_to_one)
RULE_IDS = {"fixed_indegree": 0, "fixed_outdegree": 1, "all_to_all": 2, "one_to_one": 3, "fixed_total_number": 4}
WEIGHT_IDS = {"uniform": 0, "normal": 1}
MAX_PORTS = 4
POISSON_KMAX = 128


def weight_dist_args(wd: dict):
    """(kind, a, b, lo, hi, levels) of a weight distribution: uniform on
    [low, high), or normal(mean, sd) truncated to [low, high] (default
    mean -+ 4 sd); `levels` bins (default 64)."""
    L = int(wd.get("levels", 64))
    if wd["kind"] == "uniform":
        return WEIGHT_IDS["uniform"], float(wd["low"]), float(wd["high"]), 0.0, 0.0, L
    m, sd = float(wd["mean"]), float(wd["sd"])
    return (WEIGHT_IDS["normal"], m, sd, float(wd.get("low", m - 4 * sd)), float(wd.get("high", m + 4 * sd)), L)


STDP_DEFAULTS = dict(tau_plus=20.0, tau_minus=20.0, lambda_=0.01, alpha=1.0, mu_plus=1, mu_minus=1, w_max=100.0)


def stdp_args(sd: dict):
    """(tau_plus, tau_minus, lambda, alpha, mu_plus, mu_minus, w_max) of a
    projection's "stdp" entry (NEST-like defaults)."""
    v = dict(STDP_DEFAULTS)
    v.update({("lambda_" if k == "lambda" else k): x for k, x in sd.items()})
    return (float(v["tau_plus"]), float(v["tau_minus"]), float(v["lambda_"]), float(v["alpha"]), int(v["mu_plus"]),
            int(v["mu_minus"]), float(v["w_max"]))


class PopParams(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("n_ports", C.c_uint32),
        ("tau_m", C.c_double), ("C_m", C.c_double), ("E_L", C.c_double), ("V_th", C.c_double),
        ("V_reset", C.c_double), ("t_ref", C.c_double),
        ("g_L", C.c_double), ("Delta_T", C.c_double), ("V_T", C.c_double), ("tau_w", C.c_double),
        ("a", C.c_double), ("b", C.c_double), ("V_peak", C.c_double), ("V_r", C.c_double),
        ("tau_syn", C.c_double * MAX_PORTS), ("E_rev", C.c_double * MAX_PORTS),
        ("rk_eps", C.c_double), ("rk_hmin", C.c_double), ("adex_no_exp", C.c_int32),
        ("tau_rise", C.c_double * MAX_PORTS),
    ]


def build_oracle(force: bool = False, openmp: bool = False) -> str:
    """Compile liboracle.so (or, openmp=True, liboracle_omp.so) with gcc (no
    fast-math, no FMA contraction)."""
    src = os.path.join(HERE, "snn_oracle.c")
    hdr = os.path.join(HERE, "snn_oracle.h")
    path = LIB_OMP_PATH if openmp else LIB_PATH
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    if force or not os.path.exists(path) or os.path.getmtime(path) < newest:
        tmp = path + ".tmp"
        extra = ["-fopenmp"] if openmp else []
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared"] + extra + ["-o", tmp, src, "-lm"])
        os.replace(tmp, path)
    return path


_lib = None
_lib_omp = None


def lib_omp():
    """The OpenMP build (loaded on first use)."""
    global _lib_omp
    if _lib_omp is None:
        _lib_omp = _declare(C.CDLL(build_oracle(openmp=True)))
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        _lib = _declare(C.CDLL(build_oracle()))
    return _lib


def _declare(L):
    """ctypes signatures of the oracle's C functions."""
    P64, P32, PU32, PI64, PD = (C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                C.POINTER(C.c_int64), C.POINTER(C.c_double))
    L.orc_philox4x64_10.argtypes = [P64, P64, P64]
    L.orc_delay_table.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_uint32, P64]
    L.orc_poisson_table.argtypes = [C.c_double, C.c_uint32, P64]
    L.orc_fixed_point_shift.argtypes = [C.c_double]
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.c_double, C.c_uint64, C.c_uint32, C.c_int]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_population.restype = C.c_int64
    L.orc_population.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(PopParams)]
    L.orc_set_spike_times.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, PD]
    L.orc_connect_list.argtypes = [C.c_void_p, C.c_uint64, P32, P32, PD, C.c_double, C.c_uint32]
    L.orc_weight_distribution.argtypes = [C.c_void_p, C.c_uint32, C.c_int, C.c_double, C.c_double, C.c_double,
                                          C.c_double, C.c_uint32]
    L.orc_list_weights.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, PD]
    L.orc_set_param.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, PD]
    L.orc_stdp.argtypes = [C.c_void_p, C.c_uint32, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                           C.c_int, C.c_double]
    L.orc_get_param.restype = C.c_double
    L.orc_get_param.argtypes = [C.c_void_p, C.c_uint32, C.c_int]
    L.orc_param_distribution.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, C.c_int, C.c_double,
                                         C.c_double, C.c_double, C.c_double, C.c_uint32]
    L.orc_state_distribution.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, C.c_uint32, C.c_int,
                                         C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32]
    L.orc_connect.argtypes = [C.c_void_p, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                              C.c_double, C.c_int, C.c_double, C.c_double, C.c_uint32]
    L.orc_connect_fixed_indegree.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                             C.c_uint32, C.c_double, C.c_int, C.c_double, C.c_double,
                                             C.c_uint32]
    L.orc_poisson.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_double, C.c_uint32, C.c_double,
                              C.c_uint32]
    L.orc_set_state.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, C.c_uint32, PD]
    L.orc_get_state.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, C.c_uint32, PD]
    L.orc_build.argtypes = [C.c_void_p]
    L.orc_simulate.argtypes = [C.c_void_p, C.c_uint64]
    L.orc_current_step.restype = C.c_uint64
    L.orc_current_step.argtypes = [C.c_void_p]
    L.orc_n_events.restype = C.c_uint64
    L.orc_n_events.argtypes = [C.c_void_p]
    L.orc_n_spikes.restype = C.c_uint64
    L.orc_n_spikes.argtypes = [C.c_void_p]
    L.orc_get_spikes.argtypes = [C.c_void_p, P64, P32, P32]
    L.orc_n_synapses.restype = C.c_uint64
    L.orc_n_synapses.argtypes = [C.c_void_p]
    L.orc_get_synapses.argtypes = [C.c_void_p, P32, P32, P32, P32, PI64]
    L.orc_shift_of.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32]
    L.orc_poisson_count.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, P32]
    L.orc_record_input.argtypes = [C.c_void_p, PI64, C.c_uint64]
    L.orc_replay_input.argtypes = [C.c_void_p, C.c_uint64, P64, P32, P32, C.c_uint64, PI64]
    L.orc_lif_delta_step64.argtypes = [C.POINTER(PopParams), C.c_double, PD, C.POINTER(C.c_int32),
                                       C.c_double, C.c_double]
    L.orc_lif_delta_step32.argtypes = [C.POINTER(PopParams), C.c_double, C.POINTER(C.c_float),
                                       C.POINTER(C.c_int32), C.c_float, C.c_float]
    L.orc_lif_exp_step64.argtypes = [C.POINTER(PopParams), C.c_double, PD, PD, C.POINTER(C.c_int32),
                                     C.c_double, PD]
    L.orc_lif_exp_step32.argtypes = [C.POINTER(PopParams), C.c_double, C.POINTER(C.c_float),
                                     C.POINTER(C.c_float), C.POINTER(C.c_int32), C.c_float,
                                     C.POINTER(C.c_float)]
    L.orc_lif_propagators.argtypes = [C.POINTER(PopParams), C.c_double, PD]
    L.orc_adex_step.argtypes = [C.POINTER(PopParams), C.c_double, PD, PD, C.c_double, PD,
                                P64, P64]
    L.orc_cash_karp_tableau.argtypes = [PD, PD, PD, PD]
    L.orc_adex_rhs.argtypes = [C.POINTER(PopParams), C.c_double, PD, PD]
    L.orc_prepare.argtypes = [C.c_void_p]
    L.orc_target_synapses.restype = C.c_int64
    L.orc_target_synapses.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, P32, P32, P32, PI64]
    L.orc_sampled_input.argtypes = [C.c_void_p, C.c_uint32, P32, C.c_uint64, P64, P32, P32, C.c_uint64, PI64]
    L.orc_last_error.restype = C.c_char_p
    L.orc_last_error.argtypes = [C.c_void_p]
    L.orc_threads.restype = C.c_int
    L.orc_threads.argtypes = []
    return L


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------- primitives
def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


def delay_table(kind: str, a: float, b: float, dt: float, dmax: int) -> np.ndarray:
    thr = np.zeros(dmax + 1, dtype=np.uint64)
    rc = lib().orc_delay_table(DELAY_IDS[kind], a, b, dt, dmax, _ptr(thr, C.c_uint64))
    if rc != 0:
        raise ValueError("delay table")
    return thr


def poisson_table(lam: float, kmax: int = POISSON_KMAX) -> np.ndarray:
    thr = np.zeros(kmax, dtype=np.uint64)
    if lib().orc_poisson_table(lam, kmax, _ptr(thr, C.c_uint64)) != 0:
        raise ValueError("poisson table")
    return thr


def fixed_point_shift(max_abs_w: float) -> int:
    return int(lib().orc_fixed_point_shift(max_abs_w))


def pop_params(model: str, ports: int, params: dict) -> PopParams:
    p = PopParams()
    p.model = MODEL_IDS[model]
    p.n_ports = ports
    defaults = dict(tau_m=10.0, C_m=250.0, E_L=-70.0, V_th=-55.0, V_reset=-70.0, t_ref=2.0,
                    g_L=30.0, Delta_T=2.0, V_T=-50.4, tau_w=144.0, a=4.0, b=80.5, V_peak=0.0,
                    V_r=-60.0, rk_eps=1e-6, rk_hmin=1e-8)
    for k, v in defaults.items():
        x = params.get(k, v)
        setattr(p, k, float(v if np.ndim(x) else x))  # per-neuron arrays are set afterwards
    ts = list(params.get("tau_syn", [1.0] * ports))
    er = list(params.get("E_rev", [0.0] * ports))
    tr = list(params.get("tau_rise", ts))  # default: rise = decay, the alpha function
    for i in range(MAX_PORTS):
        p.tau_syn[i] = float(ts[i]) if i < len(ts) else 1.0
        p.E_rev[i] = float(er[i]) if i < len(er) else 0.0
        p.tau_rise[i] = float(tr[i]) if i < len(tr) else 1.0
    p.adex_no_exp = int(params.get("adex_no_exp", 0))
    return p


def lif_propagators(params: PopParams, dt: float) -> np.ndarray:
    out = np.zeros(2 + 2 * MAX_PORTS)
    lib().orc_lif_propagators(C.byref(params), dt, _ptr(out, C.c_double))
    return out[: 2 + 2 * params.n_ports]


def cash_karp_tableau():
    c = np.zeros(6); a = np.zeros(36); b5 = np.zeros(6); b4 = np.zeros(6)
    lib().orc_cash_karp_tableau(_ptr(c, C.c_double), _ptr(a, C.c_double), _ptr(b5, C.c_double),
                                _ptr(b4, C.c_double))
    return c, a.reshape(6, 6), b5, b4


def adex_rhs(params: PopParams, I_e: float, y) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    dy = np.zeros_like(y)
    lib().orc_adex_rhs(C.byref(params), I_e, _ptr(y, C.c_double), _ptr(dy, C.c_double))
    return dy


def lif_delta_step32(params: PopParams, dt: float, y: float, refr: int, I_e: float, x: float):
    """One step of the fp32 same-operation-order LIF-delta update.  Returns
    (y, refr, spiked) with y = V - E_L."""
    yy = C.c_float(y)
    rr = C.c_int32(refr)
    s = lib().orc_lif_delta_step32(C.byref(params), dt, C.byref(yy), C.byref(rr), C.c_float(I_e), C.c_float(x))
    return yy.value, rr.value, int(s)


def lif_exp_step32(params: PopParams, dt: float, y: float, I, refr: int, I_e: float, x):
    """One step of the fp32 same-operation-order LIF-exp update.  Returns
    (y, I, refr, spiked) with y = V - E_L."""
    yy = C.c_float(y)
    Ia = np.ascontiguousarray(I, dtype=np.float32).copy()
    xa = np.ascontiguousarray(x, dtype=np.float32)
    rr = C.c_int32(refr)
    s = lib().orc_lif_exp_step32(C.byref(params), dt, C.byref(yy), _ptr(Ia, C.c_float), C.byref(rr),
                                 C.c_float(I_e), _ptr(xa, C.c_float))
    return yy.value, Ia, rr.value, int(s)


def adex_step(params: PopParams, dt: float, y, h: float, I_e: float, x):
    """One dt of the AdEx oracle.  Returns (y_new, h_new, mult, n_acc, n_rej)."""
    y = np.array(y, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    hh = C.c_double(h)
    na = C.c_uint64(0); nr = C.c_uint64(0)
    m = lib().orc_adex_step(C.byref(params), dt, _ptr(y, C.c_double), C.byref(hh), I_e,
                            _ptr(x, C.c_double), C.byref(na), C.byref(nr))
    return y, hh.value, int(m), na.value, nr.value


# -------------------------------------------------------------------- network
class OracleNet:
    """Oracle instance built from a specification dictionary."""

    def __init__(self, spec: dict, mode: int = FP64, build: bool = True, openmp: bool = False):
        """build=False prepares state, Poisson drive and fixed-point exponents
        but draws no synapse table: for the sampled checks of networks whose
        table does not fit (target_synapses, sampled_input, poisson_count,
        shift_of); such a network cannot be simulated.  openmp=True runs on
        the OpenMP build (all host cores, same results)."""
        self.L = lib_omp() if openmp else lib()
        self.threads = int(self.L.orc_threads())
        self.spec = spec
        self.mode = mode
        self.h = self.L.orc_create(spec["dt"], spec["seed"], spec["dmax"], mode)
        if not self.h:
            raise ValueError("orc_create failed")
        self.ranges = {}
        for p in spec["populations"]:
            pp = pop_params(p["model"], p["ports"], p["params"])
            first = self.L.orc_population(self.h, p["n"], C.byref(pp))
            self._check(first >= 0)
            self.ranges[p["name"]] = (int(first), p["n"])
        self.N = sum(p["n"] for p in spec["populations"])
        for p in spec["populations"]:  # per-neuron parameters: after every population, before any state
            t0, tn = self.ranges[p["name"]]
            for k, x in p["params"].items():
                if k in PARAM_IDS and np.ndim(x):
                    v = np.ascontiguousarray(x, dtype=np.float64)
                    assert len(v) == tn
                    self._check(self.L.orc_set_param(self.h, t0, tn, PARAM_IDS[k], _ptr(v, C.c_double)) == 0)
            for k, wd in (p.get("param_dists") or {}).items():
                kind, a, b, lo, hi, _ = weight_dist_args(wd)
                self._check(self.L.orc_param_distribution(self.h, t0, tn, PARAM_IDS[k], kind, a, b, lo, hi,
                                                          int(wd.get("levels", 1024))) == 0)
        for p in spec["populations"]:  # after every population: state is sized then
            for j, times in enumerate(p.get("spike_times", []) or []):
                t = np.ascontiguousarray(times, dtype=np.float64)
                self._check(self.L.orc_set_spike_times(self.h, self.ranges[p["name"]][0] + j, len(t),
                                                       _ptr(t, C.c_double)) == 0)
        self.P = max(p["ports"] for p in spec["populations"])
        for ip, pr in enumerate(spec["projections"]):
            if pr.get("rule") == "list":  # user-defined: gids counted from the specification's first neuron
                src = np.ascontiguousarray(pr["src_gids"], dtype=np.uint32)
                tgt = np.ascontiguousarray(pr["tgt_gids"], dtype=np.uint32)
                dl = np.ascontiguousarray(pr["delays_ms"], dtype=np.float64)
                self._check(self.L.orc_connect_list(self.h, len(src), _ptr(src, C.c_uint32), _ptr(tgt, C.c_uint32),
                                                    _ptr(dl, C.c_double), pr.get("weight", 0.0), pr["port"]) == 0)
                if pr.get("weights") is not None and len(src):
                    w = np.ascontiguousarray(pr["weights"], dtype=np.float64)
                    self._check(self.L.orc_list_weights(self.h, ip, len(w), _ptr(w, C.c_double)) == 0)
                continue
            s0, sn = self.ranges[pr["src"]]
            t0, tn = self.ranges[pr["tgt"]]
            kind, a, b = (list(pr["delay"]) + [0.0, 0.0])[:3]
            rule = RULE_IDS[pr.get("rule", "fixed_indegree")]
            self._check(self.L.orc_connect(self.h, rule, int(pr.get("K", 0)), s0, sn, t0, tn, pr.get("weight", 0.0),
                                           DELAY_IDS[kind], a, b, pr["port"]) == 0)
            if pr.get("weight_dist") is not None:
                self._check(self.L.orc_weight_distribution(self.h, ip, *weight_dist_args(pr["weight_dist"])) == 0)
            if pr.get("stdp") is not None:
                self._check(self.L.orc_stdp(self.h, ip, *stdp_args(pr["stdp"])) == 0)
        for q in spec.get("poisson", []):
            t0, tn = self.ranges[q["tgt"]]
            self._check(self.L.orc_poisson(self.h, t0, tn, q["rate"], q["n_inputs"], q["weight"],
                                           q["port"]) == 0)
        for p in spec["populations"]:
            t0, tn = self.ranges[p["name"]]
            if p.get("V0") is not None:
                self.set_state("V_m", t0, np.asarray(p["V0"], dtype=np.float64))
            ie = p.get("I_e", 0.0)
            if np.ndim(ie) == 0:
                ie = np.full(tn, float(ie))
            self.set_state("I_e", t0, np.asarray(ie, dtype=np.float64))
            # state drawn from distributions, after the arrays: {"V_m": {...}, "I_e": {...}, ...}
            for var, wd in (p.get("state_dists") or {}).items():
                kind, a, b, lo, hi, _ = weight_dist_args(wd)
                self._check(self.L.orc_state_distribution(self.h, t0, tn, VAR_IDS[var], int(wd.get("port", 0)),
                                                          kind, a, b, lo, hi, int(wd.get("levels", 1024))) == 0)
        self._check((self.L.orc_build(self.h) if build else self.L.orc_prepare(self.h)) == 0)

    def _check(self, ok):
        if not ok:
            raise RuntimeError(self.L.orc_last_error(self.h).decode())

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    def set_state(self, var: str, first: int, values, port: int = 0):
        v = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self.L.orc_set_state(self.h, first, len(v), VAR_IDS[var], port, _ptr(v, C.c_double)) == 0)

    def get_param(self, name: str, first: int = 0, n: int | None = None) -> np.ndarray:
        """Model parameter `name` of every neuron of [first, first + n)."""
        n = self.N - first if n is None else n
        return np.array([self.L.orc_get_param(self.h, first + j, PARAM_IDS[name]) for j in range(n)])

    def get_state(self, var: str, first: int = 0, n: int | None = None, port: int = 0) -> np.ndarray:
        n = self.N - first if n is None else n
        out = np.zeros(n, dtype=np.float64)
        self._check(self.L.orc_get_state(self.h, first, n, VAR_IDS[var], port, _ptr(out, C.c_double)) == 0)
        return out

    def simulate(self, steps: int):
        self._check(self.L.orc_simulate(self.h, steps) == 0)

    @property
    def step(self) -> int:
        return int(self.L.orc_current_step(self.h))

    @property
    def events(self) -> int:
        return int(self.L.orc_n_events(self.h))

    def spikes(self):
        """(step, gid, mult) arrays sorted by (step, gid)."""
        n = int(self.L.orc_n_spikes(self.h))
        st = np.zeros(n, dtype=np.uint64); gid = np.zeros(n, dtype=np.uint32); m = np.zeros(n, dtype=np.uint32)
        if n:
            self.L.orc_get_spikes(self.h, _ptr(st, C.c_uint64), _ptr(gid, C.c_uint32), _ptr(m, C.c_uint32))
        return st, gid, m

    def synapses(self):
        """Canonical synapse list: dict of arrays src, delay, tgt, port, wq."""
        n = int(self.L.orc_n_synapses(self.h))
        src = np.zeros(n, np.uint32); d = np.zeros(n, np.uint32); tgt = np.zeros(n, np.uint32)
        port = np.zeros(n, np.uint32); wq = np.zeros(n, np.int64)
        if n:
            self.L.orc_get_synapses(self.h, _ptr(src, C.c_uint32), _ptr(d, C.c_uint32), _ptr(tgt, C.c_uint32),
                                    _ptr(port, C.c_uint32), _ptr(wq, C.c_int64))
        return dict(src=src, delay=d, tgt=tgt, port=port, wq=wq)

    def shift_of(self, gid: int, port: int = 0) -> int:
        return int(self.L.orc_shift_of(self.h, gid, port))

    def poisson_count(self, gid: int, step: int) -> int:
        k = C.c_uint32(0)
        if self.L.orc_poisson_count(self.h, gid, step, C.byref(k)) != 0:
            return -1
        return int(k.value)

    def target_synapses(self, t: int):
        """(source, delay, port, w_q) of the synapses onto target t, drawn one
        by one by the fixed-indegree rule."""
        n = self.L.orc_target_synapses(self.h, t, 0, None, None, None, None)
        self._check(n >= 0)
        src = np.zeros(n, np.uint32); d = np.zeros(n, np.uint32); port = np.zeros(n, np.uint32)
        wq = np.zeros(n, np.int64)
        self.L.orc_target_synapses(self.h, t, n, _ptr(src, C.c_uint32), _ptr(d, C.c_uint32), _ptr(port, C.c_uint32),
                                   _ptr(wq, C.c_int64))
        return src, d, port, wq

    def sampled_input(self, targets, step, gid, mult, target_step: int) -> np.ndarray:
        """Input delivered at target_step to the given targets by the spikes
        (step, gid, mult), sorted by (step, gid): array [len(targets)][P]."""
        t = np.ascontiguousarray(targets, dtype=np.uint32)
        st = np.ascontiguousarray(step, dtype=np.uint64)
        g = np.ascontiguousarray(gid, dtype=np.uint32)
        m = np.ascontiguousarray(mult, dtype=np.uint32)
        out = np.zeros((len(t), self.P), dtype=np.int64)
        self._check(self.L.orc_sampled_input(self.h, len(t), _ptr(t, C.c_uint32), len(st), _ptr(st, C.c_uint64),
                                             _ptr(g, C.c_uint32), _ptr(m, C.c_uint32), target_step,
                                             _ptr(out, C.c_int64)) == 0)
        return out

    def record_input(self, max_steps: int) -> np.ndarray:
        buf = np.zeros((max_steps, self.N, self.P), dtype=np.int64)
        self._rec = buf
        self.L.orc_record_input(self.h, _ptr(buf, C.c_int64), max_steps)
        return buf

    def replay_input(self, step, gid, mult, target_step: int) -> np.ndarray:
        st = np.ascontiguousarray(step, dtype=np.uint64)
        g = np.ascontiguousarray(gid, dtype=np.uint32)
        m = np.ascontiguousarray(mult, dtype=np.uint32)
        out = np.zeros((self.N, self.P), dtype=np.int64)
        self._check(self.L.orc_replay_input(self.h, len(st), _ptr(st, C.c_uint64), _ptr(g, C.c_uint32),
                                            _ptr(m, C.c_uint32), target_step, _ptr(out, C.c_int64)) == 0)
        return out
