"""Python binding of libsnn.so (argument marshalling only).

Every step of the simulation runs in the HIP kernels behind the C ABI of
include/snn.h; this module converts a network specification dictionary (see
workloads.py) into those calls and hands the library device memory from
PyTorch's allocator and PyTorch's current stream.  If libsnn.so is missing it
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnn.so")

SNN_OK = 0
ERRORS = {-1: "INVALID", -2: "NOMEM", -3: "STATE", -4: "OVERFLOW", -5: "DEVICE", -6: "BUDGET", -7: "UNSUPPORTED"}
MODELS = {"lif_delta": 0, "lif_exp": 1, "aeif_cond_exp": 2, "aeif_cond_beta": 3, "spike_generator": 4,
          "parrot_neuron": 5}
PARAMS = {"tau_m": 0, "C_m": 1, "E_L": 2, "V_th": 3, "V_reset": 4, "t_ref": 5, "g_L": 6, "Delta_T": 7,
          "V_T": 8, "tau_w": 9, "a": 10, "b": 11, "V_peak": 12, "V_r": 13, "rk_eps": 14, "rk_hmin": 15}
PORT_PARAMS = {"tau_syn": 0, "E_rev": 1, "tau_rise": 2}
STATE = {"V_m": 0, "I_e": 1, "w": 2, "g": 3, "I_syn": 4, "refr": 5, "h": 6, "g_rise": 7}
DELAYS = {"const": 0, "uniform": 1, "normal": 2}
WEIGHT_DISTS = {"uniform": 0, "normal": 1}
# connection rules; a projection's "K" is the in-degree, the out-degree or the
# number of synapses (unused for all_to_all and one_to_one)
RULES = {"fixed_indegree": 0, "fixed_outdegree": 1, "all_to_all": 2, "one_to_one": 3, "fixed_total_number": 4}
F_NO_SPIKE_RECORD = 1
F_DELIVERY_DIRECT = 2
F_DELIVERY_BINNED = 4
DELIVERY = {"auto": 0, "direct": F_DELIVERY_DIRECT, "binned": F_DELIVERY_BINNED}
STDP_DEFAULTS = dict(tau_plus=20.0, tau_minus=20.0, lambda_=0.01, alpha=1.0, mu_plus=1, mu_minus=1, w_max=100.0)


class SnnError(RuntimeError):
    pass


class Config(C.Structure):
    _fields_ = [("dt_ms", C.c_double), ("seed", C.c_uint64), ("max_delay_steps", C.c_uint32),
                ("flags", C.c_uint32), ("tile_neurons", C.c_uint32), ("bin_capacity", C.c_uint32),
                ("delivery_blocks", C.c_uint32), ("reserved", C.c_uint32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Device(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p), ("stream", C.c_void_p)]


class Counters(C.Structure):
    _fields_ = [("steps", C.c_uint64), ("spikes", C.c_uint64), ("events", C.c_uint64), ("pairs", C.c_uint64),
                ("rk_accepted", C.c_uint64), ("rk_rejected", C.c_uint64), ("n_neurons", C.c_uint64),
                ("n_synapses", C.c_uint64), ("n_groups", C.c_uint64), ("device_bytes", C.c_uint64),
                ("build_ms", C.c_double), ("simulate_ms", C.c_double), ("overflow", C.c_uint32),
                ("max_delay_used", C.c_uint32), ("spill_events", C.c_uint64), ("delivery", C.c_uint32),
                ("tile_neurons", C.c_uint32), ("delivery_blocks", C.c_uint32), ("delivery_queue", C.c_uint32),
                ("last_call_device_ms", C.c_double), ("tile_runs", C.c_uint32),
                ("tile_window", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class JobInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("attempts", C.c_uint32), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double), ("device_bytes_peak", C.c_uint64), ("error", C.c_char * 200)]


class ServerStats(C.Structure):
    _fields_ = [("budget", C.c_uint64), ("in_use", C.c_uint64), ("peak", C.c_uint64), ("queued", C.c_uint32),
                ("running", C.c_uint32), ("done", C.c_uint64), ("failed", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3

# function name -> (restype, argtypes) as declared in include/snn.h
_P = C.c_void_p
_SIGS = {
    "snn_create_net": (C.c_int32, [C.POINTER(Config), C.POINTER(Device), C.POINTER(C.c_void_p)]),
    "snn_destroy_net": (None, [_P]),
    "snn_last_error": (C.c_char_p, [_P]),
    "snn_create": (C.c_int32, [_P, C.c_int32, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32)]),
    "snn_begin_instance": (C.c_int32, [_P, C.c_uint64, C.POINTER(C.c_uint32)]),
    "snn_set_param": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_int32, C.POINTER(C.c_double), C.c_size_t]),
    "snn_param_distribution": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_int32, C.c_int32, C.c_double,
                                           C.c_double, C.c_double, C.c_double, C.c_uint32]),
    "snn_set_port_param": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int32, C.c_double]),
    "snn_connect_fixed_indegree": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                               C.c_double, C.c_int32, C.c_double, C.c_double, C.c_uint32]),
    "snn_snapshot_size": (C.c_int32, [_P, C.POINTER(C.c_size_t)]),
    "snn_snapshot": (C.c_int32, [_P, C.c_void_p, C.c_size_t]),
    "snn_restore": (C.c_int32, [_P, C.c_void_p, C.c_size_t]),
    "snn_set_spike_times": (C.c_int32, [_P, C.c_uint32, C.POINTER(C.c_double), C.c_size_t]),
    "snn_multimeter": (C.c_int32, [_P, C.c_int32, C.c_uint32, C.POINTER(C.c_uint32), C.c_size_t, C.c_uint32,
                                   C.POINTER(C.c_uint32)]),
    "snn_get_samples": (C.c_int32, [_P, C.c_uint32, C.POINTER(C.c_uint64), C.POINTER(C.c_double), C.c_size_t,
                                    C.POINTER(C.c_size_t)]),
    "snn_connect_list": (C.c_int32, [_P, C.c_size_t, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                     C.POINTER(C.c_double), C.c_double, C.c_uint32]),
    "snn_connect": (C.c_int32, [_P, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                C.c_double, C.c_int32, C.c_double, C.c_double, C.c_uint32]),
    "snn_weight_distribution": (C.c_int32, [_P, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                            C.c_uint32]),
    "snn_list_weights": (C.c_int32, [_P, C.POINTER(C.c_double), C.c_size_t]),
    "snn_stdp": (C.c_int32, [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                             C.c_double]),
    "snn_get_weights": (C.c_int32, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
    "snn_state_distribution": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_int32, C.c_uint32, C.c_int32,
                                           C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32]),
    "snn_poisson": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_double, C.c_uint32, C.c_double, C.c_uint32]),
    "snn_set_state": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_int32, C.c_uint32, C.POINTER(C.c_double),
                                  C.c_size_t]),
    "snn_get_state": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_int32, C.c_uint32, C.POINTER(C.c_double)]),
    "snn_build": (C.c_int32, [_P]),
    "snn_release": (C.c_int32, [_P]),
    "snn_simulate": (C.c_int32, [_P, C.c_double]),
    "snn_simulate_steps": (C.c_int32, [_P, C.c_uint64]),
    "snn_get_spikes": (C.c_int32, [_P, C.c_uint64, C.c_uint64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32),
                                   C.POINTER(C.c_uint32), C.c_size_t, C.POINTER(C.c_size_t)]),
    "snn_get_counters": (C.c_int32, [_P, C.POINTER(Counters)]),
    "snn_get_input": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_int64)]),
    "snn_get_input_noalloc": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_int64)]),
    "snn_get_shift": (C.c_int32, [_P, C.c_uint32, C.c_uint32, C.POINTER(C.c_int32)]),
    "snn_poisson_counts": (C.c_int32, [_P, C.c_uint64, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32)]),
    "snn_profile_steps": (C.c_int32, [_P, C.c_uint64, C.POINTER(C.c_double)]),
    "snn_server_create": (C.c_int32, [C.c_size_t, C.c_uint32, C.POINTER(C.c_void_p)]),
    "snn_server_destroy": (None, [_P]),
    "snn_server_submit": (C.c_int32, [_P, _P, C.c_uint64, C.POINTER(C.c_uint64)]),
    "snn_server_poll": (C.c_int32, [_P, C.c_uint64, C.POINTER(C.c_int32)]),
    "snn_server_wait": (C.c_int32, [_P, C.c_uint64, C.c_double]),
    "snn_server_result": (C.c_int32, [_P, C.c_uint64, C.POINTER(C.c_void_p), C.POINTER(JobInfo)]),
    "snn_server_get_stats": (C.c_int32, [_P, C.POINTER(ServerStats)]),
    "snn_export_synapses": (C.c_int32, [_P, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
}

_lib = None


def lib():
    """Load libsnn.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch's HIP runtime (and the HSA runtime it loads) must be in the
        # process before libsnn.so resolves libhsa-runtime64.so.1, so that one
        # HSA runtime serves both the library and torch's allocator
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2007_14236_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


class TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator."""

    def __init__(self, device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.live = {}
        self._alloc = ALLOC_FN(self._a)
        self._free = FREE_FN(self._f)

    def _a(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _f(self, ptr, user):
        self.live.pop(ptr, None)

    def device_struct(self) -> Device:
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        return Device(self._alloc, self._free, None, s or None)


class Net:
    """A network on the GPU, defined from a specification dictionary, or a
    batch of independent networks (one instance per specification) that
    advance together in the same kernels.

    Specification: "dt", "seed", "dmax"; "populations" (name, model, n,
    ports, params; optional V0 and I_e as scalars or arrays, "state_dists"
    {variable: distribution}, "spike_times" for spike generators);
    "projections" (src, tgt, rule, K, weight or "weight_dist", delay
    (kind, a, b), port; or rule "list" with src_gids, tgt_gids, delays_ms and
    a weight or per-connection "weights"); "poisson" (tgt, rate, n_inputs,
    weight, port); "multimeters" (var, gids, interval, port).  A distribution
    is {"kind": "uniform", "low", "high"} or {"kind": "normal", "mean", "sd",
    "low", "high"} with "levels" bins (weights 64, states 1024 by default)."""

    def __init__(self, spec, allocator: TorchAllocator | None = None, record: bool = True, build: bool = True,
                 delivery: str = "auto", tile_neurons: int = 0, bin_capacity: int = 0, delivery_blocks: int = 0):
        self.L = lib()
        specs = list(spec) if isinstance(spec, (list, tuple)) else [spec]
        self.spec = spec
        self.alloc = allocator if allocator is not None else TorchAllocator()
        dt, dmax = specs[0]["dt"], specs[0]["dmax"]
        for sp in specs:
            if sp["dt"] != dt or sp["dmax"] != dmax:
                raise ValueError("all instances of a batch share dt and Dmax")
        flags = (0 if record else F_NO_SPIKE_RECORD) | DELIVERY[delivery]
        cfg = Config(dt, specs[0]["seed"], dmax, flags, tile_neurons, bin_capacity, delivery_blocks, 0)
        self._dev = self.alloc.device_struct()
        h = C.c_void_p()
        self._check(self.L.snn_create_net(C.byref(cfg), C.byref(self._dev), C.byref(h)), None)
        self.h = h
        self.N = 0
        self.instances = []
        self.meters = []  # multimeter ids in specification order (all instances)
        for sp in specs:
            iid = C.c_uint32()
            self._check(self.L.snn_begin_instance(self.h, int(sp["seed"]), C.byref(iid)))
            self.instances.append(self._define(sp))
        self.ranges = self.instances[0]["ranges"]
        if build:
            self.build()

    def _define(self, spec) -> dict:
        first_gid = self.N
        ranges = {}
        for p in spec["populations"]:
            first = C.c_uint32()
            self._check(self.L.snn_create(self.h, MODELS[p["model"]], p["n"], p["ports"], C.byref(first)))
            ranges[p["name"]] = (first.value, p["n"])
            self.N += p["n"]
            for j, times in enumerate(p.get("spike_times", []) or []):
                t = np.ascontiguousarray(times, dtype=np.float64)
                self._check(self.L.snn_set_spike_times(self.h, first.value + j, _ptr(t, C.c_double), len(t)))
            for k, v in p["params"].items():
                if k in PARAMS:  # a scalar for the population, or one value per neuron
                    x = np.ascontiguousarray(np.atleast_1d(np.asarray(v, dtype=np.float64)))
                    self._check(self.L.snn_set_param(self.h, first.value, p["n"], PARAMS[k], _ptr(x, C.c_double),
                                                     len(x)))
                elif k in PORT_PARAMS:
                    for port, x in enumerate(v[: p["ports"]]):
                        self._check(self.L.snn_set_port_param(self.h, first.value, p["n"], port,
                                                              PORT_PARAMS[k], float(x)))
        for p in spec["populations"]:  # model parameters drawn per neuron: {"V_th": {...}, ...}
            t0, tn = ranges[p["name"]]
            for k, wd in (p.get("param_dists") or {}).items():
                self._check(self.L.snn_param_distribution(self.h, t0, tn, PARAMS[k], *self._dist_args(wd, 1024)))
        for pr in spec["projections"]:
            if pr.get("rule") == "list":  # user-defined: gids counted from the specification's first neuron
                src = np.ascontiguousarray(np.asarray(pr["src_gids"], dtype=np.int64) + first_gid, dtype=np.uint32)
                tgt = np.ascontiguousarray(np.asarray(pr["tgt_gids"], dtype=np.int64) + first_gid, dtype=np.uint32)
                dl = np.ascontiguousarray(pr["delays_ms"], dtype=np.float64)
                self._check(self.L.snn_connect_list(self.h, len(src), _ptr(src, C.c_uint32), _ptr(tgt, C.c_uint32),
                                                    _ptr(dl, C.c_double), float(pr.get("weight", 0.0)), pr["port"]))
                if pr.get("weights") is not None:  # one weight per listed connection
                    w = np.ascontiguousarray(pr["weights"], dtype=np.float64)
                    self._check(self.L.snn_list_weights(self.h, _ptr(w, C.c_double), len(w)))
                self._stdp(pr)
                continue
            s0, sn = ranges[pr["src"]]
            t0, tn = ranges[pr["tgt"]]
            kind, a, b = (list(pr["delay"]) + [0.0, 0.0])[:3]
            self._check(self.L.snn_connect(self.h, RULES[pr.get("rule", "fixed_indegree")], int(pr.get("K", 0)), s0, sn,
                                           t0, tn, float(pr.get("weight", 0.0)), DELAYS[kind], float(a), float(b),
                                           pr["port"]))
            wd = pr.get("weight_dist")
            if wd is not None:  # uniform on [low, high), or normal(mean, sd) truncated to [low, high]
                L = int(wd.get("levels", 64))
                if wd["kind"] == "uniform":
                    args = (WEIGHT_DISTS["uniform"], float(wd["low"]), float(wd["high"]), 0.0, 0.0, L)
                else:
                    m, sd = float(wd["mean"]), float(wd["sd"])
                    args = (WEIGHT_DISTS["normal"], m, sd, float(wd.get("low", m - 4 * sd)),
                            float(wd.get("high", m + 4 * sd)), L)
                self._check(self.L.snn_weight_distribution(self.h, *args))
            self._stdp(pr)
        for q in spec.get("poisson", []):
            t0, tn = ranges[q["tgt"]]
            self._check(self.L.snn_poisson(self.h, t0, tn, float(q["rate"]), int(q["n_inputs"]),
                                           float(q["weight"]), q["port"]))
        # multimeters: "var", "interval", "port" and the recorded neurons as
        # "gids" counted from the specification's first neuron
        for mm in spec.get("multimeters", []):
            g = np.ascontiguousarray(np.asarray(mm["gids"], dtype=np.int64) + first_gid, dtype=np.uint32)
            mid = C.c_uint32()
            self._check(self.L.snn_multimeter(self.h, STATE[mm["var"]], int(mm.get("port", 0)), _ptr(g, C.c_uint32),
                                              len(g), int(mm.get("interval", 1)), C.byref(mid)))
            self.meters.append(mid.value)
        for p in spec["populations"]:
            t0, tn = ranges[p["name"]]
            if p.get("V0") is not None:
                self.set_state("V_m", t0, np.asarray(p["V0"], dtype=np.float64))
            ie = p.get("I_e", 0.0)
            self.set_state("I_e", t0, np.atleast_1d(np.asarray(ie, dtype=np.float64)), n=tn)
            # state drawn from distributions, after the arrays: {"V_m": {...}, "I_e": {...}, ...}
            for var, wd in (p.get("state_dists") or {}).items():
                L = int(wd.get("levels", 1024))
                if wd["kind"] == "uniform":
                    args = (WEIGHT_DISTS["uniform"], float(wd["low"]), float(wd["high"]), 0.0, 0.0, L)
                else:
                    m, sd = float(wd["mean"]), float(wd["sd"])
                    args = (WEIGHT_DISTS["normal"], m, sd, float(wd.get("low", m - 4 * sd)),
                            float(wd.get("high", m + 4 * sd)), L)
                self._check(self.L.snn_state_distribution(self.h, t0, tn, STATE[var], int(wd.get("port", 0)), *args))
        return dict(ranges=ranges, first=first_gid, n=self.N - first_gid)

    def _stdp(self, pr: dict):
        """Nearest-neighbour STDP of the projection just created, from its "stdp"
        entry: tau_plus, tau_minus (ms), lambda, alpha, mu_plus, mu_minus (0
        additive, 1 multiplicative) and w_max, NEST-like defaults."""
        sd = pr.get("stdp")
        if sd is None:
            return
        v = dict(STDP_DEFAULTS)
        v.update({("lambda_" if k == "lambda" else k): x for k, x in sd.items()})
        self._check(self.L.snn_stdp(self.h, float(v["tau_plus"]), float(v["tau_minus"]), float(v["lambda_"]),
                                    float(v["alpha"]), int(v["mu_plus"]), int(v["mu_minus"]), float(v["w_max"])))

    @staticmethod
    def _dist_args(wd: dict, default_levels: int) -> tuple:
        """(kind, a, b, lo, hi, levels) of a distribution: uniform on [low, high), or
        normal(mean, sd) truncated to [low, high] (default mean -+ 4 sd)."""
        L = int(wd.get("levels", default_levels))
        if wd["kind"] == "uniform":
            return (WEIGHT_DISTS["uniform"], float(wd["low"]), float(wd["high"]), 0.0, 0.0, L)
        m, sd = float(wd["mean"]), float(wd["sd"])
        return (WEIGHT_DISTS["normal"], m, sd, float(wd.get("low", m - 4 * sd)), float(wd.get("high", m + 4 * sd)), L)

    def _check(self, rc, h=-1):
        if rc != SNN_OK:
            hh = self.h if h == -1 else h
            msg = self.L.snn_last_error(hh).decode() if hh else ""
            raise SnnError(f"{ERRORS.get(rc, rc)}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            self.L.snn_destroy_net(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- calls
    def build(self):
        self._check(self.L.snn_build(self.h))

    def simulate(self, steps: int):
        self._check(self.L.snn_simulate_steps(self.h, int(steps)))

    def simulate_ms(self, t_ms: float):
        self._check(self.L.snn_simulate(self.h, float(t_ms)))

    def profile(self, steps: int) -> dict:
        """Advance `steps` steps with per-kernel HIP event timing (ms summed)."""
        ms = np.zeros(1, dtype=np.float64)
        self._check(self.L.snn_profile_steps(self.h, int(steps), _ptr(ms, C.c_double)))
        return dict(step=ms[0])

    def set_state(self, var: str, first: int, values, port: int = 0, n: int | None = None):
        v = np.ascontiguousarray(values, dtype=np.float64)
        n = len(v) if n is None else n
        self._check(self.L.snn_set_state(self.h, first, n, STATE[var], port, _ptr(v, C.c_double), len(v)))

    def get_state(self, var: str, first: int = 0, n: int | None = None, port: int = 0) -> np.ndarray:
        n = self.N - first if n is None else n
        out = np.zeros(n, dtype=np.float64)
        self._check(self.L.snn_get_state(self.h, first, n, STATE[var], port, _ptr(out, C.c_double)))
        return out

    def spikes(self, step_lo: int = 0, step_hi: int = 2**63):
        """(step, gid, mult) sorted by (step, gid)."""
        n = C.c_size_t(0)
        self._check(self.L.snn_get_spikes(self.h, step_lo, step_hi, None, None, None, 0, C.byref(n)))
        m = n.value
        st = np.zeros(m, np.uint64); gid = np.zeros(m, np.uint32); mult = np.zeros(m, np.uint32)
        if m:
            self._check(self.L.snn_get_spikes(self.h, step_lo, step_hi, _ptr(st, C.c_uint64), _ptr(gid, C.c_uint32),
                                              _ptr(mult, C.c_uint32), m, C.byref(n)))
        return st, gid, mult

    def samples(self, k: int = 0):
        """(steps, values) of multimeter k: values[sample][neuron]."""
        mid, width = self.meters[k], self._meter_width(k)
        n = C.c_size_t(0)
        self._check(self.L.snn_get_samples(self.h, mid, None, None, 0, C.byref(n)))
        m = n.value
        steps = np.zeros(m, np.uint64)
        vals = np.zeros(m * width, np.float64)
        if m:
            self._check(self.L.snn_get_samples(self.h, mid, _ptr(steps, C.c_uint64), _ptr(vals, C.c_double), m,
                                               C.byref(n)))
        return steps, vals.reshape(m, width)

    def _meter_width(self, k: int) -> int:
        specs = list(self.spec) if isinstance(self.spec, (list, tuple)) else [self.spec]
        widths = [len(mm["gids"]) for sp in specs for mm in sp.get("multimeters", [])]
        return widths[k]

    def snapshot(self) -> np.ndarray:
        """The network's dynamic state after the steps simulated so far (bytes)."""
        n = C.c_size_t(0)
        self._check(self.L.snn_snapshot_size(self.h, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self.L.snn_snapshot(self.h, buf.ctypes.data_as(C.c_void_p), buf.size))
        return buf

    def restore(self, snap: np.ndarray):
        """Load a snapshot of a network built from the same specification."""
        b = np.ascontiguousarray(snap, dtype=np.uint8)
        self._check(self.L.snn_restore(self.h, b.ctypes.data_as(C.c_void_p), b.size))

    def counters(self) -> dict:
        c = Counters()
        self._check(self.L.snn_get_counters(self.h, C.byref(c)))
        return c.as_dict()

    def get_input(self, port: int = 0, first: int = 0, n: int | None = None) -> np.ndarray:
        n = self.N - first if n is None else n
        out = np.zeros(n, dtype=np.int64)
        self._check(self.L.snn_get_input(self.h, first, n, port, _ptr(out, C.c_int64)))
        return out

    def get_input_noalloc(self, port: int = 0, first: int = 0, n: int | None = None) -> np.ndarray:
        n = self.N - first if n is None else n
        out = np.zeros(n, dtype=np.int64)
        self._check(self.L.snn_get_input_noalloc(self.h, first, n, port, _ptr(out, C.c_int64)))
        return out

    def shift(self, gid: int, port: int = 0) -> int:
        s = C.c_int32()
        self._check(self.L.snn_get_shift(self.h, gid, port, C.byref(s)))
        return s.value

    def poisson_counts(self, step: int, first: int = 0, n: int | None = None) -> np.ndarray:
        n = self.N - first if n is None else n
        out = np.zeros(n, dtype=np.uint32)
        self._check(self.L.snn_poisson_counts(self.h, step, first, n, _ptr(out, C.c_uint32)))
        return out

    def weights(self) -> np.ndarray:
        """Current fixed-point weight of every synapse, canonical order."""
        n = C.c_size_t(0)
        self._check(self.L.snn_get_weights(self.h, None, C.byref(n)))
        wq = np.zeros(n.value, np.int64)
        self._check(self.L.snn_get_weights(self.h, _ptr(wq, C.c_int64), C.byref(n)))
        return wq

    def synapses(self) -> dict:
        n = C.c_size_t(0)
        self._check(self.L.snn_export_synapses(self.h, None, None, None, None, None, C.byref(n)))
        m = n.value
        src = np.zeros(m, np.uint32); d = np.zeros(m, np.uint32); tgt = np.zeros(m, np.uint32)
        port = np.zeros(m, np.uint32); wq = np.zeros(m, np.int64)
        n = C.c_size_t(m)
        self._check(self.L.snn_export_synapses(self.h, _ptr(src, C.c_uint32), _ptr(d, C.c_uint32),
                                               _ptr(tgt, C.c_uint32), _ptr(port, C.c_uint32),
                                               _ptr(wq, C.c_int64), C.byref(n)))
        return dict(src=src, delay=d, tgt=tgt, port=port, wq=wq)
