"""Seeded synthetic workloads (network specifications).

This module only describes networks: population sizes, model parameters,
projections, Poisson drives, seeds and initial membrane potentials.  It holds
none of the simulation arithmetic; both the GPU library binding and the CPU
oracle consume the same specification dictionaries.

Specification format (plain dict):
    {"dt": ms, "seed": int, "dmax": max delay in steps (<= 63),
     "populations": [{"name", "model", "n", "ports", "params": {...},
                      "V0": float64 array (mV) | None, "I_e": float | array}],
     "projections": [{"src", "tgt", "K", "weight", "delay": (kind, a, b), "port"}],
     "poisson": [{"tgt", "rate", "n_inputs", "weight", "port"}]}
Models: "lif_delta", "lif_exp", "aeif_cond_exp".  Delay kinds: "const" (a),
"uniform" [a, b), "normal" (mean a, sd b; clipped to [dt, dmax dt]).

Workload sources (Golosio et al., arXiv 2007.14236):
  brunel_lif      -- Brunel-style LIF network with delta PSCs (Sec. 2.4 cites
                     Brunel 2000; LIF equation of Sec. 2.3).
  microcircuit    -- stand-in for the Potjans-Diesmann microcircuit (Sec. 2.3):
                     the eight population sizes are the model's, the 8x8
                     connection-probability table is NOT reproduced (it is not
                     given in the paper); a seeded synthetic table with the same
                     layered structure is scaled to 3e8 synapses instead.
  adex_balanced   -- balanced AdEx network of Sec. 2.4 with Table 1 weights and
                     Table 2 neuron parameters, exponential conductances.
  brunel_sweep    -- per-instance parameters of a batched sweep of Brunel nets.
"""
from __future__ import annotations

import math

import numpy as np

DT = 0.1

# Population sizes of the cortical microcircuit (Sec. 2.3): L2/3E, L2/3I, L4E,
# L4I, L5E, L5I, L6E, L6I.
MC_NAMES = ["L23E", "L23I", "L4E", "L4I", "L5E", "L5I", "L6E", "L6I"]
MC_SIZES = [20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948]

# AdEx parameters, Table 2 (pF, nS, mV, ms, pA); V_peak, t_ref and I_e are not
# listed there: V_peak = 0 mV, no refractory period, I_e = 0.
ADEX_T2 = dict(C_m=281.0, g_L=30.0, E_L=-70.6, V_T=-50.4, Delta_T=2.0, tau_w=144.0,
               a=4.0, b=80.5, V_r=-60.0, V_peak=0.0, t_ref=0.0,
               E_rev=[0.0, -85.0], tau_syn=[1.0, 1.0], rk_eps=1e-6)


def _uniform01(seed: int, n: int, stream: int) -> np.ndarray:
    """n values r = (u32 >> 8) * 2^-24 in [0, 1), exact in float32, from
    numpy's Philox with key (seed, stream)."""
    g = np.random.Generator(np.random.Philox(key=[seed, stream]))
    u = g.integers(0, 2**32, size=n, dtype=np.uint64)
    return ((u >> np.uint64(8)).astype(np.float64)) * 2.0**-24


def initial_v(seed: int, n: int, lo: float, hi: float, stream: int = 7) -> np.ndarray:
    """Initial membrane potentials lo + (hi - lo) r, rounded to float32 values."""
    r = _uniform01(seed, n, stream).astype(np.float32)
    lo32, span = np.float32(lo), np.float32(hi) - np.float32(lo)
    return (lo32 + span * r).astype(np.float32).astype(np.float64)


def brunel_lif(n: int = 1000, k: int = 100, g: float = 5.0, j: float = 0.1,
               nu_ext: float = 20.0, c_ext: int = 80, delay=("const", 1.5, 0.0),
               seed: int = 1, dmax: int = 63) -> dict:
    """Brunel network of LIF neurons with delta PSCs, 80% E / 20% I, fixed
    in-degree k (80% from E, 20% from I), E weight j (mV), I weight -g j,
    tau_m 20 ms, V_th 20 mV, V_reset 10 mV, t_ref 2 ms, E_L 0, Poisson drive of
    c_ext inputs at nu_ext Hz with weight j."""
    ne = (n * 4) // 5
    ni = n - ne
    ke = (k * 4) // 5
    ki = k - ke
    params = dict(tau_m=20.0, C_m=250.0, E_L=0.0, V_th=20.0, V_reset=10.0, t_ref=2.0)
    pops = [
        dict(name="E", model="lif_delta", n=ne, ports=1, params=dict(params),
             V0=initial_v(seed, ne, 0.0, 20.0, stream=7), I_e=0.0),
        dict(name="I", model="lif_delta", n=ni, ports=1, params=dict(params),
             V0=initial_v(seed, ni, 0.0, 20.0, stream=8), I_e=0.0),
    ]
    projs = []
    for tgt in ("E", "I"):
        projs.append(dict(src="E", tgt=tgt, K=ke, weight=j, delay=tuple(delay), port=0))
        projs.append(dict(src="I", tgt=tgt, K=ki, weight=-g * j, delay=tuple(delay), port=0))
    pois = [dict(tgt=t, rate=nu_ext, n_inputs=c_ext, weight=j, port=0) for t in ("E", "I")]
    return dict(name=f"brunel_lif_n{n}", dt=DT, seed=seed, dmax=dmax, populations=pops,
                projections=projs, poisson=pois)


def c0(active: bool = False) -> dict:
    """1,000-neuron Brunel LIF net, in-degree 100, g = 5, delay 1.5 ms, Poisson
    20 Hz x 80 inputs (active=True: 250 Hz, the asynchronous-irregular regime)."""
    return brunel_lif(nu_ext=250.0 if active else 20.0)


MC_TABLE = (0.08, 0.16, 0.25, 0.25, 0.02, 0.01)


def _mc_table(seed: int = 11, base=MC_TABLE) -> np.ndarray:
    """Synthetic 8x8 connection probabilities p[target, source] from the base
    values (same-layer E->E, E->I, I->E, I->I, cross-layer from E, cross-layer
    from I), each times U[0.5, 1.5) (numpy Philox, key (seed, 0)).
    Inhibition dominates every population's input and inhibitory populations
    receive more excitation than excitatory ones, as in layered cortical
    models."""
    ee, ei, ie, ii, xe, xi = base
    g = np.random.Generator(np.random.Philox(key=[seed, 0]))
    mult = g.uniform(0.5, 1.5, size=(8, 8))
    p = np.zeros((8, 8))
    for t in range(8):
        for s in range(8):
            same = (t // 2) == (s // 2)
            src_e, tgt_e = (s % 2) == 0, (t % 2) == 0
            if same:
                p[t, s] = (ee if tgt_e else ei) if src_e else (ie if tgt_e else ii)
            else:
                p[t, s] = xe if src_e else xi
    return p * mult


def microcircuit(scale: float = 1.0, k_scale: float | None = None, k_ext: int = 2800,
                 nu_bg: float = 8.0, seed: int = 1, total_synapses: float = 3.0e8,
                 dmax: int = 63, table=MC_TABLE, weight_sd: float = 0.0, weight_levels: int = 32) -> dict:
    """Microcircuit stand-in: LIF neurons with exponential PSCs (one port,
    signed weights), tau_m 10 ms, C_m 250 pF, tau_syn 0.5 ms, E_L = V_reset =
    -65 mV, V_th -50 mV, t_ref 2 ms; w_E 87.8 pA (L4E->L2/3E doubled), w_I =
    -4 w_E; delays normal 1.5 +- 0.75 ms (E sources) and 0.75 +- 0.375 ms (I
    sources); Poisson background nu_bg x k_ext inputs with weight w_E.
    Population sizes are scaled by `scale`; in-degrees by `k_scale` (default:
    `scale`, i.e. fixed connection probabilities).  weight_sd > 0 draws every
    synaptic weight from a normal distribution of that relative deviation
    around the projection's weight (truncated to mean +- 4 sd, which keeps
    the sign for weight_sd < 0.25), discretised into `weight_levels` bins."""
    if k_scale is None:
        k_scale = scale
    p = _mc_table(base=table)
    n_full = np.array(MC_SIZES, dtype=np.float64)
    # global factor so that sum_ij p_ij N_i N_j = total_synapses at full scale
    p = p * (total_synapses / float(np.sum(p * np.outer(n_full, n_full))))
    sizes = [max(1, int(round(s * scale))) for s in MC_SIZES]
    w_e = 87.8
    params = dict(tau_m=10.0, C_m=250.0, E_L=-65.0, V_th=-50.0, V_reset=-65.0, t_ref=2.0,
                  tau_syn=[0.5])
    pops = []
    for i, (name, n) in enumerate(zip(MC_NAMES, sizes)):
        pops.append(dict(name=name, model="lif_exp", n=n, ports=1, params=dict(params),
                         V0=initial_v(seed, n, -65.0, -50.0, stream=100 + i), I_e=0.0))
    projs = []
    for t in range(8):
        for s in range(8):
            k = int(round(p[t, s] * MC_SIZES[s] * k_scale))
            if k <= 0:
                continue
            src_e = (s % 2) == 0
            w = w_e if src_e else -4.0 * w_e
            if s == 2 and t == 0:
                w = 2.0 * w_e
            d = ("normal", 1.5, 0.75) if src_e else ("normal", 0.75, 0.375)
            pr = dict(src=MC_NAMES[s], tgt=MC_NAMES[t], K=k, weight=w, delay=d, port=0)
            if weight_sd > 0:
                pr["weight_dist"] = dict(kind="normal", mean=w, sd=abs(w) * weight_sd, levels=weight_levels)
            projs.append(pr)
    pois = [dict(tgt=nm, rate=nu_bg, n_inputs=int(round(k_ext * k_scale)), weight=w_e, port=0)
            for nm in MC_NAMES]
    return dict(name=f"microcircuit_s{scale:g}", dt=DT, seed=seed, dmax=dmax, populations=pops,
                projections=projs, poisson=pois)


def adex_balanced(n: int = 1_000_000, k: int = 1000, seed: int = 1, dmax: int = 63,
                  delay=("uniform", 1.0, 2.0), w_ex: float = 0.05 * math.e, w_in: float = 0.35 * math.e,
                  poisson_rate: float = 20000.0, w_poisson: float = 0.37 * math.e) -> dict:
    """Balanced AdEx network (Sec. 2.4): N_in = N_ex/4, CI = CE/4, Table 2
    neuron parameters, Poisson 20 kHz on port 0, delays U[1, 2) ms, RK45
    tolerance 1e-6, exponential conductances (tau 1 ms; port 0 E_rev 0 mV,
    port 1 E_rev -85 mV).  Table 1 gives the peak conductances W_ex 0.05,
    W_in 0.35, W_poisson 0.37 nS of the paper's alpha-shaped conductance; an
    alpha kernel with peak w carries e w tau of charge, an exponential kernel
    with jump w carries w tau, so the exponential weights are the Table 1
    values times e (same charge per spike)."""
    ne = (n * 4) // 5
    ni = n - ne
    ke = (k * 4) // 5
    ki = k - ke
    prm = dict(ADEX_T2)
    pops = [
        dict(name="E", model="aeif_cond_exp", n=ne, ports=2, params=dict(prm),
             V0=initial_v(seed, ne, prm["E_L"], prm["V_T"], stream=7), I_e=0.0),
        dict(name="I", model="aeif_cond_exp", n=ni, ports=2, params=dict(prm),
             V0=initial_v(seed, ni, prm["E_L"], prm["V_T"], stream=8), I_e=0.0),
    ]
    projs = []
    for tgt in ("E", "I"):
        projs.append(dict(src="E", tgt=tgt, K=ke, weight=w_ex, delay=tuple(delay), port=0))
        projs.append(dict(src="I", tgt=tgt, K=ki, weight=w_in, delay=tuple(delay), port=1))
    pois = [dict(tgt=t, rate=poisson_rate, n_inputs=1, weight=w_poisson, port=0) for t in ("E", "I")]
    return dict(name=f"adex_balanced_n{n}", dt=DT, seed=seed, dmax=dmax, populations=pops,
                projections=projs, poisson=pois)


def adex_balanced_alpha(n: int = 1_000_000, k: int = 1000, seed: int = 1, dmax: int = 63,
                        delay=("normal", 0.5, 0.25), w_ex: float = 0.05, w_in: float = 0.35,
                        poisson_rate: float = 20000.0, w_poisson: float = 0.37) -> dict:
    """The balanced network as Sec. 2.4 and Table 1 give it: AdEx neurons with
    alpha-function conductances (beta ports with rise = decay = 1 ms; port 0
    E_rev 0 mV, port 1 E_rev -85 mV), N_in = N_ex/4, CI = CE/4, peak
    conductances W_ex 0.05, W_in 0.35, W_poisson 0.37 nS, Poisson 20 kHz on
    port 0, delays normal with mean 0.5 ms and standard deviation 0.25 ms
    (clipped to at least one step), Table 2 neuron parameters, RK45 tolerance
    1e-6."""
    ne = (n * 4) // 5
    ni = n - ne
    ke = (k * 4) // 5
    ki = k - ke
    prm = dict(ADEX_T2)
    prm["tau_rise"] = list(prm["tau_syn"])
    pops = [
        dict(name="E", model="aeif_cond_beta", n=ne, ports=2, params=dict(prm),
             V0=initial_v(seed, ne, prm["E_L"], prm["V_T"], stream=7), I_e=0.0),
        dict(name="I", model="aeif_cond_beta", n=ni, ports=2, params=dict(prm),
             V0=initial_v(seed, ni, prm["E_L"], prm["V_T"], stream=8), I_e=0.0),
    ]
    projs = []
    for tgt in ("E", "I"):
        projs.append(dict(src="E", tgt=tgt, K=ke, weight=w_ex, delay=tuple(delay), port=0))
        projs.append(dict(src="I", tgt=tgt, K=ki, weight=w_in, delay=tuple(delay), port=1))
    pois = [dict(tgt=t, rate=poisson_rate, n_inputs=1, weight=w_poisson, port=0) for t in ("E", "I")]
    return dict(name=f"adex_alpha_n{n}_k{k}", dt=DT, seed=seed, dmax=dmax, populations=pops,
                projections=projs, poisson=pois)


def brunel_sweep_instance(i: int) -> dict:
    """Instance i of the batched sweep: N ~ U[2000, 40000] (multiple of 5,
    80/20), in-degree 0.1 N, g ~ U[3, 7], drive nu ~ U[10, 30] Hz from
    0.08 N inputs, J = 0.1 mV, delays U[0.1, 3) ms, seed 1000 + i."""
    g = np.random.Generator(np.random.Philox(key=[3, i]))
    n = int(round(g.uniform(2000, 40000) / 5.0)) * 5
    gg = float(g.uniform(3.0, 7.0))
    nu = float(g.uniform(10.0, 30.0))
    return brunel_lif(n=n, k=max(5, int(round(0.1 * n))), g=gg, j=0.1, nu_ext=nu,
                      c_ext=int(round(0.08 * n)), delay=("uniform", 0.1, 3.0), seed=1000 + i)


def count_synapses(spec: dict) -> int:
    sizes = {p["name"]: p["n"] for p in spec["populations"]}
    total = 0
    for pr in spec["projections"]:
        if pr.get("rule") == "list":
            total += len(pr["src_gids"])
            continue
        rule, ns, nt = pr.get("rule", "fixed_indegree"), sizes[pr["src"]], sizes[pr["tgt"]]
        total += {"fixed_indegree": pr.get("K", 0) * nt, "fixed_outdegree": pr.get("K", 0) * ns if nt else 0,
                  "all_to_all": ns * nt, "one_to_one": nt,
                  "fixed_total_number": pr.get("K", 0) if nt else 0}[rule]
    return int(total)


def population_ranges(spec: dict) -> dict:
    """name -> (first gid, n) in creation order."""
    out, first = {}, 0
    for p in spec["populations"]:
        out[p["name"]] = (first, p["n"])
        first += p["n"]
    return out


def total_neurons(spec: dict) -> int:
    return int(sum(p["n"] for p in spec["populations"]))


def steps_for(t_ms: float, dt: float = DT) -> int:
    return int(math.floor(t_ms / dt + 0.5))
