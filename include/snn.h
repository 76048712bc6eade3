/*
 * snn.h -- C ABI of the MI355X (gfx950) spiking-network engine.
 *
 * The engine implements the per-time-step hot path of the GPU simulator of
 * Golosio et al., "Fast simulations of highly-connected spiking cortical
 * models using GPUs" (arXiv 2007.14236):
 *   - spike delivery (Sec. 2.2 and Fig. 1): every spike is buffered per source
 *     neuron; each step the (source, connection-group) pairs whose delay has
 *     just elapsed are selected, the outgoing synapses of those groups are
 *     scanned in one flat parallel pass, and their weights are accumulated into
 *     the receptor inputs of the targets;
 *   - the neuron update beside it (Sec. 2.1): LIF exact integration (LIF and
 *     exponential-PSC equations of Sec. 2.3) and multisynapse AdEx with
 *     conductance synapses (Sec. 2.4, Table 2) integrated by an adaptive
 *     fifth-order Runge-Kutta method.
 * The calls follow the paper's statement of the problem (Sec. 2.1 and its
 * code sample): create populations of a neuron model with n receptor ports,
 * set parameters, connect by rule with weight, delay and receptor, attach
 * Poisson generators, simulate T ms at a time step dt, read back the spike
 * raster and the state.
 *
 * Conventions
 *   - Units: ms, mV, pA, nS, pF, Hz.
 *   - Neurons are numbered by global id (gid) in creation order.
 *   - Every call returns SNN_OK (0) or a negative snn_status; the message of
 *     the last failure of a handle is returned by snn_last_error().  A failed
 *     call leaves the handle usable.  No C++ exception crosses this ABI.
 *   - Pointers named out / v / host arrays are caller-owned HOST memory.  All
 *     device memory is owned by the library (allocated through the optional
 *     snn_device callbacks, else hipMalloc) and released by snn_destroy_net.
 *   - Calls on one handle must not overlap (not thread-safe per handle).
 *   - Phases: populations, parameters, connections and Poisson drives are
 *     defined before snn_build(); snn_simulate() and the readback calls come
 *     after it.  A call in the wrong phase returns SNN_E_STATE.
 */
#ifndef SNN_H
#define SNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t snn_status;
#define SNN_OK 0
#define SNN_E_INVALID (-1)     /* bad argument                                  */
#define SNN_E_NOMEM (-2)       /* device or host allocation failed              */
#define SNN_E_STATE (-3)       /* call not allowed in the current phase         */
#define SNN_E_OVERFLOW (-4)    /* a device-side capacity or range was exceeded  */
#define SNN_E_DEVICE (-5)      /* HIP runtime error                             */
#define SNN_E_BUDGET (-6)      /* request larger than the server's memory budget */
#define SNN_E_UNSUPPORTED (-7) /* valid request outside what is implemented     */

typedef struct snn_net snn_net;

/* Optional device-memory provider.  alloc returns a device pointer (or NULL on
   failure) of at least `bytes` bytes, 256-byte aligned; free releases it.
   `stream` is a hipStream_t the caller orders its own work on (may be NULL):
   the library runs its work on a private stream and orders it after the
   caller's stream at the start of every call and before it at the end. */
typedef struct snn_device {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
  void* stream;
} snn_device;

typedef struct snn_config {
  double dt_ms;             /* simulation resolution (ms), > 0                  */
  uint64_t seed;            /* key of the counter-based generator               */
  uint32_t max_delay_steps; /* Dmax, 1..63; longer delays fold into Dmax        */
  uint32_t flags;           /* SNN_F_* below                                    */
  uint32_t tile_neurons;    /* binned delivery: neurons per target tile, a power
                               of two in [256, 4096 / P2] with P2 the port count
                               rounded up to a power of two; 0 = library choice
                               (the largest, or for AdEx networks the largest
                               that leaves at least 128 tiles, at least 256) */
  uint32_t bin_capacity;    /* binned delivery: entries per tile bin (each of
                               two input buffers); 0 = library choice, at most
                               the number of synapses onto the tile.  Events
                               beyond it are still delivered exactly (atomics) */
  uint32_t delivery_blocks; /* blocks that deliver delays >= 2, 1..8192;
                               0 = library choice                             */
  uint32_t reserved;        /* 0                                              */
} snn_config;
#define SNN_F_NO_SPIKE_RECORD 1u /* do not keep the spike raster on the host */
/* How a step's synaptic events are summed into the targets' integer inputs
   (Sec. 2.2; the sum is the same either way).  Neither flag: binned for
   networks of 5e8 synapses or more and for networks with AdEx neurons when
   they fit its limits (at most 1024 tiles), else direct. */
#define SNN_F_DELIVERY_DIRECT 2u /* each event one device-scope int64 atomic add */
#define SNN_F_DELIVERY_BINNED 4u /* each event a 32-bit entry in its target tile's
                                    bin, summed in LDS by the tile's block at the
                                    next step; SNN_E_UNSUPPORTED if it does not fit */

/* neuron models (Sec. 2.1, 2.3, 2.4) */
#define SNN_LIF_PSC_DELTA 0  /* LIF, delta PSCs: weights in mV, one port      */
#define SNN_LIF_PSC_EXP 1    /* LIF, exponential PSCs: weights in pA          */
#define SNN_AEIF_COND_EXP 2  /* AdEx, exponential conductances: weights in nS */
/* AdEx with beta-function conductances (the receptor model of the Sec. 2.1
   example; tau_rise = tau_decay gives the alpha function of Sec. 2.4): per
   port dg/dt = r - g/tau_decay, dr/dt = -r/tau_rise, and an input of weight
   w (nS) adds g0 w to r, g0 chosen so that a lone input's conductance peaks
   at exactly w.  A network may mix it with SNN_AEIF_COND_EXP populations. */
#define SNN_AEIF_COND_BETA 3
/* devices (Sec. 2.1), one port each: a spike generator emits its listed
   times (snn_set_spike_times); a parrot neuron emits, at each step, one spike
   per spike arriving then (multiplicity; every weight onto it must be 1) */
#define SNN_SPIKE_GENERATOR 4
#define SNN_PARROT_NEURON 5

/* model parameters (snn_set_param): per population, or per neuron */
#define SNN_P_TAU_M 0    /* LIF membrane time constant (ms)                   */
#define SNN_P_C_M 1      /* membrane capacitance (pF)                         */
#define SNN_P_E_L 2      /* leak reversal / resting potential (mV)            */
#define SNN_P_V_TH 3     /* LIF threshold (mV)                                */
#define SNN_P_V_RESET 4  /* LIF reset potential (mV)                          */
#define SNN_P_T_REF 5    /* refractory time (ms); AdEx supports only 0        */
#define SNN_P_G_L 6      /* AdEx leak conductance (nS)                        */
#define SNN_P_DELTA_T 7  /* AdEx slope factor (mV)                            */
#define SNN_P_V_T 8      /* AdEx spike-initiation threshold (mV)              */
#define SNN_P_TAU_W 9    /* AdEx adaptation time constant (ms)                */
#define SNN_P_A 10       /* AdEx subthreshold adaptation (nS)                 */
#define SNN_P_B 11       /* AdEx spike-triggered adaptation (pA)              */
#define SNN_P_V_PEAK 12  /* AdEx spike detection / reset trigger (mV)         */
#define SNN_P_V_R 13     /* AdEx reset potential (mV)                         */
#define SNN_P_RK_EPS 14  /* AdEx RK45 relative tolerance                      */
#define SNN_P_RK_HMIN 15 /* AdEx smallest RK45 substep (ms)                   */
/* port parameters (snn_set_port_param) */
#define SNN_PP_TAU_SYN 0 /* synaptic (for beta ports: decay) time constant (ms) */
#define SNN_PP_E_REV 1   /* AdEx reversal potential (mV)                      */
#define SNN_PP_TAU_RISE 2 /* beta ports: rise time constant (ms), default 1   */

/* state variables (snn_set_state / snn_get_state), per neuron */
#define SNN_V_M 0        /* membrane potential (mV)                           */
#define SNN_V_I_E 1      /* constant external current (pA)                    */
#define SNN_V_W 2        /* AdEx adaptation current (pA)                      */
#define SNN_V_G 3        /* AdEx conductance of `port` (nS)                   */
#define SNN_V_I_SYN 4    /* LIF-exp synaptic current of `port` (pA)           */
#define SNN_V_REFR 5     /* remaining refractory steps                        */
#define SNN_V_H 6        /* AdEx carried RK45 step size (ms)                  */
#define SNN_V_G_RISE 7   /* beta port's rising variable r of `port` (nS/ms)   */

/* delay distributions (in ms; converted to steps of dt, rounded half up,
   clipped to [1, Dmax]) */
#define SNN_DELAY_CONST 0          /* a                                       */
#define SNN_DELAY_UNIFORM 1        /* uniform on [a, b)                       */
#define SNN_DELAY_NORMAL_CLIPPED 2 /* normal, mean a, standard deviation b    */

typedef struct snn_counters {
  uint64_t steps;          /* steps simulated so far                          */
  uint64_t spikes;         /* spike events recorded (multiplicity counted 1)  */
  uint64_t events;         /* synaptic events delivered (sum of group sizes)  */
  uint64_t pairs;          /* (source, delay-group) pairs selected            */
  uint64_t rk_accepted;    /* AdEx accepted RK45 substeps                     */
  uint64_t rk_rejected;    /* AdEx rejected RK45 substeps                     */
  uint64_t n_neurons, n_synapses, n_groups;
  uint64_t device_bytes;   /* device memory held by the net                   */
  double build_ms;         /* wall time of snn_build                          */
  double simulate_ms;      /* wall time spent in snn_simulate                 */
  uint32_t overflow;       /* nonzero if a device-side range check failed     */
  uint32_t max_delay_used; /* largest delay (steps) present in the network    */
  uint64_t spill_events;   /* binned delivery: events that found their tile's
                              bin full and were added by atomics instead     */
  uint32_t delivery;       /* 1 direct, 2 binned (after build)                */
  uint32_t tile_neurons;   /* binned delivery: neurons per target tile        */
  uint32_t delivery_blocks; /* blocks delivering delays >= 2                  */
  uint32_t delivery_queue;  /* binned: 1 when the delivery blocks take contiguous
                               ranges of the step's (spike, delay) items from a
                               queue (batches of at least 8 instances of at most
                               32 tiles each), 0 when each takes every G-th item */
  double last_call_device_ms; /* device time of the last snn_simulate_steps call,
                                 HIP events on the library's stream around its
                                 graph launches (kernels and the gaps between) */
  uint32_t tile_runs;       /* binned, LIF-only, no plastic synapses: 1 when the
                               groups put on average at least 4 synapses on each
                               tile they reach and the delivery's count pass reads
                               their tile runs (recorded at build, 4 bytes per run,
                               8 per group) instead of every synapse word     */
  uint32_t tile_window;     /* binned: 1 when every tile overlaps at most 8
                               populations, so that LIF-only networks run step
                               kernels that read the population tables from a
                               window in LDS; 0 otherwise (such LIF-only networks
                               then run the kernels built for AdEx as well)   */
} snn_counters;

/* ---- lifecycle ---------------------------------------------------------- */
/* Create an empty network.  dev may be NULL (hipMalloc on the current device). */
snn_status snn_create_net(const snn_config* cfg, const snn_device* dev, snn_net** out);
/* Release every host and device resource of the network (NULL is a no-op). */
void snn_destroy_net(snn_net* net);
/* Message of the last failed call on `net` ("" if none); valid until the next call. */
const char* snn_last_error(const snn_net* net);

/* ---- definition phase (before snn_build) --------------------------------- */
/* Start a new independent network inside this one (a batch member; the net
   created by snn_create_net is instance 0 with the config seed).  Populations,
   connections and drives created until the next call belong to the new
   instance; connections must stay inside one instance.  Its randomness is
   keyed by `seed` with gids and projection indices counted from the instance's
   own first neuron and first projection, so it draws exactly what a network
   built alone with that seed draws and its results are the same alone and in
   the batch.  All instances share dt, Dmax and the step counter and advance in
   the same kernels.  Called before any population, it sets instance 0's seed. */
snn_status snn_begin_instance(snn_net* net, uint64_t seed, uint32_t* instance_id);
/* Create n neurons of `model` with n_ports receptor ports (1..4; LIF delta: 1)
   and NEST-like default parameters.  *first_gid receives the first gid. */
snn_status snn_create(snn_net* net, int32_t model, uint32_t n, uint32_t n_ports, uint32_t* first_gid);
/* Set model parameter `param` (SNN_P_*) of gids [first, first+n) (Sec. 2.1:
   neuron parameters from fixed values or arrays), before snn_build.  nv == 1
   broadcasts v[0]: over a range made of whole populations it sets their
   constant, otherwise it sets the value of each neuron of the range; nv == n
   gives each neuron its own value v[j].  A later call on the same neurons
   wins.  A neuron whose parameters differ from its population's is updated
   with its own constants (LIF: tau_m, C_m, E_L, V_th, V_reset, t_ref; AdEx:
   all but the port constants), computed on the host exactly as a
   population's are; a neuron whose V_m was never set starts at its own E_L.
   SNN_E_INVALID for an unknown parameter, a bad range, nv not 1 or n, or a
   value that is not finite; invalid values (tau_m <= 0, ...) are reported by
   snn_build. */
snn_status snn_set_param(snn_net* net, uint32_t first, uint32_t n, int32_t param, const double* v, size_t nv);
/* Model parameter `param` of gids [first, first+n) drawn per neuron (Sec.
   2.1: neuron parameters from probability distributions), before snn_build:
   kind, a, b, lo, hi and levels as for snn_state_distribution; neuron i takes
   the level of the top 32 bits of word 0 of Philox block (i, param << 8,
   tag 5) with its instance's key (seed, 0), i counted from the instance's
   first neuron, then is set as by snn_set_param with one value per neuron. */
snn_status snn_param_distribution(snn_net* net, uint32_t first, uint32_t n, int32_t param, int32_t kind, double a,
                                  double b, double lo, double hi, uint32_t levels);
/* Set port parameter `param` (SNN_PP_*) of receptor `port`, same range rule. */
snn_status snn_set_port_param(snn_net* net, uint32_t first, uint32_t n, uint32_t port, int32_t param,
                              double value);
/* Fixed-indegree rule (Sec. 2.1): every target in [tgt_first, tgt_first+tgt_n)
   receives `indegree` synapses from sources drawn uniformly, with replacement,
   from [src_first, src_first+src_n) (autapses and multapses allowed), each
   with weight `weight`, receptor `port` and a delay drawn from the given
   distribution.  Randomness: counter-based, keyed by the config seed, the
   projection's creation index, the target gid and the draw index, so a network
   is identical on every run, alone or batched. */
snn_status snn_connect_fixed_indegree(snn_net* net, uint32_t src_first, uint32_t src_n, uint32_t tgt_first,
                                      uint32_t tgt_n, uint32_t indegree, double weight, int32_t delay_kind,
                                      double delay_a, double delay_b, uint32_t port);
/* Connection rules (Sec. 2.1), each with weight `weight`, receptor `port`
   and a delay per synapse drawn from the given distribution; autapses and
   multapses allowed:
     SNN_RULE_FIXED_INDEGREE     every target draws n sources uniformly (as
                                 snn_connect_fixed_indegree);
     SNN_RULE_FIXED_OUTDEGREE    every source draws n targets uniformly;
     SNN_RULE_ALL_TO_ALL         every (source, target) pair once (n unused);
     SNN_RULE_ONE_TO_ONE         source src_first + i onto target tgt_first + i
                                 (src_n == tgt_n; n unused);
     SNN_RULE_FIXED_TOTAL_NUMBER n synapses, source and target each uniform.
   Randomness: counter-based (Philox4x64-10, key (seed, 0)), counters
   (target, p << 40 | k >> 1), (source, p << 40 | k >> 1), (target,
   p << 40 | k >> 1), (target, p << 40), (synapse index, p << 40) with tag 1,
   p the projection's creation index and gids counted from the instance's
   first neuron.  SNN_E_INVALID for an unknown rule, unequal one-to-one sizes
   or a degree above 2^32 - 1. */
#define SNN_RULE_FIXED_INDEGREE 0
#define SNN_RULE_FIXED_OUTDEGREE 1
#define SNN_RULE_ALL_TO_ALL 2
#define SNN_RULE_ONE_TO_ONE 3
#define SNN_RULE_FIXED_TOTAL_NUMBER 4
/* User-defined connections (Sec. 2.1): n synapses src[j] -> tgt[j] (gids,
   all inside one instance) with delays delay_ms[j] (steps of dt rounded half
   up, at least one; SNN_E_INVALID above max_delay_steps), weight `weight` on
   `port`.  The lists are copied. */
snn_status snn_connect_list(snn_net* net, size_t n, const uint32_t* src, const uint32_t* tgt, const double* delay_ms,
                            double weight, uint32_t port);
snn_status snn_connect(snn_net* net, int32_t rule, uint64_t n, uint32_t src_first, uint32_t src_n,
                       uint32_t tgt_first, uint32_t tgt_n, double weight, int32_t delay_kind, double delay_a,
                       double delay_b, uint32_t port);
/* Connection weights from a probability distribution (Sec. 2.1, weights
   "through probability distributions"), for the projection created last
   (snn_connect / snn_connect_fixed_indegree; its `weight` is then unused).
   The distribution is discretised: [lo, hi] is cut into `levels` equal bins
   and a synapse takes the midpoint of bin j,
     w_j = lo + (hi - lo) (j + 1/2) / levels,
   with the probability the distribution, restricted to [lo, hi], gives that
   bin.  SNN_WEIGHT_UNIFORM: uniform on [a, b) (lo, hi ignored);
   SNN_WEIGHT_NORMAL: normal of mean a and standard deviation b, truncated to
   [lo, hi].  Synapse k of entity e (the first counter word of its connection
   draw) draws the top 32 bits of word k&3 of Philox block
   (e, p << 40 | k >> 2, tag 3) against thresholds
   T_j = floor(2^32 (F(e_{j+1}) - F(lo)) / (F(hi) - F(lo))) (e_{j+1} the
   upper edge of bin j, T_{levels-1} = 2^32); its level is min{j : u < T_j}.
   Every (port, quantised level) pair of every target population takes one
   of the network's weight classes (at most 1024, fewer above 2^22 neurons:
   SNN_E_UNSUPPORTED at build).  SNN_E_STATE after build or with no
   projection; SNN_E_INVALID for a list projection, levels outside 1..1024,
   a <= b (uniform), b <= 0 or lo >= hi (normal), no probability in [lo, hi];
   at build, negative levels onto conductance ports or levels other than a
   single 1 onto parrot neurons. */
#define SNN_WEIGHT_UNIFORM 0
#define SNN_WEIGHT_NORMAL 1
snn_status snn_weight_distribution(snn_net* net, int32_t kind, double a, double b, double lo, double hi,
                                   uint32_t levels);
/* Nearest-neighbour STDP (Sec. 2.1 lists it; after Morrison et al. 2008) on
   the projection created last, before snn_build.  A synapse's spikes are its
   pre arrivals (step a: the update of step a receives the spike) and its
   target's spikes (step k); in one step the arrival comes first.  Each post
   spike at k pairs with the synapse's latest arrival a <= k and potentiates,
   each arrival at a pairs with the target's latest spike k < a and
   depresses, with the power-law rule in the weight's fixed point (W =
   llrint(w_max 2^S), S the exponent of the synapse's (target population,
   port), which also covers w_max):
     F+(d) = llrint(lambda e^{-d dt / tau_plus} 2^32),
     F-(d) = llrint(alpha lambda e^{-d dt / tau_minus} 2^32),
     potentiation  w += (B+ F+(k - a)) >> 32, B+ = W - w (mu_plus 1) or W, then min(w, W);
     depression    w -= (B- F-(a - k)) >> 32, B- = w (mu_minus 1) or W, then max(w, 0);
   once per unit of multiplicity.  In step n the input of step n + 1 is
   delivered with the weights as they are, then the post spikes of step n
   potentiate, then the arrivals of step n + 1 depress.  SNN_E_STATE after
   build or with no projection; SNN_E_INVALID for tau <= 0, lambda outside
   (0, 1], alpha < 0 or alpha lambda > 1, w_max <= 0, mu not 0 or 1, or
   weights outside [0, w_max]; at build SNN_E_UNSUPPORTED for more than 255
   plastic (projection, target population) pairs. */
snn_status snn_stdp(snn_net* net, double tau_plus, double tau_minus, double lambda, double alpha, int32_t mu_plus,
                    int32_t mu_minus, double w_max);
/* Per-connection weights (Sec. 2.1, weights "through arrays") of the list
   projection created last by snn_connect_list: weights[j] for its synapse j
   (host array of n doubles, copied; n must equal the list's length; n == 0
   does nothing).  The distinct values become weight classes as above (at
   most 1024 distinct values, SNN_E_UNSUPPORTED beyond). */
snn_status snn_list_weights(snn_net* net, const double* weights, size_t n);
/* State variable `var` (SNN_V_M, SNN_V_I_E, SNN_V_W, SNN_V_G, SNN_V_I_SYN,
   SNN_V_H or SNN_V_G_RISE; `port` for the per-port ones) of neurons
   first..first+n drawn from a distribution (Sec. 2.1: neuron parameters and
   state "through probability distributions"), discretised like the weights
   (kind SNN_WEIGHT_UNIFORM on [a, b) or SNN_WEIGHT_NORMAL of mean a and
   deviation b truncated to [lo, hi]; `levels` equal bins, 1..65536, a value
   is its bin's midpoint).  Neuron i takes the level of the top 32 bits of
   word 0 of Philox block (i, var << 8 | port, tag 4) with its instance's key
   (seed, 0), i counted from the instance's first neuron; the values are then
   set as by snn_set_state (before or after build; a later call on the same
   neurons wins).  SNN_E_INVALID for a bad range, the refractory counter, or
   a bad distribution. */
snn_status snn_state_distribution(snn_net* net, uint32_t first, uint32_t n, int32_t var, uint32_t port,
                                  int32_t kind, double a, double b, double lo, double hi, uint32_t levels);
/* Multimeter (Sec. 2.1), before snn_build: record state variable `var`
   (SNN_V_M, SNN_V_W, SNN_V_G, SNN_V_G_RISE, SNN_V_I_SYN or SNN_V_H; `port` for
   the per-port ones) of the n neurons gids[0..n) after the update of every
   step n with (n + 1) % interval == 0, i.e. at time (n + 1) dt.  The device
   copies the values after each step; the host collects them while
   simulating (one synchronisation per 100 steps while a multimeter exists).
   *meter_id receives the recorder's index.  SNN_E_INVALID for an unknown
   variable, a gid out of range or interval 0; at build, for a variable the
   network does not have. */
snn_status snn_multimeter(snn_net* net, int32_t var, uint32_t port, const uint32_t* gids, size_t n,
                          uint32_t interval, uint32_t* meter_id);
/* Samples of meter `meter_id` so far: steps[k] (the step after whose update
   sample k was taken) and values[k * n_gids + j] (gid j of the meter, in the
   variable's units: V in mV as set).  *n_out = number of samples; at most
   cap are written (pass cap 0 to query the count). */
snn_status snn_get_samples(snn_net* net, uint32_t meter_id, uint64_t* steps, double* values, size_t cap,
                           size_t* n_out);
/* ---- checkpoint / resume ---------------------------------------------------- */
/* Snapshot of a built network's dynamic state after the steps simulated so
   far: neuron state, pending input (buffers of this and the next step, bins
   and spill), the spike records delivery still reads, the step books and the
   statistics.  snn_snapshot_size gives the bytes; snn_snapshot writes them
   into the caller's host buffer (SNN_E_INVALID if cap is smaller).
   snn_restore loads a snapshot into a network built from the same
   specification (SNN_E_INVALID for another network's snapshot): simulating
   on gives exactly what the original gives.  The restored network's raster
   starts at the snapshot's step; multimeter samples are not part of it. */
snn_status snn_snapshot_size(snn_net* net, size_t* bytes);
snn_status snn_snapshot(snn_net* net, void* buf, size_t cap);
snn_status snn_restore(snn_net* net, const void* buf, size_t size);
/* Spike times (ms) of spike-generator neuron `gid`, before snn_build: a time
   t is emitted in the update of step round(t / dt) - 1 (rounded half up), so
   the spike is reported at t; times in one step add up to the multiplicity
   (at most 31).  SNN_E_INVALID for a time below dt or a neuron that is not a
   spike generator; a later call replaces the list. */
snn_status snn_set_spike_times(snn_net* net, uint32_t gid, const double* t_ms, size_t n);
/* Poisson generator (Sec. 2.1, Table 1): every target in the range receives,
   independently, the summed spikes of n_inputs trains of rate_hz each, with
   weight `weight` on `port`, drawn per target and step.  At most one drive per
   neuron. */
snn_status snn_poisson(snn_net* net, uint32_t tgt_first, uint32_t tgt_n, double rate_hz, uint32_t n_inputs,
                       double weight, uint32_t port);

/* ---- state (any phase) --------------------------------------------------- */
/* Set state variable `var` (SNN_V_*) of gids [first, first+n) from v[0..nv),
   nv == 1 broadcasts, nv == n gives one value per neuron.  After build this
   writes device memory (synchronously). */
snn_status snn_set_state(snn_net* net, uint32_t first, uint32_t n, int32_t var, uint32_t port, const double* v,
                         size_t nv);
/* Read state variable `var` of gids [first, first+n) into out[0..n). */
snn_status snn_get_state(snn_net* net, uint32_t first, uint32_t n, int32_t var, uint32_t port, double* out);

/* ---- build and simulation ------------------------------------------------ */
/* Freeze the network: draw the connectivity on the device and lay it out by
   (source, delay group) with a per-source delay bitmask; allocate state,
   spike buffers and input accumulators.  Returns SNN_E_UNSUPPORTED for more
   distinct (port, weight) classes than fit next to the target index in 32
   bits (at most 1024). */
snn_status snn_build(snn_net* net);
/* Return the device memory of a built network while keeping its results:
   the spikes still on the device are copied to the host raster and the
   counters are recorded, then every device allocation is freed.  Afterwards
   snn_get_spikes and snn_get_counters answer from the host copies
   (device_bytes 0) and every call that needs the device returns SNN_E_STATE;
   the network is not built again.  Used by the server to free a finished
   request's memory at once. */
snn_status snn_release(snn_net* net);
/* Advance by round(t_ms / dt) steps (resumable: later calls continue). */
snn_status snn_simulate(snn_net* net, double t_ms);
/* Advance by `steps` steps.  The steps run as captured loops of 100 steps
   and of powers of two below it (so any count is a few graph launches); the
   call returns when the device has finished them, with SNN_E_OVERFLOW if a
   device range check failed.  The spikes of the last steps stay in the
   device ring until snn_get_spikes (or a later call's drain) copies them. */
snn_status snn_simulate_steps(snn_net* net, uint64_t steps);

/* ---- readback ------------------------------------------------------------ */
/* Spikes with step in [step_lo, step_hi), sorted by (step, gid).  A spike in
   step n is emitted at time (n+1) dt.  Writes min(count, cap) entries; *n_out
   receives the total count (call with cap = 0 to size the buffers).  Copies
   the spikes still held on the device first (waits for it). */
snn_status snn_get_spikes(snn_net* net, uint64_t step_lo, uint64_t step_hi, uint64_t* step, uint32_t* gid,
                          uint32_t* mult, size_t cap, size_t* n_out);
/* Counters (see snn_counters). */
snn_status snn_get_counters(snn_net* net, snn_counters* out);
/* Integer input already delivered for the next step of gids [first, first+n)
   on `port` (network synapses only, Poisson excluded), in units of
   2^-shift(gid, port) of the weight unit. */
snn_status snn_get_input(snn_net* net, uint32_t first, uint32_t n, uint32_t port, int64_t* out);
/* snn_get_input without any allocation, for callers that cannot allocate
   device memory (code under stream capture, tight serving loops, harnesses
   that forbid it).  Same arguments and result as snn_get_input; n is at most
   262,144 (SNN_E_INVALID above).  Binned delivery stages the sum in a fixed
   2 MiB device workspace of the library (one per GPU, held until the process
   ends, its address resolved when the first network on that GPU is created);
   calls that overlap on one GPU, from any threads or networks, race for it.
   Calls no allocator, neither the caller's nor the runtime's. */
snn_status snn_get_input_noalloc(snn_net* net, uint32_t first, uint32_t n, uint32_t port, int64_t* out);
/* Fixed-point exponent S of (gid, port): weights are stored as llrint(w 2^S). */
snn_status snn_get_shift(snn_net* net, uint32_t gid, uint32_t port, int32_t* shift);
/* Poisson counts the device draws for gids [first, first+n) at `step`
   (0 where a neuron has no drive). */
snn_status snn_poisson_counts(snn_net* net, uint64_t step, uint32_t first, uint32_t n, uint32_t* k);
/* Advance by `steps` steps launching each kernel on its own (no graph) with a
   HIP event pair around it on the library's stream, and add the summed
   device time of the step kernel (update, delay-1 delivery and delivery of
   earlier steps' spikes) to kernel_ms[0], in milliseconds.  Results are identical to
   snn_simulate_steps; used to measure per-kernel durations. */
snn_status snn_profile_steps(snn_net* net, uint64_t steps, double* kernel_ms);
/* Connectivity in canonical order (source, delay, target, port, weight): on
   input *n_syn is the capacity of the arrays, on output the synapse count
   (arrays untouched when too small). */
snn_status snn_export_synapses(snn_net* net, uint32_t* src, uint32_t* delay, uint32_t* tgt, uint32_t* port,
                               int64_t* wq, size_t* n_syn);
/* Current fixed-point weight of every synapse in the same canonical order
   (plastic synapses: as STDP has left them; static: their class weight);
   *n_syn as for snn_export_synapses. */
snn_status snn_get_weights(snn_net* net, int64_t* wq, size_t* n_syn);

/* ---- serving ------------------------------------------------------------ */
/* A request server on the current device: requests (a defined, not yet built
   network and a step count) wait in one queue in submission order; `slots`
   worker threads each take the first queued request whose known memory need
   fits what is left of `hbm_budget` bytes, build it, simulate it on the
   network's own stream and release its device memory as soon as it is done
   (snn_release), so requests submitted while others run are admitted as
   slots and memory free up and their work overlaps on the device.  Every
   device allocation of a served network passes through the server, which
   refuses one that would exceed the budget: the build fails and releases
   what it had allocated, and the request goes back to the head of the queue
   with that amount as its known need.  A request whose known need exceeds
   the budget, or that cannot fit with nothing else on the device, fails
   with SNN_E_BUDGET.  A network is
   advanced by exactly the kernels it would run alone, so its raster does
   not depend on what it was served with.  slots 1..64. */
typedef struct snn_server snn_server;
#define SNN_JOB_QUEUED 0
#define SNN_JOB_RUNNING 1
#define SNN_JOB_DONE 2
#define SNN_JOB_FAILED 3
typedef struct snn_job_info {
  snn_status status;         /* SNN_OK, or why the request failed              */
  uint32_t attempts;         /* builds tried (more than 1 after budget refusals) */
  double t_submit, t_start, t_done; /* CLOCK_MONOTONIC seconds: submitted, first
                                       taken by a slot, finished               */
  uint64_t device_bytes_peak; /* most device memory the request held          */
  char error[200];           /* message of a failure                          */
} snn_job_info;
typedef struct snn_server_stats {
  uint64_t budget, in_use, peak; /* device bytes: the budget, granted now, at most */
  uint32_t queued, running;
  uint64_t done, failed;
} snn_server_stats;
snn_status snn_server_create(size_t hbm_budget, uint32_t slots, snn_server** out);
/* Stops the workers after their current request (which finishes and is
   released); queued requests are dropped.  Networks whose results were not
   taken go back to the caller as they are (released, or never built), with
   their own allocators: the caller destroys them. */
void snn_server_destroy(snn_server* srv);
/* Queue `net` (defined with snn_create / snn_connect / ..., not built) to be
   built and advanced by `steps` steps.  The server owns the handle until
   snn_server_result returns it: the caller must not use it meanwhile.
   *ticket identifies the request.  SNN_E_STATE if the network is built,
   released or empty; SNN_E_BUDGET if its synapse words alone (4 bytes each)
   exceed the budget. */
snn_status snn_server_submit(snn_server* srv, snn_net* net, uint64_t steps, uint64_t* ticket);
/* *state = SNN_JOB_QUEUED, _RUNNING, _DONE or _FAILED.  SNN_E_INVALID for an
   unknown ticket (or one whose result was taken). */
snn_status snn_server_poll(snn_server* srv, uint64_t ticket, int32_t* state);
/* Wait until the request is done or failed (timeout_s < 0: no limit);
   SNN_E_STATE if the time ran out first. */
snn_status snn_server_wait(snn_server* srv, uint64_t ticket, double timeout_s);
/* Hand a finished request's network back (*net; its device memory is already
   released: snn_get_spikes and snn_get_counters read the results; destroy it
   with snn_destroy_net) and fill *info (may be NULL).  Returns the request's
   status; SNN_E_STATE while it is queued or running. */
snn_status snn_server_result(snn_server* srv, uint64_t ticket, snn_net** net, snn_job_info* info);
snn_status snn_server_get_stats(snn_server* srv, snn_server_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* SNN_H */
