/*
 * snn_oracle.h -- plain, slow CPU oracle for the spiking-network hot path of
 * Golosio et al., "Fast simulations of highly-connected spiking cortical
 * models using GPUs" (arXiv 2007.14236).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library: it has its own counter-based generator, its
 * own distribution tables, its own connectivity builder, neuron updates and
 * delivery loop, each written from the paper's definitions.
 *
 * Modes:
 *   ORC_FP64  : every floating-point quantity in double (physics reference).
 *   ORC_FP32SO: LIF updates in float with a fixed, FMA-free operation order
 *               (used for bit-exact raster comparison).  AdEx always runs in
 *               double.
 *
 * Units: ms, mV, pA, nS, pF, Hz.
 */
#ifndef SNN_ORACLE_H
#define SNN_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FP64 = 0, ORC_FP32SO = 1 };
enum { ORC_LIF_DELTA = 0, ORC_LIF_EXP = 1, ORC_AEIF_COND_EXP = 2, ORC_AEIF_COND_BETA = 3,
       ORC_SPIKE_GENERATOR = 4, ORC_PARROT = 5 };
enum { ORC_DELAY_CONST = 0, ORC_DELAY_UNIFORM = 1, ORC_DELAY_NORMAL_CLIPPED = 2 };
enum { ORC_TAG_CONN = 1, ORC_TAG_POISSON = 2, ORC_TAG_WEIGHT = 3, ORC_TAG_STATE = 4, ORC_TAG_PARAM = 5 };
enum { ORC_WEIGHT_UNIFORM = 0, ORC_WEIGHT_NORMAL = 1, ORC_WEIGHT_LEVELS_MAX = 1024, ORC_STATE_LEVELS_MAX = 65536 };
/* connection rules (Sec. 2.1): the count n is the in-degree, the out-degree,
   unused, unused, and the number of synapses, in that order */
enum { ORC_RULE_FIXED_INDEGREE = 0, ORC_RULE_FIXED_OUTDEGREE = 1, ORC_RULE_ALL_TO_ALL = 2,
       ORC_RULE_ONE_TO_ONE = 3, ORC_RULE_FIXED_TOTAL_NUMBER = 4, ORC_RULE_LIST = 5 };
enum { ORC_MAX_PORTS = 4, ORC_POISSON_KMAX = 128 };

/* Neuron-model parameters of one population (double, NEST units). */
typedef struct {
  int32_t model;        /* ORC_LIF_DELTA, ORC_LIF_EXP, ORC_AEIF_COND_EXP,
                           ORC_AEIF_COND_BETA                            */
  uint32_t n_ports;     /* receptor ports (1..ORC_MAX_PORTS)              */
  double tau_m, C_m, E_L, V_th, V_reset, t_ref;               /* LIF      */
  double g_L, Delta_T, V_T, tau_w, a, b, V_peak, V_r;         /* AdEx     */
  double tau_syn[ORC_MAX_PORTS];   /* ms; the decay time for beta ports     */
  double E_rev[ORC_MAX_PORTS];                                /* mV (AdEx)*/
  double rk_eps;        /* relative tolerance of the adaptive RK45 (AdEx) */
  double rk_hmin;       /* smallest substep; accepted regardless (ms)     */
  int32_t adex_no_exp;  /* test switch: drop the exponential term         */
  double tau_rise[ORC_MAX_PORTS];  /* ms; rise time of beta ports          */
} orc_pop_params;

typedef struct orc_net orc_net;

/* ---- counter-based generator: Philox4x64-10 (Salmon et al., SC'11) ---- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* ---- discretised distribution tables (thresholds on a 32-bit uniform) ---- */
/* thr[k] for k = 1..dmax; draw D = min{k : u32 < thr[k]}; thr[dmax] = 2^32. */
int orc_delay_table(int kind, double a, double b, double dt, uint32_t dmax, uint64_t* thr);
/* thr[k] for k = 0..kmax-1; draw k = min{k : u32 < thr[k]}; thr[kmax-1] = 2^32. */
int orc_poisson_table(double lambda, uint32_t kmax, uint64_t* thr);
/* fixed-point exponent: largest S with max_abs_w * 2^S < 2^30 (0 if max_abs_w == 0) */
int orc_fixed_point_shift(double max_abs_w);

/* ---- network ---- */
orc_net* orc_create(double dt_ms, uint64_t seed, uint32_t max_delay_steps, int mode);
void     orc_destroy(orc_net*);
/* returns first gid of the new population, or -1 */
int64_t  orc_population(orc_net*, uint32_t n, const orc_pop_params* p);
int      orc_connect_fixed_indegree(orc_net*, uint32_t src_first, uint32_t src_n,
                                    uint32_t tgt_first, uint32_t tgt_n, uint32_t indegree,
                                    double weight, int delay_kind, double da, double db,
                                    uint32_t port);
/* user-defined connections (Sec. 2.1): synapse j from src[j] onto tgt[j]
   with delay delay_ms[j] (steps: rounded half up, at least 1, at most Dmax,
   else an error), all with weight `weight` on `port` */
int      orc_connect_list(orc_net*, uint64_t n, const uint32_t* src, const uint32_t* tgt, const double* delay_ms,
                          double weight, uint32_t port);
/* any rule; fixed in-degree is rule 0 with n = the in-degree */
int      orc_connect(orc_net*, int rule, uint64_t n, uint32_t src_first, uint32_t src_n,
                     uint32_t tgt_first, uint32_t tgt_n, double weight, int delay_kind, double da,
                     double db, uint32_t port);
/* Weights drawn from a probability distribution (Sec. 2.1), discretised:
   the range [lo, hi] is cut into `levels` equal bins and a synapse takes the
   midpoint of bin j, w_j = lo + (hi - lo) (j + 1/2) / levels, with the
   probability the distribution, restricted to [lo, hi], gives that bin.
   kind ORC_WEIGHT_UNIFORM: uniform on [a, b) (lo, hi ignored; a < b);
   kind ORC_WEIGHT_NORMAL: normal of mean a and deviation b > 0, truncated to
   [lo, hi].  The draw of synapse k of entity e (the first counter word of its
   connection draw) is the top 32 bits of word k&3 of block
   (e, p<<40 | k>>2, ORC_TAG_WEIGHT, 0) against thresholds
   T_j = floor(2^32 (F(e_{j+1}) - F(lo)) / (F(hi) - F(lo))), e_{j+1} the upper
   edge of bin j, T_{levels-1} = 2^32: the level is min{j : u32 < T_j}.
   Applies to projection `proj` (creation index, not a list). */
int      orc_weight_distribution(orc_net*, uint32_t proj, int kind, double a, double b, double lo, double hi,
                                 uint32_t levels);
/* per-connection weights of a user-defined list projection (weights[j] for
   synapse j); at most ORC_WEIGHT_LEVELS_MAX distinct values */
int      orc_list_weights(orc_net*, uint32_t proj, uint64_t n, const double* weights);
/* Nearest-neighbour STDP (Sec. 2.1, after Morrison et al. 2008) on
   projection `proj`: time constants tau_plus and tau_minus (ms), learning
   rate lambda (0, 1], depression factor alpha (alpha lambda <= 1), weight
   dependence mu_plus, mu_minus in {0 (additive), 1 (multiplicative)},
   largest weight w_max > 0 (the weights start in [0, w_max]).  The rule and
   its timing are stated at the top of the simulation loop in
   snn_oracle.c.  orc_get_synapses reports a plastic synapse's current
   weight. */
int      orc_stdp(orc_net*, uint32_t proj, double tau_plus, double tau_minus, double lambda, double alpha, int mu_plus,
                  int mu_minus, double w_max);
int      orc_poisson(orc_net*, uint32_t tgt_first, uint32_t tgt_n, double rate_hz,
                     uint32_t n_inputs, double weight, uint32_t port);
/* Devices (Sec. 2.1).  A spike generator emits, in the update of step n, as
   many spikes as it has times t with round(t / dt) - 1 = n (t >= dt; the
   spike is then reported at t).  A parrot neuron emits, in the update of step
   n, one spike per spike arriving at step n; the connections onto it (and a
   Poisson drive) must have weight 1. */
int      orc_set_spike_times(orc_net*, uint32_t gid, uint64_t n, const double* t_ms);
/* state variables (per neuron).  var: 0 V_m (mV), 1 I_e (pA), 2 w (pA),
   3 g[port] (nS), 4 I_syn[port] (pA), 5 refractory counter, 6 h (ms) */
int      orc_set_state(orc_net*, uint32_t first, uint32_t n, int var, uint32_t port, const double* v);
int      orc_get_state(orc_net*, uint32_t first, uint32_t n, int var, uint32_t port, double* v);
/* State variable `var` (not the refractory counter) of neurons first..first+n
   drawn from a distribution, discretised as the weights are (uniform kind 0
   on [a, b), truncated normal kind 1 of mean a and deviation b on [lo, hi],
   `levels` <= ORC_STATE_LEVELS_MAX bins, midpoints): neuron i takes the
   level of the top 32 bits of word 0 of block (i, var << 8 | port,
   ORC_TAG_STATE, 0), then is set as by orc_set_state. */
/* Per-neuron model parameters (Sec. 2.1: neuron parameters from arrays or
   probability distributions): parameter `param` (0 tau_m, 1 C_m, 2 E_L, 3 V_th,
   4 V_reset, 5 t_ref, 6 g_L, 7 Delta_T, 8 V_T, 9 tau_w, 10 a, 11 b, 12 V_peak,
   13 V_r, 14 rk_eps, 15 rk_hmin) of neurons first..first+n-1 set to v[j]; the
   other parameters stay the population's.  Must come before any state is set
   or drawn (a neuron starts at its own E_L). */
int      orc_set_param(orc_net*, uint32_t first, uint32_t n, int param, const double* v);
/* parameter `param` of neuron gid (NaN for a bad gid or parameter) */
double   orc_get_param(const orc_net*, uint32_t gid, int param);
/* The same parameter drawn per neuron: neuron i takes the level of the top 32
   bits of word 0 of block (i, param << 8, ORC_TAG_PARAM, 0), key (seed, 0),
   of the discretised distribution (as orc_state_distribution). */
int      orc_param_distribution(orc_net*, uint32_t first, uint32_t n, int param, int kind, double a, double b,
                                double lo, double hi, uint32_t levels);
int      orc_state_distribution(orc_net*, uint32_t first, uint32_t n, int var, uint32_t port, int kind, double a,
                                double b, double lo, double hi, uint32_t levels);
int      orc_build(orc_net*);
int      orc_simulate(orc_net*, uint64_t steps);
uint64_t orc_current_step(const orc_net*);
/* synapse deliveries so far (sum of the sizes of the delivered groups) */
uint64_t orc_n_events(const orc_net*);

/* spikes recorded so far, sorted by (step, gid) */
uint64_t orc_n_spikes(const orc_net*);
void     orc_get_spikes(const orc_net*, uint64_t* step, uint32_t* gid, uint32_t* mult);

/* synapses in canonical order (source, delay steps, target, port, w_q) */
uint64_t orc_n_synapses(const orc_net*);
void     orc_get_synapses(const orc_net*, uint32_t* src, uint32_t* delay, uint32_t* tgt,
                          uint32_t* port, int64_t* wq);
/* fixed-point exponent used for (neuron gid, port) */
int      orc_shift_of(const orc_net*, uint32_t gid, uint32_t port);
/* quantised Poisson weight and lambda table of neuron gid (-1 if none) */
int      orc_poisson_count(const orc_net*, uint32_t gid, uint64_t step, uint32_t* k);

/* record the integer input sum (network delivery only, Poisson excluded) that
   every neuron reads at every simulated step: buffer of steps*N*P int64 */
int      orc_record_input(orc_net*, int64_t* buf, uint64_t max_steps);

/* Delivery from an external spike history (plain definition): the integer
   input each (target, port) receives at step target_step from the spikes
   (step[i], gid[i], mult[i]).  out has N*P entries. */
int      orc_replay_input(const orc_net*, uint64_t n_spk, const uint64_t* step, const uint32_t* gid,
                          const uint32_t* mult, uint64_t target_step, int64_t* out);

/* ---- sampled checks at sizes where the synapse table does not fit ---- */
/* State, Poisson drive and fixed-point exponents without the synapse table
   (orc_shift_of, orc_poisson_count and the two calls below then work). */
int      orc_prepare(orc_net*);
/* Synapses onto target t (projection order, then draw index): up to cap of
   them into the arrays; returns how many there are, -1 on error (also when a
   projection onto t draws per source or per synapse: fixed out-degree, fixed
   total number). */
int64_t  orc_target_synapses(orc_net*, uint32_t t, uint64_t cap, uint32_t* src, uint32_t* delay, uint32_t* port,
                             int64_t* wq);
/* Input delivered to targets tgt[0..nt) at target_step by the spikes given
   (sorted by (step, gid)): out[j*P + port]. */
int      orc_sampled_input(orc_net*, uint32_t nt, const uint32_t* tgt, uint64_t n_spk, const uint64_t* step,
                           const uint32_t* gid, const uint32_t* mult, uint64_t target_step, int64_t* out);

/* ---- single-neuron update steps, exposed for the pins ---- */
/* LIF: y = V - E_L.  x[] = converted input per port.  Returns 1 on spike. */
int orc_lif_delta_step64(const orc_pop_params*, double dt, double* y, int32_t* refr, double I_e, double x);
int orc_lif_delta_step32(const orc_pop_params*, double dt, float* y, int32_t* refr, float I_e, float x);
int orc_lif_exp_step64(const orc_pop_params*, double dt, double* y, double* I, int32_t* refr, double I_e, const double* x);
int orc_lif_exp_step32(const orc_pop_params*, double dt, float* y, float* I, int32_t* refr, float I_e, const float* x);
/* LIF propagators in double: out = {P22, P20, P11[0..P-1], P21[0..P-1]} */
void orc_lif_propagators(const orc_pop_params*, double dt, double* out);
/* AdEx: y = {V, w, g_0..g_{P-1}} (exponential ports) or
   {V, w, g_0..g_{P-1}, r_0..r_{P-1}} (beta ports, r the rising variable);
   h carried step size.  At step start the delivered weight x[p] is added to
   g_p (exponential) or g0_p x[p] to r_p (beta, g0_p from orc_beta_g0), then
   one dt is integrated with Cash-Karp RK45.  Returns the number of resets
   (multiplicity).  acc/rej count accepted/rejected substeps. */
int orc_adex_step(const orc_pop_params*, double dt, double* y, double* h, double I_e,
                  const double* x, uint64_t* acc, uint64_t* rej);
/* Cash-Karp tableau as used: c[6], a[6*6] (row-major, strictly lower), b5[6], b4[6] */
void orc_cash_karp_tableau(double* c, double* a, double* b5, double* b4);
/* AdEx right-hand side (for pins): dy = f(y) */
void orc_adex_rhs(const orc_pop_params*, double I_e, const double* y, double* dy);
/* Beta-port normalisation: the value added to r per unit weight, so that a
   lone input of weight w gives a conductance peaking at exactly w. */
double orc_beta_g0(double tau_rise, double tau_decay);

const char* orc_last_error(const orc_net*);
/* Threads the simulation loops use: 1, or OpenMP's thread count in a build
   with -fopenmp (same results either way). */
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
