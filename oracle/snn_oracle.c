/*
 * snn_oracle.c -- plain CPU oracle (TEST INFRASTRUCTURE ONLY; see header).
 *
 * Follows Golosio et al., arXiv 2007.14236:
 *   - LIF exact integration on the dt grid (Sec. 2.1; membrane and exponential
 *     PSC equations of Sec. 2.3, after Rotter & Diesmann 1999),
 *   - multisynapse AdEx with conductance synapses (Sec. 2.4, AdEx membrane,
 *     conductance-current and adaptation equations, Table 2) integrated by a
 *     fifth-order Runge-Kutta method with adaptive step-size control
 *     (Sec. 2.1, after Press et al. 1992: the Cash-Karp embedded pair),
 *   - spike delivery (Sec. 2.2, Fig. 1): a spike emitted at step n by source s
 *     reaches, at step n + d, exactly the synapses of s whose delay is d steps.
 *     Here that is computed as its plain definition: for every target step,
 *     loop over d = 1..Dmax, over the spikes emitted at step (target - d), and
 *     over the synapses of that source with delay d.
 *   - the fixed-indegree connection rule (Sec. 2.1) and Poisson generators
 *     (Sec. 2.1; Table 1), with randomness from Philox4x64-10.
 *
 * No blocking, fusion or reordering beyond those definitions.  Compiled with
 * -O2 -ffp-contract=off -fno-fast-math so that every float operation rounds as
 * written.
 */
#include "snn_oracle.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Round: two 64x64->128 products of counter words */
/* 0 and 2 with the published multipliers, output permuted and xored with    */
/* the key; the key is bumped by the published Weyl constants between rounds. */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Discretised distributions.                                                */
/* A delay of d ms is d/dt steps rounded half up, at least 1 step (delays are */
/* clipped at dt) and at most Dmax (upper tail folded into Dmax).  Hence      */
/* P(D <= k) = F((k + 1/2) dt) for 1 <= k < Dmax and 1 for k = Dmax, and a    */
/* 32-bit uniform u maps to D = min{k : u < floor(2^32 P(D <= k))}.           */
/* ------------------------------------------------------------------------ */
static double delay_cdf(int kind, double a, double b, double x) {
  if (kind == ORC_DELAY_CONST) {
    return x >= a ? 1.0 : 0.0;
  } else if (kind == ORC_DELAY_UNIFORM) {
    double f = (x - a) / (b - a);
    if (f < 0.0) f = 0.0;
    if (f > 1.0) f = 1.0;
    return f;
  } else {
    /* normal with mean a, standard deviation b */
    return 0.5 * erfc(-(x - a) / (b * sqrt(2.0)));
  }
}

static uint64_t prob_to_threshold(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return 4294967296ULL;
  double t = floor(ldexp(p, 32));
  if (t >= 4294967296.0) return 4294967296ULL;
  return (uint64_t)t;
}

int orc_delay_table(int kind, double a, double b, double dt, uint32_t dmax, uint64_t* thr) {
  if (dmax < 1 || dmax > 63 || !(dt > 0)) return -1;
  if (kind == ORC_DELAY_UNIFORM && !(b > a)) return -1;
  if (kind == ORC_DELAY_NORMAL_CLIPPED && !(b > 0)) return -1;
  thr[0] = 0;
  if (kind == ORC_DELAY_CONST) {
    double q = floor(a / dt + 0.5);
    uint32_t d0 = q < 1.0 ? 1u : (q > (double)dmax ? dmax : (uint32_t)q);
    for (uint32_t k = 1; k <= dmax; ++k) thr[k] = (k >= d0) ? 4294967296ULL : 0;
    return 0;
  }
  for (uint32_t k = 1; k < dmax; ++k) {
    double x = ((double)k + 0.5) * dt;
    thr[k] = prob_to_threshold(delay_cdf(kind, a, b, x));
  }
  thr[dmax] = 4294967296ULL;
  return 0;
}

/* Poisson(lambda): p_0 = e^-lambda, p_k = p_{k-1} lambda / k, cumulated in   */
/* order; the tail beyond kmax-1 is folded into kmax-1.                       */
int orc_poisson_table(double lambda, uint32_t kmax, uint64_t* thr) {
  if (!(lambda >= 0) || kmax < 2) return -1;
  double p = exp(-lambda);
  double c = p;
  for (uint32_t k = 0; k + 1 < kmax; ++k) {
    if (k > 0) { p = p * lambda / (double)k; c = c + p; }
    thr[k] = prob_to_threshold(c);
  }
  thr[kmax - 1] = 4294967296ULL;
  return 0;
}

int orc_fixed_point_shift(double max_abs_w) {
  if (!(max_abs_w > 0)) return 0;
  int e;
  (void)frexp(max_abs_w, &e); /* max_abs_w = m 2^e, 0.5 <= m < 1 */
  return 30 - e;
}

/* ------------------------------------------------------------------------ */
/* Network                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t src_first, src_n, tgt_first, tgt_n, K, port;
  int rule;
  uint64_t n;     /* the rule's count (in-degree, out-degree, synapses) */
  uint32_t* lsrc; uint32_t* ltgt; uint8_t* ldel;  /* user-defined list */
  double weight;
  uint64_t dthr[64];
  /* weight levels (0: the fixed weight): values, draw thresholds (drawn
     levels) or the level of every listed synapse (lists) */
  uint32_t wlevels;
  double* wlev;
  uint64_t* wthr;
  uint16_t* lwl;
  /* nearest-neighbour STDP (orc_stdp): plastic != 0 */
  int plastic, mu_plus, mu_minus;
  double tau_plus, tau_minus, lambda, alpha, w_max;
} orc_proj;

typedef struct {
  uint32_t tgt_first, tgt_n, port;
  double weight, lambda;
  uint64_t thr[ORC_POISSON_KMAX];
} orc_pois;

typedef struct {
  uint32_t src, tgt;
  uint8_t d, port;
  int64_t wq;
  int32_t plast;  /* projection index of a plastic synapse, -1 for a static one */
} orc_syn;

struct orc_net {
  double dt;
  uint64_t seed;
  uint32_t dmax;
  int mode;
  int built;
  char err[256];
  /* populations */
  uint32_t n_pops;
  orc_pop_params* pops;
  uint32_t* pop_first;
  uint32_t N;
  uint32_t P;               /* ports per neuron slot (max over populations) */
  uint32_t* pop_of;         /* N */
  orc_pop_params* npar;     /* N: each neuron's own parameters once any is set per neuron, else NULL */
  /* projections and Poisson drives */
  uint32_t n_proj; orc_proj* proj;
  uint32_t n_pois; orc_pois* pois;
  int32_t* pois_of;         /* N: index into pois or -1 */
  /* fixed point shifts per (population, port) */
  int* shift;               /* n_pops * P */
  /* synapses sorted canonically and offsets per (source, delay) */
  uint64_t n_syn;
  orc_syn* syn;
  uint64_t* off;            /* N*(dmax+1)+1 */
  /* state (double; FP32SO mode keeps float copies for LIF) */
  double* V; double* Ie; double* w; double* g; double* gr; double* I; double* h; int32_t* refr;
  /* spike generators: per neuron its emission steps (ascending) and cursor */
  uint64_t** gen_steps; uint64_t* gen_n; uint64_t* gen_pos;
  float* Vf; float* If; float* Ief;
  /* integer input accumulator for the next step, N*P */
  int64_t* acc;
  uint32_t* mult_now;       /* N: spike multiplicity of each neuron in the current step */
  uint64_t step;
  /* spike record */
  uint64_t n_spk, cap_spk;
  uint64_t* spk_step; uint32_t* spk_gid; uint32_t* spk_mult;
  /* per-step spike-record offsets: spikes of step n at [spk_at[n], spk_at[n+1]) */
  uint64_t* spk_at; uint64_t cap_at;
  /* optional input recording */
  int64_t* rec; uint64_t rec_max;
  /* counters */
  uint64_t rk_acc, rk_rej;
  /* plasticity: per synapse (canonical index) its weight, the step of its
     latest pre arrival (-1: none), the multiplicity arriving now and its
     largest weight W; per neuron its latest spike step (-1: none); the
     plastic synapses onto each target (tptr[t] .. tptr[t+1] in tidx) */
  uint64_t n_plastic;
  int64_t* pw; int64_t* last_pre; uint32_t* arr_m; int64_t* pwmax; int64_t* last_post;
  uint64_t* tptr; uint64_t* tidx;
  uint64_t n_events;        /* synapse deliveries (group sizes summed) */
};

static void set_err(orc_net* o, const char* m) { snprintf(o->err, sizeof o->err, "%s", m); }
static int is_adex(const orc_pop_params* pp) {
  return pp->model == ORC_AEIF_COND_EXP || pp->model == ORC_AEIF_COND_BETA;
}
const char* orc_last_error(const orc_net* o) { return o ? o->err : "null net"; }
/* the parameters neuron i is updated with (pop: its population) */
static const orc_pop_params* neuron_params(const orc_net* o, uint32_t i, uint32_t pop) {
  return o->npar ? &o->npar[i] : &o->pops[pop];
}

orc_net* orc_create(double dt_ms, uint64_t seed, uint32_t max_delay_steps, int mode) {
  if (!(dt_ms > 0) || max_delay_steps < 1 || max_delay_steps > 63) return NULL;
  orc_net* o = (orc_net*)calloc(1, sizeof(orc_net));
  o->dt = dt_ms; o->seed = seed; o->dmax = max_delay_steps; o->mode = mode;
  return o;
}

void orc_destroy(orc_net* o) {
  if (!o) return;
  for (uint32_t p = 0; p < o->n_proj; ++p) {
    free(o->proj[p].lsrc); free(o->proj[p].ltgt); free(o->proj[p].ldel);
    free(o->proj[p].wlev); free(o->proj[p].wthr); free(o->proj[p].lwl);
  }
  free(o->pops); free(o->pop_first); free(o->pop_of); free(o->npar); free(o->proj); free(o->pois); free(o->pois_of);
  free(o->shift); free(o->syn); free(o->off);
  free(o->pw); free(o->last_pre); free(o->arr_m); free(o->pwmax); free(o->last_post); free(o->tptr); free(o->tidx);
  free(o->V); free(o->Ie); free(o->w); free(o->g); free(o->gr); free(o->I); free(o->h); free(o->refr);
  if (o->gen_steps) for (uint32_t i = 0; i < o->N; ++i) free(o->gen_steps[i]);
  free(o->gen_steps); free(o->gen_n); free(o->gen_pos);
  free(o->Vf); free(o->If); free(o->Ief); free(o->acc); free(o->mult_now);
  free(o->spk_step); free(o->spk_gid); free(o->spk_mult); free(o->spk_at);
  free(o);
}

int64_t orc_population(orc_net* o, uint32_t n, const orc_pop_params* p) {
  if (o->built || o->shift) { set_err(o, "population after build"); return -1; }
  if (n == 0 || p->n_ports < 1 || p->n_ports > ORC_MAX_PORTS) { set_err(o, "bad population"); return -1; }
  if (o->V) { set_err(o, "population after state was set"); return -1; }
  if (o->npar) { set_err(o, "population after per-neuron parameters"); return -1; }
  if (p->model < ORC_LIF_DELTA || p->model > ORC_PARROT) { set_err(o, "bad model"); return -1; }
  if ((p->model == ORC_SPIKE_GENERATOR || p->model == ORC_PARROT) && p->n_ports != 1) {
    set_err(o, "devices have one port"); return -1;
  }
  if (p->model == ORC_LIF_DELTA && p->n_ports != 1) { set_err(o, "lif_delta has one port"); return -1; }
  if (p->model == ORC_AEIF_COND_BETA)
    for (uint32_t q = 0; q < p->n_ports; ++q)
      if (!(p->tau_rise[q] > 0) || !(p->tau_syn[q] > 0)) { set_err(o, "beta time constants"); return -1; }
  o->pops = (orc_pop_params*)realloc(o->pops, (o->n_pops + 1) * sizeof(orc_pop_params));
  o->pop_first = (uint32_t*)realloc(o->pop_first, (o->n_pops + 1) * sizeof(uint32_t));
  o->pops[o->n_pops] = *p;
  o->pop_first[o->n_pops] = o->N;
  o->n_pops++;
  int64_t first = o->N;
  o->N += n;
  return first;
}

static uint32_t pop_index(const orc_net* o, uint32_t gid) {
  uint32_t k = 0;
  while (k + 1 < o->n_pops && o->pop_first[k + 1] <= gid) ++k;
  return k;
}

/* Connection rules (Sec. 2.1), autapses and multapses allowed:
   fixed in-degree  -- every target draws n sources uniformly;
   fixed out-degree -- every source draws n targets uniformly;
   all-to-all       -- every (source, target) pair once;
   one-to-one       -- source first + i onto target first + i (equal sizes);
   fixed total      -- n synapses, source and target each drawn uniformly.
   Every synapse draws its delay from the projection's table. */
int orc_connect(orc_net* o, int rule, uint64_t n, uint32_t src_first, uint32_t src_n, uint32_t tgt_first,
                uint32_t tgt_n, double weight, int delay_kind, double da, double db, uint32_t port) {
  if (o->built || o->shift) { set_err(o, "connect after build"); return -1; }
  if ((uint64_t)src_first + src_n > o->N || (uint64_t)tgt_first + tgt_n > o->N || src_n == 0) {
    set_err(o, "range"); return -1;
  }
  if (rule < ORC_RULE_FIXED_INDEGREE || rule > ORC_RULE_FIXED_TOTAL_NUMBER) { set_err(o, "rule"); return -1; }
  if (rule == ORC_RULE_ONE_TO_ONE && src_n != tgt_n) { set_err(o, "one-to-one needs equal sizes"); return -1; }
  if ((rule == ORC_RULE_FIXED_INDEGREE || rule == ORC_RULE_FIXED_OUTDEGREE) && n > 0xffffffffull) {
    set_err(o, "degree"); return -1;
  }
  if (rule == ORC_RULE_FIXED_TOTAL_NUMBER && tgt_n == 0 && n) { set_err(o, "range"); return -1; }
  orc_proj pr;
  memset(&pr, 0, sizeof pr);
  pr.src_first = src_first; pr.src_n = src_n; pr.tgt_first = tgt_first; pr.tgt_n = tgt_n;
  pr.rule = rule; pr.n = n; pr.port = port; pr.weight = weight;
  pr.K = (rule == ORC_RULE_FIXED_INDEGREE || rule == ORC_RULE_FIXED_OUTDEGREE) ? (uint32_t)n
       : (rule == ORC_RULE_ALL_TO_ALL) ? src_n : (rule == ORC_RULE_ONE_TO_ONE) ? 1u : 0u;
  if (orc_delay_table(delay_kind, da, db, o->dt, o->dmax, pr.dthr) != 0) { set_err(o, "delay"); return -1; }
  o->proj = (orc_proj*)realloc(o->proj, (o->n_proj + 1) * sizeof(orc_proj));
  o->proj[o->n_proj++] = pr;
  return 0;
}

/* synapses the projection makes */
static uint64_t proj_synapses(const orc_proj* pr) {
  switch (pr->rule) {
    case ORC_RULE_FIXED_INDEGREE: return (uint64_t)pr->K * pr->tgt_n;
    case ORC_RULE_FIXED_OUTDEGREE: return pr->tgt_n ? (uint64_t)pr->K * pr->src_n : 0;
    case ORC_RULE_ALL_TO_ALL: return (uint64_t)pr->src_n * pr->tgt_n;
    case ORC_RULE_ONE_TO_ONE: return pr->tgt_n;
    default: return pr->tgt_n ? pr->n : 0;  /* fixed total number, list */
  }
}

int orc_connect_list(orc_net* o, uint64_t n, const uint32_t* src, const uint32_t* tgt, const double* delay_ms,
                     double weight, uint32_t port) {
  if (o->built || o->shift) { set_err(o, "connect after build"); return -1; }
  if (n == 0) return 0;
  orc_proj pr;
  memset(&pr, 0, sizeof pr);
  uint32_t smin = UINT32_MAX, smax = 0, tmin = UINT32_MAX, tmax = 0;
  pr.lsrc = (uint32_t*)malloc(n * sizeof(uint32_t));
  pr.ltgt = (uint32_t*)malloc(n * sizeof(uint32_t));
  pr.ldel = (uint8_t*)malloc(n);
  for (uint64_t j = 0; j < n; ++j) {
    double r = floor(delay_ms[j] / o->dt + 0.5);
    if (r < 1.0) r = 1.0;
    if (src[j] >= o->N || tgt[j] >= o->N || !(r <= (double)o->dmax)) {
      free(pr.lsrc); free(pr.ltgt); free(pr.ldel);
      set_err(o, "list entry out of range"); return -1;
    }
    pr.lsrc[j] = src[j]; pr.ltgt[j] = tgt[j]; pr.ldel[j] = (uint8_t)r;
    if (src[j] < smin) smin = src[j];
    if (src[j] > smax) smax = src[j];
    if (tgt[j] < tmin) tmin = tgt[j];
    if (tgt[j] > tmax) tmax = tgt[j];
  }
  /* ranges: the bounding intervals of the listed gids */
  pr.src_first = smin; pr.src_n = smax - smin + 1; pr.tgt_first = tmin; pr.tgt_n = tmax - tmin + 1;
  pr.rule = ORC_RULE_LIST; pr.n = n; pr.K = 1; pr.port = port; pr.weight = weight;
  o->proj = (orc_proj*)realloc(o->proj, (o->n_proj + 1) * sizeof(orc_proj));
  o->proj[o->n_proj++] = pr;
  return 0;
}

int orc_connect_fixed_indegree(orc_net* o, uint32_t src_first, uint32_t src_n, uint32_t tgt_first,
                               uint32_t tgt_n, uint32_t indegree, double weight, int delay_kind,
                               double da, double db, uint32_t port) {
  return orc_connect(o, ORC_RULE_FIXED_INDEGREE, indegree, src_first, src_n, tgt_first, tgt_n, weight, delay_kind,
                     da, db, port);
}

/* Weight distributions: the discretisation stated in the header.  F is the
   distribution function (uniform: (x - a) / (b - a); normal:
   erfc(-(x - a) / (b sqrt 2)) / 2). */
static int dbl_cmp(const void* pa, const void* pb) {
  double a = *(const double*)pa, b = *(const double*)pb;
  return a < b ? -1 : a > b ? 1 : 0;
}

static double weight_cdf(int kind, double a, double b, double x) {
  if (kind == ORC_WEIGHT_UNIFORM) return (x - a) / (b - a);
  return 0.5 * erfc(-(x - a) / (b * sqrt(2.0)));
}

/* levels and thresholds of a discretised distribution (weights and states
   alike); returns an error message or NULL */
static const char* dist_levels(int kind, double a, double b, double lo, double hi, uint32_t levels, double* lev,
                               uint64_t* thr) {
  if (kind == ORC_WEIGHT_UNIFORM) {
    if (!(a < b)) return "uniform needs a < b";
    lo = a; hi = b;
  } else if (kind == ORC_WEIGHT_NORMAL) {
    if (!(b > 0) || !(lo < hi)) return "normal needs sigma > 0 and lo < hi";
  } else {
    return "distribution";
  }
  double Flo = weight_cdf(kind, a, b, lo), Fhi = weight_cdf(kind, a, b, hi);
  if (!(Fhi > Flo)) return "no probability in [lo, hi]";
  for (uint32_t j = 0; j < levels; ++j) {
    lev[j] = lo + (hi - lo) * (((double)j + 0.5) / (double)levels);
    if (j + 1 == levels) { thr[j] = 1ull << 32; continue; }
    double edge = lo + (hi - lo) * ((double)(j + 1) / (double)levels);
    double q = (weight_cdf(kind, a, b, edge) - Flo) / (Fhi - Flo);
    double t = floor(q * 4294967296.0);
    if (t < 0) t = 0;
    if (t > 4294967296.0) t = 4294967296.0;
    thr[j] = (uint64_t)t;
  }
  return NULL;
}

int orc_weight_distribution(orc_net* o, uint32_t proj, int kind, double a, double b, double lo, double hi,
                            uint32_t levels) {
  if (o->built || o->shift) { set_err(o, "weights after build"); return -1; }
  if (proj >= o->n_proj || o->proj[proj].rule == ORC_RULE_LIST) { set_err(o, "projection"); return -1; }
  if (levels < 1 || levels > ORC_WEIGHT_LEVELS_MAX) { set_err(o, "levels"); return -1; }
  double* lev = (double*)malloc(levels * sizeof(double));
  uint64_t* thr = (uint64_t*)malloc(levels * sizeof(uint64_t));
  const char* e = dist_levels(kind, a, b, lo, hi, levels, lev, thr);
  if (e) { free(lev); free(thr); set_err(o, e); return -1; }
  orc_proj* pr = &o->proj[proj];
  free(pr->wlev); free(pr->wthr);
  pr->wlev = lev; pr->wthr = thr; pr->wlevels = levels;
  return 0;
}

int orc_set_param(orc_net* o, uint32_t first, uint32_t n, int param, const double* v) {
  if (o->N == 0 || (uint64_t)first + n > o->N) { set_err(o, "range"); return -1; }
  if (o->V) { set_err(o, "per-neuron parameters come before any state"); return -1; }
  if (!o->npar) {
    o->npar = (orc_pop_params*)malloc((size_t)o->N * sizeof(orc_pop_params));
    for (uint32_t i = 0; i < o->N; ++i) o->npar[i] = o->pops[pop_index(o, i)];
  }
  for (uint32_t j = 0; j < n; ++j) {
    orc_pop_params* q = &o->npar[first + j];
    double x = v[j];
    switch (param) {
      case 0: q->tau_m = x; break;
      case 1: q->C_m = x; break;
      case 2: q->E_L = x; break;
      case 3: q->V_th = x; break;
      case 4: q->V_reset = x; break;
      case 5: q->t_ref = x; break;
      case 6: q->g_L = x; break;
      case 7: q->Delta_T = x; break;
      case 8: q->V_T = x; break;
      case 9: q->tau_w = x; break;
      case 10: q->a = x; break;
      case 11: q->b = x; break;
      case 12: q->V_peak = x; break;
      case 13: q->V_r = x; break;
      case 14: q->rk_eps = x; break;
      case 15: q->rk_hmin = x; break;
      default: set_err(o, "param"); return -1;
    }
  }
  return 0;
}

double orc_get_param(const orc_net* o, uint32_t gid, int param) {
  if (gid >= o->N) return NAN;
  const orc_pop_params* q = neuron_params(o, gid, pop_index(o, gid));
  const double v[16] = {q->tau_m, q->C_m, q->E_L, q->V_th, q->V_reset, q->t_ref, q->g_L, q->Delta_T,
                        q->V_T, q->tau_w, q->a, q->b, q->V_peak, q->V_r, q->rk_eps, q->rk_hmin};
  return (param >= 0 && param < 16) ? v[param] : NAN;
}

int orc_param_distribution(orc_net* o, uint32_t first, uint32_t n, int param, int kind, double a, double b,
                           double lo, double hi, uint32_t levels) {
  if (o->N == 0 || (uint64_t)first + n > o->N) { set_err(o, "range"); return -1; }
  if (param < 0 || param > 15) { set_err(o, "param"); return -1; }
  if (levels < 1 || levels > ORC_STATE_LEVELS_MAX) { set_err(o, "levels"); return -1; }
  double* lev = (double*)malloc(levels * sizeof(double));
  uint64_t* thr = (uint64_t*)malloc(levels * sizeof(uint64_t));
  double* v = (double*)malloc((n ? n : 1) * sizeof(double));
  const char* e = dist_levels(kind, a, b, lo, hi, levels, lev, thr);
  if (e) { free(lev); free(thr); free(v); set_err(o, e); return -1; }
  uint64_t key[2] = {o->seed, 0};
  for (uint32_t j = 0; j < n; ++j) {
    uint64_t ctr[4] = {first + j, (uint64_t)param << 8, ORC_TAG_PARAM, 0}, blk[4];
    orc_philox4x64_10(ctr, key, blk);
    uint32_t u = (uint32_t)(blk[0] >> 32), l = 0;
    while ((uint64_t)u >= thr[l]) ++l;
    v[j] = lev[l];
  }
  int rc = orc_set_param(o, first, n, param, v);
  free(lev); free(thr); free(v);
  return rc;
}

/* State drawn from a distribution: neuron i takes the level of the top 32
   bits of word 0 of block (i, var << 8 | port, ORC_TAG_STATE, 0), key
   (seed, 0), then is set as by orc_set_state. */
int orc_state_distribution(orc_net* o, uint32_t first, uint32_t n, int var, uint32_t port, int kind, double a,
                           double b, double lo, double hi, uint32_t levels) {
  if (o->N == 0 || (uint64_t)first + n > o->N) { set_err(o, "range"); return -1; }
  if (var == 5 || var < 0 || var > 7) { set_err(o, "var"); return -1; }
  if (levels < 1 || levels > ORC_STATE_LEVELS_MAX) { set_err(o, "levels"); return -1; }
  double* lev = (double*)malloc(levels * sizeof(double));
  uint64_t* thr = (uint64_t*)malloc(levels * sizeof(uint64_t));
  double* v = (double*)malloc((n ? n : 1) * sizeof(double));
  const char* e = dist_levels(kind, a, b, lo, hi, levels, lev, thr);
  if (e) { free(lev); free(thr); free(v); set_err(o, e); return -1; }
  uint64_t key[2] = {o->seed, 0};
  for (uint32_t j = 0; j < n; ++j) {
    uint64_t ctr[4] = {first + j, ((uint64_t)var << 8) | port, ORC_TAG_STATE, 0}, blk[4];
    orc_philox4x64_10(ctr, key, blk);
    uint32_t u = (uint32_t)(blk[0] >> 32), l = 0;
    while ((uint64_t)u >= thr[l]) ++l;
    v[j] = lev[l];
  }
  int rc = orc_set_state(o, first, n, var, port, v);
  free(lev); free(thr); free(v);
  return rc;
}

int orc_stdp(orc_net* o, uint32_t proj, double tau_plus, double tau_minus, double lambda, double alpha, int mu_plus,
             int mu_minus, double w_max) {
  if (o->built || o->shift) { set_err(o, "stdp after build"); return -1; }
  if (proj >= o->n_proj) { set_err(o, "no such projection"); return -1; }
  if (!(tau_plus > 0) || !(tau_minus > 0) || !(lambda > 0) || !(lambda <= 1) || !(alpha >= 0) ||
      !(alpha * lambda <= 1) || !(w_max > 0) || (mu_plus != 0 && mu_plus != 1) || (mu_minus != 0 && mu_minus != 1)) {
    set_err(o, "bad stdp parameters"); return -1;
  }
  orc_proj* pr = &o->proj[proj];
  double lo = pr->wlevels ? pr->wlev[0] : pr->weight, hi = pr->wlevels ? pr->wlev[pr->wlevels - 1] : pr->weight;
  if (lo < 0 || hi > w_max) { set_err(o, "plastic weights must lie in [0, w_max]"); return -1; }
  pr->plastic = 1; pr->tau_plus = tau_plus; pr->tau_minus = tau_minus; pr->lambda = lambda; pr->alpha = alpha;
  pr->mu_plus = mu_plus; pr->mu_minus = mu_minus; pr->w_max = w_max;
  return 0;
}

int orc_list_weights(orc_net* o, uint32_t proj, uint64_t n, const double* weights) {
  if (o->built || o->shift) { set_err(o, "weights after build"); return -1; }
  if (proj >= o->n_proj || o->proj[proj].rule != ORC_RULE_LIST || o->proj[proj].n != n) {
    set_err(o, "list projection"); return -1;
  }
  /* levels: the distinct listed values, ascending (a library sort) */
  double* v = (double*)malloc((n ? n : 1) * sizeof(double));
  memcpy(v, weights, n * sizeof(double));
  qsort(v, (size_t)n, sizeof(double), dbl_cmp);
  uint64_t m = 0;
  for (uint64_t j = 0; j < n; ++j)
    if (m == 0 || v[j] != v[m - 1]) v[m++] = v[j];
  if (m > ORC_WEIGHT_LEVELS_MAX) { free(v); set_err(o, "too many distinct weights"); return -1; }
  orc_proj* pr = &o->proj[proj];
  free(pr->wlev); free(pr->lwl);
  pr->wlev = v; pr->wlevels = (uint32_t)m;
  pr->lwl = (uint16_t*)malloc((n ? n : 1) * sizeof(uint16_t));
  for (uint64_t j = 0; j < n; ++j) {
    uint64_t lo = 0, hi = m;  /* the level holding weights[j] */
    while (hi - lo > 1) { uint64_t mid = (lo + hi) / 2; if (v[mid] <= weights[j]) lo = mid; else hi = mid; }
    pr->lwl[j] = (uint16_t)lo;
  }
  return 0;
}

static void alloc_state(orc_net* o);

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : x > y;
}

int orc_set_spike_times(orc_net* o, uint32_t gid, uint64_t n, const double* t_ms) {
  if (o->built) { set_err(o, "spike times after build"); return -1; }
  if (gid >= o->N) { set_err(o, "range"); return -1; }
  alloc_state(o);
  if (o->pops[o->pop_of[gid]].model != ORC_SPIKE_GENERATOR) { set_err(o, "not a spike generator"); return -1; }
  uint64_t* st = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  for (uint64_t j = 0; j < n; ++j) {
    double r = floor(t_ms[j] / o->dt + 0.5);  /* steps of dt, half up */
    if (!(r >= 1.0)) { free(st); set_err(o, "spike time below dt"); return -1; }
    st[j] = (uint64_t)r - 1;
  }
  qsort(st, (size_t)n, sizeof(uint64_t), cmp_u64);
  free(o->gen_steps[gid]);
  o->gen_steps[gid] = st; o->gen_n[gid] = n; o->gen_pos[gid] = 0;
  return 0;
}

int orc_poisson(orc_net* o, uint32_t tgt_first, uint32_t tgt_n, double rate_hz, uint32_t n_inputs,
                double weight, uint32_t port) {
  if (o->built || o->shift) { set_err(o, "poisson after build"); return -1; }
  if ((uint64_t)tgt_first + tgt_n > o->N) { set_err(o, "range"); return -1; }
  orc_pois q;
  memset(&q, 0, sizeof q);
  q.tgt_first = tgt_first; q.tgt_n = tgt_n; q.port = port; q.weight = weight;
  /* n_inputs independent trains of rate_hz each, summed: Poisson(n nu dt) */
  q.lambda = (double)n_inputs * rate_hz * o->dt * 1e-3;
  if (orc_poisson_table(q.lambda, ORC_POISSON_KMAX, q.thr) != 0) { set_err(o, "poisson"); return -1; }
  o->pois = (orc_pois*)realloc(o->pois, (o->n_pois + 1) * sizeof(orc_pois));
  o->pois[o->n_pois++] = q;
  return 0;
}

static void alloc_state(orc_net* o) {
  if (o->V) return;
  o->P = 1;
  for (uint32_t k = 0; k < o->n_pops; ++k) if (o->pops[k].n_ports > o->P) o->P = o->pops[k].n_ports;
  size_t N = o->N, P = o->P;
  o->pop_of = (uint32_t*)malloc(N * sizeof(uint32_t));
  for (uint32_t i = 0; i < o->N; ++i) o->pop_of[i] = pop_index(o, i);
  o->V = (double*)calloc(N, sizeof(double));
  o->Ie = (double*)calloc(N, sizeof(double));
  o->w = (double*)calloc(N, sizeof(double));
  o->g = (double*)calloc(N * P, sizeof(double));
  o->gr = (double*)calloc(N * P, sizeof(double));
  o->I = (double*)calloc(N * P, sizeof(double));
  o->h = (double*)malloc(N * sizeof(double));
  for (size_t i = 0; i < N; ++i) o->h[i] = o->dt;
  o->refr = (int32_t*)calloc(N, sizeof(int32_t));
  o->gen_steps = (uint64_t**)calloc(N, sizeof(uint64_t*));
  o->gen_n = (uint64_t*)calloc(N, sizeof(uint64_t));
  o->gen_pos = (uint64_t*)calloc(N, sizeof(uint64_t));
  o->Vf = (float*)calloc(N, sizeof(float));
  o->If = (float*)calloc(N * P, sizeof(float));
  o->Ief = (float*)calloc(N, sizeof(float));
  o->acc = (int64_t*)calloc(N * P, sizeof(int64_t));
  o->mult_now = (uint32_t*)calloc(N, sizeof(uint32_t));
  for (size_t i = 0; i < N; ++i) o->V[i] = neuron_params(o, (uint32_t)i, o->pop_of[i])->E_L; /* rest */
  for (size_t i = 0; i < N; ++i) {
    const orc_pop_params* pp = neuron_params(o, (uint32_t)i, o->pop_of[i]);
    if (!is_adex(pp)) o->Vf[i] = (float)(o->V[i] - pp->E_L);
  }
}

/* var: 0 V_m, 1 I_e, 2 w, 3 g[port], 4 I_syn[port], 5 refractory, 6 h,
   7 r[port] (rising variable of a beta port) */
int orc_set_state(orc_net* o, uint32_t first, uint32_t n, int var, uint32_t port, const double* v) {
  if (o->N == 0 || (uint64_t)first + n > o->N) { set_err(o, "range"); return -1; }
  alloc_state(o);
  if ((var == 3 || var == 4 || var == 7) && port >= o->P) { set_err(o, "port"); return -1; }
  for (uint32_t j = 0; j < n; ++j) {
    uint32_t i = first + j;
    const orc_pop_params* pp = neuron_params(o, i, o->pop_of[i]);
    switch (var) {
      case 0:
        o->V[i] = v[j];
        /* LIF keeps y = V - E_L; the float copy is rounded once from double */
        if (!is_adex(pp)) o->Vf[i] = (float)(v[j] - pp->E_L);
        break;
      case 1: o->Ie[i] = v[j]; o->Ief[i] = (float)v[j]; break;
      case 2: o->w[i] = v[j]; break;
      case 3: o->g[(size_t)i * o->P + port] = v[j]; break;
      case 4: o->I[(size_t)i * o->P + port] = v[j]; o->If[(size_t)i * o->P + port] = (float)v[j]; break;
      case 5: o->refr[i] = (int32_t)v[j]; break;
      case 6: o->h[i] = v[j]; break;
      case 7: o->gr[(size_t)i * o->P + port] = v[j]; break;
      default: set_err(o, "var"); return -1;
    }
  }
  return 0;
}

int orc_get_state(orc_net* o, uint32_t first, uint32_t n, int var, uint32_t port, double* v) {
  if (o->N == 0 || (uint64_t)first + n > o->N) { set_err(o, "range"); return -1; }
  alloc_state(o);
  if ((var == 3 || var == 4 || var == 7) && port >= o->P) { set_err(o, "port"); return -1; }
  int f32 = (o->mode == ORC_FP32SO);
  for (uint32_t j = 0; j < n; ++j) {
    uint32_t i = first + j;
    const orc_pop_params* pp = neuron_params(o, i, o->pop_of[i]);
    int lif = !is_adex(pp);
    switch (var) {
      case 0: v[j] = (lif && f32) ? (double)o->Vf[i] + pp->E_L : o->V[i]; break;
      case 1: v[j] = o->Ie[i]; break;
      case 2: v[j] = o->w[i]; break;
      case 3: v[j] = o->g[(size_t)i * o->P + port]; break;
      case 4: v[j] = (lif && f32) ? (double)o->If[(size_t)i * o->P + port] : o->I[(size_t)i * o->P + port]; break;
      case 5: v[j] = (double)o->refr[i]; break;
      case 6: v[j] = o->h[i]; break;
      case 7: v[j] = o->gr[(size_t)i * o->P + port]; break;
      default: set_err(o, "var"); return -1;
    }
  }
  return 0;
}

/* canonical order: source, delay, target, port, quantised weight */
static int syn_cmp(const void* pa, const void* pb) {
  const orc_syn* a = (const orc_syn*)pa;
  const orc_syn* b = (const orc_syn*)pb;
  if (a->src != b->src) return a->src < b->src ? -1 : 1;
  if (a->d != b->d) return a->d < b->d ? -1 : 1;
  if (a->tgt != b->tgt) return a->tgt < b->tgt ? -1 : 1;
  if (a->port != b->port) return a->port < b->port ? -1 : 1;
  if (a->wq != b->wq) return a->wq < b->wq ? -1 : 1;
  if ((a->plast >= 0) != (b->plast >= 0)) return a->plast < 0 ? -1 : 1;  /* static before plastic */
  return 0;
}

/* draw delay steps from a table */
static uint32_t draw_delay(const uint64_t* thr, uint32_t dmax, uint32_t u) {
  for (uint32_t k = 1; k <= dmax; ++k) if ((uint64_t)u < thr[k]) return k;
  return dmax;
}

/* Everything of the build but the synapse table: state, Poisson drive per
   neuron, fixed-point exponents.  Idempotent. */
static int prepare(orc_net* o) {
  if (o->shift) return 0;
  if (o->N == 0) { set_err(o, "empty"); return -1; }
  alloc_state(o);
  uint32_t P = o->P;
  /* Poisson drive per neuron (at most one) */
  o->pois_of = (int32_t*)malloc(o->N * sizeof(int32_t));
  for (uint32_t i = 0; i < o->N; ++i) o->pois_of[i] = -1;
  for (uint32_t q = 0; q < o->n_pois; ++q) {
    for (uint32_t j = 0; j < o->pois[q].tgt_n; ++j) {
      uint32_t i = o->pois[q].tgt_first + j;
      if (o->pois_of[i] >= 0) { set_err(o, "two poisson drives on one neuron"); return -1; }
      o->pois_of[i] = (int32_t)q;
    }
  }
  /* fixed-point shift per (target population, port): the largest S such that
     every weight arriving on that port satisfies |w| 2^S < 2^30 */
  o->shift = (int*)calloc((size_t)o->n_pops * P, sizeof(int));
  double* maxw = (double*)calloc((size_t)o->n_pops * P, sizeof(double));
  for (uint32_t p = 0; p < o->n_proj; ++p) {
    const orc_proj* pr = &o->proj[p];
    if (proj_synapses(pr) == 0) continue;
    for (uint32_t k = 0; k < o->n_pops; ++k) {
      uint32_t lo = o->pop_first[k];
      uint32_t hi = (k + 1 < o->n_pops) ? o->pop_first[k + 1] : o->N;
      if (pr->tgt_first < hi && pr->tgt_first + pr->tgt_n > lo) {
        if (pr->port >= o->pops[k].n_ports) { set_err(o, "port out of range"); free(maxw); return -1; }
        double aw = fabs(pr->weight);
        for (uint32_t j = 0; j < pr->wlevels; ++j) aw = j ? fmax(aw, fabs(pr->wlev[j])) : fabs(pr->wlev[j]);
        if (pr->plastic) aw = fmax(aw, pr->w_max);  /* a plastic weight grows up to w_max */
        if (aw > maxw[k * P + pr->port]) maxw[k * P + pr->port] = aw;
        /* conductances jump by the weight: none may be negative */
        int cond = o->pops[k].model == ORC_AEIF_COND_EXP || o->pops[k].model == ORC_AEIF_COND_BETA;
        int neg = pr->wlevels ? pr->wlev[0] < 0 : pr->weight < 0;
        if (cond && neg) { set_err(o, "conductance weights must be >= 0"); free(maxw); return -1; }
      }
    }
  }
  for (uint32_t q = 0; q < o->n_pois; ++q) {
    const orc_pois* pq = &o->pois[q];
    for (uint32_t k = 0; k < o->n_pops; ++k) {
      uint32_t lo = o->pop_first[k];
      uint32_t hi = (k + 1 < o->n_pops) ? o->pop_first[k + 1] : o->N;
      if (pq->tgt_n && pq->tgt_first < hi && pq->tgt_first + pq->tgt_n > lo) {
        if (pq->port >= o->pops[k].n_ports) { set_err(o, "port out of range"); free(maxw); return -1; }
        double aw = fabs(pq->weight);
        if (aw > maxw[k * P + pq->port]) maxw[k * P + pq->port] = aw;
      }
    }
  }
  for (size_t k = 0; k < (size_t)o->n_pops * P; ++k) o->shift[k] = orc_fixed_point_shift(maxw[k]);
  free(maxw);
  /* parrots count arriving spikes: every weight onto them must be 1 */
  for (uint32_t k = 0; k < o->n_pops; ++k) {
    if (o->pops[k].model != ORC_PARROT) continue;
    uint32_t lo = o->pop_first[k], hi = (k + 1 < o->n_pops) ? o->pop_first[k + 1] : o->N;
    for (uint32_t p = 0; p < o->n_proj; ++p) {
      const orc_proj* pr = &o->proj[p];
      int unit = pr->wlevels ? (pr->wlevels == 1 && pr->wlev[0] == 1.0) : pr->weight == 1.0;
      if (proj_synapses(pr) && pr->tgt_first < hi && pr->tgt_first + pr->tgt_n > lo && !unit) {
        set_err(o, "weights onto parrot neurons must be 1"); return -1;
      }
    }
    for (uint32_t q = 0; q < o->n_pois; ++q) {
      const orc_pois* pq = &o->pois[q];
      if (pq->tgt_n && pq->tgt_first < hi && pq->tgt_first + pq->tgt_n > lo && pq->weight != 1.0) {
        set_err(o, "weights onto parrot neurons must be 1"); return -1;
      }
    }
  }
  return 0;
}

/* Counters of the connection draws, key (seed, 0), tag CONN; p is the
   projection's creation index, x << y a shift:
   fixed in-degree  -- target t, draw k < n: block (t, p<<40 | k>>1), words
                       2(k&1) (source) and 2(k&1)+1 (delay);
   fixed out-degree -- source s, draw k < n: block (s, p<<40 | k>>1), words
                       2(k&1) (target) and 2(k&1)+1 (delay);
   all-to-all       -- target t, source index k: block (t, p<<40 | k>>1),
                       word 2(k&1)+1 (delay);
   one-to-one       -- target t: block (t, p<<40), word 1 (delay);
   fixed total      -- synapse j < n: block (j, p<<40), words 0 (source),
                       1 (target), 2 (delay).
   A uniform index in a range of m is floor(u m / 2^64); a delay uses the top
   32 bits of its word against the projection's threshold table. */
static uint32_t uniform_index(uint64_t u, uint32_t m) { return (uint32_t)(((unsigned __int128)u * m) >> 64); }

/* synapse k of entity e (target, source or synapse index, by rule) of
   projection p; blk holds the block of the pair k belongs to */
static void draw_synapse(const orc_net* o, uint32_t p, uint64_t e, uint32_t k, uint64_t blk[4], uint32_t* src,
                         uint32_t* tgt, uint32_t* d) {
  const orc_proj* pr = &o->proj[p];
  uint64_t key[2] = {o->seed, 0};
  if (pr->rule == ORC_RULE_LIST) {  /* user-defined: synapse e as listed */
    *src = pr->lsrc[e]; *tgt = pr->ltgt[e]; *d = pr->ldel[e];
    return;
  }
  if (pr->rule == ORC_RULE_ONE_TO_ONE || pr->rule == ORC_RULE_FIXED_TOTAL_NUMBER) {
    uint64_t ctr[4] = {e, (uint64_t)p << 40, ORC_TAG_CONN, 0};
    orc_philox4x64_10(ctr, key, blk);
    if (pr->rule == ORC_RULE_ONE_TO_ONE) {
      *tgt = (uint32_t)e; *src = pr->src_first + ((uint32_t)e - pr->tgt_first);
      *d = draw_delay(pr->dthr, o->dmax, (uint32_t)(blk[1] >> 32));
    } else {
      *src = pr->src_first + uniform_index(blk[0], pr->src_n);
      *tgt = pr->tgt_first + uniform_index(blk[1], pr->tgt_n);
      *d = draw_delay(pr->dthr, o->dmax, (uint32_t)(blk[2] >> 32));
    }
    return;
  }
  if ((k & 1u) == 0) {
    uint64_t ctr[4] = {e, ((uint64_t)p << 40) | (uint64_t)(k >> 1), ORC_TAG_CONN, 0};
    orc_philox4x64_10(ctr, key, blk);
  }
  uint64_t u = blk[2 * (k & 1u)];
  *d = draw_delay(pr->dthr, o->dmax, (uint32_t)(blk[2 * (k & 1u) + 1] >> 32));
  if (pr->rule == ORC_RULE_FIXED_INDEGREE) { *tgt = (uint32_t)e; *src = pr->src_first + uniform_index(u, pr->src_n); }
  else if (pr->rule == ORC_RULE_FIXED_OUTDEGREE) { *src = (uint32_t)e; *tgt = pr->tgt_first + uniform_index(u, pr->tgt_n); }
  else { *tgt = (uint32_t)e; *src = pr->src_first + k; }  /* all-to-all */
}

/* quantised weight of synapse k of entity e of projection p onto target t:
   the fixed weight, the level of a listed synapse, or the level drawn by the
   weight distribution (block of tag WEIGHT; wblk holds the block of the four
   draws k belongs to) */
static int64_t synapse_wq(const orc_net* o, uint32_t p, uint64_t e, uint32_t k, uint32_t t, uint64_t wblk[4]) {
  const orc_proj* pr = &o->proj[p];
  int S = o->shift[o->pop_of[t] * o->P + pr->port];
  if (pr->wlevels == 0) return llrint(ldexp(pr->weight, S));
  if (pr->rule == ORC_RULE_LIST) return llrint(ldexp(pr->wlev[pr->lwl[e]], S));
  if ((k & 3u) == 0) {
    uint64_t key[2] = {o->seed, 0};
    uint64_t ctr[4] = {e, ((uint64_t)p << 40) | (uint64_t)(k >> 2), ORC_TAG_WEIGHT, 0};
    orc_philox4x64_10(ctr, key, wblk);
  }
  uint32_t u = (uint32_t)(wblk[k & 3u] >> 32);
  uint32_t j = 0;
  while ((uint64_t)u >= pr->wthr[j]) ++j;
  return llrint(ldexp(pr->wlev[j], S));
}

int orc_prepare(orc_net* o) { return prepare(o); }

int orc_build(orc_net* o) {
  if (o->built) { set_err(o, "built twice"); return -1; }
  if (prepare(o) != 0) return -1;
  uint32_t P = o->P, D1 = o->dmax + 1;
  uint64_t total = 0;
  for (uint32_t p = 0; p < o->n_proj; ++p) total += proj_synapses(&o->proj[p]);
  o->n_syn = total;
  o->syn = (orc_syn*)malloc((total ? total : 1) * sizeof(orc_syn));
  uint64_t pos = 0;
  for (uint32_t p = 0; p < o->n_proj; ++p) {
    const orc_proj* pr = &o->proj[p];
    if (proj_synapses(pr) == 0) continue;
    /* entities: targets, sources (out-degree) or synapses (total number);
       draws per entity: n, n, n_src, 1, 1 */
    int per_syn = pr->rule == ORC_RULE_FIXED_TOTAL_NUMBER || pr->rule == ORC_RULE_LIST;
    uint64_t ne = pr->rule == ORC_RULE_FIXED_OUTDEGREE ? pr->src_n : per_syn ? pr->n : pr->tgt_n;
    uint64_t first = pr->rule == ORC_RULE_FIXED_OUTDEGREE ? pr->src_first : per_syn ? 0 : pr->tgt_first;
    uint32_t kn = per_syn ? 1u : pr->K;
    for (uint64_t j = 0; j < ne; ++j) {
      uint64_t blk[4] = {0, 0, 0, 0}, wblk[4] = {0, 0, 0, 0};
      for (uint32_t k = 0; k < kn; ++k) {
        uint32_t s, t, d;
        draw_synapse(o, p, first + j, k, blk, &s, &t, &d);
        orc_syn sy;
        sy.src = s; sy.tgt = t; sy.port = (uint8_t)pr->port; sy.d = (uint8_t)d;
        sy.wq = synapse_wq(o, p, first + j, k, t, wblk);
        sy.plast = pr->plastic ? (int32_t)p : -1;
        o->syn[pos++] = sy;
      }
    }
  }
  /* canonical order (a library sort), then offsets of each (source, delay) run */
  qsort(o->syn, (size_t)o->n_syn, sizeof(orc_syn), syn_cmp);
  o->off = (uint64_t*)calloc((size_t)o->N * D1 + 1, sizeof(uint64_t));
  for (uint64_t e = 0; e < o->n_syn; ++e) o->off[(size_t)o->syn[e].src * D1 + o->syn[e].d + 1]++;
  for (size_t k = 1; k <= (size_t)o->N * D1; ++k) o->off[k] += o->off[k - 1];
  /* plastic synapses: their weights, last arrivals and the index by target */
  for (uint64_t e = 0; e < o->n_syn; ++e) o->n_plastic += o->syn[e].plast >= 0;
  if (o->n_plastic) {
    o->pw = (int64_t*)malloc(o->n_syn * sizeof(int64_t));
    o->pwmax = (int64_t*)malloc(o->n_syn * sizeof(int64_t));
    o->last_pre = (int64_t*)malloc(o->n_syn * sizeof(int64_t));
    o->arr_m = (uint32_t*)calloc(o->n_syn, sizeof(uint32_t));
    o->last_post = (int64_t*)malloc((size_t)o->N * sizeof(int64_t));
    o->tptr = (uint64_t*)calloc((size_t)o->N + 1, sizeof(uint64_t));
    o->tidx = (uint64_t*)malloc(o->n_plastic * sizeof(uint64_t));
    for (uint32_t i = 0; i < o->N; ++i) o->last_post[i] = -1;
    for (uint64_t e = 0; e < o->n_syn; ++e) {
      const orc_syn* sy = &o->syn[e];
      o->pw[e] = sy->wq;
      o->last_pre[e] = -1;
      o->pwmax[e] = 0;
      if (sy->plast < 0) continue;
      o->pwmax[e] = llrint(ldexp(o->proj[sy->plast].w_max, o->shift[o->pop_of[sy->tgt] * P + sy->port]));
      o->tptr[sy->tgt + 1]++;
    }
    for (uint32_t i = 0; i < o->N; ++i) o->tptr[i + 1] += o->tptr[i];
    uint64_t* fill = (uint64_t*)calloc((size_t)o->N, sizeof(uint64_t));
    for (uint64_t e = 0; e < o->n_syn; ++e)
      if (o->syn[e].plast >= 0) o->tidx[o->tptr[o->syn[e].tgt] + fill[o->syn[e].tgt]++] = e;
    free(fill);
  }
  /* spike record */
  o->cap_spk = 1024;
  o->spk_step = (uint64_t*)malloc(o->cap_spk * sizeof(uint64_t));
  o->spk_gid = (uint32_t*)malloc(o->cap_spk * sizeof(uint32_t));
  o->spk_mult = (uint32_t*)malloc(o->cap_spk * sizeof(uint32_t));
  o->cap_at = 1024;
  o->spk_at = (uint64_t*)calloc(o->cap_at, sizeof(uint64_t));
  o->built = 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* LIF exact integration (Sec. 2.1 and the LIF / exponential-PSC equations   */
/* of Sec. 2.3).  With y = V - E_L the linear system                          */
/*   dy/dt = -y/tau_m + (I + I_e)/C,  dI/dt = -I/tau_s                       */
/* is propagated exactly over dt:                                             */
/*   P22 = e^{-dt/tau_m},  P11 = e^{-dt/tau_s},  P20 = tau_m/C (1 - P22),     */
/*   P21 = tau_m tau_s / (C (tau_s - tau_m)) (e^{-dt/tau_s} - e^{-dt/tau_m})  */
/*       = (dt/C) e^{-dt/tau_m} (e^x - 1)/x,  x = dt (tau_s - tau_m)/(tau_m tau_s) */
/*   (the second form has no cancellation when tau_s is close to tau_m; its   */
/*   limit dt/C e^{-dt/tau} when tau_s = tau_m is x = 0).                     */
/* A delta PSC adds its weight (mV) to y at the step it arrives.              */
/* ------------------------------------------------------------------------ */
void orc_lif_propagators(const orc_pop_params* pp, double dt, double* out) {
  double P22 = exp(-dt / pp->tau_m);
  double P20 = pp->tau_m / pp->C_m * (1.0 - P22);
  out[0] = P22; out[1] = P20;
  for (uint32_t p = 0; p < pp->n_ports; ++p) {
    double ts = pp->tau_syn[p];
    double P11 = (ts > 0) ? exp(-dt / ts) : 0.0;
    double P21 = 0.0;
    if (ts > 0) {
      double x = dt * (ts - pp->tau_m) / (pp->tau_m * ts);
      double q = (x == 0.0) ? 1.0 : expm1(x) / x;
      P21 = dt / pp->C_m * exp(-dt / pp->tau_m) * q;
    }
    out[2 + p] = P11;
    out[2 + pp->n_ports + p] = P21;
  }
}

static int32_t refr_steps(const orc_pop_params* pp, double dt) {
  return (int32_t)floor(pp->t_ref / dt + 0.5);
}

/* Refractoriness: during the n_ref steps after a spike the membrane is held
   at V_reset and (delta PSC) arriving input is discarded; the step counter is
   decremented at each of those steps.  Threshold test V >= V_th. */
int orc_lif_delta_step64(const orc_pop_params* pp, double dt, double* y, int32_t* refr, double I_e, double x) {
  double pr[2 + 2 * ORC_MAX_PORTS];
  orc_lif_propagators(pp, dt, pr);
  double theta = pp->V_th - pp->E_L, yr = pp->V_reset - pp->E_L;
  if (*refr > 0) {
    *refr -= 1;
  } else {
    double t1 = pr[0] * (*y);
    double t2 = pr[1] * I_e;
    *y = (t1 + t2) + x;
  }
  if (*refr == 0 && *y >= theta) { *y = yr; *refr = refr_steps(pp, dt); return 1; }
  return 0;
}

int orc_lif_delta_step32(const orc_pop_params* pp, double dt, float* y, int32_t* refr, float I_e, float x) {
  double pr[2 + 2 * ORC_MAX_PORTS];
  orc_lif_propagators(pp, dt, pr);
  float P22 = (float)pr[0], P20 = (float)pr[1];
  float theta = (float)(pp->V_th - pp->E_L), yr = (float)(pp->V_reset - pp->E_L);
  if (*refr > 0) {
    *refr -= 1;
  } else {
    float t1 = P22 * (*y);
    float t2 = P20 * I_e;
    float t3 = t1 + t2;
    *y = t3 + x;
  }
  if (*refr == 0 && *y >= theta) { *y = yr; *refr = refr_steps(pp, dt); return 1; }
  return 0;
}

int orc_lif_exp_step64(const orc_pop_params* pp, double dt, double* y, double* I, int32_t* refr, double I_e,
                       const double* x) {
  double pr[2 + 2 * ORC_MAX_PORTS];
  orc_lif_propagators(pp, dt, pr);
  uint32_t P = pp->n_ports;
  double theta = pp->V_th - pp->E_L, yr = pp->V_reset - pp->E_L;
  if (*refr == 0) {
    double v = pr[0] * (*y);
    for (uint32_t p = 0; p < P; ++p) v = v + pr[2 + P + p] * I[p];
    v = v + pr[1] * I_e;
    *y = v;
  } else {
    *refr -= 1;
  }
  for (uint32_t p = 0; p < P; ++p) I[p] = pr[2 + p] * I[p] + x[p];
  if (*refr == 0 && *y >= theta) { *y = yr; *refr = refr_steps(pp, dt); return 1; }
  return 0;
}

int orc_lif_exp_step32(const orc_pop_params* pp, double dt, float* y, float* I, int32_t* refr, float I_e,
                       const float* x) {
  double pr[2 + 2 * ORC_MAX_PORTS];
  orc_lif_propagators(pp, dt, pr);
  uint32_t P = pp->n_ports;
  float theta = (float)(pp->V_th - pp->E_L), yr = (float)(pp->V_reset - pp->E_L);
  if (*refr == 0) {
    float v = (float)pr[0] * (*y);
    for (uint32_t p = 0; p < P; ++p) {
      float t = (float)pr[2 + P + p] * I[p];
      v = v + t;
    }
    float te = (float)pr[1] * I_e;
    v = v + te;
    *y = v;
  } else {
    *refr -= 1;
  }
  for (uint32_t p = 0; p < P; ++p) {
    float t = (float)pr[2 + p] * I[p];
    I[p] = t + x[p];
  }
  if (*refr == 0 && *y >= theta) { *y = yr; *refr = refr_steps(pp, dt); return 1; }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* AdEx with conductance synapses (Sec. 2.4, Table 2):                        */
/*   C dV/dt = -g_L (V - E_L) + g_L Delta_T exp((V - V_T)/Delta_T)            */
/*             - sum_p g_p (V - E_rev,p) - w + I_e                            */
/*   tau_w dw/dt = a (V - E_L) - w                                            */
/* Conductance of port p, either                                              */
/*   exponential:  dg_p/dt = -g_p / tau_syn,p                                 */
/*   beta (Sec. 2.1 example; alpha when tau_rise = tau_decay, Sec. 2.4):      */
/*                 dg_p/dt = r_p - g_p / tau_decay,p,  dr_p/dt = -r_p/tau_rise */
/*   an input of weight w at t0 adds g0 w to r_p, giving                       */
/*   g(t) = g0 w (e^{-s/td} - e^{-s/tr}) / (1/tr - 1/td), s = t - t0           */
/*   (g0 w s e^{-s/t} for tr = td = t), whose peak is w (see orc_beta_g0).     */
/* The synaptic current is taken with the sign that makes an excitatory       */
/* conductance depolarise.  The exponential uses min(V, V_peak).  At a reset  */
/* (V >= V_peak after an accepted substep) V -> V_r and w -> w + b.           */
/* ------------------------------------------------------------------------ */
double orc_beta_g0(double tr, double td) {
  /* alpha limit: g = g0 w s e^{-s/t} peaks at s = t with value g0 w t / e */
  if (fabs(td - tr) <= 1e-12 * td) return exp(1.0) / td;
  /* peak of e^{-s/td} - e^{-s/tr} at s* = ln(td/tr) / (1/tr - 1/td) */
  double rate = 1.0 / tr - 1.0 / td;
  double sp = log(td / tr) / rate;
  double peak = (exp(-sp / td) - exp(-sp / tr)) / rate;
  return 1.0 / peak;
}

void orc_adex_rhs(const orc_pop_params* pp, double I_e, const double* y, double* dy) {
  uint32_t P = pp->n_ports;
  double V = y[0], w = y[1];
  double Vc = V < pp->V_peak ? V : pp->V_peak;
  double isyn = 0.0;
  for (uint32_t p = 0; p < P; ++p) isyn += y[2 + p] * (V - pp->E_rev[p]);
  double ex = pp->adex_no_exp ? 0.0 : pp->g_L * pp->Delta_T * exp((Vc - pp->V_T) / pp->Delta_T);
  dy[0] = (-pp->g_L * (V - pp->E_L) + ex - isyn - w + I_e) / pp->C_m;
  dy[1] = (pp->a * (V - pp->E_L) - w) / pp->tau_w;
  if (pp->model == ORC_AEIF_COND_BETA) {
    for (uint32_t p = 0; p < P; ++p) {
      dy[2 + p] = y[2 + P + p] - y[2 + p] / pp->tau_syn[p];
      dy[2 + P + p] = -y[2 + P + p] / pp->tau_rise[p];
    }
  } else {
    for (uint32_t p = 0; p < P; ++p) dy[2 + p] = -y[2 + p] / pp->tau_syn[p];
  }
}

/* Cash-Karp embedded 5(4) Runge-Kutta pair (Cash & Karp 1990), the adaptive
   fifth-order method of Press et al. 1992. */
static const double CK_C[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
static const double CK_A[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
static const double CK_B5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
static const double CK_B4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0,
                                277.0 / 14336.0, 1.0 / 4.0};

void orc_cash_karp_tableau(double* c, double* a, double* b5, double* b4) {
  for (int i = 0; i < 6; ++i) {
    c[i] = CK_C[i]; b5[i] = CK_B5[i]; b4[i] = CK_B4[i];
    for (int j = 0; j < 6; ++j) a[i * 6 + j] = (j < 5) ? CK_A[i][j] : 0.0;
  }
}

/* Step-size control of Press et al. (rkqs): error measured relative to
   |y| + |h dy/dt| + 1 (state units: mV, pA, nS; the unit floor keeps the test
   meaningful for variables that are exactly zero, such as w and g at rest),
   scaled by eps; a failed step shrinks h by 0.9 e^{-1/4} (at most 10x), an
   accepted one grows it by 0.9 e^{-1/5} (at most 5x). */
#define RK_SAFETY 0.9
#define RK_PGROW (-0.2)
#define RK_PSHRNK (-0.25)
#define RK_FLOOR 1.0
#define RK_MAXIT 1000000

int orc_adex_step(const orc_pop_params* pp, double dt, double* y, double* hcar, double I_e, const double* x,
                  uint64_t* nacc, uint64_t* nrej) {
  int beta = pp->model == ORC_AEIF_COND_BETA;
  uint32_t P = pp->n_ports, NV = beta ? 2 + 2 * P : 2 + P;
  double errcon = pow(5.0 / RK_SAFETY, 1.0 / RK_PGROW);
  double eps = pp->rk_eps > 0 ? pp->rk_eps : 1e-6;
  double hmin = pp->rk_hmin > 0 ? pp->rk_hmin : 1e-8;
  /* jump by the weight delivered at this step: of the conductance itself
     (exponential), or of its rising variable (beta) */
  for (uint32_t p = 0; p < P; ++p) {
    if (beta) y[2 + P + p] += orc_beta_g0(pp->tau_rise[p], pp->tau_syn[p]) * x[p];
    else y[2 + p] += x[p];
  }
  double k[6][2 + 2 * ORC_MAX_PORTS], ytmp[2 + 2 * ORC_MAX_PORTS], y5[2 + 2 * ORC_MAX_PORTS],
      err[2 + 2 * ORC_MAX_PORTS];
  double t = 0.0;
  double h = *hcar;
  if (!(h > 0) || h > dt) h = dt;
  int mult = 0;
  long it = 0;
  while (t < dt) {
    if (++it > RK_MAXIT) break;
    int last = 0;
    if (h >= dt - t) { h = dt - t; last = 1; }
    orc_adex_rhs(pp, I_e, y, k[0]);
    for (int s = 1; s < 6; ++s) {
      for (uint32_t i = 0; i < NV; ++i) {
        double acc = 0.0;
        for (int j = 0; j < s; ++j) acc += CK_A[s][j] * k[j][i];
        ytmp[i] = y[i] + h * acc;
      }
      orc_adex_rhs(pp, I_e, ytmp, k[s]);
    }
    double errmax = 0.0;
    for (uint32_t i = 0; i < NV; ++i) {
      double s5 = 0.0, se = 0.0;
      for (int j = 0; j < 6; ++j) { s5 += CK_B5[j] * k[j][i]; se += (CK_B5[j] - CK_B4[j]) * k[j][i]; }
      y5[i] = y[i] + h * s5;
      err[i] = h * se;
      double scale = fabs(y[i]) + fabs(h * k[0][i]) + RK_FLOOR;
      double r = fabs(err[i]) / scale;
      if (r > errmax) errmax = r;
    }
    errmax /= eps;
    if (errmax > 1.0 && h > hmin) {
      double htemp = RK_SAFETY * h * pow(errmax, RK_PSHRNK);
      h = htemp > 0.1 * h ? htemp : 0.1 * h;
      if (h < hmin) h = hmin;
      (*nrej)++;
      continue;
    }
    (*nacc)++;
    t = last ? dt : t + h;
    for (uint32_t i = 0; i < NV; ++i) y[i] = y5[i];
    double hnext = (errmax > errcon) ? RK_SAFETY * h * pow(errmax, RK_PGROW) : 5.0 * h;
    if (hnext < hmin) hnext = hmin; /* the floor also bounds the proposed step */
    if (y[0] >= pp->V_peak) { y[0] = pp->V_r; y[1] += pp->b; mult++; }
    h = hnext;
  }
  if (h > dt) h = dt;
  *hcar = h;
  return mult;
}

/* ------------------------------------------------------------------------ */
/* Simulation loop.  Step n: every neuron reads the integer input delivered   */
/* for step n (plus its Poisson count for step n), converts it once with its  */
/* fixed-point exponent, updates, and records a spike (n, gid, multiplicity). */
/* Then the input for step n+1 is formed by the plain delivery definition:    */
/* for d = 1..Dmax, every spike (s, m) of step n+1-d adds m w_q of each       */
/* synapse of s with delay d to its (target, port).                           */
/* ------------------------------------------------------------------------ */
static void record_spike(orc_net* o, uint64_t n, uint32_t gid, uint32_t m) {
  if (o->n_spk == o->cap_spk) {
    o->cap_spk *= 2;
    o->spk_step = (uint64_t*)realloc(o->spk_step, o->cap_spk * sizeof(uint64_t));
    o->spk_gid = (uint32_t*)realloc(o->spk_gid, o->cap_spk * sizeof(uint32_t));
    o->spk_mult = (uint32_t*)realloc(o->spk_mult, o->cap_spk * sizeof(uint32_t));
  }
  o->spk_step[o->n_spk] = n; o->spk_gid[o->n_spk] = gid; o->spk_mult[o->n_spk] = m;
  o->n_spk++;
}

static uint32_t poisson_draw(const orc_net* o, const orc_pois* q, uint32_t gid, uint64_t n) {
  uint64_t ctr[4] = {gid, n, ORC_TAG_POISSON, 0};
  uint64_t key[2] = {o->seed, 0};
  uint64_t blk[4];
  orc_philox4x64_10(ctr, key, blk);
  uint32_t u = (uint32_t)(blk[0] >> 32);
  for (uint32_t k = 0; k < ORC_POISSON_KMAX; ++k) if ((uint64_t)u < q->thr[k]) return k;
  return ORC_POISSON_KMAX - 1;
}

int orc_poisson_count(const orc_net* o, uint32_t gid, uint64_t step, uint32_t* k) {
  if (!o->shift || gid >= o->N || o->pois_of[gid] < 0) return -1;
  *k = poisson_draw(o, &o->pois[o->pois_of[gid]], gid, step);
  return 0;
}

int orc_record_input(orc_net* o, int64_t* buf, uint64_t max_steps) {
  o->rec = buf; o->rec_max = max_steps;
  return 0;
}

static void deliver_into(const orc_net* o, uint64_t target_step, uint64_t n_spk, const uint64_t* st,
                         const uint32_t* gid, const uint32_t* mult, int64_t* out) {
  uint32_t D1 = o->dmax + 1, P = o->P;
  for (uint32_t d = 1; d <= o->dmax; ++d) {
    if (target_step < d) break;
    uint64_t nf = target_step - d;
    for (uint64_t i = 0; i < n_spk; ++i) {
      if (st[i] != nf) continue;
      uint32_t s = gid[i];
      int64_t m = (int64_t)mult[i];
      uint64_t b = o->off[(size_t)s * D1 + d], e = o->off[(size_t)s * D1 + d + 1];
      for (uint64_t q = b; q < e; ++q) {
        const orc_syn* sy = &o->syn[q];
        out[(size_t)sy->tgt * P + sy->port] += m * sy->wq;
      }
    }
  }
}

int orc_replay_input(const orc_net* o, uint64_t n_spk, const uint64_t* step, const uint32_t* gid,
                     const uint32_t* mult, uint64_t target_step, int64_t* out) {
  if (!o->built) return -1;
  memset(out, 0, (size_t)o->N * o->P * sizeof(int64_t));
  deliver_into(o, target_step, n_spk, step, gid, mult, out);
  return 0;
}

/* Sampled checks of networks too large for the synapse table: the synapses
   onto one target, drawn one by one by the rule above (in projection order,
   then draw index), and the delivered input of sampled targets by the
   definition -- for each synapse (s, d, port, w_q) onto t, the multiplicity
   of the spike of s at step target_step - d times w_q -- from a spike list
   sorted by (step, gid). */
int64_t orc_target_synapses(orc_net* o, uint32_t t, uint64_t cap, uint32_t* src, uint32_t* d, uint32_t* port,
                            int64_t* wq) {
  if (prepare(o) != 0 || t >= o->N) return -1;
  uint64_t n = 0;
  for (uint32_t p = 0; p < o->n_proj; ++p) {
    const orc_proj* pr = &o->proj[p];
    if (t < pr->tgt_first || t - pr->tgt_first >= pr->tgt_n || proj_synapses(pr) == 0) continue;
    if (pr->rule == ORC_RULE_FIXED_OUTDEGREE || pr->rule == ORC_RULE_FIXED_TOTAL_NUMBER || pr->rule == ORC_RULE_LIST) {
      set_err(o, "the rule does not draw per target"); return -1;
    }
    uint64_t blk[4] = {0, 0, 0, 0}, wblk[4] = {0, 0, 0, 0};
    for (uint32_t k = 0; k < pr->K; ++k, ++n) {
      uint32_t s, tt, dd;
      draw_synapse(o, p, t, k, blk, &s, &tt, &dd);
      int64_t w = synapse_wq(o, p, t, k, t, wblk);
      if (n < cap) { src[n] = s; d[n] = dd; port[n] = pr->port; wq[n] = w; }
    }
  }
  return (int64_t)n;
}

static uint32_t spike_mult(uint64_t n_spk, const uint64_t* st, const uint32_t* gid, const uint32_t* mult,
                           uint64_t step, uint32_t g) {
  uint64_t lo = 0, hi = n_spk;  /* first entry >= (step, g) */
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (st[mid] < step || (st[mid] == step && gid[mid] < g)) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n_spk && st[lo] == step && gid[lo] == g) ? mult[lo] : 0;
}

int orc_sampled_input(orc_net* o, uint32_t nt, const uint32_t* tgt, uint64_t n_spk, const uint64_t* step,
                      const uint32_t* gid, const uint32_t* mult, uint64_t target_step, int64_t* out) {
  if (prepare(o) != 0) return -1;
  for (uint64_t i = 1; i < n_spk; ++i)
    if (step[i] < step[i - 1] || (step[i] == step[i - 1] && gid[i] <= gid[i - 1])) {
      set_err(o, "spikes not sorted by (step, gid)"); return -1;
    }
  uint32_t P = o->P;
  for (uint32_t j = 0; j < nt; ++j) {
    uint32_t t = tgt[j];
    if (t >= o->N) { set_err(o, "target out of range"); return -1; }
    for (uint32_t q = 0; q < P; ++q) out[(size_t)j * P + q] = 0;
    for (uint32_t p = 0; p < o->n_proj; ++p) {
      const orc_proj* pr = &o->proj[p];
      if (t < pr->tgt_first || t - pr->tgt_first >= pr->tgt_n || proj_synapses(pr) == 0) continue;
      if (pr->rule == ORC_RULE_FIXED_OUTDEGREE || pr->rule == ORC_RULE_FIXED_TOTAL_NUMBER ||
          pr->rule == ORC_RULE_LIST) {
        set_err(o, "the rule does not draw per target"); return -1;
      }
      uint64_t blk[4] = {0, 0, 0, 0}, wblk[4] = {0, 0, 0, 0};
      for (uint32_t k = 0; k < pr->K; ++k) {
        uint32_t s, tt, d;
        draw_synapse(o, p, t, k, blk, &s, &tt, &d);
        int64_t w = synapse_wq(o, p, t, k, t, wblk);
        if (target_step < d) continue;
        out[(size_t)j * P + pr->port] += (int64_t)spike_mult(n_spk, step, gid, mult, target_step - d, s) * w;
      }
    }
  }
  return 0;
}

/* Update of neuron i at step n; returns its spike multiplicity.  The
   accepted and rejected RK45 substeps are added to *ra and *rr. */
static int update_neuron(orc_net* o, uint64_t n, uint32_t i, uint64_t* ra, uint64_t* rr) {
  uint32_t P = o->P;
  int f32 = (o->mode == ORC_FP32SO);
  double xd[ORC_MAX_PORTS]; float xf[ORC_MAX_PORTS];
  uint32_t pk = o->pop_of[i];
  const orc_pop_params* pp = neuron_params(o, i, pk);
  int64_t xin[ORC_MAX_PORTS];
  for (uint32_t p = 0; p < P; ++p) { xin[p] = o->acc[(size_t)i * P + p]; o->acc[(size_t)i * P + p] = 0; }
  if (o->pois_of[i] >= 0) {
    const orc_pois* q = &o->pois[o->pois_of[i]];
    int S = o->shift[pk * P + q->port];
    int64_t wq = llrint(ldexp(q->weight, S));
    xin[q->port] += (int64_t)poisson_draw(o, q, i, n) * wq;
  }
  for (uint32_t p = 0; p < pp->n_ports; ++p) {
    int S = o->shift[pk * P + p];
    xd[p] = ldexp((double)xin[p], -S);
    xf[p] = ldexpf((float)xin[p], -S);
  }
  int m = 0;
  if (pp->model == ORC_SPIKE_GENERATOR) {
    /* skip times already passed, then count the ones of this step */
    while (o->gen_pos[i] < o->gen_n[i] && o->gen_steps[i][o->gen_pos[i]] < n) o->gen_pos[i]++;
    while (o->gen_pos[i] < o->gen_n[i] && o->gen_steps[i][o->gen_pos[i]] == n) { o->gen_pos[i]++; m++; }
  } else if (pp->model == ORC_PARROT) {
    /* unit weights: the input is the number of arriving spikes */
    m = xin[0] > 0 ? (int)(xin[0] >> o->shift[pk * P]) : 0;
  } else if (pp->model == ORC_LIF_DELTA) {
    if (f32) m = orc_lif_delta_step32(pp, o->dt, &o->Vf[i], &o->refr[i], o->Ief[i], xf[0]);
    else {
      double y = o->V[i] - pp->E_L;
      m = orc_lif_delta_step64(pp, o->dt, &y, &o->refr[i], o->Ie[i], xd[0]);
      o->V[i] = y + pp->E_L;
    }
  } else if (pp->model == ORC_LIF_EXP) {
    if (f32) m = orc_lif_exp_step32(pp, o->dt, &o->Vf[i], &o->If[(size_t)i * P], &o->refr[i], o->Ief[i], xf);
    else {
      double y = o->V[i] - pp->E_L;
      m = orc_lif_exp_step64(pp, o->dt, &y, &o->I[(size_t)i * P], &o->refr[i], o->Ie[i], xd);
      o->V[i] = y + pp->E_L;
    }
  } else {
    double yv[2 + 2 * ORC_MAX_PORTS];
    uint32_t np = pp->n_ports;
    yv[0] = o->V[i]; yv[1] = o->w[i];
    for (uint32_t p = 0; p < np; ++p) yv[2 + p] = o->g[(size_t)i * P + p];
    for (uint32_t p = 0; p < np; ++p) yv[2 + np + p] = o->gr[(size_t)i * P + p];
    m = orc_adex_step(pp, o->dt, yv, &o->h[i], o->Ie[i], xd, ra, rr);
    o->V[i] = yv[0]; o->w[i] = yv[1];
    for (uint32_t p = 0; p < np; ++p) o->g[(size_t)i * P + p] = yv[2 + p];
    if (pp->model == ORC_AEIF_COND_BETA)
      for (uint32_t p = 0; p < np; ++p) o->gr[(size_t)i * P + p] = yv[2 + np + p];
  }
  return m;
}

/* Nearest-neighbour STDP (Sec. 2.1, after Morrison et al. 2008), with the
   power-law weight dependence of Guetig et al. (2003) in fixed point.  A
   synapse's spikes are its pre arrivals (step a: the update of step a
   receives the spike) and its target's spikes (step k: emitted in the
   update of step k); in one step the arrival comes first.  Pairs are
   nearest neighbours: each post spike at k pairs with the synapse's latest
   arrival a <= k (potentiation, time difference (k - a) dt), each arrival
   at a with the target's latest spike k < a (depression, (a - k) dt).  With
   W = w_max in the weight's fixed-point units and
     F+(d) = round(lambda e^{-d dt / tau_plus} 2^32),
     F-(d) = round(alpha lambda e^{-d dt / tau_minus} 2^32),
   potentiation is w += floor(B+ F+ / 2^32), B+ = W (mu_plus = 0, additive)
   or W - w (mu_plus = 1, multiplicative), then w = min(w, W); depression is
   w -= floor(B- F- / 2^32), B- = W (mu_minus = 0) or w (mu_minus = 1), then
   w = max(w, 0).  A spike of multiplicity m pairs m times.  Step n: the
   input of step n + 1 is delivered with the weights as they are, then the
   post spikes of step n potentiate, then the arrivals of step n + 1 depress
   (and become the synapses' latest arrivals). */
static int64_t stdp_fraction(double scale, double tau, double dt, uint64_t d) {
  return llrint(ldexp(scale * exp(-((double)d * dt) / tau), 32));
}

static void stdp_step(orc_net* o, uint64_t n) {
  for (uint64_t q = o->spk_at[n]; q < o->spk_at[n + 1]; ++q) {
    uint32_t t = o->spk_gid[q], m = o->spk_mult[q];
    for (uint64_t k = o->tptr[t]; k < o->tptr[t + 1]; ++k) {
      uint64_t j = o->tidx[k];
      if (o->last_pre[j] < 0) continue;
      const orc_proj* pr = &o->proj[o->syn[j].plast];
      int64_t F = stdp_fraction(pr->lambda, pr->tau_plus, o->dt, n - (uint64_t)o->last_pre[j]);
      for (uint32_t c = 0; c < m; ++c) {
        int64_t B = pr->mu_plus ? o->pwmax[j] - o->pw[j] : o->pwmax[j];
        o->pw[j] += (B * F) >> 32;
        if (o->pw[j] > o->pwmax[j]) o->pw[j] = o->pwmax[j];
      }
    }
    o->last_post[t] = (int64_t)n;
  }
  for (uint64_t j = 0; j < o->n_syn; ++j) {
    if (!o->arr_m[j]) continue;
    const orc_proj* pr = &o->proj[o->syn[j].plast];
    int64_t k = o->last_post[o->syn[j].tgt];
    if (k >= 0) {
      int64_t F = stdp_fraction(pr->alpha * pr->lambda, pr->tau_minus, o->dt, n + 1 - (uint64_t)k);
      for (uint32_t c = 0; c < o->arr_m[j]; ++c) {
        int64_t B = pr->mu_minus ? o->pw[j] : o->pwmax[j];
        o->pw[j] -= (B * F) >> 32;
        if (o->pw[j] < 0) o->pw[j] = 0;
      }
    }
    o->last_pre[j] = (int64_t)(n + 1);
    o->arr_m[j] = 0;
  }
}

/* The neuron loop and the delivery loop carry OpenMP pragmas, which a plain
   build ignores: the neurons of a step are independent (their spikes are
   recorded afterwards, in gid order) and the delivered sums are integers
   added atomically, so a build with OpenMP gives the same results. */
int orc_simulate(orc_net* o, uint64_t steps) {
  if (!o->built) { set_err(o, "simulate before build"); return -1; }
  uint32_t P = o->P, D1 = o->dmax + 1;
  for (uint64_t it = 0; it < steps; ++it) {
    uint64_t n = o->step;
    if (o->rec && n < o->rec_max) memcpy(o->rec + (size_t)n * o->N * P, o->acc, (size_t)o->N * P * sizeof(int64_t));
    if (n + 1 >= o->cap_at) {
      o->cap_at *= 2;
      o->spk_at = (uint64_t*)realloc(o->spk_at, o->cap_at * sizeof(uint64_t));
    }
    o->spk_at[n] = o->n_spk;
    /* update of step n */
    uint64_t ra = 0, rr = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : ra, rr)
    for (int64_t i = 0; i < (int64_t)o->N; ++i) o->mult_now[i] = (uint32_t)update_neuron(o, n, (uint32_t)i, &ra, &rr);
    o->rk_acc += ra; o->rk_rej += rr;
    for (uint32_t i = 0; i < o->N; ++i)
      if (o->mult_now[i] > 0) record_spike(o, n, i, o->mult_now[i]);
    o->spk_at[n + 1] = o->n_spk;
    /* delivery: input of step n+1 */
    uint64_t ev = 0;
    int64_t dtop = (int64_t)(o->dmax < n + 1 ? o->dmax : n + 1);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ev)
    for (int64_t d = 1; d <= dtop; ++d) {
      uint64_t nf = n + 1 - (uint64_t)d;
      for (uint64_t q = o->spk_at[nf]; q < o->spk_at[nf + 1]; ++q) {
        uint32_t s = o->spk_gid[q];
        int64_t m = (int64_t)o->spk_mult[q];
        uint64_t b = o->off[(size_t)s * D1 + d], e = o->off[(size_t)s * D1 + d + 1];
        ev += e - b;
        for (uint64_t r = b; r < e; ++r) {
          const orc_syn* sy = &o->syn[r];
          int64_t w = sy->plast >= 0 ? o->pw[r] : sy->wq;
#pragma omp atomic
          o->acc[(size_t)sy->tgt * P + sy->port] += m * w;
          if (sy->plast >= 0) o->arr_m[r] = (uint32_t)m;  /* one source spike per step: one arrival */
        }
      }
    }
    o->n_events += ev;
    if (o->n_plastic) stdp_step(o, n);
    o->step = n + 1;
  }
  return 0;
}

/* Threads the simulation loops run on (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

uint64_t orc_current_step(const orc_net* o) { return o->step; }
uint64_t orc_n_events(const orc_net* o) { return o->n_events; }
uint64_t orc_n_spikes(const orc_net* o) { return o->n_spk; }

void orc_get_spikes(const orc_net* o, uint64_t* step, uint32_t* gid, uint32_t* mult) {
  /* spikes are appended in (step, gid) order by construction */
  for (uint64_t i = 0; i < o->n_spk; ++i) { step[i] = o->spk_step[i]; gid[i] = o->spk_gid[i]; mult[i] = o->spk_mult[i]; }
}

uint64_t orc_n_synapses(const orc_net* o) { return o->built ? o->n_syn : 0; }

void orc_get_synapses(const orc_net* o, uint32_t* src, uint32_t* delay, uint32_t* tgt, uint32_t* port, int64_t* wq) {
  for (uint64_t e = 0; e < o->n_syn; ++e) {
    src[e] = o->syn[e].src; delay[e] = o->syn[e].d; tgt[e] = o->syn[e].tgt;
    port[e] = o->syn[e].port; wq[e] = o->syn[e].plast >= 0 ? o->pw[e] : o->syn[e].wq;
  }
}

int orc_shift_of(const orc_net* o, uint32_t gid, uint32_t port) {
  if (!o->shift || gid >= o->N || port >= o->P) return -1000;
  return o->shift[o->pop_of[gid] * o->P + port];
}
