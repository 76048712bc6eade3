/*
 * sanitize_driver.c -- runs the oracle's C API through its main paths so that
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer can check the
 * oracle's memory handling (TEST INFRASTRUCTURE ONLY, like the oracle).
 *
 * Networks: a LIF-delta Brunel network with Poisson drive and normal delays;
 * exponential-PSC LIF neurons with per-neuron and drawn parameters, drawn
 * weights and a plastic projection; AdEx neurons with exponential and beta
 * ports; spike generators into parrots through a user-defined list with
 * per-connection weights; every connection rule.  Each is built, simulated,
 * read back (spikes, state, synapses, recorded and replayed input, sampled
 * synapses) and destroyed.  Exit status 0 when every call succeeded.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "snn_oracle.h"

#define CHECK(x)                                                                   \
  do {                                                                             \
    if (!(x)) {                                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #x);              \
      return 1;                                                                    \
    }                                                                              \
  } while (0)

static orc_pop_params lif(int model, double tau_syn) {
  orc_pop_params p;
  memset(&p, 0, sizeof p);
  p.model = model; p.n_ports = 1;
  p.tau_m = 20.0; p.C_m = 250.0; p.E_L = 0.0; p.V_th = 20.0; p.V_reset = 10.0; p.t_ref = 2.0;
  p.tau_syn[0] = tau_syn; p.rk_eps = 1e-6; p.rk_hmin = 1e-8;
  return p;
}

static orc_pop_params adex(int model) {
  orc_pop_params p;
  memset(&p, 0, sizeof p);
  p.model = model; p.n_ports = 2;
  p.C_m = 281.0; p.g_L = 30.0; p.E_L = -70.6; p.V_T = -50.4; p.Delta_T = 2.0; p.tau_w = 144.0;
  p.a = 4.0; p.b = 80.5; p.V_r = -60.0; p.V_peak = 0.0;
  p.tau_syn[0] = 1.0; p.tau_syn[1] = 2.0; p.E_rev[0] = 0.0; p.E_rev[1] = -85.0;
  p.tau_rise[0] = 0.5; p.tau_rise[1] = 1.0; p.rk_eps = 1e-6; p.rk_hmin = 1e-8;
  return p;
}

/* read everything back, then destroy */
static int drain(orc_net* o, uint64_t steps) {
  uint64_t ns = orc_n_spikes(o);
  uint64_t* st = malloc((ns + 1) * sizeof *st);
  uint32_t* gid = malloc((ns + 1) * sizeof *gid);
  uint32_t* mult = malloc((ns + 1) * sizeof *mult);
  orc_get_spikes(o, st, gid, mult);
  uint64_t nsyn = orc_n_synapses(o);
  uint32_t* a = malloc((nsyn + 1) * 4);
  uint32_t* b = malloc((nsyn + 1) * 4);
  uint32_t* c = malloc((nsyn + 1) * 4);
  uint32_t* d = malloc((nsyn + 1) * 4);
  int64_t* w = malloc((nsyn + 1) * 8);
  orc_get_synapses(o, a, b, c, d, w);
  double v[64];
  CHECK(orc_get_state(o, 0, 16, 0, 0, v) == 0);
  int64_t out[4096];
  CHECK(orc_replay_input(o, ns, st, gid, mult, steps, out) == 0);
  free(st); free(gid); free(mult); free(a); free(b); free(c); free(d); free(w);
  orc_destroy(o);
  return 0;
}

int main(void) {
  /* 1: Brunel LIF-delta, Poisson drive, normal delays, recorded input */
  {
    orc_net* o = orc_create(0.1, 7, 30, ORC_FP32SO);
    CHECK(o);
    orc_pop_params p = lif(ORC_LIF_DELTA, 0.0);
    int64_t e = orc_population(o, 400, &p), i = orc_population(o, 100, &p);
    CHECK(e == 0 && i == 400);
    CHECK(orc_connect_fixed_indegree(o, 0, 400, 0, 500, 40, 0.1, ORC_DELAY_NORMAL_CLIPPED, 1.5, 0.75, 0) == 0);
    CHECK(orc_connect_fixed_indegree(o, 400, 100, 0, 500, 10, -0.5, ORC_DELAY_UNIFORM, 0.1, 2.0, 0) == 0);
    CHECK(orc_poisson(o, 0, 500, 250.0, 80, 0.1, 0) == 0);
    double v0[500];
    for (int k = 0; k < 500; ++k) v0[k] = 0.04 * k;
    CHECK(orc_set_state(o, 0, 500, 0, 0, v0) == 0);
    CHECK(orc_build(o) == 0);
    int64_t* rec = malloc((size_t)201 * 500 * sizeof(int64_t));
    CHECK(orc_record_input(o, rec, 201) == 0);
    CHECK(orc_simulate(o, 200) == 0);
    CHECK(orc_n_spikes(o) > 0);
    uint32_t t[3] = {0, 17, 499}, k = 0;
    uint32_t src[256], del[256], port[256];
    int64_t wq[256];
    CHECK(orc_target_synapses(o, 17, 256, src, del, port, wq) == 50);
    CHECK(orc_poisson_count(o, 3, 5, &k) == 0);
    (void)t;
    if (drain(o, 200)) return 1;
    free(rec);
  }
  /* 2: exponential-PSC LIF, per-neuron and drawn parameters, drawn weights, STDP */
  {
    orc_net* o = orc_create(0.1, 11, 20, ORC_FP64);
    CHECK(o);
    orc_pop_params p = lif(ORC_LIF_EXP, 0.5);
    p.E_L = -65.0; p.V_th = -50.0; p.V_reset = -65.0; p.tau_m = 10.0;
    CHECK(orc_population(o, 300, &p) == 0);
    double tau[300];
    for (int k = 0; k < 300; ++k) tau[k] = 8.0 + 0.01 * k;
    CHECK(orc_set_param(o, 0, 300, 0, tau) == 0);
    CHECK(orc_param_distribution(o, 0, 300, 3, ORC_WEIGHT_NORMAL, -50.0, 1.0, -54.0, -46.0, 256) == 0);
    CHECK(orc_connect(o, ORC_RULE_FIXED_INDEGREE, 30, 0, 300, 0, 300, 80.0, ORC_DELAY_UNIFORM, 0.2, 1.5, 0) == 0);
    CHECK(orc_weight_distribution(o, 0, ORC_WEIGHT_UNIFORM, 60.0, 100.0, 0.0, 0.0, 32) == 0);
    CHECK(orc_stdp(o, 0, 15.0, 30.0, 0.05, 0.9, 1, 1, 200.0) == 0);
    CHECK(orc_poisson(o, 0, 300, 8.0, 3500, 87.8, 0) == 0);
    CHECK(orc_state_distribution(o, 0, 300, 0, 0, ORC_WEIGHT_UNIFORM, -65.0, -50.0, 0.0, 0.0, 1024) == 0);
    CHECK(orc_build(o) == 0);
    CHECK(orc_simulate(o, 300) == 0);
    if (drain(o, 300)) return 1;
  }
  /* 3: AdEx, exponential and beta ports, every connection rule */
  {
    orc_net* o = orc_create(0.1, 3, 25, ORC_FP64);
    CHECK(o);
    orc_pop_params pe = adex(ORC_AEIF_COND_EXP), pb = adex(ORC_AEIF_COND_BETA);
    CHECK(orc_population(o, 60, &pe) == 0);
    CHECK(orc_population(o, 40, &pb) == 60);
    CHECK(orc_connect(o, ORC_RULE_FIXED_OUTDEGREE, 10, 0, 60, 0, 100, 0.3, ORC_DELAY_UNIFORM, 1.0, 2.0, 0) == 0);
    CHECK(orc_connect(o, ORC_RULE_ALL_TO_ALL, 0, 60, 40, 60, 40, 0.2, ORC_DELAY_CONST, 0.5, 0.0, 1) == 0);
    CHECK(orc_connect(o, ORC_RULE_ONE_TO_ONE, 0, 0, 40, 60, 40, 0.5, ORC_DELAY_CONST, 0.3, 0.0, 0) == 0);
    CHECK(orc_connect(o, ORC_RULE_FIXED_TOTAL_NUMBER, 500, 0, 100, 0, 100, 0.1, ORC_DELAY_NORMAL_CLIPPED, 1.0,
                      0.5, 1) == 0);
    CHECK(orc_poisson(o, 0, 100, 20000.0, 1, 1.0, 0) == 0);
    double ie[100];
    for (int k = 0; k < 100; ++k) ie[k] = 2.0 * k;
    CHECK(orc_set_state(o, 0, 100, 1, 0, ie) == 0);
    CHECK(orc_build(o) == 0);
    CHECK(orc_simulate(o, 150) == 0);
    if (drain(o, 150)) return 1;
  }
  /* 4: spike generators into parrots through a weighted list */
  {
    orc_net* o = orc_create(0.1, 5, 8, ORC_FP32SO);
    CHECK(o);
    orc_pop_params g = lif(ORC_SPIKE_GENERATOR, 0.0), q = lif(ORC_PARROT, 0.0), l = lif(ORC_LIF_DELTA, 0.0);
    CHECK(orc_population(o, 4, &g) == 0);
    CHECK(orc_population(o, 4, &q) == 4);
    CHECK(orc_population(o, 8, &l) == 8);
    double times[3] = {0.5, 1.2, 1.2};
    for (uint32_t k = 0; k < 4; ++k) CHECK(orc_set_spike_times(o, k, 3, times) == 0);
    uint32_t src[8] = {0, 1, 2, 3, 4, 5, 6, 7}, tgt[8] = {4, 5, 6, 7, 8, 9, 10, 11};
    double dl[8] = {0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8};
    double wl[8] = {1, 1, 1, 1, 5.0, 6.0, 5.0, 7.0};
    CHECK(orc_connect_list(o, 4, src, tgt, dl, 1.0, 0) == 0);
    CHECK(orc_connect_list(o, 4, src + 4, tgt + 4, dl + 4, 0.0, 0) == 0);
    CHECK(orc_list_weights(o, 1, 4, wl + 4) == 0);
    CHECK(orc_build(o) == 0);
    CHECK(orc_simulate(o, 40) == 0);
    if (drain(o, 40)) return 1;
  }
  /* 5: refused calls leave the handle valid */
  {
    orc_net* o = orc_create(0.1, 1, 4, ORC_FP64);
    CHECK(o);
    orc_pop_params p = lif(ORC_LIF_DELTA, 0.0);
    CHECK(orc_population(o, 10, &p) == 0);
    CHECK(orc_connect_fixed_indegree(o, 0, 10, 5, 10, 3, 0.1, ORC_DELAY_CONST, 0.1, 0.0, 0) != 0);
    CHECK(orc_stdp(o, 7, 20.0, 20.0, 0.01, 1.0, 1, 1, 1.0) != 0);
    CHECK(orc_last_error(o) != NULL);
    orc_destroy(o);
  }
  printf("sanitized oracle run ok\n");
  return 0;
}
