// snn_api.cpp -- host runtime behind the C ABI of include/snn.h.
//
// Owns the network description, the host-side tables the kernels read
// (propagators, fixed-point exponents, weight classes, delay and Poisson
// thresholds), device memory, the build sequence and the step loop (hipGraph
// of K one-kernel steps plus a raster tail, replayed; the spike
// ring is drained to the host raster between replays).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/snn.h"
#include "kernels.h"
#include "snn_types.h"

using namespace snn;

namespace {

constexpr uint32_t kGraphSteps = 100;
constexpr int kNumParams = 16;  // SNN_P_TAU_M .. SNN_P_RK_HMIN
constexpr uint64_t kChunkRing = 4096;  // >= drain interval + graph length
constexpr uint64_t kBinnedMinSynapses = 500000000;  // default delivery: binned from this size on
constexpr uint64_t kRunMinMean = 4;  // tile runs when groups average this many synapses per touched tile
constexpr uint64_t kQueueMinInstances = 8;          // binned batches with at least this many instances ...
constexpr uint64_t kQueueMaxTilesPerInstance = 32;  // ... of at most this many tiles each use the delivery queue

struct HostPop {
  int32_t model = 0;
  uint32_t n = 0, ports = 1, first = 0;
  uint32_t inst = 0;
  double tau_m = 10.0, C_m = 250.0, E_L = -70.0, V_th = -55.0, V_reset = -70.0, t_ref = 2.0;
  double g_L = 30.0, Delta_T = 2.0, V_T = -50.4, tau_w = 144.0, a = 4.0, b = 80.5, V_peak = 0.0, V_r = -60.0;
  double rk_eps = 1e-6, rk_hmin = 1e-8;
  double tau_syn[kMaxPorts] = {2.0, 2.0, 2.0, 2.0};
  double E_rev[kMaxPorts] = {0.0, -85.0, 0.0, 0.0};
  double tau_rise[kMaxPorts] = {1.0, 1.0, 1.0, 1.0};
  bool adex() const { return model == SNN_AEIF_COND_EXP || model == SNN_AEIF_COND_BETA; }
  // model parameter SNN_P_* by id (nullptr for an unknown id)
  double* param(int32_t id) {
    switch (id) {
      case SNN_P_TAU_M: return &tau_m;
      case SNN_P_C_M: return &C_m;
      case SNN_P_E_L: return &E_L;
      case SNN_P_V_TH: return &V_th;
      case SNN_P_V_RESET: return &V_reset;
      case SNN_P_T_REF: return &t_ref;
      case SNN_P_G_L: return &g_L;
      case SNN_P_DELTA_T: return &Delta_T;
      case SNN_P_V_T: return &V_T;
      case SNN_P_TAU_W: return &tau_w;
      case SNN_P_A: return &a;
      case SNN_P_B: return &b;
      case SNN_P_V_PEAK: return &V_peak;
      case SNN_P_V_R: return &V_r;
      case SNN_P_RK_EPS: return &rk_eps;
      case SNN_P_RK_HMIN: return &rk_hmin;
      default: return nullptr;
    }
  }
  const double* param(int32_t id) const { return const_cast<HostPop*>(this)->param(id); }
};

struct HostProj {
  uint32_t src_first, src_n, tgt_first, tgt_n;
  uint32_t K;      // draws per entity: in-degree, out-degree, n_src (all-to-all), 1 (one-to-one, total)
  uint32_t port;
  uint32_t inst, local;  // instance and creation index within it
  double weight;
  int32_t kind;
  double da, db;
  int32_t rule = SNN_RULE_FIXED_INDEGREE;
  uint64_t n = 0;  // the rule's count (fixed total number, list: synapses)
  std::vector<uint32_t> lsrc, ltgt;  // user-defined list (rule kRuleList)
  std::vector<uint8_t> ldel;
  // weight levels (empty: the single weight): values, draw thresholds
  // (distributions) or the level of every listed synapse (lists)
  std::vector<double> wlev;
  std::vector<uint64_t> wthr;
  std::vector<uint16_t> lwl;
  // nearest-neighbour STDP (snn_stdp)
  bool plastic = false;
  int32_t mu_plus = 1, mu_minus = 1;
  double tau_plus = 20.0, tau_minus = 20.0, lambda = 0.01, alpha = 1.0, w_max = 100.0;
  double wmin() const { return wlev.empty() ? weight : wlev.front(); }
  double wmax_abs() const {
    return wlev.empty() ? fabs(weight) : std::max(fabs(wlev.front()), fabs(wlev.back()));
  }
  // synapses the projection makes
  uint64_t synapses() const {
    switch (rule) {
      case SNN_RULE_FIXED_OUTDEGREE: return tgt_n ? (uint64_t)K * src_n : 0;
      case SNN_RULE_FIXED_TOTAL_NUMBER:
      case kRuleList: return tgt_n ? n : 0;
      default: return (uint64_t)K * tgt_n;
    }
  }
  // work-item entities: sources (out-degree), synapses (total) or targets
  uint64_t entities() const {
    return rule == SNN_RULE_FIXED_OUTDEGREE ? src_n : (rule == SNN_RULE_FIXED_TOTAL_NUMBER || rule == kRuleList) ? n
                                                                                                       : tgt_n;
  }
  // synapses onto a target: exact for the rules drawn per target, the mean otherwise
  double per_target() const {
    if (rule == SNN_RULE_FIXED_OUTDEGREE) return tgt_n ? (double)K * src_n / tgt_n : 0.0;
    if (rule == SNN_RULE_FIXED_TOTAL_NUMBER || rule == kRuleList) return tgt_n ? (double)n / tgt_n : 0.0;
    return (double)K;
  }
};

struct HostPois {
  uint32_t tgt_first, tgt_n, n_inputs, port;
  double rate, weight;
};

// An independent network inside this one (a batch member): randomness keyed
// by its own seed, gids and projection indices counted from its own start.
struct Inst {
  uint64_t seed;
  uint32_t first_gid;
  uint32_t n_proj;
};

struct DevAlloc {
  void* p;
  size_t bytes;
};

// ---------------------------------------------------------------- tables
// Delay d (ms) -> steps: d/dt rounded half up, at least 1, at most Dmax, so
// P(D <= k) = F((k + 1/2) dt) below Dmax; a 32-bit uniform u selects
// D = min{k : u < floor(2^32 P(D <= k))}.
double delay_cdf_at(int32_t kind, double a, double b, double x) {
  switch (kind) {
    case SNN_DELAY_CONST: return (x >= a) ? 1.0 : 0.0;
    case SNN_DELAY_UNIFORM: {
      const double f = (x - a) / (b - a);
      return f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    }
    default: return 0.5 * erfc(-(x - a) / (b * sqrt(2.0)));
  }
}

uint64_t threshold_of(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return 1ull << 32;
  const double t = floor(ldexp(p, 32));
  return (t >= 4294967296.0) ? (1ull << 32) : (uint64_t)t;
}

void delay_thresholds(int32_t kind, double a, double b, double dt, uint32_t dmax, uint64_t* thr) {
  for (uint32_t k = 0; k < 64; ++k) thr[k] = 1ull << 32;
  thr[0] = 0;
  if (kind == SNN_DELAY_CONST) {
    const double q = floor(a / dt + 0.5);
    const uint32_t d0 = q < 1.0 ? 1u : (q > (double)dmax ? dmax : (uint32_t)q);
    for (uint32_t k = 1; k <= dmax; ++k) thr[k] = (k >= d0) ? (1ull << 32) : 0;
    return;
  }
  for (uint32_t k = 1; k < dmax; ++k) thr[k] = threshold_of(delay_cdf_at(kind, a, b, ((double)k + 0.5) * dt));
  thr[dmax] = 1ull << 32;
}

// Poisson(lambda) cumulative thresholds (tail folded into the last entry).
void poisson_thresholds(double lambda, uint64_t* thr) {
  double p = exp(-lambda), c = p;
  for (int k = 0; k + 1 < kPoisKmax; ++k) {
    if (k > 0) {
      p = p * lambda / (double)k;
      c = c + p;
    }
    thr[k] = threshold_of(c);
  }
  thr[kPoisKmax - 1] = 1ull << 32;
}

// Largest S with max_w * 2^S < 2^30.
int fixed_shift(double max_w) {
  if (!(max_w > 0)) return 0;
  int e;
  (void)frexp(max_w, &e);
  return 30 - e;
}

}  // namespace

struct snn_net {
  snn_config cfg{};
  snn_device dev{};
  bool have_dev = false;
  hipStream_t stream = nullptr;
  int device = 0;  // the device current at creation: the stream's and every allocation's
  hipEvent_t ev_user = nullptr;
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;  // timing: first and last launch of a simulate call
  double last_dev_ms = 0.0;                      // device time between them in the last call
  std::string err;
  bool built = false;

  std::vector<Inst> insts;
  std::vector<HostPop> pops;
  std::vector<HostProj> projs;
  std::vector<HostPois> pois;
  std::map<uint32_t, std::vector<uint64_t>> gen_steps;  // spike generator gid -> emission steps, ascending
  // multimeters: channel c = one variable of one neuron; the device keeps the
  // last kGraphSteps steps of every channel, the host the due samples
  struct Meter {
    int32_t var;
    uint32_t port, interval, ch0;
    std::vector<uint32_t> gids;
    std::vector<uint64_t> steps;
    std::vector<double> values;  // [sample][gid]
  };
  std::vector<Meter> meters;
  const float** d_addr = nullptr;
  float* d_mbuf = nullptr;
  uint32_t nch = 0;
  std::vector<float> h_mbuf;
  uint32_t N = 0;
  // host state before build (per port arrays are [N][kMaxPorts])
  std::vector<double> V, Ie, w, h;
  // per-neuron model parameters: pn[param] is empty while every neuron takes
  // its population's value, else one value per neuron
  std::vector<double> pn[kNumParams];
  std::vector<double> g, gr, Isyn;
  std::vector<int32_t> refr;

  // after build
  uint32_t P = 1;
  uint32_t dmax_used = 1;
  std::vector<int> shift;          // [npop][P]
  std::vector<int64_t> cls_wq;     // classes sorted by (port, w_q, STDP rule)
  std::vector<uint32_t> cls_port;
  std::vector<uint8_t> cls_rule;   // 0 static, r + 1 plastic under STDP rule r
  uint32_t cls_bits = 6;
  bool has_lif = false, has_adex = false, has_beta = false;
  NetDev nd{};
  std::vector<DevAlloc> allocs;
  size_t dev_bytes = 0;
  uint64_t n_syn = 0, n_groups = 0;
  uint64_t cur_step = 0, drained_step = 0;
  uint64_t log_cap = 0;
  uint64_t drain_steps = 0;
  // captured step loops: kGraphSteps steps and every power of two below it,
  // so that any step count is a few graph launches
  std::vector<std::pair<uint32_t, hipGraphExec_t>> graphs;  // descending length
  Ctrl* pin_ctrl = nullptr;     // pinned copy of the device flags, read at the end of a call
  // raster drain, pipelined: the per-step counts and then the ring segment of
  // a window of steps are copied to pinned memory behind the graphs, each
  // collected one graph later, so the device never waits for the host
  struct Drain {
    int stage = 0;              // 0 idle, 1 counts copy in flight, 2 ring copy in flight
    uint64_t a = 0, b = 0;      // window [a, b) of steps
    uint64_t total = 0;         // entries of the window
    std::vector<uint64_t> base; // ring position of each step of the window, then the end
  } dj;
  hipEvent_t ev_drain = nullptr;
  uint64_t* pin_cb = nullptr;   // [kChunkRing] copy of the per-step ring positions
  uint32_t* pin_rc = nullptr;   // [R] copy of the per-step spike counts
  uint32_t* pinned = nullptr;   // staging of a window's ring entries
  size_t pinned_words = 0;
  uint32_t tile_neurons = 0;       // binned delivery (0: direct)

  // host raster
  // host raster: drained entries (gid | mult << 27) with their step, in step
  // order; within a step sorted by gid from index r_sorted on only when read
  std::vector<uint64_t> r_step;
  std::vector<uint32_t> r_entry;
  size_t r_sorted = 0;

  double build_ms = 0.0, sim_ms = 0.0;
  // snn_release: device memory returned, raster and counters kept on the host
  bool released = false;
  snn_counters final_ctr{};
};

namespace {

// Copies on the library's own stream, waited for: never on the legacy default
// stream, which would have to order itself against every blocking stream of
// the process (and fails while another thread captures a graph).
hipError_t copy_sync(snn_net* net, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, net->stream);
  return e == hipSuccess ? hipStreamSynchronize(net->stream) : e;
}

hipError_t copy2d_sync(snn_net* net, void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                       size_t height, hipMemcpyKind kind) {
  hipError_t e = hipMemcpy2DAsync(dst, dpitch, src, spitch, width, height, kind, net->stream);
  return e == hipSuccess ? hipStreamSynchronize(net->stream) : e;
}

snn_status fail(snn_net* net, snn_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (net) net->err = buf;
  return code;
}

#define HIPCHK(net, expr)                                                                     \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return fail((net), SNN_E_DEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

void* dev_alloc(snn_net* net, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (net->have_dev && net->dev.alloc) {
    p = net->dev.alloc(bytes, net->dev.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    net->allocs.push_back({p, bytes});
    net->dev_bytes += bytes;
  }
  return p;
}

void dev_free(snn_net* net, void* p) {
  if (!p) return;
  for (size_t i = 0; i < net->allocs.size(); ++i) {
    if (net->allocs[i].p == p) {
      net->dev_bytes -= net->allocs[i].bytes;
      net->allocs.erase(net->allocs.begin() + (long)i);
      break;
    }
  }
  if (net->have_dev && net->dev.free) net->dev.free(p, net->dev.user);
  else (void)hipFree(p);
}

template <typename T>
T* dalloc(snn_net* net, size_t count) {
  return static_cast<T*>(dev_alloc(net, count * sizeof(T)));
}

int pop_of(const snn_net* net, uint32_t gid) {
  for (size_t k = 0; k < net->pops.size(); ++k)
    if (gid >= net->pops[k].first && gid < net->pops[k].first + net->pops[k].n) return (int)k;
  return -1;
}

// populations exactly covering [first, first+n), or empty if the range is not a union of whole populations
std::vector<int> whole_pops(const snn_net* net, uint32_t first, uint32_t n) {
  std::vector<int> out;
  uint64_t cur = first, end = (uint64_t)first + n;
  while (cur < end) {
    int k = pop_of(net, (uint32_t)cur);
    if (k < 0 || net->pops[k].first != cur || net->pops[k].first + net->pops[k].n > end) return {};
    out.push_back(k);
    cur += net->pops[k].n;
  }
  return out;
}

// The parameters neuron i is updated with: its population's, with every
// parameter that is set per neuron replaced by the neuron's own value.
HostPop neuron_params(const snn_net* net, uint32_t i) {
  HostPop p = net->pops[pop_of(net, i)];
  for (int32_t id = 0; id < kNumParams; ++id)
    if (!net->pn[id].empty()) *p.param(id) = net->pn[id][i];
  return p;
}

bool any_per_neuron(const snn_net* net) {
  for (int32_t id = 0; id < kNumParams; ++id)
    if (!net->pn[id].empty()) return true;
  return false;
}

snn_status enter(snn_net* net) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->have_dev && net->dev.stream) {
    HIPCHK(net, hipEventRecord(net->ev_user, (hipStream_t)net->dev.stream));
    HIPCHK(net, hipStreamWaitEvent(net->stream, net->ev_user, 0));
  }
  return SNN_OK;
}

snn_status leave(snn_net* net) {
  if (net->have_dev && net->dev.stream) {
    HIPCHK(net, hipEventRecord(net->ev_user, net->stream));
    HIPCHK(net, hipStreamWaitEvent((hipStream_t)net->dev.stream, net->ev_user, 0));
  }
  return SNN_OK;
}

// Beta-port input scale: a lone input of weight w adds g0 w to r; then
// g(s) = g0 w (e^{-s/td} - e^{-s/tr}) / (1/tr - 1/td), whose maximum, at
// s* = ln(td/tr) / (1/tr - 1/td), must equal w.  Equal time constants give
// the alpha function g0 w s e^{-s/t}, maximal at s = t: g0 = e / t.
double beta_g0(double tr, double td) {
  if (std::fabs(td - tr) <= 1e-12 * td) return std::exp(1.0) / td;
  const double k = 1.0 / tr - 1.0 / td;
  const double s_star = std::log(td / tr) / k;
  return k / (std::exp(-s_star / td) - std::exp(-s_star / tr));
}

void lif_propagators(const HostPop& p, double dt, PopDev& d) {
  const double P22 = exp(-dt / p.tau_m);
  const double P20 = p.tau_m / p.C_m * (1.0 - P22);
  d.P22 = (float)P22;
  d.P20 = (float)P20;
  for (uint32_t q = 0; q < kMaxPorts; ++q) {
    double P11 = 0.0, P21 = 0.0;
    if (q < p.ports) {
      const double ts = p.tau_syn[q];
      if (ts > 0) {
        P11 = exp(-dt / ts);
        // tau_m tau_s / (C (tau_s - tau_m)) (e^{-dt/tau_s} - e^{-dt/tau_m}), rewritten
        // around e^{-dt/tau_m} so that close time constants do not cancel:
        // (dt / C) e^{-dt/tau_m} (e^u - 1) / u with u = dt (1/tau_m - 1/tau_s)
        const double u = dt * (ts - p.tau_m) / (p.tau_m * ts);
        const double ratio = (u == 0.0) ? 1.0 : expm1(u) / u;
        P21 = dt / p.C_m * exp(-dt / p.tau_m) * ratio;
      }
    }
    d.P11[q] = (float)P11;
    d.P21[q] = (float)P21;
  }
  d.theta = (float)(p.V_th - p.E_L);
  d.y_reset = (float)(p.V_reset - p.E_L);
  d.n_ref = (int32_t)floor(p.t_ref / dt + 0.5);
}

uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// device value of state variable `var` for neuron i (and the inverse)
// resting potential of neuron i (its own when E_L is set per neuron)
double rest_of(const snn_net* net, uint32_t i) {
  return net->pn[SNN_P_E_L].empty() ? net->pops[pop_of(net, i)].E_L : net->pn[SNN_P_E_L][i];
}

float to_device_state(const snn_net* net, int var, uint32_t i, double v) {
  const HostPop& pp = net->pops[pop_of(net, i)];
  if (var == SNN_V_M && !pp.adex()) return (float)(v - rest_of(net, i));
  return (float)v;
}

double from_device_state(const snn_net* net, int var, uint32_t i, float v) {
  const HostPop& pp = net->pops[pop_of(net, i)];
  if (var == SNN_V_M && !pp.adex()) return (double)v + rest_of(net, i);
  return (double)v;
}

snn_status drain(snn_net* net);
snn_status drain_start(snn_net* net);
snn_status drain_advance(snn_net* net);
void sort_raster(snn_net* net);
snn_status build_graphs(snn_net* net);
snn_status collect_samples(snn_net* net, uint64_t from, uint64_t to);

// ---- snapshot layout: a header, then the dynamic device arrays in order ----
struct SnapHeader {
  char magic[8];
  uint32_t version, N, P, R;
  uint64_t n_tiles, bins_total, n_syn, n_groups, nblk, sel_grid, cur_step, bytes;
};

// The device arrays that change while simulating, with their sizes.
std::vector<std::pair<void*, size_t>> state_arrays(const snn_net* net) {
  const NetDev& nd = net->nd;
  const size_t N = nd.N, P = nd.P;
  std::vector<std::pair<void*, size_t>> a;
  auto add = [&](const void* p, size_t bytes) {
    if (p && bytes) a.push_back({const_cast<void*>(p), bytes});
  };
  add(nd.V, N * 4); add(nd.Ie, N * 4); add(nd.Isyn, N * P * 4); add(nd.refr, N * 4);
  add(nd.w, N * 4); add(nd.g, N * P * 4); add(nd.gr, N * P * 4); add(nd.h, N * 4);
  add(nd.gen_next, N * 4);
  add(nd.acc, (size_t)kInBuf * N * P * 8);
  if (nd.n_tiles) {
    add(nd.bins, (size_t)kInBuf * nd.bins_total * 4);
    add(nd.bin_cnt, (size_t)kInBuf * nd.n_tiles * 4);
    add(nd.ovf_flag, (size_t)kInBuf * nd.n_tiles * 4);
  }
  add(nd.recent, (size_t)nd.R * N * sizeof(SpikeRec));
  add(nd.ring_cnt, (size_t)nd.R * 4); add(nd.ring_base, (size_t)nd.R * 8);
  add(nd.chunk_base, (size_t)nd.chunk_ring * 8);
  add(nd.ctrl, sizeof(Ctrl));
  add(nd.blk_stats, (size_t)kBlkStats * nd.nblk_upd * 8);
  add(nd.sel_stats, (size_t)2 * nd.sel_grid * 8);
  if (nd.n_rules) {  // plastic weights and the spike books of the plasticity
    add(nd.pw, (size_t)nd.n_syn * 4); add(nd.last_pre, (size_t)nd.n_syn * 4); add(nd.arr_m, (size_t)nd.n_syn);
    add(nd.last_post, N * 4); add(nd.arr_list, (size_t)2 * nd.n_plastic * 8); add(nd.arr_cnt, 8);
  }
  return a;
}

SnapHeader snap_header(const snn_net* net) {
  SnapHeader h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, "SNNSNAP1", 8);
  h.version = 1; h.N = net->nd.N; h.P = net->nd.P; h.R = net->nd.R;
  h.n_tiles = net->nd.n_tiles; h.bins_total = net->nd.bins_total; h.n_syn = net->n_syn; h.n_groups = net->n_groups;
  h.nblk = net->nd.nblk_upd; h.sel_grid = net->nd.sel_grid; h.cur_step = net->cur_step;
  h.bytes = sizeof(SnapHeader);
  for (const auto& x : state_arrays(net)) h.bytes += x.second;
  return h;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

snn_status snn_create_net(const snn_config* cfg, const snn_device* dev, snn_net** out) {
  if (!cfg || !out) return SNN_E_INVALID;
  *out = nullptr;
  if (!(cfg->dt_ms > 0) || cfg->max_delay_steps < 1 || cfg->max_delay_steps > 63) return SNN_E_INVALID;
  if ((cfg->flags & SNN_F_DELIVERY_DIRECT) && (cfg->flags & SNN_F_DELIVERY_BINNED)) return SNN_E_INVALID;
  if (cfg->flags & ~(SNN_F_NO_SPIKE_RECORD | SNN_F_DELIVERY_DIRECT | SNN_F_DELIVERY_BINNED)) return SNN_E_INVALID;
  if (cfg->delivery_blocks > 8192 || cfg->reserved) return SNN_E_INVALID;
  if (cfg->tile_neurons && (cfg->tile_neurons < 256 || cfg->tile_neurons > (uint32_t)kTileAccWords ||
                            (cfg->tile_neurons & (cfg->tile_neurons - 1))))
    return SNN_E_INVALID;
  snn_net* net = new (std::nothrow) snn_net();
  if (!net) return SNN_E_NOMEM;
  net->cfg = *cfg;
  net->insts.push_back({cfg->seed, 0, 0});
  if (dev) {
    net->dev = *dev;
    net->have_dev = true;
    if ((dev->alloc == nullptr) != (dev->free == nullptr)) {
      delete net;
      return SNN_E_INVALID;
    }
  }
  if (hipGetDevice(&net->device) != hipSuccess) {
    delete net;
    return SNN_E_DEVICE;
  }
  {  // set-up of the allocation-free readback: its workspace address on this device, once
    int64_t* ws = nullptr;
    (void)input_workspace(net->device, true, &ws);  // a failure is reported by that entry point
  }
  if (hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&net->ev_user, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&net->ev_t0) != hipSuccess || hipEventCreate(&net->ev_t1) != hipSuccess) {
    delete net;
    return SNN_E_DEVICE;
  }
  *out = net;
  return SNN_OK;
}

void snn_destroy_net(snn_net* net) {
  if (!net) return;
  if (net->stream) (void)hipStreamSynchronize(net->stream);
  for (auto& gx : net->graphs) (void)hipGraphExecDestroy(gx.second);
  while (!net->allocs.empty()) dev_free(net, net->allocs.back().p);
  if (net->pinned) (void)hipHostFree(net->pinned);
  if (net->pin_cb) (void)hipHostFree(net->pin_cb);
  if (net->pin_rc) (void)hipHostFree(net->pin_rc);
  if (net->pin_ctrl) (void)hipHostFree(net->pin_ctrl);
  if (net->ev_drain) (void)hipEventDestroy(net->ev_drain);
  if (net->ev_user) (void)hipEventDestroy(net->ev_user);
  if (net->ev_t0) (void)hipEventDestroy(net->ev_t0);
  if (net->ev_t1) (void)hipEventDestroy(net->ev_t1);
  if (net->stream) (void)hipStreamDestroy(net->stream);
  delete net;
}

const char* snn_last_error(const snn_net* net) { return net ? net->err.c_str() : "null network"; }

snn_status snn_create(snn_net* net, int32_t model, uint32_t n, uint32_t n_ports, uint32_t* first_gid) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "snn_create after snn_build");
  if (model < SNN_LIF_PSC_DELTA || model > SNN_PARROT_NEURON) return fail(net, SNN_E_INVALID, "unknown model %d", model);
  if (n == 0 || n_ports < 1 || n_ports > (uint32_t)kMaxPorts) return fail(net, SNN_E_INVALID, "bad size or port count");
  if (model == SNN_LIF_PSC_DELTA && n_ports != 1) return fail(net, SNN_E_INVALID, "LIF delta has one port");
  if ((model == SNN_SPIKE_GENERATOR || model == SNN_PARROT_NEURON) && n_ports != 1)
    return fail(net, SNN_E_INVALID, "devices have one port");
  if ((uint64_t)net->N + n > kMaxNeurons) return fail(net, SNN_E_UNSUPPORTED, "more than 2^26 neurons");
  HostPop p;
  p.model = model;
  p.n = n;
  p.ports = n_ports;
  p.first = net->N;
  p.inst = (uint32_t)net->insts.size() - 1;
  if (p.adex()) {
    p.C_m = 281.0; p.E_L = -70.6; p.t_ref = 0.0;
    for (int q = 0; q < kMaxPorts; ++q) p.tau_syn[q] = 1.0;
  }
  net->pops.push_back(p);
  net->N += n;
  for (int32_t id = 0; id < kNumParams; ++id)  // parameters set per neuron: the new neurons take p's value
    if (!net->pn[id].empty()) net->pn[id].resize(net->N, *p.param(id));
  net->V.resize(net->N, std::nan(""));
  net->Ie.resize(net->N, 0.0);
  net->w.resize(net->N, 0.0);
  net->h.resize(net->N, net->cfg.dt_ms);
  net->refr.resize(net->N, 0);
  net->g.resize((size_t)net->N * kMaxPorts, 0.0);
  net->gr.resize((size_t)net->N * kMaxPorts, 0.0);
  net->Isyn.resize((size_t)net->N * kMaxPorts, 0.0);
  if (first_gid) *first_gid = p.first;
  return SNN_OK;
}

snn_status snn_begin_instance(snn_net* net, uint64_t seed, uint32_t* instance_id) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "snn_begin_instance after snn_build");
  if (net->insts.back().first_gid == net->N && net->insts.size() > 1)
    return fail(net, SNN_E_STATE, "the current instance has no populations yet");
  if (net->N == 0) {  // no population yet: the first instance takes this seed
    net->insts.back().seed = seed;
  } else {
    net->insts.push_back({seed, net->N, 0});
  }
  if (instance_id) *instance_id = (uint32_t)net->insts.size() - 1;
  return SNN_OK;
}

snn_status snn_set_param(snn_net* net, uint32_t first, uint32_t n, int32_t param, const double* v, size_t nv) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "parameters are frozen after snn_build");
  if (param < 0 || param >= kNumParams) return fail(net, SNN_E_INVALID, "unknown parameter %d", param);
  if ((uint64_t)first + n > net->N) return fail(net, SNN_E_INVALID, "range [%u, %u) beyond the network", first, first + n);
  if (n == 0) return SNN_OK;
  if (!v || (nv != 1 && nv != n)) return fail(net, SNN_E_INVALID, "nv must be 1 (broadcast) or n (one value per neuron)");
  for (size_t j = 0; j < nv; ++j)
    if (!std::isfinite(v[j])) return fail(net, SNN_E_INVALID, "parameter values must be finite");
  std::vector<int> ks = (nv == 1) ? whole_pops(net, first, n) : std::vector<int>();
  std::vector<double>& pn = net->pn[param];
  if (!ks.empty()) {  // one value for whole populations: the populations' constant
    for (int k : ks) *net->pops[k].param(param) = v[0];
    if (!pn.empty()) std::fill(pn.begin() + first, pn.begin() + first + n, v[0]);
    return SNN_OK;
  }
  if (pn.empty()) {  // first per-neuron value of this parameter: every neuron starts from its population's
    pn.resize(net->N);
    for (size_t k = 0; k < net->pops.size(); ++k) {
      HostPop& p = net->pops[k];
      std::fill(pn.begin() + p.first, pn.begin() + p.first + p.n, *p.param(param));
    }
  }
  for (uint32_t j = 0; j < n; ++j) pn[first + j] = v[nv == 1 ? 0 : j];
  return SNN_OK;
}

constexpr uint64_t kTagParam = 5;  // Philox tag of per-neuron parameter draws

snn_status snn_set_port_param(snn_net* net, uint32_t first, uint32_t n, uint32_t port, int32_t param, double value) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "parameters are frozen after snn_build");
  std::vector<int> ks = whole_pops(net, first, n);
  if (ks.empty()) return fail(net, SNN_E_INVALID, "range is not a union of whole populations");
  for (int k : ks) {
    HostPop& p = net->pops[k];
    if (port >= p.ports) return fail(net, SNN_E_INVALID, "port %u out of range", port);
    if (param == SNN_PP_TAU_SYN) {
      if (!(value > 0)) return fail(net, SNN_E_INVALID, "tau_syn must be positive");
      p.tau_syn[port] = value;
    } else if (param == SNN_PP_E_REV) {
      p.E_rev[port] = value;
    } else if (param == SNN_PP_TAU_RISE) {
      if (!(value > 0)) return fail(net, SNN_E_INVALID, "tau_rise must be positive");
      p.tau_rise[port] = value;
    } else {
      return fail(net, SNN_E_INVALID, "unknown port parameter %d", param);
    }
  }
  return SNN_OK;
}

snn_status snn_connect(snn_net* net, int32_t rule, uint64_t n, uint32_t src_first, uint32_t src_n,
                       uint32_t tgt_first, uint32_t tgt_n, double weight, int32_t delay_kind, double delay_a,
                       double delay_b, uint32_t port) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "connect after snn_build");
  if (src_n == 0 || (uint64_t)src_first + src_n > net->N || (uint64_t)tgt_first + tgt_n > net->N)
    return fail(net, SNN_E_INVALID, "source or target range outside the network");
  if (delay_kind < SNN_DELAY_CONST || delay_kind > SNN_DELAY_NORMAL_CLIPPED)
    return fail(net, SNN_E_INVALID, "unknown delay distribution %d", delay_kind);
  if (delay_kind == SNN_DELAY_UNIFORM && !(delay_b > delay_a)) return fail(net, SNN_E_INVALID, "uniform delay needs b > a");
  if (delay_kind == SNN_DELAY_NORMAL_CLIPPED && !(delay_b > 0)) return fail(net, SNN_E_INVALID, "normal delay needs sd > 0");
  if (!std::isfinite(weight)) return fail(net, SNN_E_INVALID, "weight must be finite");
  if (rule < SNN_RULE_FIXED_INDEGREE || rule > SNN_RULE_FIXED_TOTAL_NUMBER)
    return fail(net, SNN_E_INVALID, "unknown connection rule %d", rule);
  if (rule == SNN_RULE_ONE_TO_ONE && src_n != tgt_n) return fail(net, SNN_E_INVALID, "one-to-one needs src_n == tgt_n");
  if ((rule == SNN_RULE_FIXED_INDEGREE || rule == SNN_RULE_FIXED_OUTDEGREE) && n > 0xffffffffull)
    return fail(net, SNN_E_INVALID, "degree above 2^32 - 1");
  const uint32_t inst = net->pops[pop_of(net, src_first)].inst;
  for (uint32_t t = src_first; t < src_first + src_n;) {
    const HostPop& pp = net->pops[pop_of(net, t)];
    if (pp.inst != inst) return fail(net, SNN_E_INVALID, "a projection must stay inside one instance");
    t = pp.first + pp.n;
  }
  for (uint32_t t = tgt_first; t < tgt_first + tgt_n;) {
    const HostPop& pp = net->pops[pop_of(net, t)];
    if (pp.inst != inst) return fail(net, SNN_E_INVALID, "a projection must stay inside one instance");
    if (port >= pp.ports) return fail(net, SNN_E_INVALID, "port %u out of range for target population", port);
    if (pp.adex() && weight < 0) return fail(net, SNN_E_INVALID, "conductance weights must be >= 0");
    t = pp.first + pp.n;
  }
  if (net->projs.size() >= (1u << 23)) return fail(net, SNN_E_UNSUPPORTED, "too many projections");
  const uint32_t K = (rule == SNN_RULE_FIXED_INDEGREE || rule == SNN_RULE_FIXED_OUTDEGREE) ? (uint32_t)n
                   : rule == SNN_RULE_ALL_TO_ALL ? src_n : 1u;
  net->projs.push_back({src_first, src_n, tgt_first, tgt_n, K, port, inst, net->insts[inst].n_proj++, weight,
                        delay_kind, delay_a, delay_b, rule, n});
  return SNN_OK;
}

snn_status snn_connect_list(snn_net* net, size_t n, const uint32_t* src, const uint32_t* tgt, const double* delay_ms,
                            double weight, uint32_t port) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "connect after snn_build");
  if (n == 0) return SNN_OK;
  if (!src || !tgt || !delay_ms) return fail(net, SNN_E_INVALID, "null list");
  if (!std::isfinite(weight)) return fail(net, SNN_E_INVALID, "weight must be finite");
  if (net->projs.size() >= (1u << 23)) return fail(net, SNN_E_UNSUPPORTED, "too many projections");
  HostProj pr{};
  pr.lsrc.assign(src, src + n);
  pr.ltgt.assign(tgt, tgt + n);
  pr.ldel.resize(n);
  uint32_t smin = UINT32_MAX, smax = 0, tmin = UINT32_MAX, tmax = 0;
  for (size_t j = 0; j < n; ++j) {
    if (src[j] >= net->N || tgt[j] >= net->N) return fail(net, SNN_E_INVALID, "list entry %zu out of range", j);
    const double r = std::max(1.0, std::floor(delay_ms[j] / net->cfg.dt_ms + 0.5));  // steps, half up, >= 1
    if (!(r <= (double)net->cfg.max_delay_steps))
      return fail(net, SNN_E_INVALID, "delay %g ms above max_delay_steps", delay_ms[j]);
    pr.ldel[j] = (uint8_t)r;
    smin = std::min(smin, src[j]); smax = std::max(smax, src[j]);
    tmin = std::min(tmin, tgt[j]); tmax = std::max(tmax, tgt[j]);
  }
  const uint32_t inst = net->pops[pop_of(net, smin)].inst;
  if (net->pops[pop_of(net, smax)].inst != inst || net->pops[pop_of(net, tmin)].inst != inst ||
      net->pops[pop_of(net, tmax)].inst != inst)
    return fail(net, SNN_E_INVALID, "a projection must stay inside one instance");
  for (uint32_t t = tmin; t <= tmax;) {  // ports of the target populations in the bounding range
    const HostPop& pp = net->pops[pop_of(net, t)];
    if (port >= pp.ports) return fail(net, SNN_E_INVALID, "port %u out of range for target population", port);
    if (pp.adex() && weight < 0) return fail(net, SNN_E_INVALID, "conductance weights must be >= 0");
    t = pp.first + pp.n;
  }
  // ranges: the bounding intervals of the listed gids (fixed-point exponents
  // and weight classes are taken over the target range)
  pr.src_first = smin; pr.src_n = smax - smin + 1; pr.tgt_first = tmin; pr.tgt_n = tmax - tmin + 1;
  pr.K = 1; pr.port = port; pr.inst = inst; pr.local = net->insts[inst].n_proj++; pr.weight = weight;
  pr.kind = SNN_DELAY_CONST; pr.da = net->cfg.dt_ms; pr.db = 0.0;
  pr.rule = kRuleList; pr.n = n;
  net->projs.push_back(std::move(pr));
  return SNN_OK;
}

snn_status snn_connect_fixed_indegree(snn_net* net, uint32_t src_first, uint32_t src_n, uint32_t tgt_first,
                                      uint32_t tgt_n, uint32_t indegree, double weight, int32_t delay_kind,
                                      double delay_a, double delay_b, uint32_t port) {
  return snn_connect(net, SNN_RULE_FIXED_INDEGREE, indegree, src_first, src_n, tgt_first, tgt_n, weight, delay_kind,
                     delay_a, delay_b, port);
}

// Weight distributions (Sec. 2.1), discretised: `levels` equal bins of
// [lo, hi], bin j taking its midpoint with the probability the distribution,
// restricted to [lo, hi], gives the bin.  F: uniform (x - a) / (b - a),
// normal erfc(-(x - a) / (b sqrt 2)) / 2.
static double weight_cdf(int32_t kind, double a, double b, double x) {
  if (kind == SNN_WEIGHT_UNIFORM) return (x - a) / (b - a);
  return 0.5 * erfc(-(x - a) / (b * sqrt(2.0)));
}

// Levels (bin midpoints) and draw thresholds of a discretised distribution;
// returns an error message or nullptr.
constexpr uint64_t kTagState = 4;           // Philox tag of state draws (connections 1, Poisson 2, weights 3)
constexpr uint32_t kStateLevelsMax = 65536;  // bins of a state distribution

static const char* dist_levels(int32_t kind, double a, double b, double lo, double hi, uint32_t levels,
                               std::vector<double>& lev, std::vector<uint64_t>& thr) {
  if (kind == SNN_WEIGHT_UNIFORM) {
    if (!(a < b) || !std::isfinite(a) || !std::isfinite(b)) return "uniform distribution needs a < b";
    lo = a; hi = b;
  } else if (kind == SNN_WEIGHT_NORMAL) {
    if (!(b > 0) || !(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi))
      return "normal distribution needs sd > 0 and lo < hi";
  } else {
    return "unknown distribution";
  }
  const double Flo = weight_cdf(kind, a, b, lo), Fhi = weight_cdf(kind, a, b, hi);
  if (!(Fhi > Flo)) return "the distribution has no probability in [lo, hi]";
  lev.resize(levels);
  thr.resize(levels);
  for (uint32_t j = 0; j < levels; ++j) {
    lev[j] = lo + (hi - lo) * (((double)j + 0.5) / (double)levels);
    if (j + 1 == levels) { thr[j] = 1ull << 32; break; }
    const double edge = lo + (hi - lo) * ((double)(j + 1) / (double)levels);
    const double q = (weight_cdf(kind, a, b, edge) - Flo) / (Fhi - Flo);
    thr[j] = (uint64_t)std::min(4294967296.0, std::max(0.0, floor(q * 4294967296.0)));
  }
  return nullptr;
}

snn_status snn_weight_distribution(snn_net* net, int32_t kind, double a, double b, double lo, double hi,
                                   uint32_t levels) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "weights after snn_build");
  if (net->projs.empty()) return fail(net, SNN_E_STATE, "no projection to give weights to");
  HostProj& pr = net->projs.back();
  if (pr.rule == kRuleList) return fail(net, SNN_E_INVALID, "list projections take snn_list_weights");
  if (levels < 1 || levels > (uint32_t)kMaxClasses) return fail(net, SNN_E_INVALID, "levels must be 1..%d", kMaxClasses);
  std::vector<double> lev;
  std::vector<uint64_t> thr;
  if (const char* e = dist_levels(kind, a, b, lo, hi, levels, lev, thr)) return fail(net, SNN_E_INVALID, "%s", e);
  pr.wlev = std::move(lev);
  pr.wthr = std::move(thr);
  pr.lwl.clear();
  return SNN_OK;
}

snn_status snn_stdp(snn_net* net, double tau_plus, double tau_minus, double lambda, double alpha, int32_t mu_plus,
                    int32_t mu_minus, double w_max) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "plasticity after snn_build");
  if (net->projs.empty()) return fail(net, SNN_E_STATE, "no projection to make plastic");
  if (!(tau_plus > 0) || !(tau_minus > 0) || !(lambda > 0) || !(lambda <= 1) || !(alpha >= 0) ||
      !(alpha * lambda <= 1) || !(w_max > 0) || !std::isfinite(w_max) || (mu_plus != 0 && mu_plus != 1) ||
      (mu_minus != 0 && mu_minus != 1))
    return fail(net, SNN_E_INVALID, "bad STDP parameters");
  HostProj& pr = net->projs.back();
  const double lo = pr.wlev.empty() ? pr.weight : pr.wlev.front();
  const double hi = pr.wlev.empty() ? pr.weight : pr.wlev.back();
  if (lo < 0 || hi > w_max) return fail(net, SNN_E_INVALID, "plastic weights must lie in [0, w_max]");
  pr.plastic = true;
  pr.tau_plus = tau_plus; pr.tau_minus = tau_minus; pr.lambda = lambda; pr.alpha = alpha;
  pr.mu_plus = mu_plus; pr.mu_minus = mu_minus; pr.w_max = w_max;
  return SNN_OK;
}

// Philox4x64-10 on the host (Salmon et al., SC'11; the same published
// definition the device kernels use) for draws made while the network is
// defined.
static void philox_host(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    const unsigned __int128 p0 = (unsigned __int128)M0 * c[0], p1 = (unsigned __int128)M1 * c[2];
    const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c[1] ^ k0, n2 = (uint64_t)(p0 >> 64) ^ c[3] ^ k1;
    c[0] = n0; c[1] = (uint64_t)p1; c[2] = n2; c[3] = (uint64_t)p0;
    k0 += W0; k1 += W1;
  }
}

snn_status snn_state_distribution(snn_net* net, uint32_t first, uint32_t n, int32_t var, uint32_t port,
                                  int32_t kind, double a, double b, double lo, double hi, uint32_t levels) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if ((uint64_t)first + n > net->N) return fail(net, SNN_E_INVALID, "bad state range");
  if (var == SNN_V_REFR || var < SNN_V_M || var > SNN_V_G_RISE)
    return fail(net, SNN_E_INVALID, "state variable %d cannot be drawn", var);
  if (levels < 1 || levels > kStateLevelsMax) return fail(net, SNN_E_INVALID, "levels must be 1..%u", kStateLevelsMax);
  std::vector<double> lev;
  std::vector<uint64_t> thr;
  if (const char* e = dist_levels(kind, a, b, lo, hi, levels, lev, thr)) return fail(net, SNN_E_INVALID, "%s", e);
  std::vector<double> v(std::max<uint32_t>(1, n));
  for (uint32_t i = first; i < first + n;) {  // population by population: instance seed and first gid
    const HostPop& pp = net->pops[pop_of(net, i)];
    const uint64_t seed = net->insts[pp.inst].seed, g0 = net->insts[pp.inst].first_gid;
    const uint32_t end = std::min(first + n, pp.first + pp.n);
    for (; i < end; ++i) {
      uint64_t c[4] = {i - g0, ((uint64_t)var << 8) | port, kTagState, 0};
      philox_host(c, seed, 0);
      const uint32_t u = (uint32_t)(c[0] >> 32);
      const size_t l = std::upper_bound(thr.begin(), thr.end(), (uint64_t)u) - thr.begin();  // min{l : u < thr[l]}
      v[i - first] = lev[l];
    }
  }
  return snn_set_state(net, first, n, var, port, v.data(), n);
}

snn_status snn_param_distribution(snn_net* net, uint32_t first, uint32_t n, int32_t param, int32_t kind, double a,
                                  double b, double lo, double hi, uint32_t levels) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "parameters are frozen after snn_build");
  if ((uint64_t)first + n > net->N) return fail(net, SNN_E_INVALID, "bad parameter range");
  if (param < 0 || param >= kNumParams) return fail(net, SNN_E_INVALID, "unknown parameter %d", param);
  if (levels < 1 || levels > kStateLevelsMax) return fail(net, SNN_E_INVALID, "levels must be 1..%u", kStateLevelsMax);
  std::vector<double> lev;
  std::vector<uint64_t> thr;
  if (const char* e = dist_levels(kind, a, b, lo, hi, levels, lev, thr)) return fail(net, SNN_E_INVALID, "%s", e);
  if (n == 0) return SNN_OK;
  std::vector<double> v(n);
  for (uint32_t i = first; i < first + n;) {  // population by population: instance seed and first gid
    const HostPop& pp = net->pops[pop_of(net, i)];
    const uint64_t seed = net->insts[pp.inst].seed, g0 = net->insts[pp.inst].first_gid;
    const uint32_t end = std::min(first + n, pp.first + pp.n);
    for (; i < end; ++i) {
      uint64_t c[4] = {i - g0, (uint64_t)param << 8, kTagParam, 0};
      philox_host(c, seed, 0);
      const uint32_t u = (uint32_t)(c[0] >> 32);
      v[i - first] = lev[std::upper_bound(thr.begin(), thr.end(), (uint64_t)u) - thr.begin()];
    }
  }
  return snn_set_param(net, first, n, param, v.data(), n);
}

snn_status snn_list_weights(snn_net* net, const double* weights, size_t n) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "weights after snn_build");
  if (n == 0) return SNN_OK;
  if (!weights) return fail(net, SNN_E_INVALID, "null weights");
  if (net->projs.empty() || net->projs.back().rule != kRuleList || net->projs.back().n != n)
    return fail(net, SNN_E_INVALID, "the last projection is not a list of %zu connections", n);
  HostProj& pr = net->projs.back();
  std::vector<double> v(weights, weights + n);
  for (double x : v)
    if (!std::isfinite(x)) return fail(net, SNN_E_INVALID, "weights must be finite");
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  if (v.size() > (size_t)kMaxClasses) return fail(net, SNN_E_UNSUPPORTED, "more than %d distinct weights", kMaxClasses);
  pr.lwl.resize(n);
  for (size_t j = 0; j < n; ++j)
    pr.lwl[j] = (uint16_t)(std::lower_bound(v.begin(), v.end(), weights[j]) - v.begin());
  pr.wlev = std::move(v);
  pr.wthr.clear();
  return SNN_OK;
}

snn_status snn_multimeter(snn_net* net, int32_t var, uint32_t port, const uint32_t* gids, size_t n,
                          uint32_t interval, uint32_t* meter_id) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "multimeter after snn_build");
  if (var != SNN_V_M && var != SNN_V_W && var != SNN_V_G && var != SNN_V_G_RISE && var != SNN_V_I_SYN && var != SNN_V_H)
    return fail(net, SNN_E_INVALID, "variable %d cannot be recorded", var);
  if (interval == 0 || port >= (uint32_t)kMaxPorts || (n && !gids)) return fail(net, SNN_E_INVALID, "bad meter");
  for (size_t j = 0; j < n; ++j)
    if (gids[j] >= net->N) return fail(net, SNN_E_INVALID, "gid %u out of range", gids[j]);
  if ((uint64_t)net->nch + n >= (1ull << 24)) return fail(net, SNN_E_UNSUPPORTED, "too many recorded channels");
  snn_net::Meter m;
  m.var = var; m.port = port; m.interval = interval; m.ch0 = net->nch;
  m.gids.assign(gids, gids + n);
  net->nch += (uint32_t)n;
  net->meters.push_back(std::move(m));
  if (meter_id) *meter_id = (uint32_t)net->meters.size() - 1;
  return SNN_OK;
}

snn_status snn_get_samples(snn_net* net, uint32_t meter_id, uint64_t* steps, double* values, size_t cap,
                           size_t* n_out) {
  if (!net || !n_out) return SNN_E_INVALID;
  net->err.clear();
  if (meter_id >= net->meters.size()) return fail(net, SNN_E_INVALID, "no meter %u", meter_id);
  const snn_net::Meter& m = net->meters[meter_id];
  *n_out = m.steps.size();
  const size_t k = std::min(cap, m.steps.size());
  if (k && (!steps || !values)) return fail(net, SNN_E_INVALID, "null output");
  for (size_t i = 0; i < k; ++i) steps[i] = m.steps[i];
  std::copy(m.values.begin(), m.values.begin() + k * m.gids.size(), values);
  return SNN_OK;
}

snn_status snn_snapshot_size(snn_net* net, size_t* bytes) {
  if (!net || !bytes) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "snapshot before snn_build");
  *bytes = snap_header(net).bytes;
  return SNN_OK;
}

snn_status snn_snapshot(snn_net* net, void* buf, size_t cap) {
  if (!net || !buf) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "snapshot before snn_build");
  snn_status st = enter(net);
  if (st) return st;
  st = drain(net);  // the raster so far, and no copy in flight
  if (st) return st;
  HIPCHK(net, hipStreamSynchronize(net->stream));
  const SnapHeader h = snap_header(net);
  if (cap < h.bytes) return fail(net, SNN_E_INVALID, "snapshot needs %llu bytes", (unsigned long long)h.bytes);
  char* out = static_cast<char*>(buf);
  memcpy(out, &h, sizeof h);
  size_t off = sizeof h;
  for (const auto& x : state_arrays(net)) {
    HIPCHK(net, copy_sync(net, out + off, x.first, x.second, hipMemcpyDeviceToHost));
    off += x.second;
  }
  return leave(net);
}

snn_status snn_restore(snn_net* net, const void* buf, size_t size) {
  if (!net || !buf) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "restore before snn_build");
  SnapHeader h;
  if (size < sizeof h) return fail(net, SNN_E_INVALID, "not a snapshot");
  memcpy(&h, buf, sizeof h);
  SnapHeader mine = snap_header(net);
  if (memcmp(h.magic, mine.magic, 8) || h.version != mine.version || h.N != mine.N || h.P != mine.P ||
      h.R != mine.R || h.n_tiles != mine.n_tiles || h.bins_total != mine.bins_total || h.n_syn != mine.n_syn ||
      h.n_groups != mine.n_groups || h.nblk != mine.nblk || h.sel_grid != mine.sel_grid || h.bytes != mine.bytes ||
      size < h.bytes)
    return fail(net, SNN_E_INVALID, "the snapshot is of another network");
  snn_status st = enter(net);
  if (st) return st;
  st = drain(net);
  if (st) return st;
  HIPCHK(net, hipStreamSynchronize(net->stream));
  const char* in = static_cast<const char*>(buf);
  size_t off = sizeof h;
  for (const auto& x : state_arrays(net)) {
    HIPCHK(net, copy_sync(net, x.first, in + off, x.second, hipMemcpyHostToDevice));
    off += x.second;
  }
  net->cur_step = net->drained_step = h.cur_step;
  net->dj = snn_net::Drain();
  net->r_step.clear();
  net->r_entry.clear();
  net->r_sorted = 0;
  return leave(net);
}

snn_status snn_set_spike_times(snn_net* net, uint32_t gid, const double* t_ms, size_t n) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "spike times after snn_build");
  if (gid >= net->N || (n && !t_ms)) return fail(net, SNN_E_INVALID, "bad neuron or times");
  if (net->pops[pop_of(net, gid)].model != SNN_SPIKE_GENERATOR)
    return fail(net, SNN_E_INVALID, "neuron %u is not a spike generator", gid);
  std::vector<uint64_t> st(n);
  for (size_t j = 0; j < n; ++j) {
    const double r = std::floor(t_ms[j] / net->cfg.dt_ms + 0.5);  // steps of dt, rounded half up
    if (!(r >= 1.0) || r > 1e15) return fail(net, SNN_E_INVALID, "spike time %g below dt", t_ms[j]);
    st[j] = (uint64_t)r - 1;  // emitted in this step's update, reported at t
  }
  std::sort(st.begin(), st.end());
  net->gen_steps[gid] = std::move(st);
  return SNN_OK;
}

snn_status snn_poisson(snn_net* net, uint32_t tgt_first, uint32_t tgt_n, double rate_hz, uint32_t n_inputs,
                       double weight, uint32_t port) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "poisson after snn_build");
  if ((uint64_t)tgt_first + tgt_n > net->N || !(rate_hz >= 0)) return fail(net, SNN_E_INVALID, "bad Poisson drive");
  std::vector<int> ks = whole_pops(net, tgt_first, tgt_n);
  if (ks.empty()) return fail(net, SNN_E_UNSUPPORTED, "a Poisson drive must cover whole populations");
  for (int k : ks)
    if (port >= net->pops[k].ports) return fail(net, SNN_E_INVALID, "port out of range");
  const double lam = (double)n_inputs * rate_hz * net->cfg.dt_ms * 1e-3;
  if (lam > 60.0) return fail(net, SNN_E_UNSUPPORTED, "Poisson mean per step %.3g > 60", lam);
  net->pois.push_back({tgt_first, tgt_n, n_inputs, port, rate_hz, weight});
  return SNN_OK;
}

snn_status snn_set_state(snn_net* net, uint32_t first, uint32_t n, int32_t var, uint32_t port, const double* v,
                         size_t nv) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if ((uint64_t)first + n > net->N || !v || (nv != 1 && nv != n)) return fail(net, SNN_E_INVALID, "bad state range");
  if (port >= (uint32_t)kMaxPorts) return fail(net, SNN_E_INVALID, "bad port");
  if (!net->built) {
    for (uint32_t j = 0; j < n; ++j) {
      const double x = v[nv == 1 ? 0 : j];
      const uint32_t i = first + j;
      switch (var) {
        case SNN_V_M: net->V[i] = x; break;
        case SNN_V_I_E: net->Ie[i] = x; break;
        case SNN_V_W: net->w[i] = x; break;
        case SNN_V_G: net->g[(size_t)i * kMaxPorts + port] = x; break;
        case SNN_V_I_SYN: net->Isyn[(size_t)i * kMaxPorts + port] = x; break;
        case SNN_V_REFR: net->refr[i] = (int32_t)x; break;
        case SNN_V_H: net->h[i] = x; break;
        case SNN_V_G_RISE: net->gr[(size_t)i * kMaxPorts + port] = x; break;
        default: return fail(net, SNN_E_INVALID, "unknown state variable %d", var);
      }
    }
    return SNN_OK;
  }
  snn_status st = enter(net);
  if (st) return st;
  HIPCHK(net, hipStreamSynchronize(net->stream));
  const NetDev& nd = net->nd;
  if ((var == SNN_V_G || var == SNN_V_I_SYN || var == SNN_V_G_RISE) && port >= net->P)
    return fail(net, SNN_E_INVALID, "port out of range");
  if (var == SNN_V_REFR) {
    std::vector<int32_t> buf(n);
    for (uint32_t j = 0; j < n; ++j) buf[j] = (int32_t)v[nv == 1 ? 0 : j];
    if (!nd.refr) return fail(net, SNN_E_INVALID, "no refractory state in this network");
    HIPCHK(net, copy_sync(net, nd.refr + first, buf.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
    return leave(net);
  }
  float* base = nullptr;
  size_t stride = 1, off = 0;
  switch (var) {
    case SNN_V_M: base = nd.V; break;
    case SNN_V_I_E: base = nd.Ie; break;
    case SNN_V_W: base = nd.w; break;
    case SNN_V_G: base = nd.g; stride = net->P; off = port; break;
    case SNN_V_I_SYN: base = nd.Isyn; stride = net->P; off = port; break;
    case SNN_V_H: base = nd.h; break;
    case SNN_V_G_RISE: base = nd.gr; stride = net->P; off = port; break;
    default: return fail(net, SNN_E_INVALID, "unknown state variable %d", var);
  }
  if (!base) return fail(net, SNN_E_INVALID, "state variable not present in this network");
  std::vector<float> buf(n);
  for (uint32_t j = 0; j < n; ++j) buf[j] = to_device_state(net, var, first + j, v[nv == 1 ? 0 : j]);
  if (stride == 1) {
    HIPCHK(net, copy_sync(net, base + first, buf.data(), n * sizeof(float), hipMemcpyHostToDevice));
  } else {
    HIPCHK(net, copy2d_sync(net, base + (size_t)first * stride + off, stride * sizeof(float), buf.data(), sizeof(float),
                            sizeof(float), n, hipMemcpyHostToDevice));
  }
  return leave(net);
}

snn_status snn_get_state(snn_net* net, uint32_t first, uint32_t n, int32_t var, uint32_t port, double* out) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if ((uint64_t)first + n > net->N || !out) return fail(net, SNN_E_INVALID, "bad state range");
  if (!net->built) {
    for (uint32_t j = 0; j < n; ++j) {
      const uint32_t i = first + j;
      switch (var) {
        case SNN_V_M: out[j] = std::isnan(net->V[i]) ? rest_of(net, i) : net->V[i]; break;
        case SNN_V_I_E: out[j] = net->Ie[i]; break;
        case SNN_V_W: out[j] = net->w[i]; break;
        case SNN_V_G: out[j] = net->g[(size_t)i * kMaxPorts + port]; break;
        case SNN_V_I_SYN: out[j] = net->Isyn[(size_t)i * kMaxPorts + port]; break;
        case SNN_V_REFR: out[j] = net->refr[i]; break;
        case SNN_V_H: out[j] = net->h[i]; break;
        case SNN_V_G_RISE: out[j] = net->gr[(size_t)i * kMaxPorts + port]; break;
        default: return fail(net, SNN_E_INVALID, "unknown state variable %d", var);
      }
    }
    return SNN_OK;
  }
  snn_status st = enter(net);
  if (st) return st;
  HIPCHK(net, hipStreamSynchronize(net->stream));
  const NetDev& nd = net->nd;
  if ((var == SNN_V_G || var == SNN_V_I_SYN || var == SNN_V_G_RISE) && port >= net->P)
    return fail(net, SNN_E_INVALID, "port out of range");
  if (var == SNN_V_REFR) {
    if (!nd.refr) return fail(net, SNN_E_INVALID, "no refractory state in this network");
    std::vector<int32_t> buf(n);
    HIPCHK(net, copy_sync(net, buf.data(), nd.refr + first, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (uint32_t j = 0; j < n; ++j) out[j] = buf[j];
    return leave(net);
  }
  const float* base = nullptr;
  size_t stride = 1, off = 0;
  switch (var) {
    case SNN_V_M: base = nd.V; break;
    case SNN_V_I_E: base = nd.Ie; break;
    case SNN_V_W: base = nd.w; break;
    case SNN_V_G: base = nd.g; stride = net->P; off = port; break;
    case SNN_V_I_SYN: base = nd.Isyn; stride = net->P; off = port; break;
    case SNN_V_H: base = nd.h; break;
    case SNN_V_G_RISE: base = nd.gr; stride = net->P; off = port; break;
    default: return fail(net, SNN_E_INVALID, "unknown state variable %d", var);
  }
  if (!base) return fail(net, SNN_E_INVALID, "state variable not present in this network");
  std::vector<float> buf(n);
  if (stride == 1) {
    HIPCHK(net, copy_sync(net, buf.data(), base + first, n * sizeof(float), hipMemcpyDeviceToHost));
  } else {
    HIPCHK(net, copy2d_sync(net, buf.data(), sizeof(float), base + (size_t)first * stride + off, stride * sizeof(float),
                            sizeof(float), n, hipMemcpyDeviceToHost));
  }
  for (uint32_t j = 0; j < n; ++j) out[j] = from_device_state(net, var, first + j, buf[j]);
  return leave(net);
}

}  // extern "C"

namespace {

snn_status build_impl(snn_net* net);

// Everything a failed build left behind, so that the network is as before
// the call (and may be built again, e.g. once memory is available).
void release_build(snn_net* net) {
  (void)hipStreamSynchronize(net->stream);
  for (auto& gx : net->graphs) (void)hipGraphExecDestroy(gx.second);
  net->graphs.clear();
  while (!net->allocs.empty()) dev_free(net, net->allocs.back().p);
  if (net->pin_cb) (void)hipHostFree(net->pin_cb);
  if (net->pin_rc) (void)hipHostFree(net->pin_rc);
  if (net->pin_ctrl) (void)hipHostFree(net->pin_ctrl);
  if (net->ev_drain) (void)hipEventDestroy(net->ev_drain);
  net->pin_cb = nullptr; net->pin_rc = nullptr; net->pin_ctrl = nullptr; net->ev_drain = nullptr;
  net->d_addr = nullptr; net->d_mbuf = nullptr;
  net->nd = NetDev{};
  net->has_lif = net->has_adex = net->has_beta = false;
  net->built = false;
}

}  // namespace

extern "C" {

snn_status snn_release(snn_net* net) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, net->released ? "already released" : "not built");
  snn_status st = enter(net);
  if (st) return st;
  if ((st = drain(net))) return st;
  sort_raster(net);
  snn_counters c;
  if ((st = snn_get_counters(net, &c))) return st;
  if ((st = leave(net))) return st;
  release_build(net);
  c.device_bytes = net->dev_bytes;
  net->final_ctr = c;
  net->released = true;
  return SNN_OK;
}

snn_status snn_build(snn_net* net) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (net->built) return fail(net, SNN_E_STATE, "already built");
  if (net->released) return fail(net, SNN_E_STATE, "released networks are not built again");
  if (net->N == 0) return fail(net, SNN_E_INVALID, "empty network");
  const snn_status st = build_impl(net);
  if (st != SNN_OK) {
    const std::string msg = net->err;
    release_build(net);
    net->err = msg;
  }
  return st;
}

}  // extern "C"

namespace {

snn_status build_impl(snn_net* net) {
  snn_status st = enter(net);
  if (st) return st;
  const auto t0 = std::chrono::steady_clock::now();
  const double dt = net->cfg.dt_ms;
  const uint32_t npop = (uint32_t)net->pops.size();
  const uint32_t N = net->N;
  uint32_t P = 1;
  for (const HostPop& p : net->pops) {
    P = std::max(P, p.ports);
    if (p.adex()) {
      net->has_adex = true;
      if (p.model == SNN_AEIF_COND_BETA) {
        net->has_beta = true;
        for (uint32_t q = 0; q < p.ports; ++q)
          if (!(p.tau_rise[q] > 0) || !(p.tau_syn[q] > 0)) return fail(net, SNN_E_INVALID, "invalid beta time constants");
      }
      if (p.t_ref != 0.0) return fail(net, SNN_E_UNSUPPORTED, "AdEx refractory time must be 0");
      if (!(p.Delta_T > 0) || !(p.tau_w > 0) || !(p.C_m > 0) || !(p.rk_eps > 0))
        return fail(net, SNN_E_INVALID, "invalid AdEx parameters");
    } else {
      net->has_lif = true;  // LIF and devices share the kernels' non-AdEx path
      if (!(p.tau_m > 0) || !(p.C_m > 0) || p.t_ref < 0) return fail(net, SNN_E_INVALID, "invalid LIF parameters");
    }
    if (p.model == SNN_PARROT_NEURON) {  // parrots count arriving spikes: unit weights only
      for (const HostProj& pr : net->projs)
        if (pr.synapses() && pr.tgt_first < p.first + p.n && pr.tgt_first + pr.tgt_n > p.first &&
            (pr.wlev.empty() ? pr.weight != 1.0 : (pr.wlev.size() != 1 || pr.wlev[0] != 1.0)))
          return fail(net, SNN_E_INVALID, "weights onto parrot neurons must be 1");
      for (const HostPois& q : net->pois)
        if (q.tgt_n && q.tgt_first < p.first + p.n && q.tgt_first + q.tgt_n > p.first && q.weight != 1.0)
          return fail(net, SNN_E_INVALID, "weights onto parrot neurons must be 1");
    }
  }
  // populations whose neurons carry their own constants: a parameter that the
  // model uses is set per neuron somewhere inside the population
  std::vector<uint8_t> per_neuron(npop, 0);
  if (any_per_neuron(net)) {
    static const int32_t lif_ids[] = {SNN_P_TAU_M, SNN_P_C_M, SNN_P_E_L, SNN_P_V_TH, SNN_P_V_RESET, SNN_P_T_REF};
    static const int32_t adex_ids[] = {SNN_P_C_M, SNN_P_E_L, SNN_P_T_REF, SNN_P_G_L, SNN_P_DELTA_T, SNN_P_V_T,
                                       SNN_P_TAU_W, SNN_P_A, SNN_P_B, SNN_P_V_PEAK, SNN_P_V_R, SNN_P_RK_EPS,
                                       SNN_P_RK_HMIN};
    for (uint32_t k = 0; k < npop; ++k) {
      const HostPop& p = net->pops[k];
      if (p.model == SNN_SPIKE_GENERATOR || p.model == SNN_PARROT_NEURON) continue;
      const int32_t* ids = p.adex() ? adex_ids : lif_ids;
      const size_t nid = p.adex() ? sizeof adex_ids / sizeof adex_ids[0] : sizeof lif_ids / sizeof lif_ids[0];
      for (size_t q = 0; q < nid && !per_neuron[k]; ++q) {
        const std::vector<double>& v = net->pn[ids[q]];
        if (v.empty()) continue;
        const double pop_v = *p.param(ids[q]);
        for (uint32_t i = p.first; i < p.first + p.n; ++i)
          if (v[i] != pop_v) { per_neuron[k] = 1; break; }
      }
      if (!per_neuron[k]) continue;
      for (uint32_t i = p.first; i < p.first + p.n; ++i) {
        const HostPop q = neuron_params(net, i);
        if (p.adex()) {
          if (q.t_ref != 0.0) return fail(net, SNN_E_UNSUPPORTED, "AdEx refractory time must be 0 (neuron %u)", i);
          if (!(q.Delta_T > 0) || !(q.tau_w > 0) || !(q.C_m > 0) || !(q.rk_eps > 0) || !(q.rk_hmin >= 0))
            return fail(net, SNN_E_INVALID, "invalid AdEx parameters of neuron %u", i);
        } else if (!(q.tau_m > 0) || !(q.C_m > 0) || q.t_ref < 0) {
          return fail(net, SNN_E_INVALID, "invalid LIF parameters of neuron %u", i);
        }
      }
    }
  }
  net->P = P;
  // Poisson drive per population (drives cover whole populations)
  std::vector<int> pois_of_pop(npop, -1);
  for (size_t q = 0; q < net->pois.size(); ++q) {
    for (int k : whole_pops(net, net->pois[q].tgt_first, net->pois[q].tgt_n)) {
      if (pois_of_pop[k] >= 0) return fail(net, SNN_E_INVALID, "two Poisson drives on one population");
      pois_of_pop[k] = (int)q;
    }
  }
  // fixed-point exponent per (population, port)
  std::vector<double> maxw((size_t)npop * P, 0.0);
  auto overlaps = [&](uint32_t k, uint32_t first, uint32_t n) {
    const HostPop& p = net->pops[k];
    return n > 0 && first < p.first + p.n && first + n > p.first;
  };
  for (const HostProj& pr : net->projs) {
    if (pr.synapses() == 0) continue;
    for (uint32_t k = 0; k < npop; ++k)
      if (overlaps(k, pr.tgt_first, pr.tgt_n)) {
        // a plastic weight can grow up to w_max
        maxw[k * P + pr.port] = std::max(maxw[k * P + pr.port], pr.plastic ? std::max(pr.wmax_abs(), pr.w_max)
                                                                             : pr.wmax_abs());
        if (net->pops[k].adex() && pr.wmin() < 0) return fail(net, SNN_E_INVALID, "conductance weights must be >= 0");
      }
  }
  for (const HostPois& q : net->pois)
    for (uint32_t k = 0; k < npop; ++k)
      if (overlaps(k, q.tgt_first, q.tgt_n)) maxw[k * P + q.port] = std::max(maxw[k * P + q.port], fabs(q.weight));
  net->shift.assign((size_t)npop * P, 0);
  for (size_t k = 0; k < maxw.size(); ++k) net->shift[k] = fixed_shift(maxw[k]);
  // STDP rules: one per (plastic projection, target population), numbered from 1
  // in that order (0: static), with W = w_max in the population's fixed point
  std::vector<StdpRule> rules;
  std::vector<int64_t> stdp_F;
  std::vector<uint32_t> rule_of((size_t)net->projs.size() * npop, 0);
  for (size_t p = 0; p < net->projs.size(); ++p) {
    const HostProj& pr = net->projs[p];
    if (!pr.plastic || pr.synapses() == 0) continue;
    // F(d) = round(scale e^{-d dt / tau} 2^32) up to its first zero
    auto table = [&](double scale, double tau, uint32_t& len, uint64_t& off) -> bool {
      off = stdp_F.size();
      for (uint64_t d = 0;; ++d) {
        const int64_t F = llrint(ldexp(scale * exp(-((double)d * dt) / tau), 32));
        if (F == 0) break;
        if (d >= (1u << 20)) return false;
        stdp_F.push_back(F);
      }
      len = (uint32_t)(stdp_F.size() - off);
      return true;
    };
    for (uint32_t k = 0; k < npop; ++k) {
      if (!overlaps(k, pr.tgt_first, pr.tgt_n)) continue;
      if (rules.size() >= 255) return fail(net, SNN_E_UNSUPPORTED, "more than 255 plastic (projection, population) pairs");
      StdpRule r;
      memset(&r, 0, sizeof r);
      r.W = llrint(ldexp(pr.w_max, net->shift[k * P + pr.port]));
      r.mu_plus = (uint32_t)pr.mu_plus; r.mu_minus = (uint32_t)pr.mu_minus;
      if (!table(pr.lambda, pr.tau_plus, r.len_plus, r.off_plus) ||
          !table(pr.alpha * pr.lambda, pr.tau_minus, r.len_minus, r.off_minus))
        return fail(net, SNN_E_UNSUPPORTED, "STDP time constant too long for its tables (tau / dt > 2^20 / 20)");
      rules.push_back(r);
      rule_of[p * npop + k] = (uint32_t)rules.size();
    }
  }
  // weight classes: distinct (port, w_q, rule) sorted (static before plastic at
  // equal weights), per (projection, target population)
  typedef std::tuple<uint32_t, int64_t, uint32_t> ClsKey;
  std::map<ClsKey, uint32_t> classes;
  std::vector<ClsKey> cls_key((size_t)net->projs.size() * npop, ClsKey{0, 0, 0});
  // projections with weight levels: the classes of every (target population, level)
  std::vector<uint32_t> wpop0(net->projs.size(), 0);
  std::vector<std::vector<ClsKey>> wkeys(net->projs.size());
  for (size_t p = 0; p < net->projs.size(); ++p) {
    const HostProj& pr = net->projs[p];
    if (pr.synapses() == 0) continue;
    if (!pr.wlev.empty()) {
      const uint32_t k0 = pop_of(net, pr.tgt_first), k1 = pop_of(net, pr.tgt_first + pr.tgt_n - 1);
      wpop0[p] = k0;
      for (uint32_t k = k0; k <= k1; ++k)
        for (double w : pr.wlev) {
          const ClsKey key{pr.port, llrint(ldexp(w, net->shift[k * P + pr.port])), rule_of[p * npop + k]};
          wkeys[p].push_back(key);
          classes[key] = 0;
        }
      continue;
    }
    for (uint32_t k = 0; k < npop; ++k) {
      if (!overlaps(k, pr.tgt_first, pr.tgt_n)) continue;
      const int64_t wq = llrint(ldexp(pr.weight, net->shift[k * P + pr.port]));
      cls_key[p * npop + k] = ClsKey{pr.port, wq, rule_of[p * npop + k]};
      classes[cls_key[p * npop + k]] = 0;
    }
  }
  uint32_t tbits = 1;
  while (tbits < 32 && (1ull << tbits) < (uint64_t)N) ++tbits;  // bits of the largest gid
  net->cls_bits = 32 - tbits;
  const size_t max_cls = std::min<size_t>(kMaxClasses, (size_t)1 << std::min<uint32_t>(net->cls_bits, 20));
  if (classes.size() > max_cls)
    return fail(net, SNN_E_UNSUPPORTED, "%zu (port, weight) classes; at most %zu for this network size", classes.size(),
                max_cls);
  const size_t ncls = std::max<size_t>(1, classes.size());
  net->cls_wq.assign(ncls, 0);
  net->cls_port.assign(ncls, 0);
  std::vector<uint8_t> cls_rule(ncls, 0);
  {
    uint32_t id = 0;
    for (auto& kv : classes) {
      kv.second = id;
      net->cls_port[id] = std::get<0>(kv.first);
      net->cls_wq[id] = std::get<1>(kv.first);
      cls_rule[id] = (uint8_t)std::get<2>(kv.first);
      ++id;
    }
  }
  net->cls_rule = cls_rule;
  std::vector<uint16_t> cls_of((size_t)std::max<size_t>(1, net->projs.size()) * npop, 0);
  for (size_t p = 0; p < net->projs.size(); ++p)
    for (uint32_t k = 0; k < npop; ++k)
      if (overlaps(k, net->projs[p].tgt_first, net->projs[p].tgt_n) && net->projs[p].synapses() &&
          net->projs[p].wlev.empty())
        cls_of[p * npop + k] = (uint16_t)classes[cls_key[p * npop + k]];
  std::vector<uint16_t> wcls;  // level classes of all projections, each [population][level]
  std::vector<size_t> wcls_off(net->projs.size(), 0);
  for (size_t p = 0; p < net->projs.size(); ++p) {
    wcls_off[p] = wcls.size();
    for (const auto& key : wkeys[p]) wcls.push_back((uint16_t)classes[key]);
  }
  // projections, delay tables, largest delay present
  const uint32_t dmax_cfg = net->cfg.max_delay_steps;
  std::vector<ProjDev> pd(net->projs.size());
  uint64_t total_pairs = 0, total_syn = 0;
  uint32_t dmax_used = 1;
  for (size_t p = 0; p < net->projs.size(); ++p) {
    const HostProj& pr = net->projs[p];
    ProjDev& d = pd[p];
    memset(&d, 0, sizeof d);
    d.src_first = pr.src_first; d.src_n = pr.src_n; d.tgt_first = pr.tgt_first; d.tgt_n = pr.tgt_n;
    d.rule = (uint32_t)pr.rule;
    const bool single = pr.rule == SNN_RULE_ONE_TO_ONE || pr.rule == SNN_RULE_FIXED_TOTAL_NUMBER || pr.rule == kRuleList;
    d.K = pr.K; d.kpairs = single ? 1u : (pr.K + 1) / 2; d.index = pr.local;
    d.gid_base = net->insts[pr.inst].first_gid; d.seed = net->insts[pr.inst].seed;
    d.pair_begin = total_pairs;
    delay_thresholds(pr.kind, pr.da, pr.db, dt, dmax_cfg, d.thr);
    const uint64_t syn = pr.synapses();
    if (syn) total_pairs += pr.entities() * d.kpairs;
    total_syn += syn;
    if (syn && pr.rule == kRuleList) {
      for (uint8_t v : pr.ldel) dmax_used = std::max<uint32_t>(dmax_used, v);
    } else if (syn) {
      uint32_t dm = 1;
      while (dm < dmax_cfg && d.thr[dm] < (1ull << 32)) ++dm;
      dmax_used = std::max(dmax_used, dm);
    }
  }
  if (total_syn >= (1ull << 35)) return fail(net, SNN_E_UNSUPPORTED, "more than 2^35 synapses");
  net->dmax_used = dmax_used;
  const uint32_t D1 = dmax_used + 1;
  // population table
  std::vector<PopDev> popdev(npop);
  std::vector<uint64_t> pois_thr;
  for (uint32_t k = 0; k < npop; ++k) {
    const HostPop& p = net->pops[k];
    PopDev& d = popdev[k];
    memset(&d, 0, sizeof d);
    d.first = p.first; d.n = p.n; d.model = p.model; d.n_ports = (int32_t)p.ports;
    d.gid_base = net->insts[p.inst].first_gid; d.seed = net->insts[p.inst].seed;
    d.per_neuron = per_neuron[k];
    if (!p.adex()) lif_propagators(p, dt, d);
    d.inv_C = (float)(1.0 / p.C_m); d.g_L = (float)p.g_L; d.E_L = (float)p.E_L; d.Delta_T = (float)p.Delta_T;
    d.inv_Delta_T = (float)(1.0 / p.Delta_T); d.V_T = (float)p.V_T; d.inv_tau_w = (float)(1.0 / p.tau_w);
    d.a = (float)p.a; d.b = (float)p.b; d.V_peak = (float)p.V_peak; d.V_r = (float)p.V_r;
    for (int q = 0; q < kMaxPorts; ++q) {
      d.E_rev[q] = (float)p.E_rev[q];
      d.inv_tau_syn[q] = (float)(1.0 / p.tau_syn[q]);
      if (p.model == SNN_AEIF_COND_BETA) {
        d.inv_tau_rise[q] = (float)(1.0 / p.tau_rise[q]);
        d.g0[q] = (float)beta_g0(p.tau_rise[q], p.tau_syn[q]);
      } else {
        d.inv_tau_rise[q] = 1.f;  // r stays 0 for exponential ports
        d.g0[q] = 0.f;
      }
      d.scale[q] = (q < (int)P) ? (float)ldexp(1.0, -net->shift[k * P + q]) : 0.f;
    }
    d.rk_eps = (float)p.rk_eps; d.rk_hmin = (float)p.rk_hmin; d.dt = (float)dt;
    d.pois = -1;
    if (pois_of_pop[k] >= 0) {
      const HostPois& q = net->pois[pois_of_pop[k]];
      d.pois = (int32_t)(pois_thr.size() / kPoisKmax);
      d.pois_port = (int32_t)q.port;
      d.pois_wq = llrint(ldexp(q.weight, net->shift[k * P + q.port]));
      std::vector<uint64_t> thr(kPoisKmax);
      poisson_thresholds((double)q.n_inputs * q.rate * dt * 1e-3, thr.data());
      pois_thr.insert(pois_thr.end(), thr.begin(), thr.end());
    }
  }
  if (pois_thr.empty()) pois_thr.resize(kPoisKmax, 1ull << 32);

  NetDev& nd = net->nd;
  memset(&nd, 0, sizeof nd);
  nd.N = N; nd.P = P; nd.npop = npop; nd.dmax = dmax_used;
  // step slots: the steps delivery reads (n+1-Dmax .. n-1), the previous step's
  // count, the current step's counter and the next step's (cleared): >= 3
  nd.R = std::max<uint32_t>(dmax_used + 1, 3);
  nd.npois = (uint32_t)(pois_thr.size() / kPoisKmax);
  // the inverse-CDF search stops at the first threshold of 2^32, so the
  // entries past it in any table are never read
  nd.pois_len = 1;
  for (uint32_t q = 0; q < nd.npois; ++q) {
    uint32_t k = 0;
    while (k < kPoisKmax - 1 && pois_thr[(size_t)q * kPoisKmax + k] < (1ull << 32)) ++k;
    nd.pois_len = std::max<uint32_t>(nd.pois_len, k + 1);
  }
  nd.nblk_upd = (N + kUpdBlock - 1) / kUpdBlock;
  nd.pad0 = (net->has_lif ? 1u : 0u) | (net->has_adex ? 2u : 0u) | (net->has_beta ? 4u : 0u);
  hipStream_t s = net->stream;
#define ALLOC(ptr, T, count)                                                              \
  do {                                                                                    \
    ptr = dalloc<T>(net, (count));                                                        \
    if (!ptr) return fail(net, SNN_E_NOMEM, "device allocation of %zu bytes failed", (size_t)(count) * sizeof(T)); \
  } while (0)
  PopDev* d_pops; ALLOC(d_pops, PopDev, npop);
  HIPCHK(net, hipMemcpyAsync(d_pops, popdev.data(), npop * sizeof(PopDev), hipMemcpyHostToDevice, s));
  nd.pops = d_pops;
  nd.nlif = nullptr;
  nd.nadex = nullptr;
  {  // constants of the neurons of per-neuron populations, computed as the population's are
    std::vector<NeuronLif> hl;
    std::vector<NeuronAdex> ha;
    for (uint32_t k = 0; k < npop; ++k) {
      if (!per_neuron[k]) continue;
      const HostPop& p = net->pops[k];
      if (p.adex() && ha.empty()) ha.assign(N, NeuronAdex{});
      if (!p.adex() && hl.empty()) hl.assign(N, NeuronLif{});
      for (uint32_t i = p.first; i < p.first + p.n; ++i) {
        const HostPop q = neuron_params(net, i);
        PopDev d;
        memset(&d, 0, sizeof d);
        if (!p.adex()) {
          lif_propagators(q, dt, d);
          NeuronLif& c = hl[i];
          c.P22 = d.P22; c.P20 = d.P20; c.theta = d.theta; c.y_reset = d.y_reset; c.n_ref = d.n_ref;
          for (int r = 0; r < kMaxPorts; ++r) c.P21[r] = d.P21[r];
        } else {
          NeuronAdex& c = ha[i];
          c.inv_C = (float)(1.0 / q.C_m); c.g_L = (float)q.g_L; c.E_L = (float)q.E_L; c.Delta_T = (float)q.Delta_T;
          c.inv_Delta_T = (float)(1.0 / q.Delta_T); c.V_T = (float)q.V_T; c.inv_tau_w = (float)(1.0 / q.tau_w);
          c.a = (float)q.a; c.b = (float)q.b; c.V_peak = (float)q.V_peak; c.V_r = (float)q.V_r;
          c.rk_eps = (float)q.rk_eps; c.rk_hmin = (float)q.rk_hmin;
        }
      }
    }
    if (!hl.empty()) {
      NeuronLif* d_nl; ALLOC(d_nl, NeuronLif, N);
      HIPCHK(net, copy_sync(net, d_nl, hl.data(), (size_t)N * sizeof(NeuronLif), hipMemcpyHostToDevice));
      nd.nlif = d_nl;
    }
    if (!ha.empty()) {
      NeuronAdex* d_na; ALLOC(d_na, NeuronAdex, N);
      HIPCHK(net, copy_sync(net, d_na, ha.data(), (size_t)N * sizeof(NeuronAdex), hipMemcpyHostToDevice));
      nd.nadex = d_na;
    }
  }
  uint64_t* d_pthr; ALLOC(d_pthr, uint64_t, pois_thr.size());
  HIPCHK(net, hipMemcpyAsync(d_pthr, pois_thr.data(), pois_thr.size() * 8, hipMemcpyHostToDevice, s));
  nd.pois_thr = d_pthr;
  int64_t* d_cw; ALLOC(d_cw, int64_t, ncls);
  uint32_t* d_cp; ALLOC(d_cp, uint32_t, ncls);
  HIPCHK(net, hipMemcpyAsync(d_cw, net->cls_wq.data(), ncls * 8, hipMemcpyHostToDevice, s));
  HIPCHK(net, hipMemcpyAsync(d_cp, net->cls_port.data(), ncls * 4, hipMemcpyHostToDevice, s));
  nd.cls_wq = d_cw; nd.cls_port = d_cp;
  nd.n_classes = (uint32_t)ncls; nd.cls_bits = net->cls_bits;

  // ---- connectivity: count, scan, masks, group offsets, scatter, sort ----
  const uint64_t M = (uint64_t)N * D1;
  uint32_t* d_cnt; ALLOC(d_cnt, uint32_t, M);
  uint64_t* d_off; ALLOC(d_off, uint64_t, M + 1);
  uint64_t* d_ng; ALLOC(d_ng, uint64_t, N);
  uint64_t* d_gp64; ALLOC(d_gp64, uint64_t, (size_t)N + 1);
  uint64_t* d_tmp; ALLOC(d_tmp, uint64_t, scan_tmp_words(M));
  uint64_t* d_mask; ALLOC(d_mask, uint64_t, N);
  uint32_t* d_gp32; ALLOC(d_gp32, uint32_t, (size_t)N + 1);
  ProjDev* d_proj = nullptr;
  uint16_t* d_clsof = nullptr;
  uint32_t* d_popfirst = nullptr;
  ALLOC(d_proj, ProjDev, std::max<size_t>(1, pd.size()));
  std::vector<void*> list_bufs;  // user-defined lists, freed with the build's scratch
  for (size_t p = 0; p < pd.size(); ++p) {
    const HostProj& pr = net->projs[p];
    if (pr.rule != kRuleList || !pr.synapses()) continue;
    uint32_t* ls; ALLOC(ls, uint32_t, pr.n);
    uint32_t* lt; ALLOC(lt, uint32_t, pr.n);
    uint8_t* ld; ALLOC(ld, uint8_t, pr.n);
    HIPCHK(net, copy_sync(net, ls, pr.lsrc.data(), pr.n * 4, hipMemcpyHostToDevice));
    HIPCHK(net, copy_sync(net, lt, pr.ltgt.data(), pr.n * 4, hipMemcpyHostToDevice));
    HIPCHK(net, copy_sync(net, ld, pr.ldel.data(), pr.n, hipMemcpyHostToDevice));
    pd[p].lsrc = ls; pd[p].ltgt = lt; pd[p].ldel = ld;
    list_bufs.insert(list_bufs.end(), {ls, lt, ld});
  }
  // weight levels: thresholds, classes and listed levels, one table each
  std::vector<uint64_t> wthr_all;
  std::vector<uint16_t> lvl_all;
  std::vector<ProjW> pw(std::max<size_t>(1, pd.size()));
  std::vector<size_t> thr_off(pd.size(), 0), lvl_off(pd.size(), 0);
  for (size_t p = 0; p < pd.size(); ++p) {
    const HostProj& pr = net->projs[p];
    memset(&pw[p], 0, sizeof(ProjW));
    if (pr.wlev.empty() || !pr.synapses()) continue;
    pw[p].levels = (uint32_t)pr.wlev.size();
    pw[p].pop0 = wpop0[p];
    thr_off[p] = wthr_all.size();
    wthr_all.insert(wthr_all.end(), pr.wthr.begin(), pr.wthr.end());
    lvl_off[p] = lvl_all.size();
    lvl_all.insert(lvl_all.end(), pr.lwl.begin(), pr.lwl.end());
  }
  uint64_t* d_wthr; ALLOC(d_wthr, uint64_t, std::max<size_t>(1, wthr_all.size()));
  uint16_t* d_wcls; ALLOC(d_wcls, uint16_t, std::max<size_t>(1, wcls.size()));
  uint16_t* d_lvl; ALLOC(d_lvl, uint16_t, std::max<size_t>(1, lvl_all.size()));
  ProjW* d_pw; ALLOC(d_pw, ProjW, pw.size());
  for (size_t p = 0; p < pd.size(); ++p) {
    if (!pw[p].levels) continue;
    pw[p].thr = d_wthr + thr_off[p];
    pw[p].cls = d_wcls + wcls_off[p];
    pw[p].lvl = d_lvl + lvl_off[p];
  }
  if (!wthr_all.empty())
    HIPCHK(net, copy_sync(net, d_wthr, wthr_all.data(), wthr_all.size() * 8, hipMemcpyHostToDevice));
  if (!wcls.empty()) HIPCHK(net, copy_sync(net, d_wcls, wcls.data(), wcls.size() * 2, hipMemcpyHostToDevice));
  if (!lvl_all.empty()) HIPCHK(net, copy_sync(net, d_lvl, lvl_all.data(), lvl_all.size() * 2, hipMemcpyHostToDevice));
  HIPCHK(net, copy_sync(net, d_pw, pw.data(), pw.size() * sizeof(ProjW), hipMemcpyHostToDevice));
  ALLOC(d_clsof, uint16_t, cls_of.size());
  ALLOC(d_popfirst, uint32_t, npop);
  std::vector<uint32_t> pf(npop);
  for (uint32_t k = 0; k < npop; ++k) pf[k] = net->pops[k].first;
  if (!pd.empty()) HIPCHK(net, hipMemcpyAsync(d_proj, pd.data(), pd.size() * sizeof(ProjDev), hipMemcpyHostToDevice, s));
  HIPCHK(net, hipMemcpyAsync(d_clsof, cls_of.data(), cls_of.size() * 2, hipMemcpyHostToDevice, s));
  HIPCHK(net, hipMemcpyAsync(d_popfirst, pf.data(), npop * 4, hipMemcpyHostToDevice, s));
  HIPCHK(net, hipMemsetAsync(d_cnt, 0, M * sizeof(uint32_t), s));
  HIPCHK(net, launch_gen_count(d_proj, (uint32_t)pd.size(), total_pairs, dmax_cfg, D1, d_cnt, s));
  HIPCHK(net, launch_scan_u32(d_cnt, M, d_off, d_tmp, s));
  HIPCHK(net, launch_masks(d_cnt, N, D1, d_mask, d_ng, s));
  HIPCHK(net, launch_scan_u64(d_ng, N, d_gp64, d_tmp, s));
  uint64_t G = 0, S = 0;
  HIPCHK(net, hipMemcpyAsync(&G, d_gp64 + N, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(net, hipMemcpyAsync(&S, d_off + M, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(net, hipStreamSynchronize(s));
  if (S != total_syn) return fail(net, SNN_E_DEVICE, "synapse count mismatch (%llu vs %llu)",
                                  (unsigned long long)S, (unsigned long long)total_syn);
  uint64_t* d_goff; ALLOC(d_goff, uint64_t, G + 1);
  HIPCHK(net, launch_grp_off(d_cnt, d_off, d_gp64, N, D1, d_goff, d_gp32, s));
  HIPCHK(net, hipMemcpyAsync(d_goff + G, &S, 8, hipMemcpyHostToDevice, s));
  uint32_t* d_pay; ALLOC(d_pay, uint32_t, std::max<uint64_t>(1, S));
  HIPCHK(net, launch_gen_scatter(d_proj, (uint32_t)pd.size(), total_pairs, dmax_cfg, D1, d_off, d_pay, d_clsof,
                                 d_pw, d_popfirst, npop, net->cls_bits, s));
  const uint32_t big_cap = 4096;
  uint64_t* d_big; ALLOC(d_big, uint64_t, big_cap);
  uint32_t* d_nbig; ALLOC(d_nbig, uint32_t, 1);
  HIPCHK(net, hipMemsetAsync(d_nbig, 0, 4, s));
  HIPCHK(net, launch_segsort(d_goff, G, d_pay, d_big, d_nbig, big_cap, s));
  uint32_t nbig = 0;
  HIPCHK(net, hipMemcpyAsync(&nbig, d_nbig, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(net, hipStreamSynchronize(s));
  if (nbig > big_cap) return fail(net, SNN_E_UNSUPPORTED, "too many connection groups above 16384 synapses");
  if (nbig) {  // rare: very large groups are sorted on the host
    std::vector<uint64_t> big(nbig);
    HIPCHK(net, copy_sync(net, big.data(), d_big, nbig * 8, hipMemcpyDeviceToHost));
    for (uint64_t gi : big) {
      uint64_t be[2];
      HIPCHK(net, copy_sync(net, be, d_goff + gi, 16, hipMemcpyDeviceToHost));
      std::vector<uint32_t> seg(be[1] - be[0]);
      HIPCHK(net, copy_sync(net, seg.data(), d_pay + be[0], seg.size() * 4, hipMemcpyDeviceToHost));
      std::sort(seg.begin(), seg.end());
      HIPCHK(net, copy_sync(net, d_pay + be[0], seg.data(), seg.size() * 4, hipMemcpyHostToDevice));
    }
  }
  dev_free(net, d_big); dev_free(net, d_nbig);
  dev_free(net, d_cnt); dev_free(net, d_off); dev_free(net, d_ng); dev_free(net, d_gp64); dev_free(net, d_tmp);
  dev_free(net, d_proj); dev_free(net, d_clsof); dev_free(net, d_popfirst);
  dev_free(net, d_wthr); dev_free(net, d_wcls); dev_free(net, d_lvl); dev_free(net, d_pw);
  for (void* b : list_bufs) dev_free(net, b);
  nd.src_mask = d_mask; nd.grp_ptr = d_gp32; nd.grp_off = d_goff; nd.payload = d_pay;
  nd.n_groups = G; nd.n_syn = S;
  net->n_groups = G; net->n_syn = S;

  // ---- plastic synapses: rules and tables, weights, the index by target ----
  nd.n_rules = 0;
  nd.n_plastic = 0;
  if (!rules.empty()) {
    uint8_t* d_crule; ALLOC(d_crule, uint8_t, ncls);
    HIPCHK(net, hipMemcpyAsync(d_crule, cls_rule.data(), ncls, hipMemcpyHostToDevice, s));
    StdpRule* d_rules; ALLOC(d_rules, StdpRule, rules.size());
    HIPCHK(net, hipMemcpyAsync(d_rules, rules.data(), rules.size() * sizeof(StdpRule), hipMemcpyHostToDevice, s));
    int64_t* d_F; ALLOC(d_F, int64_t, std::max<size_t>(1, stdp_F.size()));
    if (!stdp_F.empty())
      HIPCHK(net, hipMemcpyAsync(d_F, stdp_F.data(), stdp_F.size() * 8, hipMemcpyHostToDevice, s));
    nd.cls_rule = d_crule; nd.rules = d_rules; nd.stdp_F = d_F;
    nd.n_rules = (uint32_t)rules.size();
    int32_t* d_pw; ALLOC(d_pw, int32_t, std::max<uint64_t>(1, S));
    uint32_t* d_lpre; ALLOC(d_lpre, uint32_t, std::max<uint64_t>(1, S));
    uint8_t* d_am; ALLOC(d_am, uint8_t, std::max<uint64_t>(1, S));
    uint32_t* d_lpost; ALLOC(d_lpost, uint32_t, N);
    HIPCHK(net, hipMemsetAsync(d_lpost, 0, (size_t)N * 4, s));
    nd.pw = d_pw; nd.last_pre = d_lpre; nd.arr_m = d_am; nd.last_post = d_lpost;
    uint32_t* d_tc; ALLOC(d_tc, uint32_t, N);
    HIPCHK(net, hipMemsetAsync(d_tc, 0, (size_t)N * 4, s));
    HIPCHK(net, launch_stdp_count(nd, d_tc, s));
    uint64_t* d_tptr; ALLOC(d_tptr, uint64_t, (size_t)N + 1);
    uint64_t* d_stmp; ALLOC(d_stmp, uint64_t, scan_tmp_words(N));
    HIPCHK(net, launch_scan_u32(d_tc, N, d_tptr, d_stmp, s));
    uint64_t n_plastic = 0;
    HIPCHK(net, copy_sync(net, &n_plastic, d_tptr + N, 8, hipMemcpyDeviceToHost));
    uint64_t* d_cur; ALLOC(d_cur, uint64_t, (size_t)N + 1);
    HIPCHK(net, hipMemcpyAsync(d_cur, d_tptr, ((size_t)N + 1) * 8, hipMemcpyDeviceToDevice, s));
    uint64_t* d_tidx; ALLOC(d_tidx, uint64_t, std::max<uint64_t>(1, n_plastic));
    HIPCHK(net, launch_stdp_scatter(nd, d_cur, d_tidx, s));
    uint64_t* d_alist; ALLOC(d_alist, uint64_t, 2 * std::max<uint64_t>(1, n_plastic));
    uint32_t* d_acnt; ALLOC(d_acnt, uint32_t, 2);
    HIPCHK(net, hipMemsetAsync(d_acnt, 0, 8, s));
    HIPCHK(net, hipStreamSynchronize(s));
    dev_free(net, d_tc); dev_free(net, d_stmp); dev_free(net, d_cur);
    nd.tptr = d_tptr; nd.tidx = d_tidx; nd.arr_list = d_alist; nd.arr_cnt = d_acnt;
    nd.n_plastic = std::max<uint64_t>(1, n_plastic);
    if (n_plastic >= (1ull << 32)) return fail(net, SNN_E_UNSUPPORTED, "more than 2^32 plastic synapses");
  }

  // ---- state ----
  float* d_V; ALLOC(d_V, float, N);
  float* d_Ie; ALLOC(d_Ie, float, N);
  std::vector<float> hv(N), hie(N);
  for (uint32_t i = 0; i < N; ++i) {
    const HostPop& pp = net->pops[pop_of(net, i)];
    const double E_L = rest_of(net, i);  // a neuron rests at its own E_L
    const double V = std::isnan(net->V[i]) ? E_L : net->V[i];
    hv[i] = pp.adex() ? (float)V : (float)(V - E_L);
    hie[i] = (float)net->Ie[i];
  }
  HIPCHK(net, copy_sync(net, d_V, hv.data(), N * 4, hipMemcpyHostToDevice));
  HIPCHK(net, copy_sync(net, d_Ie, hie.data(), N * 4, hipMemcpyHostToDevice));
  nd.V = d_V; nd.Ie = d_Ie;
  std::vector<float> hp((size_t)N * P);
  if (net->has_lif) {
    int32_t* d_r; ALLOC(d_r, int32_t, N);
    HIPCHK(net, copy_sync(net, d_r, net->refr.data(), N * 4, hipMemcpyHostToDevice));
    nd.refr = d_r;
    float* d_I; ALLOC(d_I, float, (size_t)N * P);
    for (uint32_t i = 0; i < N; ++i)
      for (uint32_t q = 0; q < P; ++q) hp[(size_t)i * P + q] = (float)net->Isyn[(size_t)i * kMaxPorts + q];
    HIPCHK(net, copy_sync(net, d_I, hp.data(), hp.size() * 4, hipMemcpyHostToDevice));
    nd.Isyn = d_I;
  }
  if (net->has_adex) {
    float* d_w; ALLOC(d_w, float, N);
    float* d_h; ALLOC(d_h, float, N);
    float* d_g; ALLOC(d_g, float, (size_t)N * P);
    std::vector<float> hw(N), hh(N);
    for (uint32_t i = 0; i < N; ++i) { hw[i] = (float)net->w[i]; hh[i] = (float)net->h[i]; }
    for (uint32_t i = 0; i < N; ++i)
      for (uint32_t q = 0; q < P; ++q) hp[(size_t)i * P + q] = (float)net->g[(size_t)i * kMaxPorts + q];
    HIPCHK(net, copy_sync(net, d_w, hw.data(), N * 4, hipMemcpyHostToDevice));
    HIPCHK(net, copy_sync(net, d_h, hh.data(), N * 4, hipMemcpyHostToDevice));
    HIPCHK(net, copy_sync(net, d_g, hp.data(), hp.size() * 4, hipMemcpyHostToDevice));
    nd.w = d_w; nd.h = d_h; nd.g = d_g;
    if (net->has_beta) {
      float* d_gr; ALLOC(d_gr, float, (size_t)N * P);
      for (uint32_t i = 0; i < N; ++i)
        for (uint32_t q = 0; q < P; ++q) hp[(size_t)i * P + q] = (float)net->gr[(size_t)i * kMaxPorts + q];
      HIPCHK(net, copy_sync(net, d_gr, hp.data(), hp.size() * 4, hipMemcpyHostToDevice));
      nd.gr = d_gr;
    }
  }
  if (!net->gen_steps.empty()) {  // spike generators: emission steps by neuron
    std::vector<uint32_t> off((size_t)N + 1, 0);
    std::vector<uint64_t> steps;
    for (uint32_t i = 0; i < N; ++i) {
      auto it = net->gen_steps.find(i);
      if (it != net->gen_steps.end()) steps.insert(steps.end(), it->second.begin(), it->second.end());
      if (steps.size() >= (1ull << 32)) return fail(net, SNN_E_UNSUPPORTED, "more than 2^32 generator times");
      off[i + 1] = (uint32_t)steps.size();
    }
    if (steps.empty()) steps.push_back(0);
    uint32_t* d_off; ALLOC(d_off, uint32_t, (size_t)N + 1);
    uint32_t* d_next; ALLOC(d_next, uint32_t, N);
    uint64_t* d_st; ALLOC(d_st, uint64_t, steps.size());
    HIPCHK(net, copy_sync(net, d_off, off.data(), ((size_t)N + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(net, copy_sync(net, d_next, off.data(), (size_t)N * 4, hipMemcpyHostToDevice));
    HIPCHK(net, copy_sync(net, d_st, steps.data(), steps.size() * 8, hipMemcpyHostToDevice));
    nd.gen_off = d_off; nd.gen_next = d_next; nd.gen_step = d_st;
  } else {
    bool gen = false;
    for (const HostPop& p : net->pops) gen |= p.model == SNN_SPIKE_GENERATOR;
    if (gen) {  // generators without times: empty lists
      uint32_t* d_z; ALLOC(d_z, uint32_t, (size_t)2 * N + 1);
      HIPCHK(net, hipMemsetAsync(d_z, 0, ((size_t)2 * N + 1) * 4, s));
      uint64_t* d_st; ALLOC(d_st, uint64_t, 1);
      nd.gen_off = d_z; nd.gen_next = d_z + N + 1; nd.gen_step = d_st;
    }
  }
  int64_t* d_acc; ALLOC(d_acc, int64_t, (size_t)kInBuf * N * P);
  HIPCHK(net, hipMemsetAsync(d_acc, 0, (size_t)kInBuf * N * P * 8, s));
  nd.acc = d_acc;

  // ---- delivery mode: direct atomics or bins per target tile ----
  {
    uint32_t P2 = 1;
    while (P2 < P) P2 <<= 1;
    const uint32_t tmax = (uint32_t)kTileAccWords / P2;
    const bool forced = net->cfg.flags & SNN_F_DELIVERY_BINNED;
    if (net->cfg.tile_neurons > tmax)
      return fail(net, SNN_E_UNSUPPORTED, "tiles of %u neurons x %u ports exceed the %d LDS accumulators",
                  net->cfg.tile_neurons, P, kTileAccWords);
    // default tile: the largest the ports allow; networks with AdEx neurons
    // take smaller tiles while that keeps at least 128 tiles: a tile's update
    // lasts as long as its slowest neuron (a spike step), so more tiles run
    // more spike steps side by side (3e4 alpha-port neurons: 129 us per step
    // with 256-neuron tiles, 187 us with 2048)
    uint32_t T = net->cfg.tile_neurons ? net->cfg.tile_neurons : tmax;
    if (!net->cfg.tile_neurons && net->has_adex)
      while (T > 256 && ((uint64_t)N + T - 1) / T < 128) T >>= 1;
    uint32_t tsh = 0;
    while ((1u << tsh) < T) ++tsh;
    const uint64_t nt = ((uint64_t)N + T - 1) / T;
    std::vector<uint64_t> indeg(nt, 0);  // synapses onto each tile: the most events it can get in one step
    for (const HostProj& pr : net->projs) {
      if (!pr.synapses()) continue;
      // rules that draw targets at random: the mean with a margin (a tile
      // that receives more in one step spills the rest, exactly)
      const bool drawn = pr.rule == SNN_RULE_FIXED_OUTDEGREE || pr.rule == SNN_RULE_FIXED_TOTAL_NUMBER;
      const uint64_t a = pr.tgt_first, b = a + pr.tgt_n;
      for (uint64_t t = a / T; t <= (b - 1) / T; ++t) {
        const uint64_t lo = std::max<uint64_t>(a, t * T), hi = std::min<uint64_t>(b, (t + 1) * T);
        const double m = pr.per_target() * (double)(hi - lo);
        indeg[t] += drawn ? (uint64_t)std::ceil(1.25 * m + 64.0) : (uint64_t)m;
      }
    }
    uint64_t max_in = 0;
    for (uint64_t v : indeg) max_in = std::max(max_in, v);
    const bool fits = nt <= kMaxTiles && max_in < (1ull << 31);
    if (forced && !fits)
      return fail(net, SNN_E_UNSUPPORTED, "binned delivery: %llu tiles (at most %u) or %llu synapses onto one tile",
                  (unsigned long long)nt, kMaxTiles, (unsigned long long)max_in);
    net->tile_neurons = 0;
    // default: binned for large networks, whose steps carry millions of events
    // (10^6 AdEx neurons, 10^9 synapses: 190 us per step binned, 611 us direct;
    // 128 Brunel instances, 8.7e9 synapses: 1.5 ms binned, 6.7 ms direct), and
    // for every network with AdEx neurons, whose tile blocks feed the RK45 from
    // a work queue (3e4-3e5 alpha-port neurons: 1.5x faster than direct); direct
    // for smaller LIF networks, where the step is latency-bound (microcircuit
    // stand-in, 3e8 synapses: 15 us direct, 24 us binned at its best tile size)
    const bool want = forced || (!(net->cfg.flags & SNN_F_DELIVERY_DIRECT) &&
                                 (total_syn >= kBinnedMinSynapses || net->has_adex));
    if (fits && want) {
      std::vector<uint64_t> off(nt);
      std::vector<uint32_t> cap(nt);
      uint64_t tot = 0;
      for (uint64_t t = 0; t < nt; ++t) {
        const uint64_t want = net->cfg.bin_capacity ? (uint64_t)net->cfg.bin_capacity
                                                    : std::max<uint64_t>(1ull << 14, indeg[t] >> 3);
        cap[t] = (uint32_t)std::min<uint64_t>(indeg[t], want);
        tot += cap[t];
      }
      // bin positions are 32-bit: shrink the capacities if they would not fit
      // (events beyond a capacity are still delivered, by the spill path)
      const uint64_t shrink = tot / (1ull << 31) + 1;
      tot = 0;
      for (uint64_t t = 0; t < nt; ++t) {
        cap[t] = (uint32_t)(cap[t] / shrink);
        off[t] = tot;
        tot += cap[t];
      }
      uint32_t* d_bins; ALLOC(d_bins, uint32_t, std::max<uint64_t>(1, kInBuf * tot));
      uint32_t* d_bcnt; ALLOC(d_bcnt, uint32_t, kInBuf * nt);
      uint32_t* d_bovf; ALLOC(d_bovf, uint32_t, kInBuf * nt);
      uint64_t* d_boff; ALLOC(d_boff, uint64_t, nt);
      uint32_t* d_bcap; ALLOC(d_bcap, uint32_t, nt);
      HIPCHK(net, hipMemsetAsync(d_bcnt, 0, kInBuf * nt * 4, s));
      HIPCHK(net, hipMemsetAsync(d_bovf, 0, kInBuf * nt * 4, s));
      HIPCHK(net, hipMemcpyAsync(d_boff, off.data(), nt * 8, hipMemcpyHostToDevice, s));
      HIPCHK(net, hipMemcpyAsync(d_bcap, cap.data(), nt * 4, hipMemcpyHostToDevice, s));
      HIPCHK(net, hipStreamSynchronize(s));
      nd.bins = d_bins; nd.bin_cnt = d_bcnt; nd.ovf_flag = d_bovf; nd.bin_off = d_boff; nd.bin_cap = d_bcap;
      nd.n_tiles = (uint32_t)nt; nd.tile_shift = tsh; nd.bins_total = tot;
      net->tile_neurons = T;
      // a batch of many small instances: consecutive spikes of a step belong to
      // one instance, whose targets lie in a few tiles, so delivery blocks take
      // contiguous item ranges from a queue (128 Brunel instances, 733 tiles:
      // 1.26 -> 1.01 ms per step); a single network keeps the strided share,
      // which balances delays with different hit rates and group sizes
      const uint64_t ni = net->insts.size();
      nd.dlv_queue = (ni >= kQueueMinInstances && nt <= kQueueMaxTilesPerInstance * ni) ? 1u : 0u;
      // populations overlapping each tile, counted as the tile block finds
      // them (the last population starting at or before its first and last
      // neuron): the LIF-only step kernels keep them in an LDS window
      {
        std::vector<uint32_t> firsts(nd.npop);
        for (size_t k = 0; k < firsts.size(); ++k) firsts[k] = net->pops[k].first;
        auto find = [&](uint64_t gid) {
          return (uint64_t)(std::upper_bound(firsts.begin(), firsts.end(), (uint32_t)gid) - firsts.begin()) - 1;
        };
        uint64_t most = 0;
        for (uint64_t t = 0; t < nt; ++t) {
          const uint64_t lo = t << tsh, hi = std::min<uint64_t>(nd.N, (t + 1) << tsh) - 1;
          most = std::max(most, find(hi) - find(lo) + 1);
        }
        nd.tile_win = most <= kTilePopLds ? 1u : 0u;
      }
      // tile runs: the synapses of a group onto one tile are contiguous (groups
      // are sorted by target); where they are long on average, the count pass of
      // the binned flush reads one descriptor per run instead of every synapse
      const uint64_t G = nd.n_groups;
      if (!nd.n_rules && !net->has_adex && nd.tile_win && G) {
        uint32_t* d_rc; ALLOC(d_rc, uint32_t, G);
        uint32_t* d_tl; ALLOC(d_tl, uint32_t, 1);
        uint64_t* d_gr; ALLOC(d_gr, uint64_t, G + 1);
        uint64_t* d_rt; ALLOC(d_rt, uint64_t, scan_tmp_words(G));
        HIPCHK(net, hipMemsetAsync(d_tl, 0, 4, s));
        HIPCHK(net, launch_runs(false, nd.grp_off, G, nd.payload, nd.cls_bits, tsh, d_rc, nullptr, nullptr, d_tl, s));
        HIPCHK(net, launch_scan_u32(d_rc, G, d_gr, d_rt, s));
        uint64_t total = 0;
        uint32_t too_long = 0;
        HIPCHK(net, hipMemcpyAsync(&total, d_gr + G, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(net, hipMemcpyAsync(&too_long, d_tl, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(net, hipStreamSynchronize(s));
        dev_free(net, d_rc); dev_free(net, d_tl); dev_free(net, d_rt);
        if (!too_long && total && nd.n_syn >= kRunMinMean * total) {
          uint32_t* d_rd; ALLOC(d_rd, uint32_t, total);
          HIPCHK(net, launch_runs(true, nd.grp_off, G, nd.payload, nd.cls_bits, tsh, nullptr, d_gr, d_rd, nullptr, s));
          nd.grp_run = d_gr; nd.run_desc = d_rd; nd.tile_runs = 1;
        } else {
          dev_free(net, d_gr);
        }
      }
    }
  }

  // ---- spike buffers ----
  net->drain_steps = std::max<uint64_t>(kGraphSteps, std::min<uint64_t>(1000, ((1ull << 25) / N) / kGraphSteps * kGraphSteps));
  // the ring holds a drain window plus the two graphs launched before its
  // entries are copied out, at one spike per neuron and step
  net->log_cap = next_pow2((uint64_t)N * (net->drain_steps + 3 * kGraphSteps + 1));
  uint32_t* d_log; ALLOC(d_log, uint32_t, net->log_cap);
  uint64_t* d_rb; ALLOC(d_rb, uint64_t, nd.R);
  uint32_t* d_rc; ALLOC(d_rc, uint32_t, nd.R);
  uint64_t* d_cb; ALLOC(d_cb, uint64_t, kChunkRing);
  HIPCHK(net, hipMemsetAsync(d_rb, 0, nd.R * 8, s));
  HIPCHK(net, hipMemsetAsync(d_rc, 0, nd.R * 4, s));
  HIPCHK(net, hipMemsetAsync(d_cb, 0, kChunkRing * 8, s));
  nd.log = d_log; nd.ring_base = d_rb; nd.ring_cnt = d_rc;
  nd.chunk_base = d_cb; nd.log_mask = net->log_cap - 1; nd.chunk_ring = kChunkRing;

  // ---- selection / delivery ----
  // delivery blocks: binned delivery reserves bin space once per touched tile
  // and chunk, so it wants few, large chunks
  // (at least 256; more for networks whose steps carry many events, about one
  // block per 4 M synapses, at most 1024)
  nd.sel_grid = nd.n_tiles ? (uint32_t)std::min<uint64_t>(1024, std::max<uint64_t>(256, net->n_syn >> 22))
                           : std::min<uint32_t>(2048, std::max<uint32_t>(64, nd.nblk_upd));
  if (net->cfg.delivery_blocks) nd.sel_grid = net->cfg.delivery_blocks;
  const size_t nstat = (size_t)2 * nd.sel_grid;
  ALLOC(nd.sel_stats, uint64_t, nstat);
  HIPCHK(net, hipMemsetAsync(nd.sel_stats, 0, nstat * 8, s));
  ALLOC(nd.recent, SpikeRec, (size_t)nd.R * N);
  ALLOC(nd.blk_stats, uint64_t, (size_t)kBlkStats * nd.nblk_upd);
  HIPCHK(net, hipMemsetAsync(nd.blk_stats, 0, (size_t)kBlkStats * nd.nblk_upd * 8, s));
  ALLOC(nd.ctrl, Ctrl, 1);
  HIPCHK(net, hipMemsetAsync(nd.ctrl, 0, sizeof(Ctrl), s));
  net->pinned_words = 0;
  HIPCHK(net, hipHostMalloc((void**)&net->pin_cb, kChunkRing * 8, hipHostMallocDefault));
  HIPCHK(net, hipHostMalloc((void**)&net->pin_rc, (size_t)nd.R * 4, hipHostMallocDefault));
  HIPCHK(net, hipHostMalloc((void**)&net->pin_ctrl, sizeof(Ctrl), hipHostMallocDefault));
  HIPCHK(net, hipEventCreateWithFlags(&net->ev_drain, hipEventDisableTiming));
  net->dj = snn_net::Drain();
  if (net->nch) {  // multimeter channels: the address of each recorded value
    std::vector<const float*> addr(net->nch);
    for (const snn_net::Meter& m : net->meters) {
      const float* base = nullptr;
      size_t stride = 1, off = 0;
      switch (m.var) {
        case SNN_V_M: base = nd.V; break;
        case SNN_V_W: base = nd.w; break;
        case SNN_V_H: base = nd.h; break;
        case SNN_V_G: base = nd.g; stride = P; off = m.port; break;
        case SNN_V_G_RISE: base = nd.gr; stride = P; off = m.port; break;
        default: base = nd.Isyn; stride = P; off = m.port; break;
      }
      if (!base || (stride > 1 && m.port >= P))
        return fail(net, SNN_E_INVALID, "a multimeter records a variable this network does not have");
      for (size_t j = 0; j < m.gids.size(); ++j) addr[m.ch0 + j] = base + (size_t)m.gids[j] * stride + off;
    }
    ALLOC(net->d_addr, const float*, net->nch);
    ALLOC(net->d_mbuf, float, (size_t)kGraphSteps * net->nch);
    HIPCHK(net, copy_sync(net, net->d_addr, addr.data(), addr.size() * sizeof(float*), hipMemcpyHostToDevice));
    net->h_mbuf.resize((size_t)kGraphSteps * net->nch);
  }
  HIPCHK(net, hipStreamSynchronize(s));
#undef ALLOC
  net->built = true;
  net->cur_step = net->drained_step = 0;
  st = build_graphs(net);
  if (st) return st;
  net->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return leave(net);
}

}  // namespace

extern "C" {

snn_status snn_simulate_steps(snn_net* net, uint64_t steps) {
  if (!net) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "simulate before snn_build");
  snn_status st = enter(net);
  if (st) return st;
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(net, hipEventRecord(net->ev_t0, net->stream));
  uint64_t left = steps;
  while (left > 0) {
    const uint64_t from = net->cur_step;
    // the longest captured loop that fits: kGraphSteps, then the binary digits of the rest
    size_t gi = 0;
    while (net->graphs[gi].first > left) ++gi;
    const uint32_t len = net->graphs[gi].first;
    HIPCHK(net, hipGraphLaunch(net->graphs[gi].second, net->stream));
    net->cur_step += len;
    left -= len;
    if (net->nch) {  // the replay's samples, before the next one overwrites the device window
      st = collect_samples(net, from, net->cur_step);
      if (st) return st;
    }
    // a pending drain stage is collected now: its copy sits before the graph
    // just launched, which keeps the device busy meanwhile
    if (net->dj.stage) {
      st = drain_advance(net);
      if (st) return st;
    }
    if (net->dj.stage == 0 && net->cur_step - net->drained_step >= net->drain_steps) {
      st = drain_start(net);
      if (st) return st;
    }
  }
  // One copy and one wait end the call: the device flags.  The raster of the
  // last steps stays on the device (its ring holds them) until it is read or
  // the next call's drain takes it.
  HIPCHK(net, hipEventRecord(net->ev_t1, net->stream));
  HIPCHK(net, hipMemcpyAsync(net->pin_ctrl, net->nd.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, net->stream));
  HIPCHK(net, hipStreamSynchronize(net->stream));
  {
    float ms = 0.f;
    net->last_dev_ms = (hipEventElapsedTime(&ms, net->ev_t0, net->ev_t1) == hipSuccess) ? (double)ms : 0.0;
  }
  net->sim_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  const uint32_t flags = net->pin_ctrl->overflow;
  if (flags) return fail(net, SNN_E_OVERFLOW, "device range check failed (flags 0x%x)", flags);
  return leave(net);
}

snn_status snn_profile_steps(snn_net* net, uint64_t steps, double* kernel_ms) {
  if (!net || !kernel_ms) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "profile before snn_build");
  snn_status st = enter(net);
  if (st) return st;
  hipEvent_t ev[2];
  for (auto& e : ev) HIPCHK(net, hipEventCreate(&e));
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t k = 0; k < steps; ++k) {
    HIPCHK(net, launch_step(net->nd, 0, net->stream, ev[0], ev[1]));
    HIPCHK(net, launch_stdp(net->nd, 0, net->stream));
    HIPCHK(net, launch_sample(net->d_addr, net->nch, net->d_mbuf, kGraphSteps, net->nd.ctrl, 0, net->stream));
    HIPCHK(net, launch_advance(net->nd.ctrl, 1, net->stream));
    HIPCHK(net, hipEventSynchronize(ev[1]));
    float ms = 0.f;
    HIPCHK(net, hipEventElapsedTime(&ms, ev[0], ev[1]));
    kernel_ms[0] += ms;
    net->cur_step += 1;
    st = collect_samples(net, net->cur_step - 1, net->cur_step);
    if (st) return st;
    if (net->cur_step - net->drained_step >= net->drain_steps || k + 1 == steps) {
      st = drain(net);
      if (st) return st;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  net->sim_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return leave(net);
}

snn_status snn_simulate(snn_net* net, double t_ms) {
  if (!net) return SNN_E_INVALID;
  if (!(t_ms >= 0)) return fail(net, SNN_E_INVALID, "negative time");
  return snn_simulate_steps(net, (uint64_t)floor(t_ms / net->cfg.dt_ms + 0.5));
}

snn_status snn_get_spikes(snn_net* net, uint64_t step_lo, uint64_t step_hi, uint64_t* step, uint32_t* gid,
                          uint32_t* mult, size_t cap, size_t* n_out) {
  if (!net || !n_out) return SNN_E_INVALID;
  net->err.clear();
  if (net->built && step_hi > net->drained_step) {  // the steps still on the device first
    snn_status st = enter(net);
    if (st) return st;
    if ((st = drain(net))) return st;
    if ((st = leave(net))) return st;
  }
  sort_raster(net);
  const auto lo = std::lower_bound(net->r_step.begin(), net->r_step.end(), step_lo);
  const auto hi = std::lower_bound(net->r_step.begin(), net->r_step.end(), step_hi);
  const size_t a = (size_t)(lo - net->r_step.begin()), b = (size_t)(hi - net->r_step.begin());
  const size_t n = (b > a) ? b - a : 0;
  *n_out = n;
  const size_t m = std::min(n, cap);
  for (size_t j = 0; j < m; ++j) {
    if (step) step[j] = net->r_step[a + j];
    if (gid) gid[j] = net->r_entry[a + j] & kGidMask;
    if (mult) mult[j] = net->r_entry[a + j] >> kMultShift;
  }
  return SNN_OK;
}

snn_status snn_get_counters(snn_net* net, snn_counters* out) {
  if (!net || !out) return SNN_E_INVALID;
  net->err.clear();
  if (net->released) {
    *out = net->final_ctr;
    return SNN_OK;
  }
  memset(out, 0, sizeof *out);
  out->n_neurons = net->N;
  out->build_ms = net->build_ms;
  out->simulate_ms = net->sim_ms;
  out->last_call_device_ms = net->last_dev_ms;
  if (!net->built) return SNN_OK;
  snn_status st = enter(net);
  if (st) return st;
  HIPCHK(net, hipStreamSynchronize(net->stream));
  Ctrl c;
  HIPCHK(net, copy_sync(net, &c, net->nd.ctrl, sizeof c, hipMemcpyDeviceToHost));
  std::vector<uint64_t> ss((size_t)2 * net->nd.sel_grid);
  HIPCHK(net, copy_sync(net, ss.data(), net->nd.sel_stats, ss.size() * 8, hipMemcpyDeviceToHost));
  for (size_t b = 0; b < ss.size() / 2; ++b) {
    out->pairs += ss[2 * b];
    out->events += ss[2 * b + 1];
  }
  std::vector<uint64_t> bs((size_t)kBlkStats * net->nd.nblk_upd);
  HIPCHK(net, copy_sync(net, bs.data(), net->nd.blk_stats, bs.size() * 8, hipMemcpyDeviceToHost));
  for (size_t b = 0; b < net->nd.nblk_upd; ++b) {
    const uint64_t* st = &bs[(size_t)kBlkStats * b];
    out->rk_accepted += st[0];
    out->rk_rejected += st[1];
    out->spikes += st[2];
    out->pairs += st[3];
    out->events += st[4];
  }
  out->steps = net->cur_step;
  out->n_synapses = net->n_syn;
  out->n_groups = net->n_groups;
  out->device_bytes = net->dev_bytes;
  out->overflow = c.overflow;
  out->max_delay_used = net->dmax_used;
  out->spill_events = c.spill_events;
  out->delivery = net->tile_neurons ? 2u : 1u;
  out->tile_neurons = net->tile_neurons;
  out->delivery_blocks = net->nd.sel_grid;
  out->delivery_queue = net->nd.dlv_queue;
  out->tile_runs = net->nd.tile_runs;
  out->tile_window = net->nd.tile_win;
  return leave(net);
}

snn_status snn_get_input(snn_net* net, uint32_t first, uint32_t n, uint32_t port, int64_t* out) {
  if (!net || !out) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "not built");
  if ((uint64_t)first + n > net->N || port >= net->P) return fail(net, SNN_E_INVALID, "bad range");
  snn_status st = enter(net);
  if (st) return st;
  HIPCHK(net, hipStreamSynchronize(net->stream));
  const uint32_t buf = (uint32_t)(net->cur_step % kInBuf);
  const int64_t* base = net->nd.acc + (size_t)buf * net->N * net->P;
  if (!net->nd.n_tiles || n == 0) {
    if (n) HIPCHK(net, copy2d_sync(net, out, 8, base + (size_t)first * net->P + port, net->P * 8, 8, n, hipMemcpyDeviceToHost));
    return leave(net);
  }
  // binned: the spilled part (acc) plus the entries waiting in the tiles' bins
  int64_t* d = dalloc<int64_t>(net, n);
  if (!d) return fail(net, SNN_E_NOMEM, "allocation failed");
  hipError_t e = hipMemcpy2DAsync(d, 8, base + (size_t)first * net->P + port, net->P * 8, 8, n,
                                  hipMemcpyDeviceToDevice, net->stream);
  if (e == hipSuccess) e = launch_pending_input(net->nd, buf, first, n, port, d, net->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e == hipSuccess) e = copy_sync(net, out, d, (size_t)n * 8, hipMemcpyDeviceToHost);
  dev_free(net, d);
  if (e != hipSuccess) return fail(net, SNN_E_DEVICE, "input readback: %s", hipGetErrorString(e));
  return leave(net);
}

snn_status snn_get_input_noalloc(snn_net* net, uint32_t first, uint32_t n, uint32_t port, int64_t* out) {
  if (!net || !out) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "not built");
  if ((uint64_t)first + n > net->N || port >= net->P) return fail(net, SNN_E_INVALID, "bad range");
  if (n > kNoAllocInputMax)
    return fail(net, SNN_E_INVALID, "%u neurons: at most %u per call of the allocation-free readback", n,
                kNoAllocInputMax);
  int64_t* ws = nullptr;  // the device address of the workspace, resolved when the network was created
  HIPCHK(net, input_workspace(net->device, false, &ws));
  if (!ws) return fail(net, SNN_E_DEVICE, "readback workspace not available on device %d", net->device);
  snn_status st = enter(net);
  if (st) return st;
  if (n == 0) return leave(net);
  const uint32_t buf = (uint32_t)(net->cur_step % kInBuf);
  const int64_t* src = net->nd.acc + (size_t)buf * net->N * net->P + (size_t)first * net->P + port;
  if (!net->nd.n_tiles) {  // direct delivery: the accumulators hold the whole input
    HIPCHK(net, copy2d_sync(net, out, 8, src, net->P * 8, 8, n, hipMemcpyDeviceToHost));
    return leave(net);
  }
  // binned: the spilled part overwrites ws[0, n), then the bin entries are added
  HIPCHK(net, hipMemcpy2DAsync(ws, 8, src, net->P * 8, 8, n, hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(net, launch_pending_input(net->nd, buf, first, n, port, ws, net->stream));
  HIPCHK(net, copy_sync(net, out, ws, (size_t)n * 8, hipMemcpyDeviceToHost));
  return leave(net);
}

snn_status snn_get_shift(snn_net* net, uint32_t gid, uint32_t port, int32_t* shift) {
  if (!net || !shift) return SNN_E_INVALID;
  if (!net->built) return fail(net, SNN_E_STATE, "not built");
  if (gid >= net->N || port >= net->P) return fail(net, SNN_E_INVALID, "bad gid or port");
  *shift = net->shift[(size_t)pop_of(net, gid) * net->P + port];
  return SNN_OK;
}

snn_status snn_poisson_counts(snn_net* net, uint64_t step, uint32_t first, uint32_t n, uint32_t* k) {
  if (!net || !k) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "not built");
  if ((uint64_t)first + n > net->N) return fail(net, SNN_E_INVALID, "bad range");
  snn_status st = enter(net);
  if (st) return st;
  uint32_t* d = dalloc<uint32_t>(net, std::max<uint32_t>(1, n));
  if (!d) return fail(net, SNN_E_NOMEM, "allocation failed");
  hipError_t e = launch_poisson_counts(net->nd, step, first, n, d, net->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e == hipSuccess) e = copy_sync(net, k, d, (size_t)n * 4, hipMemcpyDeviceToHost);
  dev_free(net, d);
  if (e != hipSuccess) return fail(net, SNN_E_DEVICE, "poisson counts: %s", hipGetErrorString(e));
  return leave(net);
}

snn_status snn_export_synapses(snn_net* net, uint32_t* src, uint32_t* delay, uint32_t* tgt, uint32_t* port,
                               int64_t* wq, size_t* n_syn) {
  if (!net || !n_syn) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "not built");
  const size_t capn = *n_syn;
  *n_syn = net->n_syn;
  if (capn < net->n_syn || !src || !delay || !tgt || !port || !wq) return SNN_OK;
  snn_status st = enter(net);
  if (st) return st;
  HIPCHK(net, hipStreamSynchronize(net->stream));
  const uint32_t N = net->N;
  std::vector<uint64_t> mask(N), goff(net->n_groups + 1);
  std::vector<uint32_t> gp((size_t)N + 1), pay(net->n_syn);
  HIPCHK(net, copy_sync(net, mask.data(), net->nd.src_mask, (size_t)N * 8, hipMemcpyDeviceToHost));
  HIPCHK(net, copy_sync(net, gp.data(), net->nd.grp_ptr, ((size_t)N + 1) * 4, hipMemcpyDeviceToHost));
  HIPCHK(net, copy_sync(net, goff.data(), net->nd.grp_off, (net->n_groups + 1) * 8, hipMemcpyDeviceToHost));
  if (net->n_syn) HIPCHK(net, copy_sync(net, pay.data(), net->nd.payload, net->n_syn * 4, hipMemcpyDeviceToHost));
  size_t e = 0;
  for (uint32_t s = 0; s < N; ++s) {
    uint64_t m = mask[s];
    uint32_t g = gp[s];
    for (uint32_t d = 1; d < 64; ++d) {
      if (!((m >> d) & 1ull)) continue;
      for (uint64_t q = goff[g]; q < goff[g + 1]; ++q, ++e) {
        const uint32_t pl = pay[q];
        const uint32_t cls = pl & ((1u << net->cls_bits) - 1u);
        src[e] = s; delay[e] = d; tgt[e] = pl >> net->cls_bits;
        port[e] = net->cls_port[cls];
        wq[e] = net->cls_wq[cls];
      }
      ++g;
    }
    if (g != gp[s + 1]) return fail(net, SNN_E_DEVICE, "group table inconsistent at source %u", s);
  }
  if (e != net->n_syn) return fail(net, SNN_E_DEVICE, "exported %zu of %llu synapses", e, (unsigned long long)net->n_syn);
  return leave(net);
}

snn_status snn_get_weights(snn_net* net, int64_t* wq, size_t* n_syn) {
  if (!net || !n_syn) return SNN_E_INVALID;
  net->err.clear();
  if (!net->built) return fail(net, SNN_E_STATE, "not built");
  const size_t capn = *n_syn;
  *n_syn = net->n_syn;
  if (capn < net->n_syn || !wq) return SNN_OK;
  snn_status st = enter(net);
  if (st) return st;
  std::vector<uint32_t> pay(net->n_syn);
  if (net->n_syn) HIPCHK(net, copy_sync(net, pay.data(), net->nd.payload, net->n_syn * 4, hipMemcpyDeviceToHost));
  std::vector<int32_t> pw;
  if (net->nd.n_rules) {
    pw.resize(net->n_syn);
    HIPCHK(net, copy_sync(net, pw.data(), net->nd.pw, net->n_syn * 4, hipMemcpyDeviceToHost));
  }
  const uint32_t cls_mask = (1u << net->cls_bits) - 1u;
  for (uint64_t j = 0; j < net->n_syn; ++j) {  // CSR position order is the canonical order
    const uint32_t cls = pay[j] & cls_mask;
    wq[j] = (!pw.empty() && net->cls_rule[cls]) ? (int64_t)pw[j] : net->cls_wq[cls];
  }
  return leave(net);
}

}  // extern "C"

namespace {

snn_status record_graph(snn_net* net, uint32_t steps, hipGraphExec_t* out) {
  hipGraph_t g;
  HIPCHK(net, hipStreamBeginCapture(net->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (uint32_t r = 0; r < steps && e == hipSuccess; ++r) {
    e = launch_step(net->nd, r, net->stream);
    if (e == hipSuccess) e = launch_stdp(net->nd, r, net->stream);
    if (e == hipSuccess) e = launch_sample(net->d_addr, net->nch, net->d_mbuf, kGraphSteps, net->nd.ctrl, r, net->stream);
  }
  if (e == hipSuccess) e = launch_advance(net->nd.ctrl, steps, net->stream);
  hipError_t e2 = hipStreamEndCapture(net->stream, &g);
  if (e != hipSuccess) return fail(net, SNN_E_DEVICE, "capture: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(net, SNN_E_DEVICE, "end capture: %s", hipGetErrorString(e2));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(net, SNN_E_DEVICE, "instantiate: %s", hipGetErrorString(e));
  return SNN_OK;
}

// Samples due in steps [from, to) (at most kGraphSteps of them, the device
// window) copied from the device and appended to their meters.
snn_status collect_samples(snn_net* net, uint64_t from, uint64_t to) {
  if (!net->nch || to <= from) return SNN_OK;
  HIPCHK(net, copy_sync(net, net->h_mbuf.data(), net->d_mbuf, net->h_mbuf.size() * sizeof(float),
                        hipMemcpyDeviceToHost));
  for (snn_net::Meter& m : net->meters) {
    for (uint64_t n = from; n < to; ++n) {
      if ((n + 1) % m.interval) continue;
      const float* row = net->h_mbuf.data() + (size_t)(n % kGraphSteps) * net->nch + m.ch0;
      m.steps.push_back(n);
      for (size_t j = 0; j < m.gids.size(); ++j) {
        double v = row[j];
        if (m.var == SNN_V_M) v = from_device_state(net, SNN_V_M, m.gids[j], row[j]);
        m.values.push_back(v);
      }
    }
  }
  return SNN_OK;
}

snn_status build_graphs(snn_net* net) {
  uint32_t lens[16], n = 0;
  lens[n++] = kGraphSteps;
  for (uint32_t len = 1u << 6; len >= 1; len >>= 1)
    if (len < kGraphSteps) lens[n++] = len;
  for (uint32_t i = 0; i < n; ++i) {
    hipGraphExec_t gx = nullptr;
    snn_status st = record_graph(net, lens[i], &gx);
    if (st) return st;
    net->graphs.push_back({lens[i], gx});
  }
  return SNN_OK;
}

// Order the entries drained since the last read by gid within each step
// (steps are independent: large rasters are split over the host's cores).
void sort_raster(snn_net* net) {
  const size_t n = net->r_entry.size(), lo = net->r_sorted;
  if (lo >= n) return;
  auto sort_steps = [net](size_t a, size_t b) {  // [a, b) starts and ends on step boundaries
    size_t i = a;
    while (i < b) {
      size_t j = i + 1;
      while (j < b && net->r_step[j] == net->r_step[i]) ++j;
      std::sort(net->r_entry.begin() + (long)i, net->r_entry.begin() + (long)j,
                [](uint32_t x, uint32_t y) { return (x & kGidMask) < (y & kGidMask); });
      i = j;
    }
  };
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n - lo < (1u << 20) || hw == 1) {
    sort_steps(lo, n);
  } else {
    std::vector<size_t> cut{lo};
    for (unsigned t = 1; t < hw; ++t) {
      size_t c = lo + (n - lo) * t / hw;
      while (c < n && c > cut.back() && net->r_step[c] == net->r_step[c - 1]) ++c;  // to a step boundary
      cut.push_back(std::max(c, cut.back()));
    }
    cut.push_back(n);
    std::vector<std::thread> th;
    for (size_t t = 0; t + 1 < cut.size(); ++t)
      if (cut[t + 1] > cut[t]) th.emplace_back(sort_steps, cut[t], cut[t + 1]);
    for (auto& x : th) x.join();
  }
  net->r_sorted = n;
}

// Drain stage 0 -> 1: copy the per-step ring positions and counts of the
// steps [drained_step, cur_step) to pinned memory behind the launched work.
snn_status drain_start(snn_net* net) {
  snn_net::Drain& d = net->dj;
  d.a = net->drained_step;
  d.b = net->cur_step;
  net->drained_step = d.b;
  if (d.b <= d.a || (net->cfg.flags & SNN_F_NO_SPIKE_RECORD)) return SNN_OK;
  const NetDev& nd = net->nd;
  HIPCHK(net, hipMemcpyAsync(net->pin_cb, nd.chunk_base, kChunkRing * 8, hipMemcpyDeviceToHost, net->stream));
  HIPCHK(net, hipMemcpyAsync(net->pin_rc, nd.ring_cnt, (size_t)nd.R * 4, hipMemcpyDeviceToHost, net->stream));
  HIPCHK(net, hipEventRecord(net->ev_drain, net->stream));
  d.stage = 1;
  return SNN_OK;
}

// Drain stage 1 -> 2 (positions known: copy the window's ring entries to the
// pinned staging buffer) or 2 -> 0 (append them to the host raster).  Waits
// for the stage's copy.
snn_status drain_advance(snn_net* net) {
  snn_net::Drain& d = net->dj;
  const NetDev& nd = net->nd;
  if (d.stage == 0) return SNN_OK;
  HIPCHK(net, hipEventSynchronize(net->ev_drain));
  if (d.stage == 1) {
    const uint64_t base_a = net->pin_cb[d.a % kChunkRing];
    const uint64_t end = net->pin_cb[(d.b - 1) % kChunkRing] + net->pin_rc[(d.b - 1) % nd.R];
    d.total = end - base_a;
    if (d.total > net->log_cap) return fail(net, SNN_E_OVERFLOW, "spike ring overrun");
    d.base.resize(d.b - d.a + 1);
    for (uint64_t n = d.a; n < d.b; ++n) d.base[n - d.a] = net->pin_cb[n % kChunkRing] - base_a;
    d.base[d.b - d.a] = d.total;
    if (d.total > net->pinned_words) {  // no copy is in flight into the staging buffer now
      if (net->pinned) HIPCHK(net, hipHostFree(net->pinned));
      net->pinned = nullptr;
      const size_t words = std::max<size_t>(d.total, 2 * net->pinned_words);
      HIPCHK(net, hipHostMalloc((void**)&net->pinned, words * 4, hipHostMallocDefault));
      net->pinned_words = words;
    }
    const uint64_t p0 = base_a & nd.log_mask;
    const uint64_t first_part = std::min<uint64_t>(d.total, net->log_cap - p0);
    if (first_part)
      HIPCHK(net, hipMemcpyAsync(net->pinned, nd.log + p0, first_part * 4, hipMemcpyDeviceToHost, net->stream));
    if (d.total > first_part)
      HIPCHK(net, hipMemcpyAsync(net->pinned + first_part, nd.log, (d.total - first_part) * 4, hipMemcpyDeviceToHost,
                                 net->stream));
    HIPCHK(net, hipEventRecord(net->ev_drain, net->stream));
    d.stage = 2;
    return SNN_OK;
  }
  const size_t need = net->r_step.size() + d.total;
  if (need > net->r_step.capacity()) {  // geometric growth: an exact reserve per window copies the raster each time
    net->r_step.reserve(std::max(need, 2 * net->r_step.capacity()));
    net->r_entry.reserve(std::max(need, 2 * net->r_entry.capacity()));
  }
  for (uint64_t n = d.a; n < d.b; ++n)
    for (uint64_t q = d.base[n - d.a]; q < d.base[n - d.a + 1]; ++q) {
      net->r_step.push_back(n);
      net->r_entry.push_back(net->pinned[q]);
    }
  d.stage = 0;
  return SNN_OK;
}

// Everything simulated so far into the host raster (waits for the device).
snn_status drain(snn_net* net) {
  snn_status st;
  while (net->dj.stage)
    if ((st = drain_advance(net))) return st;
  if (net->cur_step > net->drained_step) {
    if ((st = drain_start(net))) return st;
    while (net->dj.stage)
      if ((st = drain_advance(net))) return st;
  }
  return SNN_OK;
}

}  // namespace

// ---- hooks for the request server (snn_server.cpp) ----
namespace snn {

void net_allocator(const snn_net* net, snn_device* dev, bool* have_dev) {
  *dev = net->dev;
  *have_dev = net->have_dev;
}

void net_set_allocator(snn_net* net, const snn_device& dev, bool have_dev) {
  net->dev = dev;
  net->have_dev = have_dev;
}

int net_device(const snn_net* net) { return net->device; }

bool net_is_fresh(const snn_net* net) { return !net->built && !net->released && net->N > 0; }

uint64_t net_planned_synapses(const snn_net* net) {
  uint64_t s = 0;
  for (const HostProj& pr : net->projs) s += pr.synapses();
  return s;
}

}  // namespace snn
