// kernels_step.hip -- one simulation step on the device, one kernel launch.
//
// Step n (Golosio et al., Sec. 2.1 and 2.2): every neuron folds the integer
// input delivered for step n (plus its Poisson count) into fp32, advances its
// dynamics over dt and, if it fires, is appended to its sub-block's spike
// list (wave ballot + lane prefix + block prefix, gid order) and its delay-1
// group is delivered at once; in the same launch the delivery blocks take
// the spikes of steps n-1 .. n+1-Dmax whose delay d expires now to their
// delay-d connection group.  A spike reaches a group of delay d iff bit d of
// its source's delay mask is set; the group is found by a popcount of the
// lower bits (the groups of a source are ordered by delay), so there is no
// loop over the groups -- the role of the ordered connection-group index of
// Fig. 1.  Selected groups are scanned in LDS into one flat index space over
// their synapses; each synapse adds multiplicity x quantised weight to the
// int64 input of its (target, port) for step n+1.  Integer sums: the result
// does not depend on order.
//
// Two ways to form that sum:
//   direct: every synaptic event is one device-scope int64 atomic add into
//     acc[(n+1) & 1][target][port];
//   binned: the neurons are cut into tiles; an event becomes a 32-bit entry in
//     its target tile's bin (one device atomic per tile and chunk reserves the
//     space), and at step n+1 the tile's block sums the bin with LDS atomics
//     before updating the tile's neurons.
#include <hip/hip_ext.h>

#include <mutex>

#include "kernels.h"
#include "philox_dev.h"

namespace snn {

namespace {

constexpr int kB = 256;
constexpr uint32_t kRkMaxIter = 100000;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint32_t find_pop(const PopDev* pops, uint32_t npop, uint32_t gid) {
  uint32_t lo = 0, hi = npop;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (pops[mid].first <= gid) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// exclusive scan over the whole block (blockDim.x multiple of 64, <= 1024)
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t* lds, uint64_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t incl = wave_incl_scan(v);
  if (lane == 63) lds[wv] = incl;
  __syncthreads();
  uint64_t before = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    const uint64_t x = lds[i];
    if (i < wv) before += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return before + incl - v;
}

__device__ __forceinline__ uint64_t block_sum(uint64_t v, uint64_t* lds) {
  uint64_t tot;
  (void)block_excl_scan(v, lds, &tot);
  return tot;
}

__device__ __forceinline__ uint64_t block_max(uint64_t v, uint64_t* lds) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t t = __shfl_xor(v, o, 64);
    v = t > v ? t : v;
  }
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  uint64_t m = 0;
  for (int i = 0; i < nw; ++i) m = lds[i] > m ? lds[i] : m;
  __syncthreads();
  return m;
}

// Poisson count of neuron gid at step n: inverse CDF of a 32-bit uniform
// (top bits of Philox word 0 at counter (gid, n, POISSON, 0), gid counted
// inside the neuron's instance, key (instance seed, 0)).
__device__ __forceinline__ uint32_t poisson_draw(const uint64_t* thr, uint64_t seed, uint32_t gid, uint64_t n) {
  const U64x4 r = philox4x64_10(gid, n, kTagPoisson, 0, seed, 0);
  const uint64_t u = r.w[0] >> 32;
  uint32_t k = 0;
  while (k < kPoisKmax - 1 && u >= thr[k]) ++k;
  return k;
}

// ------------------------------------------------------------------ update
// Constants of a LIF neuron's exact propagation: its population's, or its
// own when the population's parameters are set per neuron (the synaptic
// decay P11 is always the population's).
struct LifK {
  float P22, P20, theta, y_reset;
  float P21[kMaxPorts];
  int32_t n_ref;
};

__device__ __forceinline__ LifK lif_consts(const NetDev& nd, const PopDev& pp, uint32_t i) {
  LifK k;
  if (pp.per_neuron) {
    const NeuronLif& c = nd.nlif[i];
    k.P22 = c.P22; k.P20 = c.P20; k.theta = c.theta; k.y_reset = c.y_reset; k.n_ref = c.n_ref;
#pragma unroll
    for (int p = 0; p < kMaxPorts; ++p) k.P21[p] = c.P21[p];
  } else {
    k.P22 = pp.P22; k.P20 = pp.P20; k.theta = pp.theta; k.y_reset = pp.y_reset; k.n_ref = pp.n_ref;
#pragma unroll
    for (int p = 0; p < kMaxPorts; ++p) k.P21[p] = pp.P21[p];
  }
  return k;
}

// LIF exact integration (Sec. 2.1; LIF and exponential-PSC equations of
// Sec. 2.3), y = V - E_L, fixed fp32 operation order without contraction.
__device__ __forceinline__ bool lif_delta_step(const LifK& k, float& y, int32_t& r, float Ie, float x) {
  if (r > 0) {
    r -= 1;  // refractory: held at reset, input discarded
  } else {
    const float t1 = __fmul_rn(k.P22, y);
    const float t2 = __fmul_rn(k.P20, Ie);
    y = __fadd_rn(__fadd_rn(t1, t2), x);
  }
  if (r == 0 && y >= k.theta) { y = k.y_reset; r = k.n_ref; return true; }
  return false;
}

__device__ __forceinline__ bool lif_exp_step(const PopDev& pp, const LifK& k, float& y, float* I, int32_t& r,
                                             float Ie, const float* x) {
  if (r == 0) {
    float v = __fmul_rn(k.P22, y);
    for (int p = 0; p < pp.n_ports; ++p) v = __fadd_rn(v, __fmul_rn(k.P21[p], I[p]));
    v = __fadd_rn(v, __fmul_rn(k.P20, Ie));
    y = v;
  } else {
    r -= 1;
  }
  for (int p = 0; p < pp.n_ports; ++p) I[p] = __fadd_rn(__fmul_rn(pp.P11[p], I[p]), x[p]);
  if (r == 0 && y >= k.theta) { y = k.y_reset; r = k.n_ref; return true; }
  return false;
}

// AdEx parameters of one neuron as the integrator uses them, held in
// registers for the whole step (the population record may sit behind a
// generic pointer that the compiler would otherwise reload every substep).
template <int P, bool kBeta>
struct AdexPar {
  float V_peak, g_L, gLDT_C, V_T, k_exp, E_L, inv_C, a, inv_tau_w, b, V_r;
  float dt, hmin, inv_eps;
  float E_rev[P], inv_tau_syn[P];
  float inv_tau_rise[kBeta ? P : 1];
};

// State variables of the integrator: V, w, the port conductances, and with
// beta ports their rising variables.
template <int P, bool kBeta>
constexpr int kAdexVars = kBeta ? 2 + 2 * P : 2 + P;

// The neuron constants of AdexPar from a population record or from a
// neuron's own record (both carry the same fields).
template <int P, bool kBeta, class Src>
__device__ __forceinline__ void adex_scalars(AdexPar<P, kBeta>& q, const Src& c, float dt) {
  q.V_peak = c.V_peak; q.g_L = c.g_L; q.V_T = c.V_T;
  q.gLDT_C = c.g_L * c.Delta_T * c.inv_C;
  q.k_exp = c.inv_Delta_T * 1.4426950408889634f;  // exp(x / Delta_T) = 2^(x k_exp)
  q.E_L = c.E_L; q.inv_C = c.inv_C; q.a = c.a; q.inv_tau_w = c.inv_tau_w; q.b = c.b; q.V_r = c.V_r;
  // smallest substep: the configured floor, but never below 2^-22 dt so that
  // t + h still advances in fp32
  q.hmin = fmaxf(c.rk_hmin, dt * 2.384185791015625e-7f);
  q.inv_eps = 1.f / c.rk_eps;
}

// AdexPar of neuron i of population pp.
template <int P, bool kBeta>
__device__ __forceinline__ AdexPar<P, kBeta> adex_par(const NetDev& nd, const PopDev& pp, uint32_t i) {
  AdexPar<P, kBeta> q;
  q.dt = pp.dt;
  if (pp.per_neuron) adex_scalars<P, kBeta>(q, nd.nadex[i], pp.dt);
  else adex_scalars<P, kBeta>(q, pp, pp.dt);
#pragma unroll
  for (int p = 0; p < P; ++p) { q.E_rev[p] = pp.E_rev[p]; q.inv_tau_syn[p] = pp.inv_tau_syn[p]; }
  if constexpr (kBeta) {
#pragma unroll
    for (int p = 0; p < P; ++p) q.inv_tau_rise[p] = pp.inv_tau_rise[p];
  }
  return q;
}

// AdEx with conductance synapses (Sec. 2.4, Table 2), right-hand side in
// fp32.  y = (V, w, g_0..g_{P-1}) with exponential conductances, dg/dt =
// -g / tau; with beta conductances (Sec. 2.1 example; alpha when the two
// times are equal) y continues with the rising variables r_0..r_{P-1}:
// dg/dt = r - g / tau_decay, dr/dt = -r / tau_rise (an exponential port in
// such a network keeps r = 0).  The synaptic current is sum g_p (V - E_p)
// entering with the sign that lets an excitatory conductance depolarise; the
// exponential uses min(V, V_peak).
template <int P, bool kBeta>
__device__ __forceinline__ void adex_rhs(const AdexPar<P, kBeta>& pp, float Ie, const float* y, float* dy) {
  const float V = y[0], w = y[1];
  const float Vc = fminf(V, pp.V_peak);
  const float d = V - pp.E_L;
  // the exponential is the longest chain: the other currents are summed beside
  // it and it enters last
  const float ex = __builtin_amdgcn_exp2f((Vc - pp.V_T) * pp.k_exp);
  float cur = Ie - w;
#pragma unroll
  for (int p = 0; p < P; ++p) cur = __builtin_fmaf(-y[2 + p], V - pp.E_rev[p], cur);
  cur = __builtin_fmaf(-pp.g_L, d, cur);
  dy[0] = __builtin_fmaf(pp.gLDT_C, ex, cur * pp.inv_C);
  dy[1] = __builtin_fmaf(pp.a, d, -w) * pp.inv_tau_w;
  if constexpr (kBeta) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      dy[2 + p] = __builtin_fmaf(-y[2 + p], pp.inv_tau_syn[p], y[2 + P + p]);
      dy[2 + P + p] = -y[2 + P + p] * pp.inv_tau_rise[p];
    }
  } else {
#pragma unroll
    for (int p = 0; p < P; ++p) dy[2 + p] = -y[2 + p] * pp.inv_tau_syn[p];
  }
}

// One attempted substep of the Cash-Karp embedded 5(4) pair with the
// step-size control of Press et al. (adaptive fifth-order Runge-Kutta,
// Sec. 2.1): relative error against |y| + |h dy/dt| + 1 (state units; a floor
// for variables at zero), shrink by 0.9 e^-1/4 (>= 0.1x) on failure, grow by
// 0.9 e^-1/5 (<= 5x) on success; the last substep lands on the step end.  A
// reset (V >= V_peak) is applied after every accepted substep.  t is the time
// reached inside the step, it the attempts so far, mult the resets.  Returns
// true when the step is complete (t = dt, or the attempt cap reached).  Each
// stage state is y plus one fma per earlier stage (h folded into the
// coefficients); the error ratio uses the hardware reciprocal (it only steers
// the step size).
template <int P, bool kBeta>
__device__ __forceinline__ bool adex_substep(const AdexPar<P, kBeta>& pp, float* y, float& h, float& t, uint32_t& it,
                                             uint32_t& mult, float Ie, uint32_t& nacc, uint32_t& nrej,
                                             bool& capped) {
  constexpr int NV = kAdexVars<P, kBeta>;
  const float dt = pp.dt;
  const float errcon = 1.89e-4f;  // (5 / 0.9)^-5
  const float hmin = pp.hmin;
  if (++it > kRkMaxIter) { capped = true; return true; }
  bool last = false;
  if (h >= dt - t) { h = dt - t; last = true; }
  // stage coefficients times h: each stage state is y plus one fma per
  // earlier stage, the newest last
  const float a21 = h * (1.f / 5.f);
  const float a31 = h * (3.f / 40.f), a32 = h * (9.f / 40.f);
  const float a41 = h * (3.f / 10.f), a42 = h * (-9.f / 10.f), a43 = h * (6.f / 5.f);
  const float a51 = h * (-11.f / 54.f), a52 = h * (5.f / 2.f), a53 = h * (-70.f / 27.f), a54 = h * (35.f / 27.f);
  const float a61 = h * (1631.f / 55296.f), a62 = h * (175.f / 512.f), a63 = h * (575.f / 13824.f),
              a64 = h * (44275.f / 110592.f), a65 = h * (253.f / 4096.f);
  const float b1 = 37.f / 378.f, b3 = 250.f / 621.f, b4 = 125.f / 594.f, b6 = 512.f / 1771.f;
  // error weights: fifth-order minus embedded fourth-order weights
  const float e1 = (float)(37.0 / 378.0 - 2825.0 / 27648.0), e3 = (float)(250.0 / 621.0 - 18575.0 / 48384.0),
              e4 = (float)(125.0 / 594.0 - 13525.0 / 55296.0), e5 = (float)(-277.0 / 14336.0),
              e6 = (float)(512.0 / 1771.0 - 0.25);
  float k1[NV], k2[NV], k3[NV], k4[NV], k5[NV], k6[NV], yt[NV];
  adex_rhs<P, kBeta>(pp, Ie, y, k1);
#pragma unroll
  for (int i = 0; i < NV; ++i) yt[i] = __builtin_fmaf(a21, k1[i], y[i]);
  adex_rhs<P, kBeta>(pp, Ie, yt, k2);
#pragma unroll
  for (int i = 0; i < NV; ++i) yt[i] = __builtin_fmaf(a32, k2[i], __builtin_fmaf(a31, k1[i], y[i]));
  adex_rhs<P, kBeta>(pp, Ie, yt, k3);
#pragma unroll
  for (int i = 0; i < NV; ++i)
    yt[i] = __builtin_fmaf(a43, k3[i], __builtin_fmaf(a42, k2[i], __builtin_fmaf(a41, k1[i], y[i])));
  adex_rhs<P, kBeta>(pp, Ie, yt, k4);
#pragma unroll
  for (int i = 0; i < NV; ++i)
    yt[i] = __builtin_fmaf(a54, k4[i],
                           __builtin_fmaf(a53, k3[i], __builtin_fmaf(a52, k2[i], __builtin_fmaf(a51, k1[i], y[i]))));
  adex_rhs<P, kBeta>(pp, Ie, yt, k5);
#pragma unroll
  for (int i = 0; i < NV; ++i)
    yt[i] = __builtin_fmaf(
        a65, k5[i],
        __builtin_fmaf(a64, k4[i],
                       __builtin_fmaf(a63, k3[i], __builtin_fmaf(a62, k2[i], __builtin_fmaf(a61, k1[i], y[i])))));
  adex_rhs<P, kBeta>(pp, Ie, yt, k6);
  float errmax = 0.f;
  float y5[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    y5[i] = __builtin_fmaf(
        h, __builtin_fmaf(b6, k6[i], __builtin_fmaf(b4, k4[i], __builtin_fmaf(b3, k3[i], b1 * k1[i]))), y[i]);
    const float err =
        h * __builtin_fmaf(e6, k6[i],
                           __builtin_fmaf(e5, k5[i], __builtin_fmaf(e4, k4[i], __builtin_fmaf(e3, k3[i], e1 * k1[i]))));
    const float scale = __builtin_fmaf(h, fabsf(k1[i]), fabsf(y[i])) + 1.f;  // h > 0
    errmax = fmaxf(errmax, fabsf(err) * __builtin_amdgcn_rcpf(scale));
  }
  errmax = errmax * pp.inv_eps;
  if (errmax > 1.f && h > hmin) {
    const float ht = 0.9f * h * __builtin_amdgcn_exp2f(-0.25f * __builtin_amdgcn_logf(errmax));
    h = fmaxf(ht, 0.1f * h);
    h = fmaxf(h, hmin);
    ++nrej;
    return false;
  }
  ++nacc;
  t = last ? dt : t + h;
#pragma unroll
  for (int i = 0; i < NV; ++i) y[i] = y5[i];
  const float hn =
      fmaxf((errmax > errcon) ? 0.9f * h * __builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf(errmax)) : 5.f * h, hmin);
  if (y[0] >= pp.V_peak) { y[0] = pp.V_r; y[1] += pp.b; ++mult; }
  h = hn;
  return !(t < dt);
}

// One dt of the AdEx model: substeps until the step end, h carried to the
// next step (at most dt).  Returns the number of resets.
template <int P, bool kBeta>
__device__ uint32_t adex_step(const AdexPar<P, kBeta>& pp, float* y, float& h, float Ie, uint32_t& nacc,
                              uint32_t& nrej, bool& capped) {
  const float dt = pp.dt;
  if (!(h > 0.f) || h > dt) h = dt;
  float t = 0.f;
  uint32_t it = 0, mult = 0;
  while (!adex_substep<P, kBeta>(pp, y, h, t, it, mult, Ie, nacc, nrej, capped)) {
  }
  if (h > dt) h = dt;
  return mult;
}

constexpr uint32_t kPopLds = 16;  // population tables up to this size are read from LDS
constexpr uint32_t kPoisLds = 8;  // Poisson threshold tables up to this count are read from LDS
constexpr int kSelChunk = 512;    // selected groups held in LDS at a time
constexpr uint32_t kClsLds = 256; // weight classes cached in LDS by direct delivery (more: global)
constexpr int kSelPerThread = kSelChunk / kB;
static_assert(kTilePopLds <= kPoisLds, "a tile window's Poisson tables fit the LDS table");
constexpr int kTileSubs = kTileAccWords / kB;  // most 256-neuron sub-blocks of a tile
constexpr uint32_t kHotCap = 256;
// Delays of at least this many steps are delivered by the delivery blocks
// (their spikes' records are complete when the step starts); delay-1 groups
// by the blocks that emit the spikes, within the step.
constexpr uint32_t kDlvMinDelay = 2;  // AdEx neurons of a tile queued ahead of the others

// LDS of the selection: the selected (source, delay-group) records of one
// chunk and their exclusive prefix of group sizes.
struct SelLds {
  uint64_t p_off[kSelChunk];
  uint64_t p_st[kSelChunk];
  uint32_t p_len[kSelChunk];
  uint32_t p_mult[kSelChunk];
  uint8_t p_buf[kSelChunk];  // direct delivery: input buffer of the pair's arrival step
  uint64_t red[kB / 64];
  uint64_t seg[66];
  uint32_t slot[66];
  uint32_t npair;
  uint64_t j0;  // delivery queue: first item of the block's current range
};

// direct delivery: weight classes cached for the atomic adds
struct DirectLds : SelLds {
  int64_t wq[kClsLds];
  uint32_t wp[kClsLds];
};

// binned delivery: events per target tile of the chunk, then each tile's
// reserved position in its bin
constexpr int kCidx = 1024;  // coarse index of a chunk's events
struct BinLds : SelLds {
  uint32_t tcnt[kMaxTiles];   // events per tile, then the write cursor
  uint32_t tbase[kMaxTiles];  // absolute bin index of the reserved range
  uint32_t tavail[kMaxTiles]; // entries of the range inside the bin's capacity
  uint16_t cidx[kCidx];       // the record holding event m << csh of the chunk
};

// LDS of a direct-delivery update block
struct UpdTables {
  PopDev spops[kPopLds];
  uint64_t sthr[kPoisLds * kPoisKmax];
};

struct UpdLds {
  uint32_t wcnt[kB / 64];
  uint64_t red[kB / 64];
  union {
    UpdTables t;  // population and Poisson tables, during the update
    DirectLds d;  // selection of the block's delay-1 groups, after it
  } u;
};
// the weight classes of DirectLds and its pair counter lie beyond the tables:
// the classes are loaded with the tables, the counter cleared while they are read
static_assert(offsetof(SelLds, npair) >= sizeof(UpdTables), "selection state must not overlap the update tables");

// LDS of a tile block: the tile's int64 input (dead after the update, then
// reused by the delay-1 binning), weight classes, population and Poisson tables
struct TileLds {
  union {
    int64_t acc[kTileAccWords];
    BinLds d1;
  } u;
  union {
    int64_t wq[kMaxClasses];      // weight of each class: summing the bin
    uint8_t mk[kTileAccWords];    // spike count of each neuron: after the update
  } c;
  uint8_t wp[kMaxClasses];
  PopDev spops[kTilePopLds];
  uint64_t sthr[kPoisLds * kPoisKmax];
  uint32_t wcnt[kTileSubs][kB / 64];
  uint64_t red[kB / 64];
  uint32_t emit;  // first position of the tile's spikes in the step
  // AdEx work queue: neurons at or above V_T + 4 Delta_T (about to spike: a
  // spike step takes ~100 substeps) first, from a short list, then the others
  // in index order
  uint32_t next, hq_next2, hq_n;
  uint16_t hq[kHotCap];
  uint32_t hot[kTileAccWords / 32];
};
static_assert(sizeof(BinLds) <= sizeof(int64_t) * kTileAccWords, "delay-1 binning reuses the tile input");

union StepLds {
  UpdLds upd;
  DirectLds dlv;
};

// binned delivery with tile runs: each selected group's first run and run
// count, and the exclusive prefix of the run counts
struct BinRunLds : BinLds {
  uint64_t p_run[kSelChunk];
  uint32_t p_nrun[kSelChunk];
  uint32_t q_st[kSelChunk];
};

union BinStepLds {
  TileLds tile;
  BinLds dlv;
};

union BinRunStepLds {
  TileLds tile;
  BinRunLds dlv;
};

__device__ __forceinline__ void dlv_load_classes(const NetDev& nd, DirectLds& sh) {
  const uint32_t nc = nd.n_classes < kClsLds ? nd.n_classes : kClsLds;
  for (uint32_t c = threadIdx.x; c < nc; c += kB) { sh.wq[c] = nd.cls_wq[c]; sh.wp[c] = nd.cls_port[c]; }
}

__device__ __forceinline__ void dlv_init(const NetDev& nd, DirectLds& sh) {
  dlv_load_classes(nd, sh);
  if (threadIdx.x == 0) sh.npair = 0;
}

__device__ __forceinline__ void dlv_init(const NetDev& nd, BinLds& sh) {
  for (uint32_t t = threadIdx.x; t < nd.n_tiles; t += kB) sh.tcnt[t] = 0;
  if (threadIdx.x == 0) sh.npair = 0;
}

// Selection of one in-flight spike for delay d (Sec. 2.2, Fig. 1): the spike
// reaches a connection group now iff its source has a group of delay d (bit d
// of the delay mask); that group's index among the source's groups, which are
// ordered by delay, is the number of lower bits set.
__device__ __forceinline__ uint32_t sel_add(SelLds& sh, uint64_t off, uint32_t len, uint32_t mult, uint32_t buf) {
  const uint32_t k = atomicAdd(&sh.npair, 1u);  // LDS counter; callers keep k < kSelChunk
  sh.p_off[k] = off;
  sh.p_len[k] = len;
  sh.p_mult[k] = mult;
  sh.p_buf[k] = (uint8_t)buf;
  return k;
}

__device__ __forceinline__ void dlv_probe(const NetDev& nd, SelLds& sh, uint32_t entry, uint32_t grp_ptr,
                                          uint64_t mask, uint32_t d, uint32_t buf) {
  if ((mask >> d) & 1ull) {
    const uint32_t g = grp_ptr + (uint32_t)__popcll(mask & ((1ull << d) - 1ull));
    const uint64_t off = nd.grp_off[g];
    sel_add(sh, off, (uint32_t)(nd.grp_off[g + 1] - off), entry >> kMultShift, buf);
  }
}

// the same, recording the group's tile runs
__device__ __forceinline__ void dlv_probe(const NetDev& nd, BinRunLds& sh, uint32_t entry, uint32_t grp_ptr,
                                          uint64_t mask, uint32_t d, uint32_t buf) {
  if ((mask >> d) & 1ull) {
    const uint32_t g = grp_ptr + (uint32_t)__popcll(mask & ((1ull << d) - 1ull));
    const uint64_t off = nd.grp_off[g], r0 = nd.grp_run[g];
    const uint32_t k = sel_add(sh, off, (uint32_t)(nd.grp_off[g + 1] - off), entry >> kMultShift, buf);
    sh.p_run[k] = r0;
    sh.p_nrun[k] = (uint32_t)(nd.grp_run[g + 1] - r0);
  }
}

// Exclusive prefix of the chunk's group sizes into p_st; returns the number
// of synapses (events) of the chunk.  Ends with a barrier.
__device__ __forceinline__ uint64_t sel_scan(SelLds& sh) {
  const uint32_t np = sh.npair;
  uint32_t L[kSelPerThread];
  uint64_t lsum = 0;
#pragma unroll
  for (int q = 0; q < kSelPerThread; ++q) {
    const uint32_t i = threadIdx.x * kSelPerThread + q;
    L[q] = (i < np) ? sh.p_len[i] : 0u;
    lsum += L[q];
  }
  uint64_t ev;
  uint64_t run = block_excl_scan(lsum, sh.red, &ev);
#pragma unroll
  for (int q = 0; q < kSelPerThread; ++q) {
    const uint32_t i = threadIdx.x * kSelPerThread + q;
    if (i < np) sh.p_st[i] = run;
    run += L[q];
  }
  __syncthreads();
  return ev;
}

// record holding flat event e: the last one with p_st <= e
__device__ __forceinline__ uint32_t sel_find(const SelLds& sh, uint32_t np, uint64_t e) {
  uint32_t lo = 0, hi = np;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sh.p_st[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// Record holding flat event e >= p_st[lo]: a lane's events grow by the block
// size between calls, which spans a few groups, so a short linear advance
// usually suffices; otherwise binary search over the rest.
__device__ __forceinline__ uint32_t sel_advance(const SelLds& sh, uint32_t np, uint32_t lo, uint64_t e) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (lo + 1 >= np || sh.p_st[lo + 1] > e) return lo;
    ++lo;
  }
  uint32_t hi = np;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sh.p_st[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// the same over a 32-bit prefix st[0 .. n)
__device__ __forceinline__ uint32_t st_advance(const uint32_t* st, uint32_t n, uint32_t lo, uint32_t e) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (lo + 1 >= n || st[lo + 1] > e) return lo;
    ++lo;
  }
  uint32_t hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (st[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

constexpr int kUnroll = 4;  // events per lane and round of a flat scan

// A spike of multiplicity mult reaching plastic synapse j (CSR position) at
// the step whose input buffer is buf (the arrival step's parity): its weight
// as it is now, times mult, is the input; the arrival is recorded for the
// plasticity kernel of this step (a synapse receives at most one spike per
// step, so the list never holds more than the plastic synapses).
__device__ __forceinline__ int64_t plastic_arrival(const NetDev& nd, uint64_t j, uint32_t mult, uint32_t buf) {
  nd.arr_m[j] = (uint8_t)mult;
  const uint32_t k = __hip_atomic_fetch_add(&nd.arr_cnt[buf], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  nd.arr_list[(size_t)buf * nd.n_plastic + k] = j;
  return (int64_t)nd.pw[j] * (int64_t)mult;
}

// Events e0, e0 + kB, ... (kUnroll of them, those below ev) of a lane: their
// records r[] and synapse words pl[], all loads issued before any is used.
__device__ __forceinline__ void sel_gather(const NetDev& nd, const SelLds& sh, uint32_t np, uint64_t ev,
                                           uint64_t e0, uint32_t& lo, uint32_t* r, uint32_t* pl) {
#pragma unroll
  for (int q = 0; q < kUnroll; ++q) {
    const uint64_t e = e0 + (uint64_t)q * kB;
    if (e < ev) lo = sel_advance(sh, np, lo, e);
    r[q] = lo;
  }
#pragma unroll
  for (int q = 0; q < kUnroll; ++q) {
    const uint64_t e = e0 + (uint64_t)q * kB;
    pl[q] = (e < ev) ? nd.payload[sh.p_off[r[q]] + (e - sh.p_st[r[q]])] : 0u;
  }
}

// Direct delivery of the chunk (flat scan of the synapses of its selected
// groups): every synapse is one item, consecutive lanes take consecutive
// synapses of a group, and each adds multiplicity x quantised weight to the
// int64 input of its (target, port) in the input buffer of the pair's arrival
// step with a device-scope atomic.  Called by the whole block after a barrier; returns
// the events delivered and resets the chunk.
__device__ uint64_t dlv_flush(const NetDev& nd, DirectLds& sh, uint32_t /*buf: per pair*/) {
  const uint32_t np = sh.npair;
  const uint64_t ev = sel_scan(sh);
  const size_t bstride = (size_t)nd.N * nd.P;
  const uint32_t cls_bits = nd.cls_bits, cls_mask = (1u << cls_bits) - 1u, P = nd.P;
  const bool plastic = nd.n_rules != 0;
  uint32_t lo = 0;
  for (uint64_t e0 = threadIdx.x; e0 < ev; e0 += kUnroll * kB) {  // independent events per lane and round
    uint32_t r[kUnroll], pl[kUnroll];
    sel_gather(nd, sh, np, ev, e0, lo, r, pl);
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const uint64_t e = e0 + (uint64_t)q * kB;
      if (e >= ev) break;
      const uint32_t cls = pl[q] & cls_mask;
      const bool in_lds = cls < kClsLds;
      int64_t v;
      if (plastic && nd.cls_rule[cls])
        v = plastic_arrival(nd, sh.p_off[r[q]] + (e - sh.p_st[r[q]]), sh.p_mult[r[q]], sh.p_buf[r[q]]);
      else
        v = (in_lds ? sh.wq[cls] : nd.cls_wq[cls]) * (int64_t)sh.p_mult[r[q]];
      const uint32_t port = in_lds ? sh.wp[cls] : nd.cls_port[cls];
      int64_t* acc = nd.acc + bstride * sh.p_buf[r[q]];
      __hip_atomic_fetch_add((unsigned long long*)&acc[(size_t)(pl[q] >> cls_bits) * P + port],
                             (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) sh.npair = 0;
  __syncthreads();
  return ev;
}

// An event that found its tile's bin full: added to the spill accumulator of
// its (target, port) and the tile flagged, so that the tile block of the next
// step adds the spill to the bin's sum.
__device__ __forceinline__ void bin_spill(const NetDev& nd, uint32_t buf, uint32_t tgt, uint32_t cls, uint32_t mult,
                                       uint32_t tile, uint32_t& spills) {
  const int64_t v = nd.cls_wq[cls] * (int64_t)mult;
  __hip_atomic_fetch_add((unsigned long long*)&nd.acc[((size_t)buf * nd.N + tgt) * nd.P + nd.cls_port[cls]],
                         (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  nd.ovf_flag[(size_t)buf * nd.n_tiles + tile] = 1u;
  ++spills;  // counted per lane, added to the step's total once per chunk
}

// A plastic synapse's event in binned delivery: its weight is read now (the
// plasticity kernel changes it before the tile sums its bin), so the event
// goes to the tile's spill accumulator, like an event that found its bin full.
__device__ __forceinline__ void bin_plastic(const NetDev& nd, uint32_t buf, uint64_t j, uint32_t tgt, uint32_t cls,
                                            uint32_t mult, uint32_t tile) {
  const int64_t v = plastic_arrival(nd, j, mult, buf);
  __hip_atomic_fetch_add((unsigned long long*)&nd.acc[((size_t)buf * nd.N + tgt) * nd.P + nd.cls_port[cls]],
                         (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  nd.ovf_flag[(size_t)buf * nd.n_tiles + tile] = 1u;
}

constexpr int kLaneRun = 4;  // consecutive events per lane and round of the binned flush

// Coarse index of the chunk's ev events over its np records: cidx[m] = the
// record holding event m << csh.  Returns csh; ends with a barrier.
__device__ __forceinline__ uint32_t build_cidx(BinLds& sh, uint32_t np, uint64_t ev) {
  uint32_t csh = 6;
  while (ev && ((ev - 1) >> csh) >= (uint64_t)kCidx) ++csh;
  for (uint32_t i = threadIdx.x; i < np; i += kB) {
    const uint64_t a = sh.p_st[i], b = a + sh.p_len[i];
    for (uint64_t m = (a + (1ull << csh) - 1) >> csh; (m << csh) < b; ++m) sh.cidx[m] = (uint16_t)i;
  }
  __syncthreads();
  return csh;
}

// Events e0 .. e0 + kLaneRun - 1 (those below ev) of a lane, consecutive
// synapses that mostly share a record: their records r[] and synapse words
// pl[], all loads issued before any is used.
__device__ __forceinline__ void lane_gather(const NetDev& nd, const BinLds& sh, uint32_t np, uint64_t ev,
                                            uint64_t e0, uint32_t csh, uint32_t* r, uint32_t* pl) {
  uint32_t lo = sel_advance(sh, np, sh.cidx[e0 >> csh], e0);
  uint64_t nxt = (lo + 1 < np) ? sh.p_st[lo + 1] : ~0ull;
#pragma unroll
  for (int q = 0; q < kLaneRun; ++q) {
    const uint64_t e = e0 + q;
    if (e < ev) {
      while (e >= nxt) {
        ++lo;
        nxt = (lo + 1 < np) ? sh.p_st[lo + 1] : ~0ull;
      }
    }
    r[q] = lo;
  }
#pragma unroll
  for (int q = 0; q < kLaneRun; ++q) {
    const uint64_t e = e0 + q;
    pl[q] = (e < ev) ? nd.payload[sh.p_off[r[q]] + (e - sh.p_st[r[q]])] : 0u;
  }
}

// Second half of the binned flush, called by every thread once its part of
// the count pass has added each touched tile's events to tcnt: one device
// atomic per tile reserves its range, then the chunk's synapses are written
// (as in the count pass, kLaneRun consecutive ones per lane), spills and
// plastic synapses aside.  Resets the chunk; returns ev.
__device__ __forceinline__ uint64_t bin_write(const NetDev& nd, BinLds& sh, uint32_t buf, uint32_t np, uint64_t ev,
                                              uint32_t csh, bool bad) {
  const uint32_t cls_bits = nd.cls_bits, cls_mask = (1u << cls_bits) - 1u;
  const uint32_t tsh = nd.tile_shift, lmask = (1u << tsh) - 1u, ntl = nd.n_tiles;
  const bool plastic = nd.n_rules != 0;
  constexpr uint32_t kNone = 0xffffffffu;
  const uint64_t step = (uint64_t)kB * kLaneRun;
  __syncthreads();
  uint32_t* cnt = nd.bin_cnt + (size_t)buf * ntl;
  for (uint32_t t = threadIdx.x; t < ntl; t += kB) {
    const uint32_t c = sh.tcnt[t];
    if (c) {
      const uint32_t base = __hip_atomic_fetch_add(&cnt[t], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t cap = nd.bin_cap[t];
      sh.tbase[t] = (uint32_t)nd.bin_off[t] + base;
      sh.tavail[t] = (base < cap) ? min(c, cap - base) : 0u;
      sh.tcnt[t] = 0;
    }
  }
  __syncthreads();
  uint32_t* bins = nd.bins + (size_t)buf * nd.bins_total;
  uint32_t spills = 0;
  for (uint64_t b0 = 0; b0 < ev; b0 += step) {
    const uint64_t e0 = b0 + (uint64_t)threadIdx.x * kLaneRun;
    if (e0 >= ev) break;
    uint32_t r[kLaneRun], pl[kLaneRun], tt[kLaneRun], slot[kLaneRun];
    lane_gather(nd, sh, np, ev, e0, csh, r, pl);
#pragma unroll
    for (int q = 0; q < kLaneRun; ++q) {
      uint32_t t = kNone;
      if (e0 + q < ev) {
        t = (pl[q] >> cls_bits) >> tsh;
        if (t >= ntl) {
          t = kNone;
        } else if (plastic && nd.cls_rule[pl[q] & cls_mask]) {
          bin_plastic(nd, buf, sh.p_off[r[q]] + (e0 + q - sh.p_st[r[q]]), pl[q] >> cls_bits, pl[q] & cls_mask,
                      sh.p_mult[r[q]], t);
          t = kNone;
        }
      }
      tt[q] = t;
    }
    // a run of consecutive events onto one tile: one LDS atomic, consecutive slots
#pragma unroll
    for (int q = 0; q < kLaneRun; ++q) {
      slot[q] = 0;
      if (tt[q] == kNone) continue;
      if (q > 0 && tt[q] == tt[q - 1]) {
        slot[q] = slot[q - 1] + 1;
      } else {
        uint32_t k = 1;
#pragma unroll
        for (int j = q + 1; j < kLaneRun; ++j) {
          if (tt[j] != tt[q]) break;
          ++k;
        }
        slot[q] = atomicAdd(&sh.tcnt[tt[q]], k);
      }
    }
#pragma unroll
    for (int q = 0; q < kLaneRun; ++q) {
      const uint32_t t = tt[q];
      if (t == kNone) continue;
      const uint32_t tgt = pl[q] >> cls_bits, cls = pl[q] & cls_mask, mult = sh.p_mult[r[q]];
      if (slot[q] < sh.tavail[t])
        bins[sh.tbase[t] + slot[q]] = ((tgt & lmask) << kBinLocalShift) | (mult << kBinMultShift) | cls;
      else
        bin_spill(nd, buf, tgt, cls, mult, t, spills);
    }
  }
  if (bad) atomicOr(&nd.ctrl->overflow, 4u);  // a target outside the tiles: reported, not written
  if (spills)
    __hip_atomic_fetch_add((unsigned long long*)&nd.ctrl->spill_events, (unsigned long long)spills, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < ntl; t += kB) sh.tcnt[t] = 0;
  if (threadIdx.x == 0) sh.npair = 0;
  __syncthreads();
  return ev;
}

// Binned delivery of the chunk: the same flat scan, but each event becomes
// one 32-bit entry (local target, multiplicity, weight class) in the bin of
// its target tile in input buffer buf; the tile block of that step sums its
// bin in LDS.  Two passes over the chunk's synapses: count the events per tile
// (LDS), reserve each tile's range with one device atomic, then write the
// entries.  A lane takes kLaneRun consecutive synapses per round (found from
// a coarse index of the chunk's events), and a run of them onto one tile
// takes one LDS atomic and consecutive entries.  Called by the whole block
// after a barrier; returns the events delivered and resets the chunk.
__device__ uint64_t dlv_flush(const NetDev& nd, BinLds& sh, uint32_t buf) {
  // every pair of a binned chunk arrives at the same step (buffer buf)
  const uint32_t np = sh.npair;
  const uint64_t ev = sel_scan(sh);
  const uint32_t csh = build_cidx(sh, np, ev);
  // target = pl >> cls_bits, tile = target >> tile_shift: two shifts, each
  // below 32 (their sum can exceed 31 when a tile is wider than the gid range)
  const uint32_t cls_bits = nd.cls_bits, cls_mask = (1u << cls_bits) - 1u;
  const uint32_t tsh = nd.tile_shift, ntl = nd.n_tiles;
  const bool plastic = nd.n_rules != 0;
  constexpr uint32_t kNone = 0xffffffffu;
  bool bad = false;
  const uint64_t step = (uint64_t)kB * kLaneRun;
  for (uint64_t b0 = 0; b0 < ev; b0 += step) {
    const uint64_t e0 = b0 + (uint64_t)threadIdx.x * kLaneRun;
    if (e0 >= ev) break;
    uint32_t r[kLaneRun], pl[kLaneRun];
    lane_gather(nd, sh, np, ev, e0, csh, r, pl);
    uint32_t tp = kNone, k = 0;
#pragma unroll
    for (int q = 0; q < kLaneRun; ++q) {
      uint32_t t = kNone;
      if (e0 + q < ev) {
        t = (pl[q] >> cls_bits) >> tsh;
        if (t >= ntl) { bad = true; t = kNone; }
        else if (plastic && nd.cls_rule[pl[q] & cls_mask]) t = kNone;  // plastic: no bin entry
      }
      if (t != tp) {
        if (k) atomicAdd(&sh.tcnt[tp], k);
        tp = t;
        k = 0;
      }
      if (t != kNone) ++k;
    }
    if (k) atomicAdd(&sh.tcnt[tp], k);
  }
  return bin_write(nd, sh, buf, np, ev, csh, bad);
}

// the same with the count pass over the chunk's tile runs (one 4-byte
// descriptor per run instead of every synapse word: networks whose groups put
// many synapses on each tile they touch, without plastic synapses)
__device__ __forceinline__ uint64_t dlv_flush(const NetDev& nd, BinRunLds& sh, uint32_t buf) {
  const uint32_t np = sh.npair;
  const uint64_t ev = sel_scan(sh);
  const uint32_t csh = build_cidx(sh, np, ev);
  uint64_t nr;
  {  // exclusive prefix of the groups' run counts
    uint32_t L[kSelPerThread];
    uint64_t lsum = 0;
#pragma unroll
    for (int q = 0; q < kSelPerThread; ++q) {
      const uint32_t i = threadIdx.x * kSelPerThread + q;
      L[q] = (i < np) ? sh.p_nrun[i] : 0u;
      lsum += L[q];
    }
    uint64_t run = block_excl_scan(lsum, sh.red, &nr);
#pragma unroll
    for (int q = 0; q < kSelPerThread; ++q) {
      const uint32_t i = threadIdx.x * kSelPerThread + q;
      if (i < np) sh.q_st[i] = (uint32_t)run;
      run += L[q];
    }
    __syncthreads();
  }
  const uint32_t ntl = nd.n_tiles;
  bool bad = false;
  uint32_t pr = 0;
  for (uint64_t r = threadIdx.x; r < nr; r += kB) {
    pr = st_advance(sh.q_st, np, pr, (uint32_t)r);
    const uint32_t d = nd.run_desc[sh.p_run[pr] + ((uint32_t)r - sh.q_st[pr])];
    const uint32_t t = d >> kRunLenBits;
    if (t < ntl) atomicAdd(&sh.tcnt[t], d & ((1u << kRunLenBits) - 1u));
    else bad = true;
  }
  __syncthreads();
  return bin_write(nd, sh, buf, np, ev, csh, bad);
}

// Synaptic state of AdEx neuron i into y[2..] with the step's input x (nS)
// applied: added to g (exponential port) or, scaled by g0, to r (beta port).
template <int P, bool kBeta>
__device__ __forceinline__ void adex_load_syn(const NetDev& nd, const PopDev& pp, uint32_t i, const float* x,
                                              float* y) {
  if constexpr (!kBeta) {
#pragma unroll
    for (int p = 0; p < P; ++p) y[2 + p] = nd.g[(size_t)i * nd.P + p] + x[p];
  } else {
    const bool beta = pp.model == kAdexBeta;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const float g = nd.g[(size_t)i * nd.P + p], r = nd.gr[(size_t)i * nd.P + p];
      y[2 + p] = beta ? g : g + x[p];
      y[2 + P + p] = beta ? __builtin_fmaf(pp.g0[p], x[p], r) : r;
    }
  }
}

template <int P, bool kBeta>
__device__ __forceinline__ void adex_store_syn(const NetDev& nd, uint32_t i, const float* y) {
#pragma unroll
  for (int p = 0; p < P; ++p) nd.g[(size_t)i * nd.P + p] = y[2 + p];
  if constexpr (kBeta) {
#pragma unroll
    for (int p = 0; p < P; ++p) nd.gr[(size_t)i * nd.P + p] = y[2 + P + p];
  }
}

// ------------------------------------------------------------------ update
// One neuron i at step n: Poisson count of the step added to its integer
// input a[] (network input of step n, fixed point), conversion to fp32,
// LIF exact integration (Sec. 2.1, 2.3) or AdEx RK45 (Sec. 2.1, 2.4).
// Returns the number of spikes (resets) in the step, clamped to kMaxMult.
// kAd: 0 no AdEx neurons, 1 AdEx with exponential ports only, 2 beta ports
// present (the integrator then carries the rising variables of every port).
template <bool kLif, int kAd, int P>
__device__ __forceinline__ uint32_t neuron_step(const NetDev& nd, const PopDev* pops, const uint64_t* pthr,
                                                uint64_t n, uint32_t i, int64_t* a, uint32_t& nacc, uint32_t& nrej,
                                                bool& capped, bool& mover, uint32_t npop) {
  const PopDev& pp = pops[find_pop(pops, npop, i)];
  if (pp.pois >= 0) {
    const uint32_t k = poisson_draw(pthr + (size_t)pp.pois * kPoisKmax, pp.seed, i - pp.gid_base, n);
#pragma unroll
    for (int p = 0; p < kMaxPorts; ++p)
      if (p == pp.pois_port) a[p] += (int64_t)k * pp.pois_wq;
  }
  float x[kMaxPorts];
#pragma unroll
  for (int p = 0; p < kMaxPorts; ++p) x[p] = __fmul_rn((float)a[p], pp.scale[p]);
  const float Ie = nd.Ie[i];
  uint32_t m = 0;
  if (kLif && pp.model >= kSpikeGen) {
    if (pp.model == kSpikeGen) {
      // devices (Sec. 2.1): a generator emits one spike per listed step n
      uint32_t c = nd.gen_next[i];
      const uint32_t e = nd.gen_off[i + 1];
      while (c < e && nd.gen_step[c] < n) ++c;
      while (c < e && nd.gen_step[c] == n) { ++m; ++c; }
      nd.gen_next[i] = c;
    } else {
      // a parrot repeats the spikes arriving now: with unit weights its
      // input is their number (exact in fp32 up to 2^24)
      m = a[0] > 0 ? (uint32_t)x[0] : 0u;
    }
  }
  if (kLif && pp.model < kAdex) {
    float y = nd.V[i];
    int32_t r = nd.refr[i];
    bool s;
    const LifK k = lif_consts(nd, pp, i);
    if (pp.model == kLifDelta) {
      s = lif_delta_step(k, y, r, Ie, x[0]);
    } else {
      float I[kMaxPorts];
#pragma unroll
      for (int p = 0; p < kMaxPorts; ++p) I[p] = (p < pp.n_ports) ? nd.Isyn[(size_t)i * nd.P + p] : 0.f;
      s = lif_exp_step(pp, k, y, I, r, Ie, x);
#pragma unroll
      for (int p = 0; p < kMaxPorts; ++p)
        if (p < pp.n_ports) nd.Isyn[(size_t)i * nd.P + p] = I[p];
    }
    nd.V[i] = y;
    nd.refr[i] = r;
    m = s ? 1u : 0u;
  }
  if constexpr (kAd != 0) {
    constexpr bool kBeta = kAd == 2;
    if (pp.model == kAdex || pp.model == kAdexBeta) {
      float y[kAdexVars<P, kBeta>];
      y[0] = nd.V[i];
      y[1] = nd.w[i];
      adex_load_syn<P, kBeta>(nd, pp, i, x, y);
      float h = nd.h[i];
      m = adex_step<P, kBeta>(adex_par<P, kBeta>(nd, pp, i), y, h, Ie, nacc, nrej, capped);
      nd.V[i] = y[0];
      nd.w[i] = y[1];
      adex_store_syn<P, kBeta>(nd, i, y);
      nd.h[i] = h;
    }
  }
  if (m > kMaxMult) { mover = true; m = kMaxMult; }
  return m;
}

__device__ __forceinline__ void load_tables(const NetDev& nd, PopDev* spops, uint32_t pop_cap, uint64_t* sthr,
                                            const PopDev*& pops, const uint64_t*& pthr) {
  const bool lds_pops = nd.npop <= pop_cap;
  const bool lds_thr = nd.npois <= kPoisLds;
  if (lds_pops) {
    const uint32_t words = nd.npop * (uint32_t)(sizeof(PopDev) / 4);
    for (uint32_t w = threadIdx.x; w < words; w += kB)
      reinterpret_cast<uint32_t*>(spops)[w] = reinterpret_cast<const uint32_t*>(nd.pops)[w];
  }
  if (lds_thr) {
    const uint32_t len = nd.pois_len;
    for (uint32_t w = threadIdx.x; w < nd.npois * len; w += kB) {
      const uint32_t q = w / len, k = w - q * len;
      sthr[q * kPoisKmax + k] = nd.pois_thr[q * kPoisKmax + k];
    }
  }
  pops = lds_pops ? spops : nd.pops;
  pthr = lds_thr ? sthr : nd.pois_thr;
}

// The population records p0 .. p0 + np - 1 (np <= kTilePopLds) and their
// Poisson tables in LDS, the tables renumbered by window index.
__device__ __forceinline__ void load_tile_window(const NetDev& nd, uint32_t p0, uint32_t np, PopDev* spops,
                                                 uint64_t* sthr) {
  const uint32_t words = np * (uint32_t)(sizeof(PopDev) / 4);
  for (uint32_t w = threadIdx.x; w < words; w += kB)
    reinterpret_cast<uint32_t*>(spops)[w] = reinterpret_cast<const uint32_t*>(nd.pops + p0)[w];
  const uint32_t len = nd.pois_len;
  for (uint32_t w = threadIdx.x; w < np * len; w += kB) {
    const uint32_t k = w / len, j = w - k * len;
    const int32_t q = nd.pops[p0 + k].pois;
    if (q >= 0) sthr[k * kPoisKmax + j] = nd.pois_thr[(size_t)q * kPoisKmax + j];
  }
  __syncthreads();
  if (threadIdx.x < np && spops[threadIdx.x].pois >= 0) spops[threadIdx.x].pois = (int32_t)threadIdx.x;
}

// Populations overlapping tile t: the first one and their number.
__device__ __forceinline__ uint32_t tile_pops(const NetDev& nd, uint32_t t, uint32_t& p0) {
  const uint32_t first = t << nd.tile_shift;
  const uint32_t nt = min(1u << nd.tile_shift, nd.N - first);
  p0 = find_pop(nd.pops, nd.npop, first);
  return find_pop(nd.pops, nd.npop, first + nt - 1) - p0 + 1;
}

// A tile block's population records and Poisson tables: all of them in LDS
// when they fit; otherwise, when the populations overlapping the tile (a
// contiguous run in gid order, a few even in a batch of many instances) fit,
// those, with their Poisson tables renumbered in LDS; otherwise as
// load_tables.  Returns the number of records at `pops`.  Visible after the
// caller's next barrier.
__device__ __forceinline__ uint32_t load_tile_tables(const NetDev& nd, uint32_t first, uint32_t nt, PopDev* spops,
                                                     uint64_t* sthr, const PopDev*& pops, const uint64_t*& pthr) {
  const uint32_t p0 = find_pop(nd.pops, nd.npop, first), p1 = find_pop(nd.pops, nd.npop, first + nt - 1);
  const uint32_t np = p1 - p0 + 1;
  if ((nd.npop <= kTilePopLds && nd.npois <= kPoisLds) || np > kTilePopLds || np > kPoisLds) {
    load_tables(nd, spops, kTilePopLds, sthr, pops, pthr);
    return nd.npop;
  }
  load_tile_window(nd, p0, np, spops, sthr);
  pops = spops;
  pthr = sthr;
  return np;
}

__device__ __forceinline__ uint32_t inbuf(uint64_t n) { return (uint32_t)(n % kInBuf); }

// First raster-ring position of the spikes of step n: the positions of the
// earlier steps' spikes end here.
__device__ __forceinline__ uint64_t step_pos(const NetDev& nd, uint64_t n) {
  if (n == 0) return 0;
  const uint32_t s = (uint32_t)((n - 1) % nd.R);
  return nd.ring_base[s] + nd.ring_cnt[s];
}

// Once per step (block 0): the step's raster position for the readers of the
// next steps and the drain, and the spike counter of step n + 1 cleared (its
// slot holds step n + 1 - R, which no block reads during step n).
__device__ __forceinline__ void step_books(const NetDev& nd, uint64_t n) {
  const uint64_t pos = step_pos(nd, n);
  nd.ring_base[n % nd.R] = pos;
  nd.chunk_base[n & (nd.chunk_ring - 1)] = pos;
  nd.ring_cnt[(n + 1) % nd.R] = 0;
  nd.ctrl->dlv_next[(n + 1) & 3] = 0;  // the delivery queue of step n + 1 (step n uses slot n & 3)
  // plastic arrivals: this step fills the list of arrival step n + 1; the list
  // of step n was consumed by the plasticity kernel of step n - 1
  if (nd.n_rules) nd.arr_cnt[n & 1] = 0;
}

// A spike of step n at position pos among the step's spikes: raster entry and
// the selection record that the delivery of later steps reads.
__device__ __forceinline__ void emit_spike(const NetDev& nd, uint64_t n, uint64_t pos_n, uint32_t pos,
                                           uint32_t entry, uint32_t grp_ptr, uint64_t mask) {
  nd.log[(pos_n + pos) & nd.log_mask] = entry;
  SpikeRec r;
  r.entry = entry;
  r.grp_ptr = grp_ptr;
  r.mask = mask;
  nd.recent[(size_t)(n % nd.R) * nd.N + pos] = r;
}

// Direct-delivery update block: 256 neurons, input from acc[n % 2] (read and
// cleared); spikes get their positions from one atomic per wave on the step's
// counter (wave ballot + lane prefix), their raster entries and records are
// written here, and their delay-1 groups are delivered at once by the
// block's flat scan into the buffer of step n + 1.
template <bool kLif, int kAd, int P>
__device__ void update_block(const NetDev& nd, uint64_t n, uint32_t blk, UpdLds& sl) {
  const PopDev* pops;
  const uint64_t* pthr;
  load_tables(nd, sl.u.t.spops, kPopLds, sl.u.t.sthr, pops, pthr);
  dlv_load_classes(nd, sl.u.d);
  __syncthreads();
  const uint32_t i = blk * kB + threadIdx.x;
  bool spk = false;
  uint32_t entry = 0;
  uint32_t nacc = 0, nrej = 0;
  bool capped = false, mover = false;
  if (i < nd.N) {
    int64_t* acc = nd.acc + ((size_t)inbuf(n) * nd.N + i) * nd.P;
    int64_t a[kMaxPorts];
#pragma unroll
    for (int p = 0; p < kMaxPorts; ++p) {
      a[p] = 0;
      if (p < (int)nd.P) {
        a[p] = acc[p];
        if (a[p] != 0) acc[p] = 0;
      }
    }
    const uint32_t m = neuron_step<kLif, kAd, P>(nd, pops, pthr, n, i, a, nacc, nrej, capped, mover, nd.npop);
    spk = m > 0;
    entry = i | (m << kMultShift);
    if (spk && nd.n_rules) nd.last_post[i] = (uint32_t)(n + 1);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t bal = __ballot(spk);
  // each wave reserves its spikes' positions in the step with one atomic
  uint32_t wpos = 0;
  if (bal) {
    if (lane == 0)
      wpos = __hip_atomic_fetch_add(&nd.ring_cnt[n % nd.R], (uint32_t)__popcll(bal), __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    wpos = __shfl(wpos, 0, 64) + (uint32_t)__popcll(bal & lanemask_lt());
  }
  if (lane == 0) sl.wcnt[wv] = __popcll(bal);
  // a spiking neuron's delay mask, first group and the offsets of its delay-1
  // group, loaded while the wave's atomic is in flight
  uint64_t mask = 0, o1 = 0;
  uint32_t gp = 0, l1 = 0;
  if (spk) {
    mask = nd.src_mask[i];
    gp = nd.grp_ptr[i];
    if ((mask >> 1) & 1ull) { o1 = nd.grp_off[gp]; l1 = (uint32_t)(nd.grp_off[gp + 1] - o1); }
  }
  if (spk) emit_spike(nd, n, step_pos(nd, n), wpos, entry, gp, mask);
  if (threadIdx.x == 0) sl.u.d.npair = 0;  // the tables are dead from here
  __syncthreads();
  uint32_t btot = 0;
#pragma unroll
  for (int w = 0; w < kB / 64; ++w) btot += sl.wcnt[w];
  // delay-1 groups of the block's spikes: selected into LDS and delivered by
  // the block's flat scan into the buffer of step n+1
  uint64_t pairs = 0, events = 0;
  if (btot) {  // block-uniform
    DirectLds& sh = sl.u.d;
    if (l1) sel_add(sh, o1, l1, entry >> kMultShift, inbuf(n + 1));
    __syncthreads();
    if (sh.npair) {
      pairs += sh.npair;
      events += dlv_flush(nd, sh, 0u);
    }
  }
  uint64_t sa = 0, sr = 0;
  if (kAd != 0) {
    sa = block_sum(nacc, sl.red);
    sr = block_sum(nrej, sl.red);
  } else {
    __syncthreads();
  }
  if (threadIdx.x == 0) {  // no-return atomics: the block need not wait for a read
    uint64_t* st = nd.blk_stats + (size_t)kBlkStats * blk;
    const uint64_t v[kBlkStats] = {sa, sr, btot, pairs, events};
#pragma unroll
    for (int k = 0; k < kBlkStats; ++k)
      if (v[k]) __hip_atomic_fetch_add(&st[k], v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (capped) atomicOr(&nd.ctrl->overflow, 2u);
  if (mover) atomicOr(&nd.ctrl->overflow, 1u);
}

// AdEx neuron i at step n as one lane's work item: state and folded input
// loaded, then advanced one RK45 substep per call of adex_substep.
template <int P, bool kBeta>
struct AdexItem {
  AdexPar<P, kBeta> q;
  float y[kAdexVars<P, kBeta>];
  float h, t, Ie;
  uint32_t it, mult;
};

template <int P, bool kBeta>
__device__ __forceinline__ void adex_load(const NetDev& nd, const PopDev* pops, uint32_t npop, const uint64_t* pthr,
                                          uint64_t n, uint32_t i, int64_t* a, AdexItem<P, kBeta>& w) {
  const PopDev& pp = pops[find_pop(pops, npop, i)];
  if (pp.pois >= 0) {
    const uint32_t k = poisson_draw(pthr + (size_t)pp.pois * kPoisKmax, pp.seed, i - pp.gid_base, n);
#pragma unroll
    for (int p = 0; p < kMaxPorts; ++p)
      if (p == pp.pois_port) a[p] += (int64_t)k * pp.pois_wq;
  }
  w.q = adex_par<P, kBeta>(nd, pp, i);
  w.y[0] = nd.V[i];
  w.y[1] = nd.w[i];
  float x[P];
#pragma unroll
  for (int p = 0; p < P; ++p) x[p] = __fmul_rn((float)a[p], pp.scale[p]);
  adex_load_syn<P, kBeta>(nd, pp, i, x, w.y);
  w.h = nd.h[i];
  if (!(w.h > 0.f) || w.h > pp.dt) w.h = pp.dt;
  w.Ie = nd.Ie[i];
  w.t = 0.f;
  w.it = 0;
  w.mult = 0;
}

template <int P, bool kBeta>
__device__ __forceinline__ uint32_t adex_store(const NetDev& nd, uint32_t i, AdexItem<P, kBeta>& w, bool& mover) {
  nd.V[i] = w.y[0];
  nd.w[i] = w.y[1];
  adex_store_syn<P, kBeta>(nd, i, w.y);
  nd.h[i] = (w.h > w.q.dt) ? w.q.dt : w.h;
  uint32_t m = w.mult;
  if (m > kMaxMult) { mover = true; m = kMaxMult; }
  return m;
}

// Binned-delivery tile block t at step n: sums the tile's bin (the events
// written for step n during earlier steps, plus any spill) into int64 LDS
// accumulators, updates the tile's neurons from them, emits their spikes
// (one atomic on the step's counter for the whole tile) and bins the delay-1
// groups of those spikes for step n+1.  The spike count
// of a neuron is kept in its (then dead) first LDS input slot until all
// neurons are done.  AdEx-only networks take their neurons from a work queue:
// a lane whose neuron has reached the step end takes the next one, so waves
// stay full while neurons near a spike need many RK45 substeps and the
// others one.
template <bool kLif, int kAd, int P, bool kWin = false>
__device__ void tile_block(const NetDev& nd, uint64_t n, uint32_t t, TileLds& sl) {
  const uint32_t PP = nd.P, tsh = nd.tile_shift, buf = inbuf(n);
  const uint32_t first = t << tsh;
  const uint32_t nt = min(1u << tsh, nd.N - first);
  // first raster position of this step's spikes: the previous step's books are
  // final, so it is read now rather than after the update
  const uint64_t pos_n = step_pos(nd, n);
  const PopDev* pops;
  const uint64_t* pthr;
  uint32_t npop;
  if constexpr (kWin) {
    // the caller found the tile's populations to fit the LDS window: the
    // tables are read from LDS only, with no generic loads (whose waits
    // would also cover the block's global memory operations)
    uint32_t p0;
    npop = tile_pops(nd, t, p0);
    load_tile_window(nd, p0, npop, sl.spops, sl.sthr);
    pops = sl.spops;
    pthr = sl.sthr;
  } else {
    npop = load_tile_tables(nd, first, nt, sl.spops, sl.sthr, pops, pthr);
  }
  for (uint32_t c = threadIdx.x; c < nd.n_classes; c += kB) {
    sl.c.wq[c] = nd.cls_wq[c];
    sl.wp[c] = (uint8_t)nd.cls_port[c];
  }
  for (uint32_t j = threadIdx.x; j < nt * PP; j += kB) sl.u.acc[j] = 0;
  if (threadIdx.x == 0) { sl.next = 0; sl.hq_next2 = 0; sl.hq_n = 0; }
  const size_t ti = (size_t)buf * nd.n_tiles + t;
  const uint32_t cnt = min(nd.bin_cnt[ti], nd.bin_cap[t]);
  const uint32_t ovf = nd.ovf_flag[ti];
  const uint32_t* bin = nd.bins + (size_t)buf * nd.bins_total + nd.bin_off[t];
  __syncthreads();
  bool bad = false;
  auto add = [&](uint32_t e) {
    const uint32_t cls = e & (uint32_t)(kMaxClasses - 1), loc = e >> kBinLocalShift;
    if (loc >= nt || cls >= nd.n_classes) { bad = true; return; }
    const int64_t v = sl.c.wq[cls] * (int64_t)((e >> kBinMultShift) & kMaxMult);
    atomicAdd((unsigned long long*)&sl.u.acc[loc * PP + sl.wp[cls]], (unsigned long long)v);
  };
  uint32_t j = threadIdx.x;
  // independent loads in flight per lane: 16 (8 with beta ports, whose
  // integrator leaves fewer registers)
  constexpr int kBinLoads = (kAd == 2) ? 8 : 16;
  for (; j + (kBinLoads - 1) * kB < cnt; j += kBinLoads * kB) {
    uint32_t e[kBinLoads];
#pragma unroll
    for (int q = 0; q < kBinLoads; ++q) e[q] = bin[j + q * kB];
#pragma unroll
    for (int q = 0; q < kBinLoads; ++q) add(e[q]);
  }
  for (; j < cnt; j += kB) add(bin[j]);
  if (bad) atomicOr(&nd.ctrl->overflow, 4u);  // a malformed entry: reported, not added
  __syncthreads();
  if (ovf) {  // block-uniform: events that did not fit the bin
    int64_t* g = nd.acc + ((size_t)buf * nd.N + first) * PP;
    for (uint32_t j = threadIdx.x; j < nt * PP; j += kB) {
      const int64_t v = g[j];
      if (v != 0) { sl.u.acc[j] += v; g[j] = 0; }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    nd.bin_cnt[ti] = 0;
    if (ovf) nd.ovf_flag[ti] = 0;
  }
  uint32_t nacc = 0, nrej = 0;
  bool capped = false, mover = false;
  if (kAd != 0 && !kLif) {
    // AdEx only: work queue over the tile's neurons; each lane holds its
    // current neuron and has the next one's state already loaded, so the
    // loads of a refill overlap the substeps of the current neuron
    auto fetch = [&](uint32_t l, AdexItem<P, kAd == 2>& it) {
      int64_t a[kMaxPorts];
#pragma unroll
      for (int p = 0; p < kMaxPorts; ++p) a[p] = (p < (int)PP) ? sl.u.acc[l * PP + p] : 0;
      adex_load<P, kAd == 2>(nd, pops, npop, pthr, n, first + l, a, it);
    };
    for (uint32_t l = threadIdx.x; l < nt; l += kB) {
      const uint32_t i = first + l;
      const PopDev& hp = pops[find_pop(pops, npop, i)];
      const bool hot = nd.V[i] >= hp.V_T + 4.f * hp.Delta_T;
      const uint64_t hb = __ballot(hot);
      if ((threadIdx.x & 31) == 0) sl.hot[l >> 5] = (uint32_t)(hb >> (threadIdx.x & 32));
      if (hot) {
        const uint32_t k = atomicAdd(&sl.hq_n, 1u);
        if (k < kHotCap) sl.hq[k] = (uint16_t)l;
        else atomicAnd(&sl.hot[l >> 5], ~(1u << (l & 31)));  // list full: taken in index order
      }
    }
    __syncthreads();
    // The first 64 hot neurons go to one wave (a different one in blocks b,
    // b + 256, b + 512, which dispatch places on one CU), lane by lane, and
    // that wave runs only their substeps, at raised priority: a lane whose
    // neuron is done idles, since refilling it would put neuron loads and
    // Poisson draws between the substeps of the long chains.  Then the wave
    // joins the others' queue.  Further hot neurons go to any wave first.
    if ((threadIdx.x >> 6) == ((blockIdx.x >> 8) & 3u)) {
      const uint32_t nh = min(min(sl.hq_n, kHotCap), 64u);
      if (nh) {  // wave-uniform
        __builtin_amdgcn_s_setprio(2);
        uint32_t hl = ((threadIdx.x & 63u) < nh) ? (uint32_t)sl.hq[threadIdx.x & 63u] : nt;
        AdexItem<P, kAd == 2> hw;
        if (hl < nt) fetch(hl, hw);
        while (hl < nt) {
          if (adex_substep<P, kAd == 2>(hw.q, hw.y, hw.h, hw.t, hw.it, hw.mult, hw.Ie, nacc, nrej, capped)) {
            sl.c.mk[hl] = (uint8_t)adex_store<P, kAd == 2>(nd, first + hl, hw, mover);
            hl = nt;
          }
        }
        __builtin_amdgcn_s_setprio(0);
      }
    }
    auto claim = [&]() -> uint32_t {
      const uint32_t nh = min(sl.hq_n, kHotCap);
      if (nh > 64u) {
        const uint32_t h = 64u + atomicAdd(&sl.hq_next2, 1u);
        if (h < nh) return sl.hq[h];
      }
      for (;;) {
        const uint32_t c = atomicAdd(&sl.next, 1u);
        if (c >= nt) return nt;
        if (!((sl.hot[c >> 5] >> (c & 31)) & 1u)) return c;
      }
    };
    uint32_t loc = claim(), nloc = nt;
    AdexItem<P, kAd == 2> w, nx;
    if (loc < nt) {
      fetch(loc, w);
      nloc = claim();
      if (nloc < nt) fetch(nloc, nx);
    }
    while (loc < nt) {
      if (adex_substep<P, kAd == 2>(w.q, w.y, w.h, w.t, w.it, w.mult, w.Ie, nacc, nrej, capped)) {
        sl.c.mk[loc] = (uint8_t)adex_store<P, kAd == 2>(nd, first + loc, w, mover);
        loc = nloc;
        if (loc < nt) {
          w = nx;
          nloc = claim();
          if (nloc < nt) fetch(nloc, nx);
        }
      }
    }
  } else {
    for (uint32_t loc = threadIdx.x; loc < nt; loc += kB) {
      int64_t a[kMaxPorts];
#pragma unroll
      for (int p = 0; p < kMaxPorts; ++p) a[p] = (p < (int)PP) ? sl.u.acc[loc * PP + p] : 0;
      sl.c.mk[loc] =
          (uint8_t)neuron_step<kLif, kAd, P>(nd, pops, pthr, n, first + loc, a, nacc, nrej, capped, mover, npop);
    }
  }
  __syncthreads();
  // spikes of the tile: counts per (256-neuron sub-block, wave), one atomic for
  // the tile's positions; a neuron's position follows sub-block, wave, lane
  const uint32_t nsub = (nt + kB - 1) / kB;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint32_t k = 0; k < nsub; ++k) {
    const uint32_t loc = k * kB + threadIdx.x;
    const uint64_t bal = __ballot(loc < nt && sl.c.mk[loc] != 0);
    if (lane == 0) sl.wcnt[k][wv] = __popcll(bal);
  }
  __syncthreads();
  uint32_t spikes = 0;
  for (uint32_t k = 0; k < nsub; ++k)
#pragma unroll
    for (int q = 0; q < kB / 64; ++q) spikes += sl.wcnt[k][q];
  BinLds& sh = sl.u.d1;  // the LDS input is dead from here: it holds the selection
  uint64_t pairs = 0, events = 0;
  if (spikes) {  // block-uniform
    if (threadIdx.x == 0)
      sl.emit = __hip_atomic_fetch_add(&nd.ring_cnt[n % nd.R], spikes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    dlv_init(nd, sh);
    __syncthreads();
    uint32_t before = 0;  // spikes of the sub-blocks before k
    for (uint32_t k = 0; k < nsub; ++k) {  // block-uniform
      uint32_t woff = 0, ktot = 0;
#pragma unroll
      for (int q = 0; q < kB / 64; ++q) {
        if (q < wv) woff += sl.wcnt[k][q];
        ktot += sl.wcnt[k][q];
      }
      if (ktot == 0) continue;  // block-uniform: nothing to emit or select
      const uint32_t loc = k * kB + threadIdx.x;
      const uint32_t m = loc < nt ? sl.c.mk[loc] : 0u;
      const uint64_t bal = __ballot(m != 0);
      if (m) {
        const uint32_t i = first + loc;
        const uint32_t entry = i | (m << kMultShift);
        if (nd.n_rules) nd.last_post[i] = (uint32_t)(n + 1);
        const uint64_t mask = nd.src_mask[i];
        const uint32_t gp = nd.grp_ptr[i];
        emit_spike(nd, n, pos_n, sl.emit + before + woff + (uint32_t)__popcll(bal & lanemask_lt()), entry, gp, mask);
        if ((mask >> 1) & 1ull) dlv_probe(nd, sh, entry, gp, mask, 1, inbuf(n + 1));
      }
      before += ktot;
      if (spikes > (uint32_t)(kSelChunk - kB)) {  // block-uniform: else the chunk cannot fill up
        __syncthreads();
        if (sh.npair > (uint32_t)(kSelChunk - kB)) {
          pairs += sh.npair;
          events += dlv_flush(nd, sh, inbuf(n + 1));
        }
      }
    }
    __syncthreads();
    if (sh.npair) {
      pairs += sh.npair;
      events += dlv_flush(nd, sh, inbuf(n + 1));
    }
  }
  uint64_t sa = 0, sr = 0;
  if (kAd != 0) {
    sa = block_sum(nacc, sl.red);
    sr = block_sum(nrej, sl.red);
  }
  if (threadIdx.x == 0) {  // no-return atomics: the block need not wait for a read
    uint64_t* st = nd.blk_stats + (size_t)kBlkStats * (first / kB);
    const uint64_t v[kBlkStats] = {sa, sr, (uint64_t)spikes, pairs, events};
#pragma unroll
    for (int k = 0; k < kBlkStats; ++k)
      if (v[k]) __hip_atomic_fetch_add(&st[k], v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (capped) atomicOr(&nd.ctrl->overflow, 2u);
  if (mover) atomicOr(&nd.ctrl->overflow, 1u);
}

// Delivery blocks of step n: the input of step n+1 from the spikes of steps
// n-1 .. n+1-Dmax whose delay d >= 2 expires now, read from their selection
// records.  The items (spike, d) are ordered by delay, then by the spike's
// position in its step (spikes of one tile lie together).  Two ways to share
// them among the G blocks:
//   strided: item e goes to block e mod G, so that every block sees every
//     delay (hits and group sizes vary with the delay);
//   queue (binned batches of many small instances): blocks take ranges of
//     consecutive items from a queue until it is empty, so that a chunk holds
//     spikes of few instances, whose targets lie in few tiles (longer runs per
//     tile in the bins), and blocks that start late take less.
template <class L>
__device__ void deliver_block(const NetDev& nd, uint64_t n, uint32_t b, uint32_t G, L& sh) {
  const uint32_t R = nd.R, dmax = nd.dmax;
  dlv_init(nd, sh);
  const uint32_t dseg = threadIdx.x + 1;  // delay of this item segment (threads 0..63)
  if (threadIdx.x < 64) {
    uint64_t cnt = 0;
    uint32_t slt = 0;
    if (dseg >= kDlvMinDelay && dseg <= dmax && n + 1 >= dseg) {
      slt = (uint32_t)((n + 1 - dseg) % R);
      cnt = nd.ring_cnt[slt];
    }
    const uint64_t incl = wave_incl_scan(cnt);
    sh.seg[dseg] = incl - cnt;
    if (dseg == 64) sh.seg[65] = incl;
    sh.slot[dseg] = slt;
  }
  __syncthreads();
  const uint64_t items = sh.seg[65];
  const uint32_t b1 = inbuf(n + 1);
  uint64_t pairs = 0, events = 0;
  auto select = [&](uint64_t e) {
    uint32_t lo = kDlvMinDelay, hi = 65;  // segment d: seg[d] <= e < seg[d + 1]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (sh.seg[mid] <= e) lo = mid; else hi = mid;
    }
    const SpikeRec r = nd.recent[(size_t)sh.slot[lo] * nd.N + (e - sh.seg[lo])];
    dlv_probe(nd, sh, r.entry, r.grp_ptr, r.mask, lo, b1);
  };
  if (nd.dlv_queue) {
    const uint64_t share = (items + G - 1) / G;
    const uint64_t grab = share < 1 ? 1 : (share > (uint64_t)kSelChunk ? (uint64_t)kSelChunk : share);
    for (;;) {  // block-uniform
      if (threadIdx.x == 0)
        sh.j0 = __hip_atomic_fetch_add(&nd.ctrl->dlv_next[n & 3], grab, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      const uint64_t j0 = sh.j0;
      if (j0 >= items) break;
      const uint64_t j1 = (j0 + grab < items) ? j0 + grab : items;
#pragma unroll
      for (int q = 0; q < kSelPerThread; ++q) {
        const uint64_t e = j0 + (uint64_t)q * kB + threadIdx.x;
        if (e < j1) select(e);
      }
      __syncthreads();
      pairs += sh.npair;
      events += dlv_flush(nd, sh, b1);  // ends with a barrier: j0 may be rewritten
    }
  } else {
    const uint64_t mine = (b < items) ? (items - b + G - 1) / G : 0;
    for (uint64_t j0 = 0; j0 < mine; j0 += kSelChunk) {  // block-uniform
#pragma unroll
      for (int q = 0; q < kSelPerThread; ++q) {
        const uint64_t j = j0 + (uint64_t)q * kB + threadIdx.x;
        if (j < mine) select(b + (uint64_t)G * j);
      }
      __syncthreads();
      pairs += sh.npair;
      events += dlv_flush(nd, sh, b1);
    }
  }
  if (threadIdx.x == 0 && (pairs || events)) {
    __hip_atomic_fetch_add((unsigned long long*)&nd.sel_stats[2 * b], (unsigned long long)pairs, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add((unsigned long long*)&nd.sel_stats[2 * b + 1], (unsigned long long)events,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One simulation step n, direct delivery: blocks [0, nblk_upd) update the
// neurons (LIF exact integration, Sec. 2.1/2.3; AdEx RK45, Sec. 2.1/2.4),
// emit their spikes and deliver their delay-1 groups; the remaining blocks
// deliver the earlier steps' spikes whose delay (>= 2)
// expires now.  The update reads the input buffer of step n; deliveries go to
// the buffers of the steps they arrive at.
template <bool kLif, int kAd, int P>
__global__ void __launch_bounds__(kB) k_step(NetDev nd, uint32_t rel) {
  __shared__ StepLds lds;
  const uint64_t n = nd.ctrl->step_base + rel;
  if (blockIdx.x == 0 && threadIdx.x == 0) step_books(nd, n);
  if (blockIdx.x < nd.nblk_upd) {
    update_block<kLif, kAd, P>(nd, n, blockIdx.x, lds.upd);
  } else {
    deliver_block(nd, n, blockIdx.x - nd.nblk_upd, gridDim.x - nd.nblk_upd, lds.dlv);
  }
}

// A tile block's step.  The LIF-only kernels run only where every tile's
// populations fit the LDS window (the host launches the AdEx-capable kernel
// for other LIF-only networks), so they read the tables from LDS only.
template <bool kLif, int kAd, int P>
__device__ __forceinline__ void tile_step(const NetDev& nd, uint64_t n, uint32_t t, TileLds& sl) {
  tile_block<kLif, kAd, P, kAd == 0>(nd, n, t, sl);
}

// One simulation step n, binned delivery: blocks [0, n_tiles) are the tile
// blocks (input from their bins, update, emission, delay-1 binning), the
// remaining blocks bin the earlier steps' spikes whose delay (>= 2) expires
// now.
template <bool kLif, int kAd, int P>
__global__ void __launch_bounds__(kB) k_step_binned(NetDev nd, uint32_t rel) {
  __shared__ BinStepLds lds;
  const uint64_t n = nd.ctrl->step_base + rel;
  if (blockIdx.x == 0 && threadIdx.x == 0) step_books(nd, n);
  if (blockIdx.x < nd.n_tiles) {
    tile_step<kLif, kAd, P>(nd, n, blockIdx.x, lds.tile);
  } else {
    deliver_block(nd, n, blockIdx.x - nd.n_tiles, gridDim.x - nd.n_tiles, lds.dlv);
  }
}

// The same for LIF-only networks with tile runs: the delivery blocks' count
// pass reads the runs (a kernel of its own, so that the other step kernels
// carry no code for it).
template <bool kLif, int kAd, int P>
__global__ void __launch_bounds__(kB) k_step_binned_runs(NetDev nd, uint32_t rel) {
  __shared__ BinRunStepLds lds;
  const uint64_t n = nd.ctrl->step_base + rel;
  if (blockIdx.x == 0 && threadIdx.x == 0) step_books(nd, n);
  if (blockIdx.x < nd.n_tiles) {
    tile_step<kLif, kAd, P>(nd, n, blockIdx.x, lds.tile);
  } else {
    deliver_block(nd, n, blockIdx.x - nd.n_tiles, gridDim.x - nd.n_tiles, lds.dlv);
  }
}

__global__ void k_advance(Ctrl* ctrl, uint32_t steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->step_base += steps;
}

__global__ void __launch_bounds__(kB) k_poisson_counts(NetDev nd, uint64_t step, uint32_t first, uint32_t n,
                                                       uint32_t* out) {
  const uint32_t j = blockIdx.x * kB + threadIdx.x;
  if (j >= n) return;
  const uint32_t i = first + j;
  const PopDev& pp = nd.pops[find_pop(nd.pops, nd.npop, i)];
  out[j] = (pp.pois >= 0) ? poisson_draw(nd.pois_thr + (size_t)pp.pois * kPoisKmax, pp.seed, i - pp.gid_base, step) : 0u;
}

// Readback of the binned input pending in input buffer buf, on one port, for
// gids [first, first + n): block = one tile, entries decoded and added to
// out[gid - first] (which holds the tile's spill already).
__global__ void __launch_bounds__(kB) k_pending_input(NetDev nd, uint32_t buf, uint32_t first, uint32_t n,
                                                      uint32_t port, int64_t* out) {
  const uint32_t t = (first >> nd.tile_shift) + blockIdx.x;
  const uint32_t tfirst = t << nd.tile_shift;
  const size_t ti = (size_t)buf * nd.n_tiles + t;
  const uint32_t cnt = min(nd.bin_cnt[ti], nd.bin_cap[t]);
  const uint32_t* bin = nd.bins + (size_t)buf * nd.bins_total + nd.bin_off[t];
  for (uint32_t j = threadIdx.x; j < cnt; j += kB) {
    const uint32_t e = bin[j];
    const uint32_t cls = e & (uint32_t)(kMaxClasses - 1);
    const uint32_t gid = tfirst + (e >> kBinLocalShift);
    if (cls >= nd.n_classes || gid < first || gid - first >= n || nd.cls_port[cls] != port) continue;
    const int64_t v = nd.cls_wq[cls] * (int64_t)((e >> kBinMultShift) & kMaxMult);
    atomicAdd((unsigned long long*)&out[gid - first], (unsigned long long)v);
  }
}

}  // namespace

// Launch helper: with events, the kernel is launched by hipExtLaunchKernelGGL,
// which records `start` and `stop` on the dispatch itself (kernel duration).
template <typename K, typename... Args>
static void launch(K kernel, dim3 grid, dim3 blk, hipStream_t s, hipEvent_t start, hipEvent_t stop, Args... args) {
  if (start) hipExtLaunchKernelGGL(kernel, grid, blk, 0, s, start, stop, 0, args...);
  else hipLaunchKernelGGL(kernel, grid, blk, 0, s, args...);
}

template <template <bool, int, int> class Sel, bool kLif, int kAd>
static void launch_ports(const NetDev& nd, dim3 grid, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                         uint32_t rel) {
  const dim3 blk(kB);
  switch (nd.P) {
    case 1: launch(Sel<kLif, kAd, 1>::fn(), grid, blk, s, start, stop, nd, rel); break;
    case 2: launch(Sel<kLif, kAd, 2>::fn(), grid, blk, s, start, stop, nd, rel); break;
    case 3: launch(Sel<kLif, kAd, 3>::fn(), grid, blk, s, start, stop, nd, rel); break;
    default: launch(Sel<kLif, kAd, 4>::fn(), grid, blk, s, start, stop, nd, rel); break;
  }
}

template <template <bool, int, int> class Sel>
static void launch_variant(const NetDev& nd, dim3 grid, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                           uint32_t rel) {
  // which models are present is encoded in nd.pad0: bit 0 LIF, bit 1 AdEx,
  // bit 2 AdEx with beta ports
  const bool lif = nd.pad0 & 1u, adex = nd.pad0 & 2u, beta = nd.pad0 & 4u;
  if (!adex && (nd.tile_win || !nd.n_tiles)) {
    launch(Sel<true, 0, 1>::fn(), grid, dim3(kB), s, start, stop, nd, rel);
  } else if (!adex) {  // binned, a tile overlaps more populations than its LDS window holds
    launch_ports<Sel, true, 1>(nd, grid, s, start, stop, rel);
  } else if (!beta) {
    if (lif) launch_ports<Sel, true, 1>(nd, grid, s, start, stop, rel);
    else launch_ports<Sel, false, 1>(nd, grid, s, start, stop, rel);
  } else {
    if (lif) launch_ports<Sel, true, 2>(nd, grid, s, start, stop, rel);
    else launch_ports<Sel, false, 2>(nd, grid, s, start, stop, rel);
  }
}

template <bool A, int B, int C>
struct SelDirect {
  static auto fn() { return k_step<A, B, C>; }
};
template <bool A, int B, int C>
struct SelBinned {
  static auto fn() { return k_step_binned<A, B, C>; }
};

hipError_t launch_step(const NetDev& nd, uint32_t rel, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  if (nd.n_tiles && nd.tile_runs && nd.tile_win)  // LIF-only networks
    launch(k_step_binned_runs<true, 0, 1>, dim3(nd.n_tiles + nd.sel_grid), dim3(kB), s, start, stop, nd, rel);
  else if (nd.n_tiles) launch_variant<SelBinned>(nd, dim3(nd.n_tiles + nd.sel_grid), s, start, stop, rel);
  else launch_variant<SelDirect>(nd, dim3(nd.nblk_upd + nd.sel_grid), s, start, stop, rel);
  return hipGetLastError();
}

hipError_t launch_advance(Ctrl* ctrl, uint32_t steps, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctrl, steps);
  return hipGetLastError();
}

hipError_t launch_pending_input(const NetDev& nd, uint32_t buf, uint32_t first, uint32_t n, uint32_t port,
                                int64_t* out, hipStream_t s) {
  if (n == 0 || nd.n_tiles == 0) return hipSuccess;
  const uint32_t t0 = first >> nd.tile_shift, t1 = (first + n - 1) >> nd.tile_shift;
  hipLaunchKernelGGL(k_pending_input, dim3(t1 - t0 + 1), dim3(kB), 0, s, nd, buf, first, n, port, out);
  return hipGetLastError();
}

// Workspace of the allocation-free input readback: a file-scope device array.
// Host code must not pass its name to a kernel or a copy (on the host the name
// is only a stand-in); the device address comes from hipGetSymbolAddress, once
// per device with that device current, and is kept per device.
static __device__ __align__(256) int64_t scratch[kNoAllocInputMax];

namespace {
std::mutex g_ws_mu;
int64_t* g_ws_ptr[kMaxDevices] = {};
}  // namespace

hipError_t input_workspace(int device, bool resolve, int64_t** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_ws_mu);
  if (!g_ws_ptr[device] && resolve) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ws_ptr[device] = static_cast<int64_t*>(p);
  }
  *out = g_ws_ptr[device];
  return hipSuccess;
}

hipError_t launch_poisson_counts(const NetDev& nd, uint64_t step, uint32_t first, uint32_t n, uint32_t* k,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_poisson_counts, dim3((n + kB - 1) / kB), dim3(kB), 0, s, nd, step, first, n, k);
  return hipGetLastError();
}

}  // namespace snn
