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
// LIF exact integration (Sec. 2.1; LIF and exponential-PSC equations of
// Sec. 2.3), y = V - E_L, fixed fp32 operation order without contraction.
__device__ __forceinline__ bool lif_delta_step(const PopDev& pp, float& y, int32_t& r, float Ie, float x) {
  if (r > 0) {
    r -= 1;  // refractory: held at reset, input discarded
  } else {
    const float t1 = __fmul_rn(pp.P22, y);
    const float t2 = __fmul_rn(pp.P20, Ie);
    y = __fadd_rn(__fadd_rn(t1, t2), x);
  }
  if (r == 0 && y >= pp.theta) { y = pp.y_reset; r = pp.n_ref; return true; }
  return false;
}

__device__ __forceinline__ bool lif_exp_step(const PopDev& pp, float& y, float* I, int32_t& r, float Ie,
                                             const float* x) {
  if (r == 0) {
    float v = __fmul_rn(pp.P22, y);
    for (int p = 0; p < pp.n_ports; ++p) v = __fadd_rn(v, __fmul_rn(pp.P21[p], I[p]));
    v = __fadd_rn(v, __fmul_rn(pp.P20, Ie));
    y = v;
  } else {
    r -= 1;
  }
  for (int p = 0; p < pp.n_ports; ++p) I[p] = __fadd_rn(__fmul_rn(pp.P11[p], I[p]), x[p]);
  if (r == 0 && y >= pp.theta) { y = pp.y_reset; r = pp.n_ref; return true; }
  return false;
}

// AdEx with exponential conductances (Sec. 2.4, Table 2), right-hand side in
// fp32.  y = (V, w, g_0..g_{P-1}); the synaptic current is sum g_p (V - E_p)
// entering with the sign that lets an excitatory conductance depolarise; the
// exponential uses min(V, V_peak).
template <int P>
__device__ __forceinline__ void adex_rhs(const PopDev& pp, float Ie, const float* y, float* dy) {
  const float V = y[0], w = y[1];
  const float Vc = fminf(V, pp.V_peak);
  float isyn = 0.f;
#pragma unroll
  for (int p = 0; p < P; ++p) isyn = __builtin_fmaf(y[2 + p], V - pp.E_rev[p], isyn);
  const float ex = pp.g_L * pp.Delta_T * __expf((Vc - pp.V_T) * pp.inv_Delta_T);
  dy[0] = (__builtin_fmaf(-pp.g_L, V - pp.E_L, ex) - isyn - w + Ie) * pp.inv_C;
  dy[1] = __builtin_fmaf(pp.a, V - pp.E_L, -w) * pp.inv_tau_w;
#pragma unroll
  for (int p = 0; p < P; ++p) dy[2 + p] = -y[2 + p] * pp.inv_tau_syn[p];
}

// One attempted substep of the Cash-Karp embedded 5(4) pair with the
// step-size control of Press et al. (adaptive fifth-order Runge-Kutta,
// Sec. 2.1): relative error against |y| + |h dy/dt| + 1 (state units; a floor
// for variables at zero), shrink by 0.9 e^-1/4 (>= 0.1x) on failure, grow by
// 0.9 e^-1/5 (<= 5x) on success; the last substep lands on the step end.  A
// reset (V >= V_peak) is applied after every accepted substep.  t is the time
// reached inside the step, it the attempts so far, mult the resets.  Returns
// true when the step is complete (t = dt, or the attempt cap reached).
template <int P>
__device__ __forceinline__ bool adex_substep(const PopDev& pp, float* y, float& h, float& t, uint32_t& it,
                                             uint32_t& mult, float Ie, uint32_t& nacc, uint32_t& nrej,
                                             bool& capped) {
  constexpr int NV = 2 + P;
  const float dt = pp.dt;
  const float c21 = 1.f / 5.f;
  const float c31 = 3.f / 40.f, c32 = 9.f / 40.f;
  const float c41 = 3.f / 10.f, c42 = -9.f / 10.f, c43 = 6.f / 5.f;
  const float c51 = -11.f / 54.f, c52 = 5.f / 2.f, c53 = -70.f / 27.f, c54 = 35.f / 27.f;
  const float c61 = 1631.f / 55296.f, c62 = 175.f / 512.f, c63 = 575.f / 13824.f, c64 = 44275.f / 110592.f,
              c65 = 253.f / 4096.f;
  const float b1 = 37.f / 378.f, b3 = 250.f / 621.f, b4 = 125.f / 594.f, b6 = 512.f / 1771.f;
  // error weights: fifth-order minus embedded fourth-order weights
  const float e1 = (float)(37.0 / 378.0 - 2825.0 / 27648.0), e3 = (float)(250.0 / 621.0 - 18575.0 / 48384.0),
              e4 = (float)(125.0 / 594.0 - 13525.0 / 55296.0), e5 = (float)(-277.0 / 14336.0),
              e6 = (float)(512.0 / 1771.0 - 0.25);
  const float errcon = 1.89e-4f;  // (5 / 0.9)^-5
  // smallest substep: the configured floor, but never below 2^-22 dt so that
  // t + h still advances in fp32
  const float hmin = fmaxf(pp.rk_hmin, dt * 2.384185791015625e-7f);
  if (++it > kRkMaxIter) { capped = true; return true; }
  bool last = false;
  if (h >= dt - t) { h = dt - t; last = true; }
  float k1[NV], k2[NV], k3[NV], k4[NV], k5[NV], k6[NV], yt[NV];
  adex_rhs<P>(pp, Ie, y, k1);
#pragma unroll
  for (int i = 0; i < NV; ++i) yt[i] = __builtin_fmaf(h, c21 * k1[i], y[i]);
  adex_rhs<P>(pp, Ie, yt, k2);
#pragma unroll
  for (int i = 0; i < NV; ++i) yt[i] = __builtin_fmaf(h, c31 * k1[i] + c32 * k2[i], y[i]);
  adex_rhs<P>(pp, Ie, yt, k3);
#pragma unroll
  for (int i = 0; i < NV; ++i) yt[i] = __builtin_fmaf(h, c41 * k1[i] + c42 * k2[i] + c43 * k3[i], y[i]);
  adex_rhs<P>(pp, Ie, yt, k4);
#pragma unroll
  for (int i = 0; i < NV; ++i)
    yt[i] = __builtin_fmaf(h, c51 * k1[i] + c52 * k2[i] + c53 * k3[i] + c54 * k4[i], y[i]);
  adex_rhs<P>(pp, Ie, yt, k5);
#pragma unroll
  for (int i = 0; i < NV; ++i)
    yt[i] = __builtin_fmaf(h, c61 * k1[i] + c62 * k2[i] + c63 * k3[i] + c64 * k4[i] + c65 * k5[i], y[i]);
  adex_rhs<P>(pp, Ie, yt, k6);
  float errmax = 0.f;
  float y5[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    y5[i] = __builtin_fmaf(h, b1 * k1[i] + b3 * k3[i] + b4 * k4[i] + b6 * k6[i], y[i]);
    const float err = h * (e1 * k1[i] + e3 * k3[i] + e4 * k4[i] + e5 * k5[i] + e6 * k6[i]);
    const float scale = fabsf(y[i]) + fabsf(h * k1[i]) + 1.f;
    errmax = fmaxf(errmax, fabsf(err) / scale);
  }
  errmax = errmax / pp.rk_eps;
  if (errmax > 1.f && h > hmin) {
    const float ht = 0.9f * h * exp2f(-0.25f * __log2f(errmax));
    h = fmaxf(ht, 0.1f * h);
    h = fmaxf(h, hmin);
    ++nrej;
    return false;
  }
  ++nacc;
  t = last ? dt : t + h;
#pragma unroll
  for (int i = 0; i < NV; ++i) y[i] = y5[i];
  const float hn = fmaxf((errmax > errcon) ? 0.9f * h * exp2f(-0.2f * __log2f(errmax)) : 5.f * h, hmin);
  if (y[0] >= pp.V_peak) { y[0] = pp.V_r; y[1] += pp.b; ++mult; }
  h = hn;
  return !(t < dt);
}

// One dt of the AdEx model: substeps until the step end, h carried to the
// next step (at most dt).  Returns the number of resets.
template <int P>
__device__ uint32_t adex_step(const PopDev& pp, float* y, float& h, float Ie, uint32_t& nacc, uint32_t& nrej,
                              bool& capped) {
  const float dt = pp.dt;
  if (!(h > 0.f) || h > dt) h = dt;
  float t = 0.f;
  uint32_t it = 0, mult = 0;
  while (!adex_substep<P>(pp, y, h, t, it, mult, Ie, nacc, nrej, capped)) {
  }
  if (h > dt) h = dt;
  return mult;
}

constexpr uint32_t kPopLds = 16;  // population tables up to this size are read from LDS
constexpr uint32_t kPoisLds = 8;  // Poisson threshold tables up to this count are read from LDS
constexpr int kSelChunk = 512;    // selected groups held in LDS at a time
constexpr uint32_t kClsLds = 256; // weight classes cached in LDS by direct delivery (more: global)
constexpr int kSelPerThread = kSelChunk / kB;
constexpr uint32_t kTilePopLds = 8;  // population tables a tile block keeps in LDS
constexpr int kTileSubs = kTileAccWords / kB;  // most 256-neuron sub-blocks of a tile

// LDS of the selection: the selected (source, delay-group) records of one
// chunk and their exclusive prefix of group sizes.
struct SelLds {
  uint64_t p_off[kSelChunk];
  uint64_t p_st[kSelChunk];
  uint32_t p_len[kSelChunk];
  uint32_t p_mult[kSelChunk];
  uint64_t red[kB / 64];
  uint64_t seg[66];
  uint32_t slot[66];
  uint32_t npair;
};

// direct delivery: weight classes cached for the atomic adds
struct DirectLds : SelLds {
  int64_t wq[kClsLds];
  uint32_t wp[kClsLds];
};

// binned delivery: events per target tile of the chunk, then each tile's
// reserved position in its bin
struct BinLds : SelLds {
  uint32_t tcnt[kMaxTiles];
  uint32_t tbase[kMaxTiles];
};

// LDS of a direct-delivery update block
struct UpdLds {
  uint32_t wcnt[kB / 64];
  uint64_t red[kB / 64];
  unsigned long long d1[2];
  PopDev spops[kPopLds];
  uint64_t sthr[kPoisLds * kPoisKmax];
};

// LDS of a tile block: the tile's int64 input (dead after the update, then
// reused by the delay-1 binning), weight classes, population and Poisson tables
struct TileLds {
  union {
    int64_t acc[kTileAccWords];
    BinLds d1;
  } u;
  int64_t wq[kMaxClasses];
  uint8_t wp[kMaxClasses];
  PopDev spops[kTilePopLds];
  uint64_t sthr[kPoisLds * kPoisKmax];
  uint32_t wcnt[kTileSubs][kB / 64];
  uint64_t red[kB / 64];
  uint32_t sub_cnt[kTileSubs];
  uint32_t next;  // AdEx work queue: next local neuron to take
};
static_assert(sizeof(BinLds) <= sizeof(int64_t) * kTileAccWords, "delay-1 binning reuses the tile input");

union StepLds {
  UpdLds upd;
  DirectLds dlv;
};

union BinStepLds {
  TileLds tile;
  BinLds dlv;
};

__device__ __forceinline__ void dlv_init(const NetDev& nd, DirectLds& sh) {
  const uint32_t nc = nd.n_classes < kClsLds ? nd.n_classes : kClsLds;
  for (uint32_t c = threadIdx.x; c < nc; c += kB) { sh.wq[c] = nd.cls_wq[c]; sh.wp[c] = nd.cls_port[c]; }
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
__device__ __forceinline__ void dlv_probe(const NetDev& nd, SelLds& sh, uint32_t entry, uint32_t grp_ptr,
                                          uint64_t mask, uint32_t d) {
  if ((mask >> d) & 1ull) {
    const uint32_t g = grp_ptr + (uint32_t)__popcll(mask & ((1ull << d) - 1ull));
    const uint64_t off = nd.grp_off[g];
    const uint32_t len = (uint32_t)(nd.grp_off[g + 1] - off);
    const uint32_t k = atomicAdd(&sh.npair, 1u);  // LDS counter; callers keep k < kSelChunk
    sh.p_off[k] = off;
    sh.p_len[k] = len;
    sh.p_mult[k] = entry >> kMultShift;
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

// Direct delivery of the chunk (flat scan of the synapses of its selected
// groups): every synapse is one item, consecutive lanes take consecutive
// synapses of a group, and each adds multiplicity x quantised weight to the
// int64 input of its (target, port) for the step of parity par1 with a
// device-scope atomic.  Called by the whole block after a barrier; returns
// the events delivered and resets the chunk.
__device__ uint64_t dlv_flush(const NetDev& nd, DirectLds& sh, uint32_t par1) {
  const uint32_t np = sh.npair;
  const uint64_t ev = sel_scan(sh);
  int64_t* acc = nd.acc + (size_t)par1 * nd.N * nd.P;
  const uint32_t cls_bits = nd.cls_bits, cls_mask = (1u << cls_bits) - 1u, P = nd.P;
  for (uint64_t e = threadIdx.x; e < ev; e += kB) {
    const uint32_t lo = sel_find(sh, np, e);
    const uint32_t pl = nd.payload[sh.p_off[lo] + (e - sh.p_st[lo])];
    const uint32_t cls = pl & cls_mask;
    const bool in_lds = cls < kClsLds;
    const int64_t v = (in_lds ? sh.wq[cls] : nd.cls_wq[cls]) * (int64_t)sh.p_mult[lo];
    const uint32_t port = in_lds ? sh.wp[cls] : nd.cls_port[cls];
    __hip_atomic_fetch_add((unsigned long long*)&acc[(size_t)(pl >> cls_bits) * P + port],
                           (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (threadIdx.x == 0) sh.npair = 0;
  __syncthreads();
  return ev;
}

// An event that found its tile's bin full: added to the spill accumulator of
// its (target, port) and the tile flagged, so that the tile block of the next
// step adds the spill to the bin's sum.
__device__ __forceinline__ void bin_spill(const NetDev& nd, uint32_t par1, uint32_t tgt, uint32_t cls, uint32_t mult,
                                       uint32_t tile) {
  const int64_t v = nd.cls_wq[cls] * (int64_t)mult;
  __hip_atomic_fetch_add((unsigned long long*)&nd.acc[((size_t)par1 * nd.N + tgt) * nd.P + nd.cls_port[cls]],
                         (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  nd.ovf_flag[(size_t)par1 * nd.n_tiles + tile] = 1u;
  __hip_atomic_fetch_add((unsigned long long*)&nd.ctrl->spill_events, 1ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// Binned delivery of the chunk: the same flat scan, but each event becomes
// one 32-bit entry (local target, multiplicity, weight class) in the bin of
// its target tile for the step of parity par1; the tile block of that step
// sums its bin in LDS.  Two passes over the chunk's synapses: count the
// events per tile (LDS), reserve each tile's range with one device atomic,
// then write the entries.  Called by the whole block after a barrier;
// returns the events delivered and resets the chunk.
__device__ uint64_t dlv_flush(const NetDev& nd, BinLds& sh, uint32_t par1) {
  const uint32_t np = sh.npair;
  const uint64_t ev = sel_scan(sh);
  // target = pl >> cls_bits, tile = target >> tile_shift: two shifts, each
  // below 32 (their sum can exceed 31 when a tile is wider than the gid range)
  const uint32_t cls_bits = nd.cls_bits, cls_mask = (1u << cls_bits) - 1u;
  const uint32_t tsh = nd.tile_shift, lmask = (1u << tsh) - 1u, ntl = nd.n_tiles;
  bool bad = false;
  for (uint64_t e = threadIdx.x; e < ev; e += kB) {
    const uint32_t lo = sel_find(sh, np, e);
    const uint32_t pl = nd.payload[sh.p_off[lo] + (e - sh.p_st[lo])];
    const uint32_t t = (pl >> cls_bits) >> tsh;
    if (t < ntl) atomicAdd(&sh.tcnt[t], 1u);
    else bad = true;
  }
  __syncthreads();
  uint32_t* cnt = nd.bin_cnt + (size_t)par1 * ntl;
  for (uint32_t t = threadIdx.x; t < ntl; t += kB) {
    const uint32_t c = sh.tcnt[t];
    if (c) {
      sh.tbase[t] = __hip_atomic_fetch_add(&cnt[t], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sh.tcnt[t] = 0;
    }
  }
  __syncthreads();
  uint32_t* bins = nd.bins + (size_t)par1 * nd.bins_total;
  for (uint64_t e = threadIdx.x; e < ev; e += kB) {
    const uint32_t lo = sel_find(sh, np, e);
    const uint32_t pl = nd.payload[sh.p_off[lo] + (e - sh.p_st[lo])];
    const uint32_t tgt = pl >> cls_bits, t = tgt >> tsh;
    if (t >= ntl) continue;
    const uint32_t slot = sh.tbase[t] + atomicAdd(&sh.tcnt[t], 1u);
    const uint32_t cls = pl & cls_mask, mult = sh.p_mult[lo];
    if (slot < nd.bin_cap[t])
      bins[nd.bin_off[t] + slot] = ((tgt & lmask) << kBinLocalShift) | (mult << kBinMultShift) | cls;
    else
      bin_spill(nd, par1, tgt, cls, mult, t);
  }
  if (bad) atomicOr(&nd.ctrl->overflow, 4u);  // a target outside the tiles: reported, not written
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < ntl; t += kB) sh.tcnt[t] = 0;
  if (threadIdx.x == 0) sh.npair = 0;
  __syncthreads();
  return ev;
}

// ------------------------------------------------------------------ update
// One neuron i at step n: Poisson count of the step added to its integer
// input a[] (network input of step n, fixed point), conversion to fp32,
// LIF exact integration (Sec. 2.1, 2.3) or AdEx RK45 (Sec. 2.1, 2.4).
// Returns the number of spikes (resets) in the step, clamped to kMaxMult.
template <bool kLif, bool kAdexOn, int P>
__device__ __forceinline__ uint32_t neuron_step(const NetDev& nd, const PopDev* pops, const uint64_t* pthr,
                                                uint64_t n, uint32_t i, int64_t* a, uint32_t& nacc, uint32_t& nrej,
                                                bool& capped, bool& mover) {
  const PopDev& pp = pops[find_pop(pops, nd.npop, i)];
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
  if (kLif && pp.model != kAdex) {
    float y = nd.V[i];
    int32_t r = nd.refr[i];
    bool s;
    if (pp.model == kLifDelta) {
      s = lif_delta_step(pp, y, r, Ie, x[0]);
    } else {
      float I[kMaxPorts];
#pragma unroll
      for (int p = 0; p < kMaxPorts; ++p) I[p] = (p < pp.n_ports) ? nd.Isyn[(size_t)i * nd.P + p] : 0.f;
      s = lif_exp_step(pp, y, I, r, Ie, x);
#pragma unroll
      for (int p = 0; p < kMaxPorts; ++p)
        if (p < pp.n_ports) nd.Isyn[(size_t)i * nd.P + p] = I[p];
    }
    nd.V[i] = y;
    nd.refr[i] = r;
    m = s ? 1u : 0u;
  }
  if constexpr (kAdexOn) {
    if (pp.model == kAdex) {
      float y[2 + P];
      y[0] = nd.V[i];
      y[1] = nd.w[i];
#pragma unroll
      for (int p = 0; p < P; ++p) y[2 + p] = nd.g[(size_t)i * nd.P + p] + x[p];
      float h = nd.h[i];
      m = adex_step<P>(pp, y, h, Ie, nacc, nrej, capped);
      nd.V[i] = y[0];
      nd.w[i] = y[1];
#pragma unroll
      for (int p = 0; p < P; ++p) nd.g[(size_t)i * nd.P + p] = y[2 + p];
      nd.h[i] = h;
    }
  }
  if (m > kMaxMult) { mover = true; m = kMaxMult; }
  return m;
}

// Spike list of 256-neuron sub-block ub at step n: wave ballot, lane prefix,
// block prefix (gid order), into the stage buffer of the step's parity.
// Returns the sub-block's spike count (block-uniform).  Two barriers.
__device__ __forceinline__ uint32_t stage_spikes(const NetDev& nd, uint64_t n, uint32_t ub, bool spk,
                                                 uint32_t entry, uint32_t* wcnt) {
  const size_t sb = (size_t)(n & 1) * nd.nblk_upd;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t bal = __ballot(spk);
  const uint32_t pre = __popcll(bal & lanemask_lt());
  if (lane == 0) wcnt[wv] = __popcll(bal);
  __syncthreads();
  uint32_t woff = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kB / 64; ++w) {
    if (w < wv) woff += wcnt[w];
    tot += wcnt[w];
  }
  if (spk) nd.stage[(sb + ub) * kB + woff + pre] = entry;
  if (threadIdx.x == 0) nd.stage_cnt[sb + ub] = tot;
  __syncthreads();
  return tot;
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
  if (lds_thr)
    for (uint32_t w = threadIdx.x; w < nd.npois * kPoisKmax; w += kB) sthr[w] = nd.pois_thr[w];
  pops = lds_pops ? spops : nd.pops;
  pthr = lds_thr ? sthr : nd.pois_thr;
}

// Direct-delivery update block: 256 neurons, input from acc[n & 1] (read and
// cleared), spikes staged, delay-1 groups delivered at once.
template <bool kLif, bool kAdexOn, int P>
__device__ void update_block(const NetDev& nd, uint64_t n, uint32_t blk, UpdLds& sl) {
  const PopDev* pops;
  const uint64_t* pthr;
  load_tables(nd, sl.spops, kPopLds, sl.sthr, pops, pthr);
  if (threadIdx.x == 0) { sl.d1[0] = 0; sl.d1[1] = 0; }
  __syncthreads();
  const uint32_t i = blk * kB + threadIdx.x;
  bool spk = false;
  uint32_t entry = 0;
  uint32_t nacc = 0, nrej = 0;
  bool capped = false, mover = false;
  if (i < nd.N) {
    int64_t* acc = nd.acc + ((size_t)(n & 1) * nd.N + i) * nd.P;
    int64_t a[kMaxPorts];
#pragma unroll
    for (int p = 0; p < kMaxPorts; ++p) {
      a[p] = 0;
      if (p < (int)nd.P) {
        a[p] = acc[p];
        if (a[p] != 0) acc[p] = 0;
      }
    }
    const uint32_t m = neuron_step<kLif, kAdexOn, P>(nd, pops, pthr, n, i, a, nacc, nrej, capped, mover);
    spk = m > 0;
    entry = i | (m << kMultShift);
  }
  const uint32_t btot = stage_spikes(nd, n, blk, spk, entry, sl.wcnt);
  // delay-1 groups of this block's spikes reach their targets at the next
  // step: delivered here, each group by the whole wave (consecutive lanes,
  // consecutive synapses)
  {
    const int lane = threadIdx.x & 63;
    uint64_t off = 0;
    uint32_t len = 0;
    bool has1 = false;
    if (spk) {
      const uint64_t mask = nd.src_mask[i];
      if ((mask >> 1) & 1ull) {  // the delay-1 group is the source's first group
        const uint32_t g = nd.grp_ptr[i];
        off = nd.grp_off[g];
        len = (uint32_t)(nd.grp_off[g + 1] - off);
        has1 = true;
      }
    }
    uint64_t bal = __ballot(has1);
    if (bal) {
      int64_t* accn = nd.acc + (size_t)((n + 1) & 1) * nd.N * nd.P;
      const uint32_t cls_bits = nd.cls_bits, cls_mask = (1u << cls_bits) - 1u, P2 = nd.P;
      unsigned long long wp = 0, we = 0;
      while (bal) {
        const int l = __ffsll((unsigned long long)bal) - 1;
        bal &= bal - 1;
        const uint64_t o = __shfl((unsigned long long)off, l, 64);
        const uint32_t L = __shfl(len, l, 64);
        const uint32_t mm = __shfl(entry >> kMultShift, l, 64);
        for (uint32_t j = lane; j < L; j += 64) {
          const uint32_t pl = nd.payload[o + j];
          const uint32_t cls = pl & cls_mask;
          const int64_t v = nd.cls_wq[cls] * (int64_t)mm;
          __hip_atomic_fetch_add((unsigned long long*)&accn[(size_t)(pl >> cls_bits) * P2 + nd.cls_port[cls]],
                                 (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        ++wp;
        we += L;
      }
      if (lane == 0) { atomicAdd(&sl.d1[0], wp); atomicAdd(&sl.d1[1], we); }
    }
  }
  uint64_t sa = 0, sr = 0;
  if (kAdexOn) {
    sa = block_sum(nacc, sl.red);
    sr = block_sum(nrej, sl.red);
  } else {
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    uint64_t* st = nd.blk_stats + (size_t)kBlkStats * blk;
    st[0] += sa;
    st[1] += sr;
    st[2] += btot;
    st[3] += sl.d1[0];
    st[4] += sl.d1[1];
  }
  if (capped) atomicOr(&nd.ctrl->overflow, 2u);
  if (mover) atomicOr(&nd.ctrl->overflow, 1u);
}

// AdEx neuron i at step n as one lane's work item: state and folded input
// loaded, then advanced one RK45 substep per call of adex_substep.
template <int P>
struct AdexItem {
  const PopDev* pp;
  float y[2 + P];
  float h, t, Ie;
  uint32_t it, mult;
};

template <int P>
__device__ __forceinline__ void adex_load(const NetDev& nd, const PopDev* pops, const uint64_t* pthr, uint64_t n,
                                          uint32_t i, int64_t* a, AdexItem<P>& w) {
  const PopDev& pp = pops[find_pop(pops, nd.npop, i)];
  if (pp.pois >= 0) {
    const uint32_t k = poisson_draw(pthr + (size_t)pp.pois * kPoisKmax, pp.seed, i - pp.gid_base, n);
#pragma unroll
    for (int p = 0; p < kMaxPorts; ++p)
      if (p == pp.pois_port) a[p] += (int64_t)k * pp.pois_wq;
  }
  w.pp = &pp;
  w.y[0] = nd.V[i];
  w.y[1] = nd.w[i];
#pragma unroll
  for (int p = 0; p < P; ++p) w.y[2 + p] = nd.g[(size_t)i * nd.P + p] + __fmul_rn((float)a[p], pp.scale[p]);
  w.h = nd.h[i];
  if (!(w.h > 0.f) || w.h > pp.dt) w.h = pp.dt;
  w.Ie = nd.Ie[i];
  w.t = 0.f;
  w.it = 0;
  w.mult = 0;
}

template <int P>
__device__ __forceinline__ uint32_t adex_store(const NetDev& nd, uint32_t i, AdexItem<P>& w, bool& mover) {
  nd.V[i] = w.y[0];
  nd.w[i] = w.y[1];
#pragma unroll
  for (int p = 0; p < P; ++p) nd.g[(size_t)i * nd.P + p] = w.y[2 + p];
  nd.h[i] = (w.h > w.pp->dt) ? w.pp->dt : w.h;
  uint32_t m = w.mult;
  if (m > kMaxMult) { mover = true; m = kMaxMult; }
  return m;
}

// Binned-delivery tile block t at step n: sums the tile's bin (the events
// written for step n by the previous step, plus any spill) into int64 LDS
// accumulators, updates the tile's neurons from them, stages their spikes per
// 256-neuron sub-block and bins the delay-1 groups of those spikes for step
// n+1.  The spike count of a neuron is kept in its (then dead) first LDS
// input slot until all neurons are done.  AdEx-only networks take their
// neurons from a work queue: a lane whose neuron has reached the step end
// takes the next one, so waves stay full while neurons near a spike need many
// RK45 substeps and the others one.
template <bool kLif, bool kAdexOn, int P>
__device__ void tile_block(const NetDev& nd, uint64_t n, uint32_t t, TileLds& sl) {
  const uint32_t par = (uint32_t)(n & 1), PP = nd.P, tsh = nd.tile_shift;
  const uint32_t first = t << tsh;
  const uint32_t nt = min(1u << tsh, nd.N - first);
  const PopDev* pops;
  const uint64_t* pthr;
  load_tables(nd, sl.spops, kTilePopLds, sl.sthr, pops, pthr);
  for (uint32_t c = threadIdx.x; c < nd.n_classes; c += kB) {
    sl.wq[c] = nd.cls_wq[c];
    sl.wp[c] = (uint8_t)nd.cls_port[c];
  }
  for (uint32_t j = threadIdx.x; j < nt * PP; j += kB) sl.u.acc[j] = 0;
  if (threadIdx.x == 0) sl.next = kB;
  const size_t ti = (size_t)par * nd.n_tiles + t;
  const uint32_t cnt = min(nd.bin_cnt[ti], nd.bin_cap[t]);
  const uint32_t ovf = nd.ovf_flag[ti];
  const uint32_t* bin = nd.bins + (size_t)par * nd.bins_total + nd.bin_off[t];
  __syncthreads();
  bool bad = false;
  for (uint32_t j = threadIdx.x; j < cnt; j += kB) {
    const uint32_t e = bin[j];
    const uint32_t cls = e & (uint32_t)(kMaxClasses - 1), loc = e >> kBinLocalShift;
    if (loc >= nt || cls >= nd.n_classes) { bad = true; continue; }
    const int64_t v = sl.wq[cls] * (int64_t)((e >> kBinMultShift) & kMaxMult);
    atomicAdd((unsigned long long*)&sl.u.acc[loc * PP + sl.wp[cls]], (unsigned long long)v);
  }
  if (bad) atomicOr(&nd.ctrl->overflow, 4u);  // a malformed entry: reported, not added
  __syncthreads();
  if (ovf) {  // block-uniform: events that did not fit the bin
    int64_t* g = nd.acc + ((size_t)par * nd.N + first) * PP;
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
  if (kAdexOn && !kLif) {
    // AdEx only: work queue over the tile's neurons
    uint32_t loc = threadIdx.x;
    AdexItem<P> w;
    if (loc < nt) {
      int64_t a[kMaxPorts];
#pragma unroll
      for (int p = 0; p < kMaxPorts; ++p) a[p] = (p < (int)PP) ? sl.u.acc[loc * PP + p] : 0;
      adex_load<P>(nd, pops, pthr, n, first + loc, a, w);
    }
    while (loc < nt) {
      if (adex_substep<P>(*w.pp, w.y, w.h, w.t, w.it, w.mult, w.Ie, nacc, nrej, capped)) {
        sl.u.acc[loc * PP] = (int64_t)adex_store<P>(nd, first + loc, w, mover);
        loc = atomicAdd(&sl.next, 1u);
        if (loc < nt) {
          int64_t a[kMaxPorts];
#pragma unroll
          for (int p = 0; p < kMaxPorts; ++p) a[p] = (p < (int)PP) ? sl.u.acc[loc * PP + p] : 0;
          adex_load<P>(nd, pops, pthr, n, first + loc, a, w);
        }
      }
    }
  } else {
    for (uint32_t loc = threadIdx.x; loc < nt; loc += kB) {
      int64_t a[kMaxPorts];
#pragma unroll
      for (int p = 0; p < kMaxPorts; ++p) a[p] = (p < (int)PP) ? sl.u.acc[loc * PP + p] : 0;
      sl.u.acc[loc * PP] =
          (int64_t)neuron_step<kLif, kAdexOn, P>(nd, pops, pthr, n, first + loc, a, nacc, nrej, capped, mover);
    }
  }
  __syncthreads();
  // spike lists of the tile's 256-neuron sub-blocks (gid order): ballots of
  // all sub-blocks, one barrier, then the writes
  const uint32_t ub0 = first / kB, nsub = (nt + kB - 1) / kB;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint32_t k = 0; k < nsub; ++k) {
    const uint32_t loc = k * kB + threadIdx.x;
    const bool spk = loc < nt && sl.u.acc[loc * PP] != 0;
    const uint64_t bal = __ballot(spk);
    if (lane == 0) sl.wcnt[k][wv] = __popcll(bal);
  }
  __syncthreads();
  const size_t sb = (size_t)par * nd.nblk_upd;
  uint32_t spikes = 0;
  for (uint32_t k = 0; k < nsub; ++k) {
    const uint32_t loc = k * kB + threadIdx.x;
    const uint32_t m = loc < nt ? (uint32_t)sl.u.acc[loc * PP] : 0u;
    const uint64_t bal = __ballot(m != 0);
    uint32_t woff = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kB / 64; ++q) {
      if (q < wv) woff += sl.wcnt[k][q];
      tot += sl.wcnt[k][q];
    }
    if (m) nd.stage[(sb + ub0 + k) * kB + woff + __popcll(bal & lanemask_lt())] = (first + loc) | (m << kMultShift);
    if (threadIdx.x == 0) { nd.stage_cnt[sb + ub0 + k] = tot; sl.sub_cnt[k] = tot; }
    spikes += tot;
  }
  __syncthreads();  // the LDS input is dead from here: it holds the delay-1 selection
  BinLds& sh = sl.u.d1;
  uint64_t pairs = 0, events = 0;
  if (spikes) {  // block-uniform
    dlv_init(nd, sh);
    __syncthreads();
    const uint32_t par1 = par ^ 1u;
    for (uint32_t k = 0; k < nsub; ++k) {  // block-uniform
      const uint32_t c = sl.sub_cnt[k];
      if (threadIdx.x < c) {
        const uint32_t entry = nd.stage[(sb + ub0 + k) * kB + threadIdx.x];
        const uint32_t src = entry & kGidMask;
        const uint64_t mask = nd.src_mask[src];
        if ((mask >> 1) & 1ull) dlv_probe(nd, sh, entry, nd.grp_ptr[src], mask, 1);
      }
      __syncthreads();
      if (sh.npair > (uint32_t)(kSelChunk - kB) || (k + 1 == nsub && sh.npair > 0)) {
        pairs += sh.npair;
        events += dlv_flush(nd, sh, par1);
      }
    }
  }
  uint64_t sa = 0, sr = 0;
  if (kAdexOn) {
    sa = block_sum(nacc, sl.red);
    sr = block_sum(nrej, sl.red);
  }
  if (threadIdx.x == 0) {
    uint64_t* st = nd.blk_stats + (size_t)kBlkStats * ub0;
    st[0] += sa;
    st[1] += sr;
    st[2] += spikes;
    st[3] += pairs;
    st[4] += events;
  }
  if (capped) atomicOr(&nd.ctrl->overflow, 2u);
  if (mover) atomicOr(&nd.ctrl->overflow, 1u);
}

// Spikes of step f = n-1, read from the update blocks' lists of that step:
// block b appends the entries [i0, i1) (ranks within step f, gid order) to
// the raster ring and, if kDeliver, records them for later steps and selects
// their delay-2 groups.  Entries are taken in rounds of at most one per thread.
template <bool kDeliver, class L>
__device__ void walk_step(const NetDev& nd, uint64_t f, uint64_t base_f, uint64_t i0, uint64_t i1, L& sh,
                          uint32_t par1, uint64_t& pairs, uint64_t& events) {
  const size_t sb = (size_t)(f & 1) * nd.nblk_upd;
  SpikeRec* rec = nd.recent + (size_t)(f % nd.R) * nd.N;
  uint64_t run = 0;
  for (uint32_t t0 = 0; t0 < nd.nblk_upd && run < i1; t0 += kB) {  // block-uniform
    const uint32_t ub = t0 + threadIdx.x;
    const uint32_t cc = (ub < nd.nblk_upd) ? nd.stage_cnt[sb + ub] : 0;
    uint64_t tsum;
    const uint64_t p_ub = run + block_excl_scan(cc, sh.red, &tsum);
    const uint64_t lo = p_ub > i0 ? p_ub : i0;
    const uint64_t hi = (p_ub + cc < i1) ? p_ub + cc : i1;
    const uint32_t mine = hi > lo ? (uint32_t)(hi - lo) : 0u;
    const uint32_t rounds = (uint32_t)block_max(mine, sh.red);
    for (uint32_t r = 0; r < rounds; ++r) {  // block-uniform
      if (r < mine) {
        const uint64_t e = lo + r;
        const uint32_t entry = nd.stage[(sb + ub) * kB + (e - p_ub)];
        nd.log[(base_f + e) & nd.log_mask] = entry;
        if (kDeliver) {
          const uint32_t src = entry & kGidMask;
          const uint64_t mask = nd.src_mask[src];
          const uint32_t gp = nd.grp_ptr[src];
          SpikeRec sr;
          sr.entry = entry; sr.grp_ptr = gp; sr.mask = mask;
          rec[e] = sr;
          dlv_probe(nd, sh, entry, gp, mask, 2);
        }
      }
      if (kDeliver) {
        __syncthreads();
        if (sh.npair > (uint32_t)(kSelChunk - kB)) {  // LDS nearly full: deliver now
          pairs += sh.npair;
          events += dlv_flush(nd, sh, par1);
        }
      }
    }
    run += tsum;
  }
}

// Delivery blocks of step n: the input of step n+1 from the spikes of step
// n-1 (delay 2; read from the update blocks' lists of that step, which these
// blocks also append to the raster ring and record) and of steps
// n-2 .. n+1-Dmax (delays >= 3; from the recent-spike records).  Block b owns
// an equal share of all these items (one item = one in-flight spike).
template <class L>
__device__ void deliver_block(const NetDev& nd, uint64_t n, uint32_t b, uint32_t G, L& sh) {
  const uint32_t R = nd.R, dmax = nd.dmax;
  dlv_init(nd, sh);
  const uint32_t dseg = threadIdx.x + 1;  // delay of this item segment (threads 0..63)
  uint64_t cnt = 0;
  uint32_t slt = 0;
  if (threadIdx.x < 64 && dseg >= 3 && dseg <= dmax && n + 1 >= dseg) {
    slt = (uint32_t)((n + 1 - dseg) % R);
    cnt = nd.ring_cnt[slt];
  }
  uint64_t base1 = 0;
  if (n >= 2) base1 = nd.ring_base[(n - 2) % R] + nd.ring_cnt[(n - 2) % R];
  uint64_t c = 0;
  if (n >= 1) {
    const size_t sb = (size_t)((n - 1) & 1) * nd.nblk_upd;
    for (uint32_t ub = threadIdx.x; ub < nd.nblk_upd; ub += kB) c += nd.stage_cnt[sb + ub];
  }
  const uint64_t tot1 = block_sum(c, sh.red);  // spikes of step n-1
  if (threadIdx.x < 64) {
    if (dseg == 2) cnt = tot1;
    const uint64_t incl = wave_incl_scan(cnt);
    sh.seg[dseg] = incl - cnt;
    if (dseg == 64) sh.seg[65] = incl;
    sh.slot[dseg] = slt;
  }
  __syncthreads();
  const uint64_t items = sh.seg[65];
  const uint64_t ipb = (items + G - 1) / G;
  const uint64_t i0 = (uint64_t)b * ipb;
  const uint64_t i1 = (i0 + ipb < items) ? i0 + ipb : items;
  if (b == 0 && threadIdx.x == 0 && n >= 1) {
    nd.ring_base[(n - 1) % R] = base1;
    nd.ring_cnt[(n - 1) % R] = (uint32_t)tot1;
    nd.chunk_base[(n - 1) & (nd.chunk_ring - 1)] = base1;
  }
  const uint32_t par1 = (uint32_t)((n + 1) & 1);
  uint64_t pairs = 0, events = 0;
  // delay 2: spikes of step n-1
  const uint64_t e1 = (i1 < tot1) ? i1 : tot1;
  if (i0 < e1) walk_step<true>(nd, n - 1, base1, i0, e1, sh, par1, pairs, events);
  __syncthreads();
  if (sh.npair > 0) {
    pairs += sh.npair;
    events += dlv_flush(nd, sh, par1);
  }
  // delays >= 3: recent-spike records
  const uint64_t s0 = (i0 > tot1) ? i0 : tot1;
  for (uint64_t c0 = s0; c0 < i1; c0 += kSelChunk) {  // block-uniform
#pragma unroll
    for (int q = 0; q < kSelPerThread; ++q) {
      const uint64_t e = c0 + (uint64_t)q * kB + threadIdx.x;
      if (e >= i1) continue;
      uint32_t d = 3;
      while (d < 64 && sh.seg[d + 1] <= e) ++d;
      const SpikeRec r = nd.recent[(size_t)sh.slot[d] * nd.N + (e - sh.seg[d])];
      dlv_probe(nd, sh, r.entry, r.grp_ptr, r.mask, d);
    }
    __syncthreads();
    pairs += sh.npair;
    events += dlv_flush(nd, sh, par1);
  }
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add((unsigned long long*)&nd.sel_stats[2 * b], (unsigned long long)pairs, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add((unsigned long long*)&nd.sel_stats[2 * b + 1], (unsigned long long)events,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One simulation step n, direct delivery: blocks [0, nblk_upd) update the
// neurons (LIF exact integration, Sec. 2.1/2.3; AdEx RK45, Sec. 2.1/2.4),
// stage their spikes and deliver their delay-1 groups; the remaining blocks
// deliver the earlier steps' spikes whose delay expires now.  All deliveries
// go to the input of step n+1, the update reads the input of step n
// (double-buffered by parity).
template <bool kLif, bool kAdexOn, int P>
__global__ void __launch_bounds__(kB) k_step(NetDev nd, uint32_t rel) {
  __shared__ StepLds lds;
  const uint64_t n = nd.ctrl->step_base + rel;
  if (blockIdx.x < nd.nblk_upd) {
    update_block<kLif, kAdexOn, P>(nd, n, blockIdx.x, lds.upd);
  } else {
    deliver_block(nd, n, blockIdx.x - nd.nblk_upd, gridDim.x - nd.nblk_upd, lds.dlv);
  }
}

// One simulation step n, binned delivery: blocks [0, n_tiles) are the tile
// blocks (input from their bins, update, delay-1 binning), the remaining
// blocks bin the earlier steps' spikes whose delay expires now.
template <bool kLif, bool kAdexOn, int P>
__global__ void __launch_bounds__(kB) k_step_binned(NetDev nd, uint32_t rel) {
  __shared__ BinStepLds lds;
  const uint64_t n = nd.ctrl->step_base + rel;
  if (blockIdx.x < nd.n_tiles) {
    tile_block<kLif, kAdexOn, P>(nd, n, blockIdx.x, lds.tile);
  } else {
    deliver_block(nd, n, blockIdx.x - nd.n_tiles, gridDim.x - nd.n_tiles, lds.dlv);
  }
}

// Raster ring for the last simulated step (step_base - 1): its spikes are
// otherwise appended by the next step's delivery blocks.  Idempotent.
__global__ void __launch_bounds__(kB) k_log_tail(NetDev nd) {
  __shared__ DirectLds sh;
  const uint64_t sbase = nd.ctrl->step_base;
  if (sbase == 0) return;  // block-uniform
  const uint64_t f = sbase - 1;
  const uint32_t R = nd.R;
  const uint64_t base_f = (f >= 1) ? nd.ring_base[(f - 1) % R] + nd.ring_cnt[(f - 1) % R] : 0;
  const size_t sb = (size_t)(f & 1) * nd.nblk_upd;
  uint64_t c = 0;
  for (uint32_t ub = threadIdx.x; ub < nd.nblk_upd; ub += kB) c += nd.stage_cnt[sb + ub];
  const uint64_t tot = block_sum(c, sh.red);
  const uint64_t G = gridDim.x;
  const uint64_t ipb = (tot + G - 1) / G;
  const uint64_t i0 = blockIdx.x * ipb;
  const uint64_t i1 = (i0 + ipb < tot) ? i0 + ipb : tot;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    nd.ring_base[f % R] = base_f;
    nd.ring_cnt[f % R] = (uint32_t)tot;
    nd.chunk_base[f & (nd.chunk_ring - 1)] = base_f;
  }
  uint64_t pairs = 0, events = 0;
  if (i0 < i1) walk_step<false>(nd, f, base_f, i0, i1, sh, 0u, pairs, events);
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

// Readback of the binned input pending for the step of parity par, on one
// port, for gids [first, first + n): block = one tile, entries decoded and
// added to out[gid - first] (which holds the tile's spill already).
__global__ void __launch_bounds__(kB) k_pending_input(NetDev nd, uint32_t par, uint32_t first, uint32_t n,
                                                      uint32_t port, int64_t* out) {
  const uint32_t t = (first >> nd.tile_shift) + blockIdx.x;
  const uint32_t tfirst = t << nd.tile_shift;
  const size_t ti = (size_t)par * nd.n_tiles + t;
  const uint32_t cnt = min(nd.bin_cnt[ti], nd.bin_cap[t]);
  const uint32_t* bin = nd.bins + (size_t)par * nd.bins_total + nd.bin_off[t];
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

template <template <bool, bool, int> class Sel>
static void launch_variant(const NetDev& nd, dim3 grid, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                           uint32_t rel) {
  // which models are present is encoded in nd.pad0: bit 0 LIF, bit 1 AdEx
  const bool lif = nd.pad0 & 1u, adex = nd.pad0 & 2u;
  const dim3 blk(kB);
  if (!adex) {
    launch(Sel<true, false, 1>::fn(), grid, blk, s, start, stop, nd, rel);
  } else {
    switch (nd.P) {
      case 1: if (lif) launch(Sel<true, true, 1>::fn(), grid, blk, s, start, stop, nd, rel);
              else launch(Sel<false, true, 1>::fn(), grid, blk, s, start, stop, nd, rel); break;
      case 2: if (lif) launch(Sel<true, true, 2>::fn(), grid, blk, s, start, stop, nd, rel);
              else launch(Sel<false, true, 2>::fn(), grid, blk, s, start, stop, nd, rel); break;
      case 3: if (lif) launch(Sel<true, true, 3>::fn(), grid, blk, s, start, stop, nd, rel);
              else launch(Sel<false, true, 3>::fn(), grid, blk, s, start, stop, nd, rel); break;
      default: if (lif) launch(Sel<true, true, 4>::fn(), grid, blk, s, start, stop, nd, rel);
               else launch(Sel<false, true, 4>::fn(), grid, blk, s, start, stop, nd, rel); break;
    }
  }
}

template <bool A, bool B, int C>
struct SelDirect {
  static auto fn() { return k_step<A, B, C>; }
};
template <bool A, bool B, int C>
struct SelBinned {
  static auto fn() { return k_step_binned<A, B, C>; }
};

hipError_t launch_step(const NetDev& nd, uint32_t rel, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  if (nd.n_tiles) launch_variant<SelBinned>(nd, dim3(nd.n_tiles + nd.sel_grid), s, start, stop, rel);
  else launch_variant<SelDirect>(nd, dim3(nd.nblk_upd + nd.sel_grid), s, start, stop, rel);
  return hipGetLastError();
}

hipError_t launch_log_tail(const NetDev& nd, hipStream_t s) {
  hipLaunchKernelGGL(k_log_tail, dim3(nd.fresh_grid), dim3(kB), 0, s, nd);
  return hipGetLastError();
}

hipError_t launch_advance(Ctrl* ctrl, uint32_t steps, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctrl, steps);
  return hipGetLastError();
}

hipError_t launch_pending_input(const NetDev& nd, uint32_t par, uint32_t first, uint32_t n, uint32_t port,
                                int64_t* out, hipStream_t s) {
  if (n == 0 || nd.n_tiles == 0) return hipSuccess;
  const uint32_t t0 = first >> nd.tile_shift, t1 = (first + n - 1) >> nd.tile_shift;
  hipLaunchKernelGGL(k_pending_input, dim3(t1 - t0 + 1), dim3(kB), 0, s, nd, par, first, n, port, out);
  return hipGetLastError();
}

hipError_t launch_poisson_counts(const NetDev& nd, uint64_t step, uint32_t first, uint32_t n, uint32_t* k,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_poisson_counts, dim3((n + kB - 1) / kB), dim3(kB), 0, s, nd, step, first, n, k);
  return hipGetLastError();
}

}  // namespace snn
