// kernels_step.hip -- one simulation step on the device.
//
// Step n (Golosio et al., Sec. 2.1 and 2.2) is two kernels:
//   1. k_step_main: update blocks -- every neuron folds the integer input
//      delivered for step n (plus its Poisson count) into fp32, advances its
//      dynamics over dt and, if it fires, is appended to its block's spike
//      list (wave ballot + lane prefix + block prefix, gid order); delivery
//      blocks in the same launch -- the spikes of steps n-1 .. n+1-Dmax whose
//      delay d expires now reach their delay-d connection group.
//   2. k_step_fresh: the spikes of step n are appended to the raster ring,
//      recorded for later steps, and delivered to their delay-1 groups.
// A spike reaches a group of delay d iff bit d of its source's delay mask is
// set; the group is found by a popcount of the lower bits (the groups of a
// source are ordered by delay), so there is no loop over the groups -- the
// role of the ordered connection-group index of Fig. 1.  Selected groups are
// scanned in LDS into one flat index space over their synapses; each synapse
// adds multiplicity x quantised weight to the int64 input of its (target,
// port) for step n+1.  Integer atomics: the sum does not depend on order.
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

// One dt with the Cash-Karp embedded 5(4) pair and the step-size control of
// Press et al. (adaptive fifth-order Runge-Kutta, Sec. 2.1): relative error
// against |y| + |h dy/dt| + 1 (state units; a floor for variables at zero), shrink by 0.9 e^-1/4 (>= 0.1x) on failure, grow by
// 0.9 e^-1/5 (<= 5x) on success; the last substep lands on the step end; h is
// carried to the next step.  A reset (V >= V_peak) is applied after every
// accepted substep.  Returns the number of resets.
template <int P>
__device__ uint32_t adex_step(const PopDev& pp, float* y, float& h, float Ie, uint32_t& nacc, uint32_t& nrej,
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
  float t = 0.f;
  if (!(h > 0.f) || h > dt) h = dt;
  uint32_t mult = 0, it = 0;
  float k1[NV], k2[NV], k3[NV], k4[NV], k5[NV], k6[NV], yt[NV];
  while (t < dt) {
    if (++it > kRkMaxIter) { capped = true; break; }
    bool last = false;
    if (h >= dt - t) { h = dt - t; last = true; }
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
      continue;
    }
    ++nacc;
    t = last ? dt : t + h;
#pragma unroll
    for (int i = 0; i < NV; ++i) y[i] = y5[i];
    const float hn = fmaxf((errmax > errcon) ? 0.9f * h * exp2f(-0.2f * __log2f(errmax)) : 5.f * h, hmin);
    if (y[0] >= pp.V_peak) { y[0] = pp.V_r; y[1] += pp.b; ++mult; }
    h = hn;
  }
  if (h > dt) h = dt;
  return mult;
}

constexpr uint32_t kPopLds = 16;  // population tables up to this size are read from LDS
constexpr uint32_t kPoisLds = 8;  // Poisson threshold tables up to this count are read from LDS
constexpr int kSelChunk = 512;    // selected groups held in LDS at a time
constexpr uint32_t kClsLds = 256; // weight classes cached in LDS (more are read from global memory)
constexpr int kSelPerThread = kSelChunk / kB;

// LDS of the delivery routine: the selected (source, delay-group) records of
// one chunk, their exclusive prefix of group sizes, and the weight classes.
struct DlvLds {
  uint64_t p_off[kSelChunk];
  uint64_t p_st[kSelChunk];
  uint32_t p_len[kSelChunk];
  uint32_t p_mult[kSelChunk];
  int64_t wq[kClsLds];
  uint32_t wp[kClsLds];
  uint64_t red[kB / 64];
  uint64_t seg[66];
  uint32_t slot[66];
  uint32_t npair;
};

// LDS of an update block
struct UpdLds {
  uint32_t wcnt[kB / 64];
  uint64_t red[kB / 64];
  unsigned long long d1[2];
  PopDev spops[kPopLds];
  uint64_t sthr[kPoisLds * kPoisKmax];
};

union StepLds {
  UpdLds upd;
  DlvLds dlv;
};

__device__ __forceinline__ void dlv_load_classes(const NetDev& nd, DlvLds& sh) {
  const uint32_t nc = nd.n_classes < kClsLds ? nd.n_classes : kClsLds;
  for (uint32_t c = threadIdx.x; c < nc; c += kB) { sh.wq[c] = nd.cls_wq[c]; sh.wp[c] = nd.cls_port[c]; }
  if (threadIdx.x == 0) sh.npair = 0;
}

// Selection of one in-flight spike for delay d (Sec. 2.2, Fig. 1): the spike
// reaches a connection group now iff its source has a group of delay d (bit d
// of the delay mask); that group's index among the source's groups, which are
// ordered by delay, is the number of lower bits set.
__device__ __forceinline__ void dlv_probe(const NetDev& nd, DlvLds& sh, uint32_t entry, uint32_t grp_ptr,
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

// Flat scan of the synapses of the chunk's selected groups: exclusive prefix
// of the group sizes in LDS, then every synapse of every group is one item;
// each item reads one synapse word (consecutive lanes, consecutive synapses of
// a group) and adds multiplicity x quantised weight to the int64 input of its
// (target, port) for the next step.  Called by the whole block after a
// barrier; returns the events delivered and resets the chunk.
__device__ uint64_t dlv_flush(const NetDev& nd, DlvLds& sh, int64_t* acc) {
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
  const uint32_t cls_bits = nd.cls_bits, cls_mask = (1u << cls_bits) - 1u, P = nd.P;
  for (uint64_t e = threadIdx.x; e < ev; e += kB) {
    uint32_t lo = 0, hi = np;  // last record with p_st <= e
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (sh.p_st[mid] <= e) lo = mid; else hi = mid;
    }
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

// ------------------------------------------------------------------ update
template <bool kLif, bool kAdexOn, int P>
__device__ void update_block(const NetDev& nd, uint64_t n, uint32_t blk, UpdLds& sl) {
  uint32_t* wcnt = sl.wcnt;
  PopDev* spops = sl.spops;
  uint64_t* sthr = sl.sthr;
  uint64_t* red = sl.red;
  const uint32_t i = blk * kB + threadIdx.x;
  const bool lds_pops = nd.npop <= kPopLds;
  const bool lds_thr = nd.npois <= kPoisLds;
  if (lds_pops) {
    const uint32_t words = nd.npop * (uint32_t)(sizeof(PopDev) / 4);
    for (uint32_t w = threadIdx.x; w < words; w += kB)
      reinterpret_cast<uint32_t*>(spops)[w] = reinterpret_cast<const uint32_t*>(nd.pops)[w];
  }
  if (lds_thr)
    for (uint32_t w = threadIdx.x; w < nd.npois * kPoisKmax; w += kB) sthr[w] = nd.pois_thr[w];
  __syncthreads();
  const PopDev* pops = lds_pops ? spops : nd.pops;
  const uint64_t* pthr = lds_thr ? sthr : nd.pois_thr;
  bool spk = false;
  uint32_t entry = 0;
  uint32_t nacc = 0, nrej = 0;
  bool capped = false, mover = false;
  if (i < nd.N) {
    const PopDev& pp = pops[find_pop(pops, nd.npop, i)];
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
    spk = m > 0;
    entry = i | (m << kMultShift);
  }
  // spike list of the block: wave ballot, lane prefix, block prefix (gid
  // order), into the stage buffer of this step's parity
  const size_t sb = (size_t)(n & 1) * nd.nblk_upd;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t btot;
  {
    const uint64_t bal = __ballot(spk);
    const uint32_t pre = __popcll(bal & lanemask_lt());
    if (lane == 0) wcnt[wv] = __popcll(bal);
    if (threadIdx.x == 0) { sl.d1[0] = 0; sl.d1[1] = 0; }
    __syncthreads();
    uint32_t woff = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kB / 64; ++w) {
      if (w < wv) woff += wcnt[w];
      tot += wcnt[w];
    }
    btot = tot;
    if (spk) nd.stage[(sb + blk) * kB + woff + pre] = entry;
    if (threadIdx.x == 0) nd.stage_cnt[sb + blk] = tot;
  }
  // delay-1 groups of this block's spikes reach their targets at the next
  // step: delivered here, each group by the whole wave (consecutive lanes,
  // consecutive synapses)
  {
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
    sa = block_sum(nacc, red);
    sr = block_sum(nrej, red);
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

// Spikes of step f = n-1, read from the update blocks' lists of that step:
// block b appends the entries [i0, i1) (ranks within step f, gid order) to
// the raster ring and, if kDeliver, records them for later steps and selects
// their delay-2 groups.  Entries are taken in rounds of at most one per thread.
template <bool kDeliver>
__device__ void walk_step(const NetDev& nd, uint64_t f, uint64_t base_f, uint64_t i0, uint64_t i1, DlvLds& sh,
                          int64_t* acc, uint64_t& pairs, uint64_t& events) {
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
          events += dlv_flush(nd, sh, acc);
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
__device__ void deliver_block(const NetDev& nd, uint64_t n, uint32_t b, uint32_t G, DlvLds& sh) {
  const uint32_t R = nd.R, dmax = nd.dmax;
  dlv_load_classes(nd, sh);
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
  int64_t* acc = nd.acc + (size_t)((n + 1) & 1) * nd.N * nd.P;
  uint64_t pairs = 0, events = 0;
  // delay 2: spikes of step n-1
  const uint64_t e1 = (i1 < tot1) ? i1 : tot1;
  if (i0 < e1) walk_step<true>(nd, n - 1, base1, i0, e1, sh, acc, pairs, events);
  __syncthreads();
  if (sh.npair > 0) {
    pairs += sh.npair;
    events += dlv_flush(nd, sh, acc);
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
    events += dlv_flush(nd, sh, acc);
  }
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add((unsigned long long*)&nd.sel_stats[2 * b], (unsigned long long)pairs, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add((unsigned long long*)&nd.sel_stats[2 * b + 1], (unsigned long long)events,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One simulation step n: blocks [0, nblk_upd) update the neurons (LIF exact
// integration, Sec. 2.1/2.3; AdEx RK45, Sec. 2.1/2.4), stage their spikes and
// deliver their delay-1 groups; the remaining blocks deliver the earlier
// steps' spikes whose delay expires now.  All deliveries go to the input of
// step n+1, the update reads the input of step n (double-buffered by parity).
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

// Raster ring for the last simulated step (step_base - 1): its spikes are
// otherwise appended by the next step's delivery blocks.  Idempotent.
__global__ void __launch_bounds__(kB) k_log_tail(NetDev nd) {
  __shared__ DlvLds sh;
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
  if (i0 < i1) walk_step<false>(nd, f, base_f, i0, i1, sh, nullptr, pairs, events);
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

}  // namespace

// Launch helper: with events, the kernel is launched by hipExtLaunchKernelGGL,
// which records `start` and `stop` on the dispatch itself (kernel duration).
template <typename K, typename... Args>
static void launch(K kernel, dim3 grid, dim3 blk, hipStream_t s, hipEvent_t start, hipEvent_t stop, Args... args) {
  if (start) hipExtLaunchKernelGGL(kernel, grid, blk, 0, s, start, stop, 0, args...);
  else hipLaunchKernelGGL(kernel, grid, blk, 0, s, args...);
}

hipError_t launch_step(const NetDev& nd, uint32_t rel, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  // which models are present is encoded in nd.pad0: bit 0 LIF, bit 1 AdEx
  const bool lif = nd.pad0 & 1u, adex = nd.pad0 & 2u;
  const dim3 grid(nd.nblk_upd + nd.sel_grid), blk(kB);
  if (!adex) {
    launch(k_step<true, false, 1>, grid, blk, s, start, stop, nd, rel);
  } else {
    switch (nd.P) {
      case 1: if (lif) launch(k_step<true, true, 1>, grid, blk, s, start, stop, nd, rel);
              else launch(k_step<false, true, 1>, grid, blk, s, start, stop, nd, rel); break;
      case 2: if (lif) launch(k_step<true, true, 2>, grid, blk, s, start, stop, nd, rel);
              else launch(k_step<false, true, 2>, grid, blk, s, start, stop, nd, rel); break;
      case 3: if (lif) launch(k_step<true, true, 3>, grid, blk, s, start, stop, nd, rel);
              else launch(k_step<false, true, 3>, grid, blk, s, start, stop, nd, rel); break;
      default: if (lif) launch(k_step<true, true, 4>, grid, blk, s, start, stop, nd, rel);
               else launch(k_step<false, true, 4>, grid, blk, s, start, stop, nd, rel); break;
    }
  }
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

hipError_t launch_poisson_counts(const NetDev& nd, uint64_t step, uint32_t first, uint32_t n, uint32_t* k,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_poisson_counts, dim3((n + kB - 1) / kB), dim3(kB), 0, s, nd, step, first, n, k);
  return hipGetLastError();
}

}  // namespace snn
