// kernels_step.hip -- one simulation step on the device.
//
// Step n (Golosio et al., Sec. 2.1 and 2.2):
//   1. update   : every neuron folds the integer input delivered for step n
//                 (plus its Poisson count) into fp32, advances its dynamics
//                 over dt and, if it fires, is appended to the block's spike
//                 list (wave ballot + lane prefix + block prefix, gid order).
//   2. select + deliver: compacts the block lists of step n into the spike
//                 ring and selects every (source, delay group) pair whose delay
//                 d has just elapsed: spikes of step n+1-d whose source has a
//                 group of delay d (bit d of the source's delay mask; the group
//                 is found by a popcount of the lower bits, so no loop over the
//                 groups is needed -- the role of the ordered group index of
//                 Fig. 1).  The selected groups are scanned in LDS into one
//                 flat index space over their synapses; each synapse adds
//                 multiplicity x quantised weight to the int64 input of its
//                 (target, port) for step n+1 (integer atomics: the sum does
//                 not depend on their order).
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

// spike list of the block: order-preserving compaction by gid
__device__ __forceinline__ void block_stage_spikes(const NetDev& nd, bool spk, uint32_t entry, uint32_t* wcnt) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t bal = __ballot(spk);
  const uint32_t pre = __popcll(bal & lanemask_lt());
  if (lane == 0) wcnt[wv] = __popcll(bal);
  __syncthreads();
  uint32_t woff = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kB / 64; ++i) {
    if (i < wv) woff += wcnt[i];
    tot += wcnt[i];
  }
  if (spk) nd.stage[(size_t)blockIdx.x * kB + woff + pre] = entry;
  if (threadIdx.x == 0) nd.stage_cnt[blockIdx.x] = tot;
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

template <bool kLif, bool kAdexOn, int P>
__global__ void __launch_bounds__(kB) k_update(NetDev nd, uint32_t rel) {
  __shared__ uint32_t wcnt[kB / 64];
  __shared__ PopDev spops[kPopLds];
  __shared__ uint64_t sthr[kPoisLds * kPoisKmax];
  const uint64_t n = nd.ctrl->step_base + rel;
  const uint32_t i = blockIdx.x * kB + threadIdx.x;
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
  block_stage_spikes(nd, spk, entry, wcnt);
  if (kAdexOn) {
    __shared__ uint64_t red[kB / 64];
    const uint64_t sa = block_sum(nacc, red);
    const uint64_t sr = block_sum(nrej, red);
    if (threadIdx.x == 0) {
      nd.blk_stats[2 * blockIdx.x] += sa;
      nd.blk_stats[2 * blockIdx.x + 1] += sr;
    }
  }
  if (capped) atomicOr(&nd.ctrl->overflow, 2u);
  if (mover) atomicOr(&nd.ctrl->overflow, 1u);
}

// ------------------------------------------------------------------ select
// ----------------------------------------------------------- select+deliver
// Block b owns the item range [i0, i1) of step n's selection items: first the
// spikes of step n (delay 1, read from the update blocks' lists and copied into
// the spike ring by the block that owns them), then those of steps n-1 ..
// n+1-Dmax (delays 2..Dmax, read from the ring).  Items are taken in chunks of
// kSelChunk: every item whose source has a group of the item's delay yields
// one (synapse offset, group size, multiplicity) record in LDS; the chunk's
// records are scanned in LDS (exclusive prefix of the sizes) and their
// synapses delivered in one flat pass by the whole block, so consecutive
// lanes read consecutive synapses of a group.  Integer atomics make the result
// independent of the order in which blocks and lanes deliver.
constexpr int kSelChunk = 1024;
constexpr int kSelPerThread = kSelChunk / kB;

__global__ void __launch_bounds__(kB) k_select_deliver(NetDev nd, uint32_t rel) {
  __shared__ uint64_t red[kB / 64];
  __shared__ uint64_t seg[66];
  __shared__ uint64_t sbase[66];
  __shared__ uint64_t p_off[kSelChunk];
  __shared__ uint64_t p_st[kSelChunk];
  __shared__ uint32_t p_len[kSelChunk];
  __shared__ uint32_t p_mult[kSelChunk];
  __shared__ int64_t wq[kMaxClasses];
  __shared__ uint32_t wp[kMaxClasses];
  __shared__ uint32_t npair;
  const uint64_t n = nd.ctrl->step_base + rel;
  const uint32_t R = nd.R, dmax = nd.dmax;
  for (uint32_t c = threadIdx.x; c < nd.n_classes; c += kB) { wq[c] = nd.cls_wq[c]; wp[c] = nd.cls_port[c]; }
  const uint32_t cls_bits = nd.cls_bits, cls_mask = (1u << cls_bits) - 1u;
  // ring entries of the earlier steps (independent of the reduction below)
  uint64_t cnt = 0, bb = 0;
  const uint32_t dseg = threadIdx.x + 1;  // delay of this item segment (threads 0..63)
  if (threadIdx.x < 64 && dseg >= 2 && dseg <= dmax && n + 1 >= dseg) {
    cnt = nd.ring_cnt[(n + 1 - dseg) % R];
    bb = nd.ring_base[(n + 1 - dseg) % R];
  }
  const uint64_t base_n = (n == 0) ? 0 : nd.ring_base[(n - 1) % R] + nd.ring_cnt[(n - 1) % R];
  // |S_n|: spikes staged by the update blocks of step n
  uint64_t c = 0;
  for (uint32_t ub = threadIdx.x; ub < nd.nblk_upd; ub += kB) c += nd.stage_cnt[ub];
  const uint64_t tot = block_sum(c, red);
  if (threadIdx.x < 64) {
    if (dseg == 1) { cnt = tot; bb = base_n; }
    const uint64_t incl = wave_incl_scan(cnt);
    seg[dseg] = incl - cnt;
    if (dseg == 64) seg[65] = incl;
    sbase[dseg] = bb;
  }
  __syncthreads();
  const uint64_t items = seg[65];
  const uint64_t G = gridDim.x;
  const uint64_t ipb = (items + G - 1) / G;
  const uint64_t i0 = blockIdx.x * ipb;
  const uint64_t i1 = (i0 + ipb < items) ? i0 + ipb : items;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    nd.ring_base[n % R] = base_n;
    nd.ring_cnt[n % R] = (uint32_t)tot;
    nd.chunk_base[n & (nd.chunk_ring - 1)] = base_n;
    nd.ctrl->tot_spikes += tot;
  }
  // copy this block's share of step n's spikes into the ring (gid order)
  const uint64_t e1 = (i1 < tot) ? i1 : tot;
  if (i0 < e1) {
    uint64_t run = 0;
    for (uint32_t t0 = 0; t0 < nd.nblk_upd && run < e1; t0 += kB) {
      const uint32_t ub = t0 + threadIdx.x;
      const uint32_t cc = (ub < nd.nblk_upd) ? nd.stage_cnt[ub] : 0;
      uint64_t tsum;
      const uint64_t p_ub = run + block_excl_scan(cc, red, &tsum);
      const uint64_t lo = p_ub > i0 ? p_ub : i0;
      const uint64_t hi = (p_ub + cc < e1) ? p_ub + cc : e1;
      for (uint64_t e = lo; e < hi; ++e) nd.log[(base_n + e) & nd.log_mask] = nd.stage[(size_t)ub * kB + (e - p_ub)];
      run += tsum;
    }
  }
  __syncthreads();  // the block reads back only the ring entries it wrote itself
  int64_t* acc = nd.acc + (size_t)((n + 1) & 1) * nd.N * nd.P;
  const uint32_t P = nd.P;
  uint64_t blk_pairs = 0, blk_events = 0;
  for (uint64_t c0 = i0; c0 < i1; c0 += kSelChunk) {  // block-uniform
    if (threadIdx.x == 0) npair = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSelPerThread; ++q) {
      const uint64_t e = c0 + (uint64_t)q * kB + threadIdx.x;
      if (e >= i1) continue;
      uint32_t d = 1;
      while (d < 64 && seg[d + 1] <= e) ++d;
      const uint32_t entry = nd.log[(sbase[d] + (e - seg[d])) & nd.log_mask];
      const uint32_t src = entry & kGidMask;
      if (src >= nd.N) {  // never true for entries written by this pipeline
        atomicOr(&nd.ctrl->overflow, 4u);
        continue;
      }
      const uint64_t mask = nd.src_mask[src];
      if ((mask >> d) & 1ull) {
        const uint32_t g = nd.grp_ptr[src] + (uint32_t)__popcll(mask & ((1ull << d) - 1ull));
        const uint64_t off = nd.grp_off[g];
        const uint32_t len = (uint32_t)(nd.grp_off[g + 1] - off);
        const uint32_t k = atomicAdd(&npair, 1u);  // LDS counter, k < kSelChunk
        p_off[k] = off;
        p_len[k] = len;
        p_mult[k] = entry >> kMultShift;
      }
    }
    __syncthreads();
    const uint32_t np = npair;
    // exclusive prefix of the group sizes (each thread owns kSelPerThread records)
    uint32_t L[kSelPerThread];
    uint64_t lsum = 0;
#pragma unroll
    for (int q = 0; q < kSelPerThread; ++q) {
      const uint32_t i = threadIdx.x * kSelPerThread + q;
      L[q] = (i < np) ? p_len[i] : 0u;
      lsum += L[q];
    }
    uint64_t ev;
    uint64_t run = block_excl_scan(lsum, red, &ev);
#pragma unroll
    for (int q = 0; q < kSelPerThread; ++q) {
      const uint32_t i = threadIdx.x * kSelPerThread + q;
      if (i < np) p_st[i] = run;
      run += L[q];
    }
    __syncthreads();
    for (uint64_t e = threadIdx.x; e < ev; e += kB) {
      uint32_t lo = 0, hi = np;  // last record with p_st <= e
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (p_st[mid] <= e) lo = mid; else hi = mid;
      }
      const uint32_t pl = nd.payload[p_off[lo] + (e - p_st[lo])];
      const uint32_t cls = pl & cls_mask;
      const int64_t v = wq[cls] * (int64_t)p_mult[lo];
      __hip_atomic_fetch_add((unsigned long long*)&acc[(size_t)(pl >> cls_bits) * P + wp[cls]],
                             (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    blk_pairs += np;
    blk_events += ev;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    nd.sel_stats[2 * blockIdx.x] += blk_pairs;
    nd.sel_stats[2 * blockIdx.x + 1] += blk_events;
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

}  // namespace

// Launch helper: with events, the kernel is launched by hipExtLaunchKernelGGL,
// which records `start` and `stop` on the dispatch itself (kernel duration).
template <typename K, typename... Args>
static void launch(K kernel, dim3 grid, dim3 blk, hipStream_t s, hipEvent_t start, hipEvent_t stop, Args... args) {
  if (start) hipExtLaunchKernelGGL(kernel, grid, blk, 0, s, start, stop, 0, args...);
  else hipLaunchKernelGGL(kernel, grid, blk, 0, s, args...);
}

hipError_t launch_update(const NetDev& nd, uint32_t rel, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  // which models are present is encoded in nd.pad0: bit 0 LIF, bit 1 AdEx
  const bool lif = nd.pad0 & 1u, adex = nd.pad0 & 2u;
  const dim3 grid(nd.nblk_upd), blk(kB);
  if (!adex) {
    launch(k_update<true, false, 1>, grid, blk, s, start, stop, nd, rel);
  } else {
    switch (nd.P) {
      case 1: if (lif) launch(k_update<true, true, 1>, grid, blk, s, start, stop, nd, rel);
              else launch(k_update<false, true, 1>, grid, blk, s, start, stop, nd, rel); break;
      case 2: if (lif) launch(k_update<true, true, 2>, grid, blk, s, start, stop, nd, rel);
              else launch(k_update<false, true, 2>, grid, blk, s, start, stop, nd, rel); break;
      case 3: if (lif) launch(k_update<true, true, 3>, grid, blk, s, start, stop, nd, rel);
              else launch(k_update<false, true, 3>, grid, blk, s, start, stop, nd, rel); break;
      default: if (lif) launch(k_update<true, true, 4>, grid, blk, s, start, stop, nd, rel);
               else launch(k_update<false, true, 4>, grid, blk, s, start, stop, nd, rel); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_select_deliver(const NetDev& nd, uint32_t rel, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  launch(k_select_deliver, dim3(nd.sel_grid), dim3(kB), s, start, stop, nd, rel);
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
