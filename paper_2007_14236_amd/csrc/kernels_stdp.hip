// kernels_stdp.hip -- nearest-neighbour spike-timing dependent plasticity
// (Sec. 2.1 lists it among the synapse models, after Morrison et al. 2008),
// with the power-law weight dependence of Guetig et al. (2003), in integer
// fixed point so that the result does not depend on the order of the work.
//
// A plastic synapse's spikes are its pre arrivals (step a: the update of
// step a receives the spike) and its target's spikes (step k); within one
// step the arrival comes first.  Each post spike at k pairs with the
// synapse's latest arrival a <= k (potentiation, distance k - a steps), each
// arrival at a with the target's latest spike k < a (depression, distance
// a - k).  With F+(d) = round(lambda e^{-d dt / tau_plus} 2^32) and F-(d) =
// round(alpha lambda e^{-d dt / tau_minus} 2^32) from host tables, and W the
// largest weight in the synapse's fixed-point units:
//   potentiation  w += floor(B+ F+ / 2^32),  B+ = W - w (mu_plus) or W;  w <= W
//   depression    w -= floor(B- F- / 2^32),  B- = w (mu_minus) or W;      w >= 0
// once per unit of multiplicity.  Step n, after its step kernel (which
// delivered the input of step n + 1 with the weights as they were and
// recorded the arrivals of step n + 1 and the spikes of step n): the post
// spikes of step n potentiate, then the arrivals of step n + 1 depress.
#include "kernels.h"

namespace snn {

namespace {

constexpr int kB = 256;

__device__ __forceinline__ int64_t table_at(const NetDev& nd, uint64_t off, uint32_t len, uint64_t d) {
  return d < len ? nd.stdp_F[off + d] : 0;
}

__device__ __forceinline__ const StdpRule& rule_of(const NetDev& nd, uint64_t j) {
  const uint32_t cls = nd.payload[j] & ((1u << nd.cls_bits) - 1u);
  return nd.rules[nd.cls_rule[cls] - 1];
}

// depression of w by `times` arrivals at distance d from the target's latest spike
__device__ __forceinline__ int64_t depress(const NetDev& nd, const StdpRule& r, int64_t w, uint64_t d,
                                           uint32_t times) {
  const int64_t F = table_at(nd, r.off_minus, r.len_minus, d);
  for (uint32_t c = 0; c < times; ++c) {
    const int64_t B = r.mu_minus ? w : r.W;
    w -= (B * F) >> 32;
    if (w < 0) w = 0;
  }
  return w;
}

// Plasticity of step n.  Blocks take the post spikes of step n (one spike
// per block at a time, its lanes over the plastic synapses onto it): each
// synapse is potentiated, and, if it also receives a spike at step n + 1,
// depressed at distance 1.  All lanes then take the arrivals of step n + 1
// onto targets that did not fire at step n.  The two sets of synapses are
// disjoint, and each synapse is one lane's, so no update races.
__global__ void __launch_bounds__(kB) k_stdp(NetDev nd, uint32_t rel) {
  const uint64_t n = nd.ctrl->step_base + rel;
  const uint32_t slot = (uint32_t)(n % nd.R);
  const uint32_t nsp = nd.ring_cnt[slot];
  const uint32_t b1 = (uint32_t)((n + 1) & 1);
  for (uint32_t s = blockIdx.x; s < nsp; s += gridDim.x) {
    const uint32_t entry = nd.recent[(size_t)slot * nd.N + s].entry;
    const uint32_t t = entry & kGidMask, m = entry >> kMultShift;
    const uint64_t k0 = nd.tptr[t], k1 = nd.tptr[t + 1];
    for (uint64_t k = k0 + threadIdx.x; k < k1; k += kB) {
      const uint64_t j = nd.tidx[k];
      const StdpRule& r = rule_of(nd, j);
      int64_t w = nd.pw[j];
      const uint32_t lp = nd.last_pre[j];
      if (lp) {
        const int64_t F = table_at(nd, r.off_plus, r.len_plus, n - (uint64_t)(lp - 1));
        for (uint32_t c = 0; c < m; ++c) {
          const int64_t B = r.mu_plus ? r.W - w : r.W;
          w += (B * F) >> 32;
          if (w > r.W) w = r.W;
        }
      }
      const uint32_t am = nd.arr_m[j];
      if (am) {
        w = depress(nd, r, w, 1, am);
        nd.last_pre[j] = (uint32_t)(n + 2);
        nd.arr_m[j] = 0;
      }
      nd.pw[j] = (int32_t)w;
    }
  }
  const uint32_t na = nd.arr_cnt[b1];
  const uint64_t* list = nd.arr_list + (size_t)b1 * nd.n_plastic;
  for (uint64_t a = (uint64_t)blockIdx.x * kB + threadIdx.x; a < na; a += (uint64_t)gridDim.x * kB) {
    const uint64_t j = list[a];
    const uint32_t t = nd.payload[j] >> nd.cls_bits;
    const uint32_t lpost = nd.last_post[t];
    if (lpost == (uint32_t)(n + 1)) continue;  // fired at step n: done with its spike above
    if (lpost) nd.pw[j] = (int32_t)depress(nd, rule_of(nd, j), nd.pw[j], n + 2 - (uint64_t)lpost, nd.arr_m[j]);
    nd.last_pre[j] = (uint32_t)(n + 2);
    nd.arr_m[j] = 0;
  }
}

// ---- set-up: weights, and the plastic synapses onto each target ----
__global__ void __launch_bounds__(kB) k_stdp_count(NetDev nd, uint32_t* cnt) {
  const uint32_t cls_mask = (1u << nd.cls_bits) - 1u;
  for (uint64_t j = (uint64_t)blockIdx.x * kB + threadIdx.x; j < nd.n_syn; j += (uint64_t)gridDim.x * kB) {
    const uint32_t pl = nd.payload[j];
    const uint32_t cls = pl & cls_mask;
    nd.pw[j] = (int32_t)nd.cls_wq[cls];
    nd.last_pre[j] = 0;
    nd.arr_m[j] = 0;
    if (nd.cls_rule[cls]) atomicAdd(&cnt[pl >> nd.cls_bits], 1u);
  }
}

__global__ void __launch_bounds__(kB) k_stdp_scatter(NetDev nd, uint64_t* cursor, uint64_t* tidx) {
  const uint32_t cls_mask = (1u << nd.cls_bits) - 1u;
  for (uint64_t j = (uint64_t)blockIdx.x * kB + threadIdx.x; j < nd.n_syn; j += (uint64_t)gridDim.x * kB) {
    const uint32_t pl = nd.payload[j];
    if (!nd.cls_rule[pl & cls_mask]) continue;
    const uint64_t k = atomicAdd((unsigned long long*)&cursor[pl >> nd.cls_bits], 1ull);
    tidx[k] = j;
  }
}

uint32_t grid_for(uint64_t items) {
  const uint64_t b = (items + kB - 1) / kB;
  return (uint32_t)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

hipError_t launch_stdp(const NetDev& nd, uint32_t rel, hipStream_t s) {
  if (!nd.n_rules) return hipSuccess;
  hipLaunchKernelGGL(k_stdp, dim3(512), dim3(kB), 0, s, nd, rel);
  return hipGetLastError();
}

hipError_t launch_stdp_count(const NetDev& nd, uint32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_stdp_count, dim3(grid_for(nd.n_syn)), dim3(kB), 0, s, nd, cnt);
  return hipGetLastError();
}

hipError_t launch_stdp_scatter(const NetDev& nd, uint64_t* cursor, uint64_t* tidx, hipStream_t s) {
  hipLaunchKernelGGL(k_stdp_scatter, dim3(grid_for(nd.n_syn)), dim3(kB), 0, s, nd, cursor, tidx);
  return hipGetLastError();
}

}  // namespace snn
