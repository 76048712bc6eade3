// kernels_build.hip -- on-device connectivity build (the paper keeps this on
// the host and names building it on the GPU as future work, Sec. 4).
//
// Connection rules (Sec. 2.1), one Philox4x64-10 block per work item, key
// (seed, 0), tag CONN, gids and p counted inside the projection's instance:
//   fixed in-degree  -- target t draws K sources: block (t, p << 40 | k >> 1),
//                       words 2(k&1) (source) and 2(k&1)+1 (delay);
//   fixed out-degree -- source s draws K targets: block (s, p << 40 | k >> 1),
//                       words 2(k&1) (target) and 2(k&1)+1 (delay);
//   all-to-all       -- target t, source index k: block (t, p << 40 | k >> 1),
//                       word 2(k&1)+1 (delay);
//   one-to-one       -- target t: block (t, p << 40), word 1 (delay);
//   fixed total      -- synapse j: block (j, p << 40), words 0 (source),
//                       1 (target), 2 (delay);
//   user-defined     -- synapse j as listed (no draw).
// A uniform index in a range of m is floor(u m / 2^64); a delay is the top 32
// bits of its word against the projection's threshold table.  A weight drawn
// from a distribution (Sec. 2.1) is the level of the top 32 bits of word k&3
// of block (c0, p << 40 | k >> 2) with tag WEIGHT, c0 the first counter word
// of the synapse's connection draw and k its draw index (0 for one-to-one
// and the fixed total number), against the level thresholds.
//
// Layout (Sec. 2.2, Fig. 1): synapses grouped per source into connection
// groups of equal delay, groups ordered by delay.  Build = counting sort by
// (source, delay) -- histogram, exclusive scan, scatter -- then every group is
// sorted by payload (target << 6 | class) so that the CSR is the unique
// canonical arrangement (source, delay, target, port, weight).
#include "kernels.h"
#include "philox_dev.h"

namespace snn {

namespace {

constexpr int kB = 256;
constexpr int kTagWeight = 3;  // Philox tag of the weight draws (connections 1, Poisson 2)

__device__ __forceinline__ uint32_t find_proj(const ProjDev* projs, uint32_t nproj, uint64_t q) {
  uint32_t lo = 0, hi = nproj;  // largest p with pair_begin <= q
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (projs[mid].pair_begin <= q) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t draw_delay(const uint64_t* thr, uint32_t dmax, uint32_t u) {
  // smallest d in [1, dmax] with u < thr[d]; thr is non-decreasing, thr[dmax] = 2^32
  uint32_t lo = 1, hi = dmax;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if ((uint64_t)u < thr[mid]) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t draw_level(const uint64_t* thr, uint32_t levels, uint32_t u) {
  // smallest j with u < thr[j]; thr[levels - 1] = 2^32
  uint32_t lo = 0, hi = levels - 1;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if ((uint64_t)u < thr[mid]) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t find_pop(const uint32_t* pop_first, uint32_t npop, uint32_t gid) {
  uint32_t lo = 0, hi = npop;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (pop_first[mid] <= gid) lo = mid; else hi = mid;
  }
  return lo;
}

// The synapse draw of work item q (Sec. 2.1 rules; counter layout in the
// header comment of the library): entity e and pair kp of projection p, up to
// two synapses, each counted (histogram) or scattered into its (source,
// delay) bucket.
template <bool kScatter>
__global__ void __launch_bounds__(kB) k_gen(const ProjDev* __restrict__ projs, uint32_t nproj, uint64_t total_pairs,
                                             uint32_t dmax_cfg, uint32_t D1, uint32_t* cnt,
                                             unsigned long long* cursor, uint32_t* payload, const uint16_t* cls_of,
                                             const ProjW* pw, const uint32_t* pop_first, uint32_t npop,
                                             uint32_t cls_bits) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total_pairs; q += stride) {
    const uint32_t p = find_proj(projs, nproj, q);
    const ProjDev& pr = projs[p];
    const uint64_t local = q - pr.pair_begin;
    const uint64_t e = local / pr.kpairs;
    const uint32_t kp = (uint32_t)(local - e * pr.kpairs);
    // entity gid (instance-local in the counter): target, source, or none
    const uint32_t ent = pr.rule == kRuleOutDegree ? pr.src_first + (uint32_t)e
                       : pr.rule == kRuleTotal ? 0u : pr.tgt_first + (uint32_t)e;
    if (pr.rule == kRuleList) {  // user-defined: synapse e as listed, no draw
      const uint32_t src = pr.lsrc[e], tgt = pr.ltgt[e];
      const uint64_t bucket = (uint64_t)src * D1 + pr.ldel[e];
      if (!kScatter) {
        atomicAdd(&cnt[bucket], 1u);
      } else {
        const uint32_t k = find_pop(pop_first, npop, tgt);
        const ProjW& w = pw[p];
        const uint32_t cls = w.levels ? w.cls[(k - w.pop0) * w.levels + w.lvl[e]] : cls_of[(size_t)p * npop + k];
        const unsigned long long slot = atomicAdd(&cursor[bucket], 1ull);
        payload[slot] = (tgt << cls_bits) | cls;
      }
      continue;
    }
    const uint64_t c0 = pr.rule == kRuleTotal ? e : (uint64_t)(ent - pr.gid_base);
    const uint64_t c1 = ((uint64_t)pr.index << 40) | kp;
    const U64x4 blk = philox4x64_10(c0, c1, kTagConn, 0, pr.seed, 0);
    const int nh = (pr.rule == kRuleOneToOne || pr.rule == kRuleTotal) ? 1 : 2;
    // weight draws of this item's synapses (scatter only, drawn projections)
    U64x4 wblk = {};
    if (kScatter && pw[p].levels)
      wblk = philox4x64_10(c0, ((uint64_t)pr.index << 40) | (kp >> 1), kTagWeight, 0, pr.seed, 0);
    for (int h = 0; h < nh; ++h) {
      const uint32_t k = 2 * kp + h;
      if (k >= pr.K) break;
      uint32_t src, tgt, d;
      switch (pr.rule) {
        case kRuleOutDegree:
          src = ent;
          tgt = pr.tgt_first + (uint32_t)__umul64hi(blk.w[2 * h], (uint64_t)pr.tgt_n);
          d = draw_delay(pr.thr, dmax_cfg, (uint32_t)(blk.w[2 * h + 1] >> 32));
          break;
        case kRuleAllToAll:
          src = pr.src_first + k;
          tgt = ent;
          d = draw_delay(pr.thr, dmax_cfg, (uint32_t)(blk.w[2 * h + 1] >> 32));
          break;
        case kRuleOneToOne:
          src = pr.src_first + (uint32_t)e;
          tgt = ent;
          d = draw_delay(pr.thr, dmax_cfg, (uint32_t)(blk.w[1] >> 32));
          break;
        case kRuleTotal:
          src = pr.src_first + (uint32_t)__umul64hi(blk.w[0], (uint64_t)pr.src_n);
          tgt = pr.tgt_first + (uint32_t)__umul64hi(blk.w[1], (uint64_t)pr.tgt_n);
          d = draw_delay(pr.thr, dmax_cfg, (uint32_t)(blk.w[2] >> 32));
          break;
        default:  // fixed in-degree
          src = pr.src_first + (uint32_t)__umul64hi(blk.w[2 * h], (uint64_t)pr.src_n);
          tgt = ent;
          d = draw_delay(pr.thr, dmax_cfg, (uint32_t)(blk.w[2 * h + 1] >> 32));
          break;
      }
      const uint64_t bucket = (uint64_t)src * D1 + d;
      if (!kScatter) {
        atomicAdd(&cnt[bucket], 1u);
      } else {
        const uint32_t kpop = find_pop(pop_first, npop, tgt);
        const ProjW& w = pw[p];
        uint32_t cls;
        if (w.levels) {
          const uint32_t j = draw_level(w.thr, w.levels, (uint32_t)(wblk.w[k & 3u] >> 32));
          cls = w.cls[(kpop - w.pop0) * w.levels + j];
        } else {
          cls = cls_of[(size_t)p * npop + kpop];
        }
        const unsigned long long slot = atomicAdd(&cursor[bucket], 1ull);
        payload[slot] = (tgt << cls_bits) | cls;
      }
    }
  }
}

uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

// ---------------------------------------------------------------- scan
constexpr int kScanItems = 16;
constexpr uint64_t kScanTile = (uint64_t)kB * kScanItems;

// inclusive wave scan of 64-bit values
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// exclusive block scan for blockDim.x == kB; returns exclusive prefix, *total = block sum
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t* lds4, uint64_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t incl = wave_incl_scan(v);
  if (lane == 63) lds4[wv] = incl;
  __syncthreads();
  uint64_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kB / 64; ++i) {
    const uint64_t x = lds4[i];
    if (i < wv) before += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return before + incl - v;
}

template <typename T>
__global__ void __launch_bounds__(kB) k_tile_sums(const T* __restrict__ in, uint64_t n, uint64_t* sums) {
  __shared__ uint64_t lds[kB / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const uint64_t j = base + i;
    if (j < n) s += (uint64_t)in[j];
  }
  uint64_t tot;
  (void)block_excl_scan(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(kB) k_tile_scan(const T* __restrict__ in, uint64_t n, const uint64_t* tile_off,
                                                   uint64_t* out, uint64_t* total_out) {
  __shared__ uint64_t lds[kB / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const uint64_t j = base + i;
    v[i] = (j < n) ? (uint64_t)in[j] : 0;
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan(s, lds, &tot) + (tile_off ? tile_off[blockIdx.x] : 0);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const uint64_t j = base + i;
    if (j < n) out[j] = run;
    run += v[i];
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kB - 1) *total_out = run;
}

template <typename T>
hipError_t scan_impl(const T* in, uint64_t n, uint64_t* out, uint64_t* tmp, hipStream_t s) {
  // out has n + 1 entries; out[n] = total
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (n == 0) {
    return hipMemsetAsync(out, 0, sizeof(uint64_t), s);
  }
  if (tiles == 1) {
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kB), 0, s, in, n, (const uint64_t*)nullptr, out, out + n);
    return hipGetLastError();
  }
  uint64_t* sums = tmp;             // tiles
  uint64_t* sums_scan = tmp + tiles;  // tiles + 1
  uint64_t* rest = sums_scan + tiles + 1;
  hipLaunchKernelGGL(k_tile_sums<T>, dim3((uint32_t)tiles), dim3(kB), 0, s, in, n, sums);
  hipError_t e = scan_impl<uint64_t>(sums, tiles, sums_scan, rest, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_scan<T>, dim3((uint32_t)tiles), dim3(kB), 0, s, in, n, (const uint64_t*)sums_scan, out,
                     out + n);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kB) k_masks(const uint32_t* __restrict__ cnt, uint32_t N, uint32_t D1, uint64_t* mask,
                                              uint64_t* ngroups) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  uint64_t m = 0;
  uint32_t ng = 0;
  for (uint32_t d = 1; d < D1; ++d) {
    if (cnt[(uint64_t)s * D1 + d]) { m |= 1ull << d; ++ng; }
  }
  mask[s] = m;
  ngroups[s] = ng;
}

__global__ void __launch_bounds__(kB) k_grp_off(const uint32_t* __restrict__ cnt, const uint64_t* __restrict__ off,
                                                const uint64_t* __restrict__ grp_ptr64, uint32_t N, uint32_t D1,
                                                uint64_t* grp_off, uint32_t* grp_ptr32) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > N) return;
  grp_ptr32[s] = (uint32_t)grp_ptr64[s];
  if (s == N) return;
  uint64_t g = grp_ptr64[s];
  for (uint32_t d = 1; d < D1; ++d) {
    const uint64_t b = (uint64_t)s * D1 + d;
    if (cnt[b]) grp_off[g++] = off[b];
  }
}

// ------------------------------------------------------------ group sorting
// Rank sort for short groups, one wave per group: rank(i) = #{v_j < v_i} +
// #{j < i : v_j == v_i}.  Stable, and identical values are interchangeable.
constexpr uint32_t kWaveSortMax = 512;
constexpr uint32_t kBlockSortMax = 16384;

__global__ void __launch_bounds__(kB) k_segsort_wave(const uint64_t* __restrict__ grp_off, uint64_t n_groups,
                                                     uint32_t* payload) {
  __shared__ uint32_t buf[kB / 64][kWaveSortMax];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t* v = buf[wv];
  const uint64_t nw = (uint64_t)gridDim.x * (kB / 64);
  for (uint64_t g = (uint64_t)blockIdx.x * (kB / 64) + wv; g < n_groups; g += nw) {
    const uint64_t b = grp_off[g];
    const uint32_t L = (uint32_t)(grp_off[g + 1] - b);
    if (L <= 1 || L > kWaveSortMax) continue;  // wave-uniform
    for (uint32_t i = lane; i < L; i += 64) v[i] = payload[b + i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t i = lane; i < L; i += 64) {
      const uint32_t x = v[i];
      uint32_t r = 0;
      for (uint32_t j = 0; j < L; ++j) {
        const uint32_t y = v[j];
        r += (y < x) || (y == x && j < i);
      }
      payload[b + r] = x;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Bitonic sort in LDS for groups of (kWaveSortMax, kBlockSortMax]; one block
// per group, grid-stride over groups; longer groups are listed for the host.
constexpr int kSB = 1024;
__global__ void __launch_bounds__(kSB) k_segsort_block(const uint64_t* __restrict__ grp_off, uint64_t n_groups,
                                                       uint32_t* payload, unsigned long long* big, uint32_t* nbig,
                                                       uint32_t big_cap) {
  extern __shared__ uint32_t sbuf[];
  for (uint64_t g = blockIdx.x; g < n_groups; g += gridDim.x) {
    const uint64_t b = grp_off[g];
    const uint64_t L64 = grp_off[g + 1] - b;
    if (L64 <= kWaveSortMax) continue;
    if (L64 > kBlockSortMax) {
      if (threadIdx.x == 0) {
        const uint32_t k = atomicAdd(nbig, 1u);
        if (k < big_cap) big[k] = g;
      }
      continue;
    }
    const uint32_t L = (uint32_t)L64;
    uint32_t M = 1;
    while (M < L) M <<= 1;
    for (uint32_t i = threadIdx.x; i < M; i += kSB) sbuf[i] = (i < L) ? payload[b + i] : 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t k = 2; k <= M; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t i = threadIdx.x; i < M; i += kSB) {
          const uint32_t ix = i ^ j;
          if (ix > i) {
            const uint32_t a = sbuf[i], c = sbuf[ix];
            const bool up = (i & k) == 0;
            if ((a > c) == up) { sbuf[i] = c; sbuf[ix] = a; }
          }
        }
        __syncthreads();
      }
    }
    for (uint32_t i = threadIdx.x; i < L; i += kSB) payload[b + i] = sbuf[i];
    __syncthreads();
  }
}


// ------------------------------------------------------------ tile runs
// A group's synapses are sorted by target, so those onto one tile of the
// binned delivery lie together: a run.  One wave per group finds the run
// starts (a synapse whose tile differs from its predecessor's) with a ballot
// over 64 synapses at a time.  Pass kFill = false counts them per group;
// pass kFill = true writes run k of group g as run_desc[grp_run[g] + k] =
// tile << kRunLenBits | length, in synapse order: each start closes the run
// before it (the previous start in the window, or the run still open from
// the earlier windows), and the last run closes at the group's end.  A group
// of kRunMaxGroup synapses or more sets *too_long (no runs for the network).
template <bool kFill>
__global__ void __launch_bounds__(kB) k_runs(const uint64_t* __restrict__ grp_off, uint64_t n_groups,
                                             const uint32_t* __restrict__ payload, uint32_t cls_bits, uint32_t tsh,
                                             uint32_t* __restrict__ cnt, const uint64_t* __restrict__ grp_run,
                                             uint32_t* __restrict__ run_desc, uint32_t* too_long) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t nwaves = ((uint64_t)gridDim.x * kB) >> 6;
  for (uint64_t g = ((uint64_t)blockIdx.x * kB + threadIdx.x) >> 6; g < n_groups; g += nwaves) {
    const uint64_t a = grp_off[g], b = grp_off[g + 1];
    if (!kFill && lane == 0 && b - a >= kRunMaxGroup) atomicOr(too_long, 1u);
    uint64_t runs = 0;                 // run starts before this window
    uint32_t prev_tile = 0xffffffffu;  // tile of the synapse before the window
    uint64_t open_pos = a;             // first synapse of the open run
    uint32_t open_tile = 0;
    const uint64_t base = kFill ? grp_run[g] : 0;
    for (uint64_t j0 = a; j0 < b; j0 += 64) {  // wave-uniform
      const uint64_t j = j0 + lane;
      const bool in = j < b;
      const uint32_t t = in ? (payload[j] >> cls_bits) >> tsh : 0xffffffffu;
      const uint32_t left = __shfl(t, (int)(lane ? lane - 1 : 0), 64);
      const bool start = in && t != (lane ? left : prev_tile);
      const uint64_t m = __ballot(start);
      if (kFill) {
        const uint64_t below = m & ((1ull << lane) - 1ull);
        const uint32_t pl = below ? 63u - (uint32_t)__clzll(below) : 0u;
        const uint32_t tile_pl = __shfl(t, (int)pl, 64);
        const uint64_t k = runs + (uint64_t)__popcll(below);
        if (start && k > 0) {
          const uint64_t pos = below ? j0 + pl : open_pos;
          const uint32_t tile = below ? tile_pl : open_tile;
          run_desc[base + k - 1] = (tile << kRunLenBits) | (uint32_t)(j - pos);
        }
      }
      if (m) {
        const uint32_t hb = 63u - (uint32_t)__clzll(m);
        open_pos = j0 + hb;
        open_tile = __shfl(t, (int)hb, 64);
      }
      const uint32_t last = (uint32_t)((b - j0 < 64 ? b - j0 : 64) - 1);
      prev_tile = __shfl(t, (int)last, 64);
      runs += (uint64_t)__popcll(m);
    }
    if (lane == 0) {
      if (!kFill) cnt[g] = (uint32_t)runs;
      else if (runs) run_desc[base + runs - 1] = (open_tile << kRunLenBits) | (uint32_t)(b - open_pos);
    }
  }
}

}  // namespace

hipError_t launch_gen_count(const ProjDev* projs, uint32_t nproj, uint64_t total_pairs, uint32_t dmax_cfg,
                            uint32_t D1, uint32_t* cnt, hipStream_t s) {
  if (total_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gen<false>, dim3(grid_for(total_pairs, kB, 65536)), dim3(kB), 0, s, projs, nproj, total_pairs,
                     dmax_cfg, D1, cnt, (unsigned long long*)nullptr, (uint32_t*)nullptr, (const uint16_t*)nullptr,
                     (const ProjW*)nullptr, (const uint32_t*)nullptr, 0u, 0u);
  return hipGetLastError();
}

hipError_t launch_gen_scatter(const ProjDev* projs, uint32_t nproj, uint64_t total_pairs, uint32_t dmax_cfg,
                              uint32_t D1, uint64_t* cursor, uint32_t* payload, const uint16_t* cls_of,
                              const ProjW* pw, const uint32_t* pop_first, uint32_t npop, uint32_t cls_bits,
                              hipStream_t s) {
  if (total_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gen<true>, dim3(grid_for(total_pairs, kB, 65536)), dim3(kB), 0, s, projs, nproj, total_pairs,
                     dmax_cfg, D1, (uint32_t*)nullptr, (unsigned long long*)cursor, payload, cls_of, pw, pop_first,
                     npop, cls_bits);
  return hipGetLastError();
}

size_t scan_tmp_words(uint64_t n) {
  size_t w = 0;
  uint64_t m = n;
  while (true) {
    const uint64_t tiles = (m + kScanTile - 1) / kScanTile;
    if (tiles <= 1) break;
    w += 2 * tiles + 1;
    m = tiles;
  }
  return w + 1;
}

hipError_t launch_scan_u32(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* tmp, hipStream_t s) {
  return scan_impl<uint32_t>(in, n, out, tmp, s);
}

hipError_t launch_scan_u64(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* tmp, hipStream_t s) {
  return scan_impl<uint64_t>(in, n, out, tmp, s);
}

hipError_t launch_masks(const uint32_t* cnt, uint32_t N, uint32_t D1, uint64_t* mask, uint64_t* ngroups,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_masks, dim3((N + kB - 1) / kB), dim3(kB), 0, s, cnt, N, D1, mask, ngroups);
  return hipGetLastError();
}

hipError_t launch_grp_off(const uint32_t* cnt, const uint64_t* off, const uint64_t* grp_ptr64, uint32_t N, uint32_t D1,
                          uint64_t* grp_off, uint32_t* grp_ptr32, hipStream_t s) {
  hipLaunchKernelGGL(k_grp_off, dim3((N + 1 + kB - 1) / kB), dim3(kB), 0, s, cnt, off, grp_ptr64, N, D1, grp_off,
                     grp_ptr32);
  return hipGetLastError();
}

hipError_t launch_segsort(const uint64_t* grp_off, uint64_t n_groups, uint32_t* payload, uint64_t* big,
                          uint32_t* nbig, uint32_t big_cap, hipStream_t s) {
  if (n_groups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_segsort_wave, dim3(grid_for(n_groups, kB / 64, 1u << 20)), dim3(kB), 0, s, grp_off, n_groups,
                     payload);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_segsort_block, dim3(grid_for(n_groups, 1, 4096)), dim3(kSB), kBlockSortMax * sizeof(uint32_t),
                     s, grp_off, n_groups, payload, (unsigned long long*)big, nbig, big_cap);
  return hipGetLastError();
}

hipError_t launch_runs(bool fill, const uint64_t* grp_off, uint64_t n_groups, const uint32_t* payload,
                       uint32_t cls_bits, uint32_t tsh, uint32_t* cnt, const uint64_t* grp_run, uint32_t* run_desc,
                       uint32_t* too_long, hipStream_t s) {
  if (n_groups == 0) return hipSuccess;
  const dim3 grid(grid_for(n_groups, kB / 64, 1u << 16));
  if (fill)
    hipLaunchKernelGGL(k_runs<true>, grid, dim3(kB), 0, s, grp_off, n_groups, payload, cls_bits, tsh, cnt, grp_run,
                       run_desc, too_long);
  else
    hipLaunchKernelGGL(k_runs<false>, grid, dim3(kB), 0, s, grp_off, n_groups, payload, cls_bits, tsh, cnt, grp_run,
                       run_desc, too_long);
  return hipGetLastError();
}

}  // namespace snn
