// snn_types.h -- device-visible data layout of one network (host and device).
//
// HBM layout (all arrays device-resident for the life of the network):
//   neuron state (SoA, fp32): V (LIF: V - E_L), I_e, and per model
//     LIF-exp: I_syn[N][P];  AdEx: w, g[N][P], h, and with beta ports the
//     rising variables r[N][P];  refr (int32) for LIF;  spike generators:
//     their emission steps (CSR by neuron) and a cursor per neuron.
//   acc[2][N][P]  int64 fixed-point input, one buffer per arrival step n
//                 (read) and n+1 (written) (index step % 2; direct: all input;
//                 binned delivery: only the events that did not fit their
//                 tile's bin).
//   binned delivery: targets are cut into tiles of 2^tile_shift neurons;
//     bins[2][bins_total] u32 entries local << 15 | mult << 10 | class, the
//     tile t region at bin_off[t] holding up to bin_cap[t] entries,
//     bin_cnt[2][n_tiles] entries written, ovf_flag[2][n_tiles] set when a
//     tile's events spilled into acc.
//   CSR by (source, delay group):
//     src_mask[N]   u64, bit d set <=> source has a group with delay d steps
//     grp_ptr[N+1]  u32, index of the source's first group
//     grp_off[G+1]  u64, first synapse of each group (groups ordered by delay)
//     payload[S]    u32, target << b | weight class (class -> port, w_q),
//                   b = 32 - bits(N), at most 1024 classes
//   spikes, per step slot s = step % R (R = max(Dmax + 1, 3)):
//     ring_cnt[s]   spikes of the step (the emitting blocks' atomic cursor),
//     ring_base[s]  their first position in log[CAP], the raster ring
//                   (gid | mult << 27, any order within a step),
//     recent[s][N]  16-byte selection records (entry, first group, delay
//                   mask) read by later steps' delivery.
//   selection and delivery keep the selected (synapse offset, group size,
//     multiplicity) records in LDS only.
#pragma once
#include <stdint.h>

namespace snn {

constexpr int kMaxPorts = 4;
constexpr int kMaxClasses = 1024;   // (port, quantised weight) classes per network
constexpr uint32_t kMaxNeurons = 1u << 26;
constexpr int kPoisKmax = 128;
constexpr int kMultShift = 27;
constexpr uint32_t kGidMask = (1u << kMultShift) - 1;
constexpr uint32_t kMaxMult = 31;
constexpr int kUpdBlock = 256;      // neurons per update block
constexpr int kInBuf = 2;           // input buffers: arrival steps n (read) and n+1 (written)
constexpr int kBlkStats = 5;   // per update block: rk accepted, rk rejected, spikes, delay-1 pairs, events
constexpr int kTileAccWords = 4096; // int64 LDS accumulators of a tile block (tile neurons x ports)
constexpr uint32_t kMaxTiles = 1024; // tiles of the binned delivery
constexpr int kBinLocalShift = 15;   // bin entry: local target << 15 | mult << 10 | class
constexpr int kBinMultShift = 10;
constexpr int kRunLenBits = 22;                  // tile run descriptor: tile << 22 | length
constexpr uint64_t kRunMaxGroup = 1ull << 20;     // tile runs only for groups below this size
constexpr uint32_t kNoAllocInputMax = 1u << 18;  // neurons per call of the allocation-free input readback
constexpr int kMaxDevices = 64;
constexpr int kTagConn = 1;
constexpr int kTagPoisson = 2;

enum Model : int32_t { kLifDelta = 0, kLifExp = 1, kAdex = 2, kAdexBeta = 3, kSpikeGen = 4, kParrot = 5 };

// Parameters of one population as the kernels use them (fp32, propagators
// precomputed in double on the host).
struct PopDev {
  uint32_t first, n;
  int32_t model, n_ports;
  // LIF exact integration
  float P22, P20, theta, y_reset;
  float P11[kMaxPorts], P21[kMaxPorts];
  int32_t n_ref;
  // AdEx
  float inv_C, g_L, E_L, Delta_T, inv_Delta_T, V_T, inv_tau_w, a, b, V_peak, V_r;
  float E_rev[kMaxPorts], inv_tau_syn[kMaxPorts];
  // beta ports: 1/tau_rise and the input scale g0 (exponential ports: 1, 0)
  float inv_tau_rise[kMaxPorts], g0[kMaxPorts];
  float rk_eps, rk_hmin, dt;
  // fixed-point input conversion: x = (float)acc * scale[port], scale = 2^-S
  float scale[kMaxPorts];
  // Poisson drive (index into the threshold table, -1 if none)
  int32_t pois;
  int32_t pois_port;
  int64_t pois_wq;
  // instance of the population: first gid and generator key
  uint32_t gid_base;
  // 1: the neurons carry their own constants (NetDev::nlif / nadex, indexed by
  // gid) in place of the LIF or AdEx fields above
  uint32_t per_neuron;
  uint64_t seed;
};

// Constants of one LIF neuron whose parameters are its own (tau_m, C_m, E_L,
// V_th, V_reset, t_ref per neuron; tau_syn stays per population, so P11 does).
struct NeuronLif {
  float P22, P20, theta, y_reset;
  float P21[kMaxPorts];
  int32_t n_ref, pad;
};

// Constants of one AdEx neuron whose parameters are its own (all but the
// port constants).
struct NeuronAdex {
  float inv_C, g_L, E_L, Delta_T, inv_Delta_T, V_T, inv_tau_w, a, b, V_peak, V_r, rk_eps, rk_hmin, pad;
};

static_assert(sizeof(PopDev) % 8 == 0, "PopDev is copied to LDS in 32-bit words");

// connection rules; a work item of the build is one pair of draws of one
// entity (target, source or, for the fixed total number, one synapse)
enum Rule : uint32_t { kRuleInDegree = 0, kRuleOutDegree = 1, kRuleAllToAll = 2, kRuleOneToOne = 3, kRuleTotal = 4,
                       kRuleList = 5 };

struct ProjDev {
  uint32_t src_first, src_n, tgt_first, tgt_n;
  uint32_t K;              // draws per entity (in-degree, out-degree, n_src, 1, 1)
  uint32_t kpairs;         // work items per entity: ceil(K / 2) (1 for one-to-one and fixed total)
  uint32_t index;          // creation index within its instance (Philox counter word 1, bits 40+)
  uint32_t gid_base;       // first gid of its instance (counters use instance-local gids)
  uint32_t rule, pad;
  uint64_t seed;           // generator key of its instance
  uint64_t pair_begin;     // prefix of entities * kpairs over projections
  const uint32_t* lsrc;    // user-defined list: source, target and delay (steps) of synapse j
  const uint32_t* ltgt;
  const uint8_t* ldel;
  uint64_t thr[64];        // delay thresholds, thr[d] for d = 1..Dmax
};

// Selection record of a recent spike: gid | mult << 27, the source's first
// group and its delay mask (looked up once, when the spike is emitted).
struct SpikeRec {
  uint32_t entry;
  uint32_t grp_ptr;
  uint64_t mask;
};

// Scalars written by the kernels.
struct Ctrl {
  uint64_t step_base;      // absolute step of relative step 0 of a launch
  uint32_t overflow;       // sticky flags (bit 0 mult, 1 rk iterations, 2 ranges)
  uint32_t pad;
  uint64_t spill_events;   // binned delivery: events that did not fit their tile's bin
  uint64_t dlv_next[4];    // delivery queue: items of step n taken so far, slot n % 4
};

// Nearest-neighbour STDP rule of the plastic synapses of one (projection,
// target population): W = w_max in the fixed-point units of their (target
// population, port); F+(d) = stdp_F[off_plus + d] for d < len_plus (0
// beyond), F-(d) likewise, both scaled by 2^32.
struct StdpRule {
  int64_t W;
  uint32_t mu_plus, mu_minus;
  uint32_t len_plus, len_minus;
  uint64_t off_plus, off_minus;
};

// Populations a tile block keeps in its LDS window (binned delivery): a
// LIF-only network whose every tile overlaps at most this many runs step
// kernels that read the population tables from LDS only.
constexpr uint32_t kTilePopLds = 8;

struct NetDev {
  uint32_t N, P, npop, dmax;   // dmax = largest delay present
  uint32_t npois, pois_len;    // Poisson threshold tables; entries read at most (the rest are never reached)
  uint32_t R, nblk_upd, sel_grid, pad0;  // R step slots; pad0: bit 0 LIF, bit 1 AdEx, bit 2 beta ports present
  uint32_t n_tiles, tile_shift;  // binned delivery (n_tiles == 0: direct atomics)
  uint32_t dlv_queue, tile_runs; // binned delivery blocks take contiguous item ranges from a queue (batches);
                                 // their count pass reads the groups' tile runs (grp_run, run_desc)
  uint32_t tile_win, pad_tw;     // binned: every tile overlaps at most kTilePopLds populations
  uint64_t bins_total;           // bin entries per input buffer
  uint64_t log_mask;           // CAP - 1
  uint64_t chunk_ring;         // slots of chunk_base (power of two)
  uint64_t n_groups, n_syn;
  const PopDev* pops;
  const NeuronLif* nlif;       // [N] or null: constants of neurons of per_neuron LIF populations
  const NeuronAdex* nadex;     // [N] or null: the same for AdEx populations
  const uint64_t* pois_thr;    // [npois][kPoisKmax]
  const int64_t* cls_wq;       // [n_classes]
  const uint32_t* cls_port;    // [n_classes]
  uint32_t n_classes, cls_bits; // payload = target << cls_bits | class
  // state
  float* V; float* Ie; float* Isyn; float* w; float* g; float* gr; float* h; int32_t* refr;
  // spike generators: neuron i's emission steps gen_step[gen_off[i] .. gen_off[i+1]) ascending, its cursor gen_next[i]
  const uint32_t* gen_off; const uint64_t* gen_step; uint32_t* gen_next;
  // CSR
  const uint64_t* src_mask; const uint32_t* grp_ptr; const uint64_t* grp_off; const uint32_t* payload;
  int64_t* acc;
  uint32_t* bins; uint32_t* bin_cnt; uint32_t* ovf_flag; const uint64_t* bin_off; const uint32_t* bin_cap;
  // spikes
  uint32_t* log; uint64_t* ring_base; uint32_t* ring_cnt; uint64_t* chunk_base;
  SpikeRec* recent;            // [R][N] selection records of the last R steps' spikes
  // selection / delivery
  uint64_t* sel_stats;         // [sel_grid][2]: pairs and events delivered by delivery blocks (cumulative)
  // per-update-block statistics [nblk_upd][kBlkStats]
  uint64_t* blk_stats;
  Ctrl* ctrl;
  // nearest-neighbour STDP (n_rules == 0: no plastic synapse; the rest unset).
  // Per synapse (CSR position j): its weight pw, the step + 1 of its latest
  // arrival (0: none) and the multiplicity arriving at the next step; per
  // neuron the step + 1 of its latest spike; the plastic synapses onto each
  // target, tidx[tptr[t] .. tptr[t+1]); the plastic synapses an arrival step
  // delivers to, arr_list[step & 1][0 .. arr_cnt[step & 1]).
  uint32_t n_rules, pad1;
  uint64_t n_plastic;
  const StdpRule* rules;
  const int64_t* stdp_F;
  const uint8_t* cls_rule;     // [n_classes]: 0 static, r + 1 plastic under rules[r]
  int32_t* pw;
  uint32_t* last_pre;
  uint8_t* arr_m;
  uint32_t* last_post;
  const uint64_t* tptr;
  const uint64_t* tidx;
  uint64_t* arr_list;
  uint32_t* arr_cnt;
  // tile runs of the binned delivery: the synapses of group g onto one tile are
  // run_desc[grp_run[g] .. grp_run[g+1]), each tile << kRunLenBits | length, in
  // synapse order (a group is sorted by target)
  const uint64_t* grp_run;
  const uint32_t* run_desc;
};

}  // namespace snn
