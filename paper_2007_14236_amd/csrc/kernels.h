// kernels.h -- host-callable launchers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snn_types.h"

namespace snn {

// ---- connectivity build ----
// Weight levels of one projection (empty: its single weight): the class of
// level j onto a target of population k is cls[(k - pop0) * levels + j];
// drawn projections take j from thr (u32 draws), lists from lvl[synapse].
struct ProjW {
  const uint64_t* thr;
  const uint16_t* cls;
  const uint16_t* lvl;
  uint32_t levels, pop0;
};

// total_pairs = sum over projections of tgt_n * ceil(K / 2)
hipError_t launch_gen_count(const ProjDev* projs, uint32_t nproj, uint64_t total_pairs, uint32_t dmax_cfg,
                            uint32_t D1, uint32_t* cnt, hipStream_t s);
hipError_t launch_gen_scatter(const ProjDev* projs, uint32_t nproj, uint64_t total_pairs, uint32_t dmax_cfg,
                              uint32_t D1, uint64_t* cursor, uint32_t* payload, const uint16_t* cls_of,
                              const ProjW* pw, const uint32_t* pop_first, uint32_t npop, uint32_t cls_bits,
                              hipStream_t s);
// exclusive scan of n u32 (in32) or u64 (in64) values into out; *total_dev receives the sum.
// tmp must hold scan_tmp_words(n) u64 words.
size_t scan_tmp_words(uint64_t n);
hipError_t launch_scan_u32(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* tmp, hipStream_t s);
hipError_t launch_scan_u64(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* tmp, hipStream_t s);
hipError_t launch_masks(const uint32_t* cnt, uint32_t N, uint32_t D1, uint64_t* mask, uint64_t* ngroups,
                        hipStream_t s);
hipError_t launch_grp_off(const uint32_t* cnt, const uint64_t* off, const uint64_t* grp_ptr64, uint32_t N,
                          uint32_t D1, uint64_t* grp_off, uint32_t* grp_ptr32, hipStream_t s);
// sort every group's payload ascending; groups longer than 16384 are listed in big[] (count in *nbig)
hipError_t launch_segsort(const uint64_t* grp_off, uint64_t n_groups, uint32_t* payload, uint64_t* big,
                          uint32_t* nbig, uint32_t big_cap, hipStream_t s);
// Tile runs of every group (binned delivery with tile shift tsh): fill =
// false counts them into cnt[g] (and sets *too_long for a group of
// kRunMaxGroup synapses or more), fill = true writes them at run_desc[grp_run[g] ..].
hipError_t launch_runs(bool fill, const uint64_t* grp_off, uint64_t n_groups, const uint32_t* payload,
                       uint32_t cls_bits, uint32_t tsh, uint32_t* cnt, const uint64_t* grp_run, uint32_t* run_desc,
                       uint32_t* too_long, hipStream_t s);

// ---- per-step pipeline (step = ctrl->step_base + rel) ----
// One step: update, spike emission and delay-1/-2 delivery, and delivery of
// earlier steps' spikes.  With start/stop events the events are recorded on
// the kernel's own dispatch.
hipError_t launch_step(const NetDev& nd, uint32_t rel, hipStream_t s, hipEvent_t start = nullptr,
                       hipEvent_t stop = nullptr);
hipError_t launch_advance(Ctrl* ctrl, uint32_t steps, hipStream_t s);
// Binned delivery: add the pending bin entries of input buffer `buf` on `port`
// for gids [first, first+n) to out[0..n) (device int64).
hipError_t launch_pending_input(const NetDev& nd, uint32_t buf, uint32_t first, uint32_t n, uint32_t port,
                                int64_t* out, hipStream_t s);
// Multimeter: after the step ctrl->step_base + rel, copy *addr[c] for the nch
// channels into buf[(step % window) * nch + c].
hipError_t launch_sample(const float* const* addr, uint32_t nch, float* buf, uint32_t window, const Ctrl* ctrl,
                         uint32_t rel, hipStream_t s);
// Device address of this library's fixed readback workspace on `device`
// (kNoAllocInputMax int64 values, one copy per GPU, held until the process
// ends).  Resolved once per device; call with that device current first
// (resolve = true), later calls only look it up.  Null if never resolved.
hipError_t input_workspace(int device, bool resolve, int64_t** out);
// ---- nearest-neighbour STDP ----
// Plasticity of step ctrl->step_base + rel (after that step's kernel); no-op
// without plastic synapses.
hipError_t launch_stdp(const NetDev& nd, uint32_t rel, hipStream_t s);
// Set-up: pw[j] = the class weight and cleared arrivals for every synapse;
// cnt[t] += the plastic synapses onto t (cnt zeroed by the caller).
hipError_t launch_stdp_count(const NetDev& nd, uint32_t* cnt, hipStream_t s);
// tidx[cursor[t]++] = j for every plastic synapse j onto t (cursor = tptr copy).
hipError_t launch_stdp_scatter(const NetDev& nd, uint64_t* cursor, uint64_t* tidx, hipStream_t s);
hipError_t launch_poisson_counts(const NetDev& nd, uint64_t step, uint32_t first, uint32_t n, uint32_t* k,
                                 hipStream_t s);

}  // namespace snn
