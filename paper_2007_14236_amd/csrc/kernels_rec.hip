// kernels_rec.hip -- sampled recording of state variables (the multimeter
// device of Sec. 2.1): after a step's update, each recorded channel (one
// state variable of one neuron) is copied into the slot of its step in a
// window of steps that the host collects.
#include "kernels.h"

namespace snn {

namespace {

constexpr int kB = 256;

// step = ctrl->step_base + rel; buf[(step % window) * nch + c] = *addr[c]
__global__ void __launch_bounds__(kB) k_sample(const float* const* __restrict__ addr, uint32_t nch, float* buf,
                                               uint32_t window, const Ctrl* ctrl, uint32_t rel) {
  const uint32_t c = blockIdx.x * kB + threadIdx.x;
  if (c >= nch) return;
  const uint64_t step = ctrl->step_base + rel;
  buf[(size_t)(step % window) * nch + c] = *addr[c];
}

}  // namespace

hipError_t launch_sample(const float* const* addr, uint32_t nch, float* buf, uint32_t window, const Ctrl* ctrl,
                         uint32_t rel, hipStream_t s) {
  if (nch == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample, dim3((nch + kB - 1) / kB), dim3(kB), 0, s, addr, nch, buf, window, ctrl, rel);
  return hipGetLastError();
}

}  // namespace snn
