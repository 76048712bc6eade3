// snn_internal.h -- library-internal access to a network handle for the
// request server (not part of the C ABI).
#pragma once
#include <stdint.h>

#include "../../include/snn.h"

namespace snn {

// the network's device-memory provider (have_dev false: hipMalloc)
void net_allocator(const snn_net* net, snn_device* dev, bool* have_dev);
void net_set_allocator(snn_net* net, const snn_device& dev, bool have_dev);
// the device current when the network was created
int net_device(const snn_net* net);
// defined, not yet built, never released
bool net_is_fresh(const snn_net* net);
// synapses its projections will make (4 bytes each at least on the device)
uint64_t net_planned_synapses(const snn_net* net);

}  // namespace snn
