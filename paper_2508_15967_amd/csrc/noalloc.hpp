// Static device scratch of rg_trace_rays_noalloc (noalloc.hip).
#pragma once

#include <string>

// Size of the static scratch array per device: the Dormand-Prince refill
// queue, or the per-ray state of the one-launch-per-step forms for up to
// about 260,000 rays (RK4) or 31,000 rays (Dormand-Prince, 3-D).
#define RG_NOALLOC_SCRATCH_BYTES (4u << 20)

namespace rg {
// Resolves the device address of the static scratch on `device`, which must
// be current; once per device (later calls return at once).  0 on success,
// else -1 with a message in *err.
int noalloc_resolve(int device, std::string *err);
// The address resolved for `device`, or nullptr if noalloc_resolve has not
// succeeded on it.
void *noalloc_address(int device);
}  // namespace rg
