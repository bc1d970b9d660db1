// Kernel suite: buffer specification and launch of one variant.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm.h"

namespace pm {
// bytes[i], role[i] of the kernel's buffers (see pm_buffers)
int buffers(const pm_variant &v, size_t *bytes, uint32_t *role, uint32_t *nb);
// enqueue one launch; v must already be valid
int launch(const pm_variant &v, void *const *bufs, hipStream_t s);
}  // namespace pm
