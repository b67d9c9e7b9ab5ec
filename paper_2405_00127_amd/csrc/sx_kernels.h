// Host-callable launchers of the stroke-expansion kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sx_device.h"

namespace sx {

int scan_tiles(uint32_t n);
size_t scan_status_bytes(uint32_t n);
size_t scan_ctl_bytes();

hipError_t launch_scan_tags(const uint8_t* tags, uint32_t n, uint32_t* mon, void* ctl, void* st, hipStream_t s);
hipError_t launch_scan_counts(const uint32_t* in, uint32_t n, uint64_t* out, void* ctl, void* st, hipStream_t s);
hipError_t launch_count(const SceneView& sv, const Cfg& cfg, uint32_t* counts, hipStream_t s);
hipError_t launch_emit(const SceneView& sv, const Cfg& cfg, const uint64_t* offsets, void* out, uint64_t cap_records,
                       hipStream_t s);
hipError_t launch_copy_total(const uint64_t* offsets, uint32_t n, uint64_t* dst, hipStream_t s);

}  // namespace sx
