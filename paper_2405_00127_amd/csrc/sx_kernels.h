// Host-callable launchers of the stroke-expansion kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sx_device.h"

namespace sx {

// Item workspace of the piece / record kernels: one region of region_cap
// slots per piece tile, then ovf_cap shared overflow slots at ovf_base.
struct WsCtl {
    unsigned long long ovf_n;        // overflow slots requested
    unsigned long long items_total;  // items requested by all tiles
    unsigned long long result[2];    // records and items needed, for synchronous readback
};
struct ItemWs {
    Item* items;
    uint32_t* tile_n;  // per piece tile: slots requested (clamp to region_cap)
    WsCtl* ctl;
    uint32_t tile;        // tags per piece tile (the piece kernel's block size: 64 or 256)
    uint32_t region_cap;  // slots per tile
    uint64_t ovf_base, ovf_cap;
};

// One scene's streams and where they go in a batch arena.
struct GatherDesc {
    const uint8_t* tags;
    const float2* pts;
    const StyleD* styles;
    const float* xforms;
    const uint32_t* path_map;
    uint32_t n_tags, n_pts, n_styles, n_xforms, n_paths;
    uint32_t tag_base, pt_base, style_base, xform_base, path_base;
    uint32_t pad;
};

int scan_tiles(uint32_t n);
uint32_t piece_tiles(uint32_t n, uint32_t tile);
size_t scan_status_bytes(uint32_t n);
size_t scan_ctl_bytes();

hipError_t launch_scan_tags(const uint8_t* tags, uint32_t n, uint32_t* mon, void* ctl, void* st, WsCtl* ws_reset,
                            hipStream_t s);
hipError_t launch_scan_counts(const uint32_t* in, uint32_t n, uint64_t* out, void* ctl, void* st, hipStream_t s);
hipError_t launch_pieces(const SceneView& sv, const Cfg& cfg, const ItemWs& ws, uint32_t* counts, int waves,
                         hipStream_t s);
hipError_t launch_piece_stats(const SceneView& sv, const Cfg& cfg, const ItemWs& ws, uint32_t* counts,
                              unsigned long long* stats, hipStream_t s);
hipError_t launch_records(const SceneView& sv, const ItemWs& ws, int arcs, const uint64_t* offsets, void* out,
                          uint64_t cap, hipStream_t s);
hipError_t launch_gather(const GatherDesc* descs, uint32_t n_scenes, uint8_t* tags, float2* pts, StyleD* styles,
                         float* xforms, uint32_t* path_map, hipStream_t s);
hipError_t launch_scene_offsets(const uint64_t* offsets, const GatherDesc* descs, uint32_t n_scenes, uint32_t n_tags,
                                uint64_t* scene_offsets, hipStream_t s);
hipError_t launch_finish(const uint64_t* offsets, uint32_t n, const ItemWs& ws, uint64_t* dst, hipStream_t s);

}  // namespace sx
