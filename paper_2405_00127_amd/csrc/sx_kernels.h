// Host-callable launchers of the stroke-expansion kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sx_device.h"

namespace sx {

// Item workspace of the slot / record kernels: one region of region_cap
// 64-byte units per piece tile (the slots from its first piece to the next
// tile's), then ovf_cap shared overflow units at ovf_base; and the per-slot
// spiral records (8 floats per slot).
struct WsCtl {
    unsigned long long ovf_n;        // overflow units requested
    unsigned long long items_total;  // units requested by all tiles
    unsigned long long slots_total;  // slots of the last expansion
    unsigned long long result[2];    // records and status, for synchronous readback
};
struct ItemWs {
    Unit* units;
    float* es_tab;
    uint32_t* tile_n;  // per slot tile: units requested (clamp to region_cap)
    WsCtl* ctl;
    uint32_t tile;        // pieces per tile
    uint32_t region_cap;  // units per tile
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
uint32_t slot_tiles(uint64_t n_slots);
uint32_t slot_block();
size_t scan_status_bytes(uint32_t n);
size_t scan_ctl_bytes();

hipError_t launch_scan_tags(const uint8_t* tags, uint32_t n, uint32_t* mon, void* ctl, void* st, WsCtl* ws_reset,
                            hipStream_t s);
hipError_t launch_scan_counts(const uint32_t* in, uint32_t n, uint64_t* out, void* ctl, void* st, hipStream_t s);
// out[0] = 0 by a one-thread kernel (no memset node when captured in a graph)
hipError_t launch_zero_u64(uint64_t* out, hipStream_t s);
hipError_t launch_scan_counts_dev(const uint32_t* in, const uint64_t* n_dev, uint32_t cap, uint64_t* out, void* ctl,
                                  void* st, hipStream_t s);
// piece codes kept per tag by the counting bisection pass
constexpr int kKeepCodes = 32;  // fewest piece codes kept per tag by the count pass
// Piece codes the count pass keeps per tag for n tags: a budget of 2^25 words
// shared by the tags, at least kKeepCodes and at most 1024 per tag (small
// scenes keep every code, so the write pass copies instead of re-running the
// bisection of segments with many pieces).
inline uint32_t keep_codes_of(uint32_t n) {
    const uint64_t k = (1ull << 25) / ((uint64_t)mon_stride_of(n) + 1u);
    return (uint32_t)(k < (uint64_t)kKeepCodes ? kKeepCodes : (k > 1024u ? 1024u : k));
}
// The write pass fills pcs, the piece list: piece p of the scene (canonical
// order) as {tag, code}, its slot being p + tag.
hipError_t launch_bisect(const SceneView& sv, const Cfg& cfg, uint32_t range, uint32_t keep, int waves, bool write,
                         uint32_t* nslots, uint32_t* codes, const uint64_t* base, Slot* pcs, uint64_t slot_cap,
                         unsigned long long* stats, hipStream_t s);
// pieces (one thread per piece, tiles of slot_block() pieces)
hipError_t launch_slots(const SceneView& sv, const Cfg& cfg, const ItemWs& ws, const Slot* pcs,
                        const uint64_t* n_slots_dev, uint64_t slot_cap, uint32_t* rc, int waves,
                        unsigned long long* stats, hipStream_t s);
// tail slots (one thread per tag), after launch_slots
hipError_t launch_tails(const SceneView& sv, const Cfg& cfg, const ItemWs& ws, const uint64_t* base,
                        uint64_t slot_cap, uint32_t* rc, unsigned long long* stats, hipStream_t s);
hipError_t launch_records(const SceneView& sv, const ItemWs& ws, const Cfg& cfg, const uint64_t* roff, const Slot* pcs,
                          const uint64_t* n_slots_dev, uint64_t slot_cap, void* out, uint64_t cap, hipStream_t s);
// Single-pass expansion into an unordered line soup (one thread per tag;
// records reserved with atomic adds on *counter, which ends at the total the
// scene needs even when it exceeds cap_records).
hipError_t launch_soup(const SceneView& sv, const Cfg& cfg, void* out, uint64_t cap_records,
                       unsigned long long* counter, hipStream_t s);
hipError_t launch_gather(const GatherDesc* descs, uint32_t n_scenes, uint8_t* tags, float2* pts, StyleD* styles,
                         float* xforms, uint32_t* path_map, hipStream_t s);
hipError_t launch_scene_offsets(const uint64_t* base, const uint64_t* roff, uint64_t slot_cap, const GatherDesc* descs,
                                uint32_t n_scenes, uint32_t n_tags, uint64_t* scene_offsets, hipStream_t s);
hipError_t launch_finish(const uint64_t* roff, const uint64_t* n_slots_dev, uint64_t slot_cap, uint32_t n_tags,
                         const ItemWs& ws, uint64_t* dst, hipStream_t s);
hipError_t launch_tag_records(const uint64_t* base, const uint64_t* roff, uint64_t slot_cap, uint32_t n_tags,
                              uint32_t* counts, uint64_t* offs, hipStream_t s);

// Dashing: phase 0 runs the measuring pass, the two scans and the count
// pass (otag[n], opt[n] then hold the dashed encoding's tag and point
// totals); phase 1 writes the dashed tags and points.  Scratch per source
// tag: len, cum (n + 1), subix (n + 1), cnt; sub_start (n + 2); otag, opt
// (n + 1); ctl / st: two look-back scan control and status blocks.
// Device buffers of the dashing passes (per source tag unless noted).
struct DashBufs {
    DashDesc* desc;       // per style entry
    int64_t* pat;         // pattern values on the grid
    double* panels;       // 16 panel integrals of each dashed segment (panel-major)
    uint64_t* len;        // grid length of each dashed segment
    uint64_t* cum;        // exclusive prefix of len (+ total)
    uint64_t* sub_start;  // per subpath: cum at its first tag
    uint32_t* subix;      // subpaths ended before each tag
    uint32_t* nch;        // work chunks of each tag
    uint64_t* chb;        // exclusive prefix of nch (+ total)
    uint32_t* flag;       // set when a segment needs too many chunks
    uint32_t* ch_tag;     // per chunk: its tag
    uint2* cnt;           // per chunk: (tags, points) it contributes
    uint64_t *otag, *opt; // per chunk: exclusive prefixes of cnt (+ totals)
    void *ctl0, *ctl1, *ctl2, *st0, *st1, *st2;  // scan control blocks and tile status
    uint32_t n_ch;        // number of chunks (known from phase 1 on)
};
// phase 0: lengths, positions, subpath starts, chunks and their scan;
// phase 1 (b.n_ch set): chunk owners, per-chunk counts and their scan;
// phase 2: the write pass into tags_out / pts_out.
hipError_t launch_dash(const SceneView& sv, const DashBufs& b, int phase, uint8_t* tags_out, float2* pts_out,
                       hipStream_t s);

}  // namespace sx
