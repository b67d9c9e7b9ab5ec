// HIP kernels of the stroke-expansion hot path for gfx950 (wave64).
//
//  scan_tags_kernel       tag-monoid prefix scan (Section 8.2): single pass,
//                         wave64 shuffle scan + LDS block scan + decoupled
//                         look-back over dynamically numbered tiles.
//  bisect_kernel          Algorithm 2 in FP64 with lane refill (a wave owns a
//                         range of tags; a lane whose tag is done takes the
//                         next).  Count pass: slots per tag (pieces + 1 tail)
//                         and the codes of the first pieces; write pass: every
//                         piece {tag, code} at its canonical position in the
//                         piece list.
//  scan_counts_kernel     exclusive scan of u32 counts into u64 offsets (slot
//  scan_counts_dev_kernel bases; record offsets, with the count read on the
//                         device).  Replaces the paper's atomic bump
//                         allocation: the output order is canonical.
//  slot_kernel            per piece, the Euler spiral, parallel curves,
//                         cusp split, evolutes and counts (Sections 4-6),
//                         over tiles of 256 pieces.  Writes emission items
//                         into per-tile workspace regions and the slot's
//                         record count.
//  tail_kernel            per tag, its tail slot: the join or cap
//                         (Algorithm 1), items into the same regions.
//  record_kernel          per item chunk, the FP32 per-point work: records
//                         at roff[slot] + the chunk's position in its slot,
//                         staged per tile in LDS and written coalesced.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sx_device.h"
#include "sx_kernels.h"

namespace sx {

// ------------------------------------------------------ look-back scan
// A tile publishes its aggregate, then its inclusive prefix, as four 32-bit
// parts each (the pair (a, b) split in halves), every part in its own 64-bit
// word next to the launch's epoch: (epoch << 32) | part.  A word is read and
// written with single relaxed device-scope atomics, so a reader sees a part
// only together with its epoch and no fences are needed (on this GPU a
// release or acquire at device scope writes back or invalidates the whole L2
// of the XCD).  A part is ready once its word carries the current epoch; the
// epoch (kept in device memory, advanced by the last tile of every launch,
// never 0) makes stale words of earlier launches read as "not ready", so
// nothing is cleared between launches and the kernels can be replayed inside
// a HIP graph.  Aggregate and inclusive words are separate, so a reader that
// takes a tile's aggregate never mixes in its inclusive prefix.
struct TileStatus {
    unsigned long long agg[4];
    unsigned long long inc[4];
};
static_assert(sizeof(TileStatus) == 64, "tile status layout");

struct Pair {
    uint64_t a, b;
};

struct ScanCtl {
    uint32_t ticket, done, epoch, err;
};
__device__ __forceinline__ Pair operator+(Pair x, Pair y) { return Pair{x.a + y.a, x.b + y.b}; }

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_up(lo, d, 64);
    hi = __shfl_up(hi, d, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl(lo, src, 64);
    hi = __shfl(hi, src, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_xor(lo, m, 64);
    hi = __shfl_xor(hi, m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// inclusive wave64 scan
__device__ __forceinline__ Pair wave_scan(Pair v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t ua = shfl_up_u64(v.a, d), ub = shfl_up_u64(v.b, d);
        if (lane >= d) { v.a += ua; v.b += ub; }
    }
    return v;
}
__device__ __forceinline__ Pair wave_sum(Pair v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        v.a += shfl_xor_u64(v.a, m);
        v.b += shfl_xor_u64(v.b, m);
    }
    return v;
}

__device__ __forceinline__ uint32_t pair_part(Pair v, int k) {
    const uint64_t w = (k < 2) ? v.a : v.b;
    return (k & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
}

// Lanes 0..3 of the calling wave publish the four parts of v.
__device__ __forceinline__ void publish(TileStatus* st, uint32_t tile, uint32_t epoch, bool inclusive, Pair v,
                                       int lane) {
    if (lane < 4) {
        const unsigned long long w = ((unsigned long long)epoch << 32) | pair_part(v, lane);
        unsigned long long* p = inclusive ? &st[tile].inc[lane] : &st[tile].agg[lane];
        __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ unsigned long long rd(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The four words of a status record as a pair, if all carry `epoch`.
__device__ __forceinline__ bool read4(const unsigned long long* w, uint32_t epoch, Pair& v) {
    const unsigned long long w0 = rd(w), w1 = rd(w + 1), w2 = rd(w + 2), w3 = rd(w + 3);
    const bool ok = (uint32_t)(w0 >> 32) == epoch && (uint32_t)(w1 >> 32) == epoch && (uint32_t)(w2 >> 32) == epoch &&
                    (uint32_t)(w3 >> 32) == epoch;
    v.a = (uint64_t)(uint32_t)w0 | ((uint64_t)(uint32_t)w1 << 32);
    v.b = (uint64_t)(uint32_t)w2 | ((uint64_t)(uint32_t)w3 << 32);
    return ok;
}

// Wave 0 of tile `tile` computes the exclusive prefix of all earlier tiles.
// The wait for a predecessor is bounded: after kSpinLimit polls the tile
// gives up, records the failure in *err and carries on (wrong sums, but every
// wave exits).  Predecessors always hold earlier tickets, so they are resident
// and the limit is never reached in a correct run.
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ Pair look_back(TileStatus* st, uint32_t tile, uint32_t epoch, int lane, uint32_t* err) {
    Pair excl{0, 0};
    int64_t pos = (int64_t)tile - 1;
    while (pos >= 0) {
        const int64_t idx = pos - lane;
        uint32_t state;  // 0 not ready, 1 aggregate, 2 inclusive, 3 before tile 0 (inclusive zero)
        Pair v{0, 0};
        for (uint32_t spins = 0;; spins++) {
            state = 3;
            v = Pair{0, 0};
            if (idx >= 0) {
                // both records in one round trip, the inclusive one preferred
                Pair vi, va;
                const bool ri = read4(st[idx].inc, epoch, vi);
                const bool ra = read4(st[idx].agg, epoch, va);
                state = ri ? 2u : (ra ? 1u : 0u);
                v = ri ? vi : va;
            }
            if (__ballot(state == 0u) == 0ull) break;
            if (spins >= kSpinLimit) {
                if (lane == 0) atomicOr(err, 1u);
                state = 3;
                v = Pair{0, 0};
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        const uint64_t incl_mask = __ballot(state >= 2u);
        if (incl_mask) {
            const int first = __builtin_ctzll(incl_mask);  // nearest tile with a full prefix
            if (lane > first) v = Pair{0, 0};
            excl = excl + wave_sum(v);
            break;
        }
        excl = excl + wave_sum(v);
        pos -= 64;
    }
    return excl;
}

// --------------------------------------------------------- tag monoid
constexpr int kScanBlock = 256;
constexpr int kTagItems = 16;    // tags per thread of the tag-monoid scan
constexpr int kCountItems = 32;  // counts per thread of the count scans
constexpr int kRecCountItems = 64;  // counts per thread of the record-count scan (one round of tiles)

__device__ __forceinline__ Pair tag_inc(uint32_t t) {
    uint64_t pts = (t & kTagCount) + ((t & kTagEnd) ? 1u : 0u);
    uint64_t pth = (t & kTagPath) ? 1u : 0u;
    uint64_t sty = (t & kTagStyle) ? 1u : 0u;
    uint64_t xf = (t & kTagXform) ? 1u : 0u;
    return Pair{pts | (pth << 32), sty | (xf << 32)};
}

// The last block of a launch resets the ticket and done counters and
// records the epoch it used, so the next launch starts clean without any
// memset.
// (The next launch reads these words after the kernel boundary, which
// makes them visible; no fence is needed here.)
__device__ __forceinline__ void finish_scan(ScanCtl* ctl, uint32_t epoch_used) {
    if (atomicAdd(&ctl->done, 1u) == gridDim.x - 1) {
        ctl->ticket = 0;
        ctl->done = 0;
        ctl->epoch = epoch_used;
    }
}

template <int Items, class Load, class Store>
__device__ void scan_tile(Load load, Store store, uint32_t n, ScanCtl* ctl, TileStatus* st) {
    constexpr uint32_t kTile = kScanBlock * Items;
    __shared__ uint32_t s_tile, s_epoch;
    __shared__ Pair s_wave[kScanBlock / 64];
    __shared__ Pair s_excl;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) {
        s_tile = atomicAdd(&ctl->ticket, 1u);
        // this launch's epoch: one past the last launch's, never 0 (zeroed words)
        const uint32_t e = ctl->epoch + 1u;
        s_epoch = e ? e : 1u;
    }
    __syncthreads();
    const uint32_t tile = s_tile, epoch = s_epoch;
    const uint32_t ntiles = (n + kTile - 1) / kTile;
    if (tile >= ntiles) {
        // a grid sized for a capacity larger than this launch's n: nothing to scan
        if (tid == 0) finish_scan(ctl, s_epoch);
        return;
    }
    const uint64_t base = (uint64_t)tile * kTile + (uint64_t)tid * Items;
    Pair item[Items];
    load(base, item);
    Pair run{0, 0};
#pragma unroll
    for (int j = 0; j < Items; j++) {
        run = run + item[j];
        item[j] = run;  // thread-local inclusive
    }
    Pair wincl = wave_scan(run, lane);
    if (lane == 63) s_wave[wv] = wincl;
    __syncthreads();
    Pair wpre{0, 0}, agg{0, 0};
#pragma unroll
    for (int k = 0; k < kScanBlock / 64; k++) {
        if (k < wv) wpre = wpre + s_wave[k];
        agg = agg + s_wave[k];
    }
    Pair texcl = wpre + wincl;
    texcl.a -= run.a;
    texcl.b -= run.b;
    if (wv == 0) {
        Pair excl{0, 0};
        if (tile == 0) {
            publish(st, tile, epoch, true, agg, lane);
        } else {
            publish(st, tile, epoch, false, agg, lane);
            excl = look_back(st, tile, epoch, lane, &ctl->err);
            publish(st, tile, epoch, true, excl + agg, lane);
        }
        if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    Pair pre = s_excl + texcl;
    store(base, item, pre);
    __syncthreads();
    if (tid == 0) finish_scan(ctl, s_epoch);
}

__global__ __launch_bounds__(kScanBlock) void scan_tags_kernel(const uint8_t* __restrict__ tags, uint32_t n,
                                                               uint32_t* __restrict__ mon, ScanCtl* ctl,
                                                               TileStatus* st, WsCtl* ws_reset) {
    // the workspace counters of the piece kernel that follows start at zero
    if (ws_reset && blockIdx.x == 0 && threadIdx.x == 0) {
        ws_reset->ovf_n = 0;
        ws_reset->items_total = 0;
    }
    auto load = [&](uint64_t base, Pair* item) {
        if (base + kTagItems <= n) {
            uint4 raw = *reinterpret_cast<const uint4*>(tags + base);
            uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
            for (int j = 0; j < kTagItems; j++) item[j] = tag_inc((w[j >> 2] >> (8 * (j & 3))) & 0xffu);
        } else {
#pragma unroll
            for (int j = 0; j < kTagItems; j++) item[j] = (base + j < n) ? tag_inc(tags[base + j]) : Pair{0, 0};
        }
    };
    auto store = [&](uint64_t base, const Pair* incl, Pair pre) {
        // item j: exclusive = pre + incl[j-1]; style/xform stored inclusive - 1
        uint32_t o_off[kTagItems], o_pth[kTagItems], o_sty[kTagItems], o_xf[kTagItems];
#pragma unroll
        for (int j = 0; j < kTagItems; j++) {
            Pair ex = pre;
            if (j > 0) ex = ex + incl[j - 1];
            Pair in = pre + incl[j];
            o_off[j] = (uint32_t)ex.a;
            o_pth[j] = (uint32_t)(ex.a >> 32);
            o_sty[j] = (uint32_t)in.b - 1u;
            o_xf[j] = (uint32_t)(in.b >> 32) - 1u;
        }
        // rows of mon_stride_of(n) words: 16-byte aligned, so a full run of
        // 16 tags (base a multiple of 16) stores as four uint4 per row
        const size_t stride = mon_stride_of(n);
        uint32_t* m0 = mon;
        uint32_t* m1 = mon + stride;
        uint32_t* m2 = mon + 2 * stride;
        uint32_t* m3 = mon + 3 * stride;
        if (base + kTagItems <= n) {
#pragma unroll
            for (int j = 0; j < kTagItems; j += 4) {
                *reinterpret_cast<uint4*>(m0 + base + j) = make_uint4(o_off[j], o_off[j + 1], o_off[j + 2], o_off[j + 3]);
                *reinterpret_cast<uint4*>(m1 + base + j) = make_uint4(o_pth[j], o_pth[j + 1], o_pth[j + 2], o_pth[j + 3]);
                *reinterpret_cast<uint4*>(m2 + base + j) = make_uint4(o_sty[j], o_sty[j + 1], o_sty[j + 2], o_sty[j + 3]);
                *reinterpret_cast<uint4*>(m3 + base + j) = make_uint4(o_xf[j], o_xf[j + 1], o_xf[j + 2], o_xf[j + 3]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < kTagItems; j++) {
                if (base + j < n) {
                    m0[base + j] = o_off[j];
                    m1[base + j] = o_pth[j];
                    m2[base + j] = o_sty[j];
                    m3[base + j] = o_xf[j];
                }
            }
        }
    };
    scan_tile<kTagItems>(load, store, n, ctl, st);
}

// exclusive scan of u32 counts into u64 offsets; out[n] = total
template <int Items>
__device__ __forceinline__ void scan_u32_body(const uint32_t* __restrict__ in, uint32_t n, uint64_t* __restrict__ out,
                                              ScanCtl* ctl, TileStatus* st);
__global__ __launch_bounds__(kScanBlock) void scan_counts_kernel(const uint32_t* __restrict__ in, uint32_t n,
                                                                 uint64_t* __restrict__ out, ScanCtl* ctl,
                                                                 TileStatus* st) {
    scan_u32_body<kCountItems>(in, n, out, ctl, st);
}
// the same with n read from device memory (clamped to the buffers' capacity);
// the grid covers the capacity
__global__ __launch_bounds__(kScanBlock) void scan_counts_dev_kernel(const uint32_t* __restrict__ in,
                                                                     const uint64_t* __restrict__ n_dev, uint32_t cap,
                                                                     uint64_t* __restrict__ out, ScanCtl* ctl,
                                                                     TileStatus* st) {
    const uint64_t nd = *n_dev;
    if (nd == 0 && blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
    scan_u32_body<kRecCountItems>(in, nd < cap ? (uint32_t)nd : cap, out, ctl, st);
}
template <int Items>
__device__ __forceinline__ void scan_u32_body(const uint32_t* __restrict__ in, uint32_t n, uint64_t* __restrict__ out,
                                              ScanCtl* ctl, TileStatus* st) {
    auto load = [&](uint64_t base, Pair* item) {
        if (base + Items <= n) {
#pragma unroll
            for (int j = 0; j < Items; j += 4) {
                uint4 v = *reinterpret_cast<const uint4*>(in + base + j);
                item[j] = Pair{v.x, 0};
                item[j + 1] = Pair{v.y, 0};
                item[j + 2] = Pair{v.z, 0};
                item[j + 3] = Pair{v.w, 0};
            }
        } else {
#pragma unroll
            for (int j = 0; j < Items; j++) item[j] = Pair{(base + j < n) ? (uint64_t)in[base + j] : 0ull, 0};
        }
    };
    auto store = [&](uint64_t base, const Pair* incl, Pair pre) {
#pragma unroll
        for (int j = 0; j < Items; j++) {
            const uint64_t ex = pre.a + (j > 0 ? incl[j - 1].a : 0ull);
            if (base + j < n) out[base + j] = ex;
            if (base + j == (uint64_t)n - 1u) out[n] = pre.a + incl[j].a;
        }
    };
    scan_tile<Items>(load, store, n, ctl, st);
}

// --------------------------------------------------------- bisection
// One wave per workgroup owns `range` consecutive tags.  Every lane runs the
// bisection of one segment at a time (Algorithm 2, one trial per loop turn);
// a lane whose segment is done takes the wave's next tag (lane refill), so
// the wave is busy until its range is exhausted instead of waiting for its
// longest segment.  The count pass writes, per tag, its slot count (accepted
// pieces + 1 tail) and keeps the codes of its first `keep` pieces (code
// q of tag i at codes[q * stride + i], so the lanes of a wave, holding
// consecutive tags, read and write consecutive words); the
// write pass, after the scan of those counts, writes each tag's pieces into
// the scene's piece list (canonical order; the piece of ordinal p of tag i
// has slot p + i, since every tag before it owns one tail slot besides its
// pieces): copied from the kept codes, or, for the few segments with more
// pieces, from a second run of the bisection.
constexpr int kBisectBlock = 64;
constexpr uint32_t kBisectMaxRange = 1024;  // tags per wave (the autotuner's largest range)
constexpr int kRefillLanes = 8;  // idle lanes that trigger a refill (on the map scene 8 and 12 beat 4, 16 and 32)

template <bool Write, bool Stats, int MinWaves>
__global__ __launch_bounds__(kBisectBlock, MinWaves) void bisect_kernel(
    SceneView sv, Cfg cfg, uint32_t range, uint32_t keep, uint32_t* __restrict__ nslots, uint32_t* __restrict__ codes,
    const uint64_t* __restrict__ base, Slot* __restrict__ pcs, uint64_t slot_cap,
    unsigned long long* __restrict__ stats) {
    const uint32_t lane = threadIdx.x;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const size_t cstride = mon_stride_of(sv.n_tags);  // row stride of the kept codes
    const uint32_t a = blockIdx.x * range;
    const uint32_t b = min(sv.n_tags, a + range);
    uint32_t n_trials = 0, n_lines = 0;
    // Count pass: lines (one straight piece each, reading G32), markers and
    // invalid tags need no bisection.  They are settled for the whole range
    // first, 64 consecutive tags at a time, and only the curves are listed
    // (in LDS) for the refill loop, so that a refill does not spend rounds
    // of scattered loads on tags that take no trial.
    __shared__ uint32_t s_curve[kBisectMaxRange];
    uint32_t n_curve = 0;
    if (!Write) {
        for (uint32_t t0 = a; t0 < b; t0 += 64u) {
            const uint32_t it = t0 + lane;
            bool curve = false;
            if (it < b) {
                bool line;
                const int kind = tag_kind(sv, it, line);
                if (kind == kTagSegment && !line) {
                    curve = true;
                } else if (kind == kTagSegment) {
                    nslots[it] = 2u;
                    codes[it] = slot_code(0u, 0u, false) | kCodeLine;
                    if (Stats) n_lines++;
                } else {
                    nslots[it] = 1u;  // markers and invalid tags own only their tail slot
                }
            }
            const uint64_t m = __ballot(curve);
            if (curve) s_curve[n_curve + (uint32_t)__popcll(m & below)] = it;
            n_curve += (uint32_t)__popcll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the refill loop's work list: the range's curves (count pass) or its tags
    uint32_t cursor = Write ? a : 0u;  // next unassigned entry (wave-uniform)
    const uint32_t cend = Write ? b : n_curve;
    bool busy = false;
    uint32_t i = 0, seq = 0;
    uint64_t bi = 0;  // piece ordinal of the lane's tag's first piece (write pass)
    TagInfo ti;
    Seg s;
    Bisect bs;
    for (;;) {
        // refill idle lanes with the next tags of the range, once kRefillLanes
        // lanes are idle (a refill fetches segments: its latency is shared by
        // the lanes it serves) or the wave has nothing left to run
        const uint64_t idle = __ballot(!busy);
        if (idle && cursor < cend && (__popcll(idle) >= kRefillLanes || __ballot(busy) == 0ull)) {
            const uint32_t ni = cursor + (uint32_t)__popcll(idle & below);
            cursor += (uint32_t)__popcll(idle);
            if (!busy && ni < cend) {
                i = Write ? ni : s_curve[ni];
                seq = 0;
                bool copied = false;
                if (Write) {
                    bi = base[i] - i;  // pieces of the tags before this one
                    const uint32_t np = nslots[i] - 1u;
                    if (np <= keep) {
                        // pieces known from the count pass: copy them
                        for (uint32_t q = 0; q < np; q++)
                            if (bi + q < slot_cap) pcs[bi + q] = Slot{i, codes[q * cstride + i]};
                        copied = true;
                    }
                }
                if (!copied) fetch_tag(sv, i, ti, s);
                if (copied) {
                    // done with this tag
                } else if (!Write && ti.kind == kTagSegment && ti.line) {
                    // a line is one straight piece (reading G32): no bisection
                    nslots[i] = 2u;
                    codes[i] = slot_code(0u, 0u, false) | kCodeLine;
                    if (Stats) n_lines++;
                } else if (ti.kind == kTagSegment) {
                    bisect_init(bs, s);
                    busy = true;
                } else if (!Write) {
                    nslots[i] = 1u;  // markers and invalid tags own only their tail slot
                }
            }
            continue;  // refill again until no idle lane can take a tag
        }
        if (__ballot(busy) == 0ull) break;
        if (busy) {
            uint32_t t0u = 0, depth = 0;
            bool done = false, pivot = false;
            if (Stats) {
                if (ti.line) n_lines++;
                else n_trials++;
            }
            if (bisect_step(bs, s, cfg, ti.line, t0u, depth, pivot, done)) {
                if (Write) {
                    const uint64_t at = bi + seq;
                    if (at < slot_cap) pcs[at] = Slot{i, slot_code(t0u, depth, pivot)};
                } else if (seq < keep) {
                    codes[seq * cstride + i] = slot_code(t0u, depth, pivot);
                }
                seq++;
                if (done) {
                    if (!Write) nslots[i] = seq + 1u;
                    busy = false;
                }
            }
        }
    }
    if (Stats) {
        atomicAdd(&stats[kStTrials], (unsigned long long)n_trials);
        atomicAdd(&stats[kStLines], (unsigned long long)n_lines);
    }
}

// ------------------------------------------------------------- slots
constexpr int kSlotBlock = 256;   // pieces per workgroup and per workspace tile
constexpr int kSlotGrid = 8192;   // persistent grid of the slot kernel (tiles stride by it)
constexpr int kTailBlock = 256;   // tags per tail-kernel workgroup
constexpr int kTailGrid = 8192;   // grid cap of the tail kernel (tags stride by it)
constexpr int kTailWin = 64;      // slot tiles a tail-kernel block counts in LDS
constexpr int kRecBlock = 256;
constexpr int kRecGrid = 8192;    // persistent grid of the record kernel
constexpr uint32_t kStageWords = 6400;  // LDS words staging a tile's records (25 KB)
constexpr int kOvfBlocks = 512;   // record-kernel blocks striding over the overflow slots

// Unit allocation of the piece launch.  A piece's items are first counted
// by a dry run of its puts (CountAlloc: nothing is written); the lane then
// reserves them with one LDS atomic on its tile's counter (the address
// differs between lanes, so this is a plain per-lane atomic, not a scalar
// loop over the lanes) and hands its reservation out in order (LaneAlloc).
// A reservation that does not fit in the tile's region moves as a whole to
// the shared overflow area (the part inside the region is left empty).
struct CountAlloc {
    uint32_t n;
    __device__ uint64_t alloc(uint32_t nc) {
        n += nc;
        return ~0ull;
    }
};
constexpr uint32_t kPieceGroup = 4;     // piece tiles a piece-launch workgroup orders together
constexpr uint32_t kSingleTiles = 1024;  // the last piece tiles, taken one per workgroup
struct LaneAlloc {
    uint64_t next;  // next unit of the reservation, or ~0ull (dropped)
    __device__ uint64_t alloc(uint32_t nc) {
        const uint64_t u = next;
        if (u != ~0ull) next = u + nc;
        return u;
    }
};

// Piece tiles: tile T holds the pieces of ordinals [T, T + 1) x kSlotBlock
// and owns the slots from the first of them up to the first slot of tile
// T + 1 (so also the tails of the tags whose last piece it holds; tile 0
// starts at slot 0, and there is always at least one tile).  Its item
// region and its contiguous range of output records follow from that.
__device__ __forceinline__ uint32_t piece_tile_count(uint64_t n_pieces) {
    return n_pieces ? (uint32_t)((n_pieces + kSlotBlock - 1) / kSlotBlock) : 1u;
}
__device__ __forceinline__ uint64_t tile_first_slot(const Slot* pcs, uint32_t tile, uint32_t n_tiles,
                                                    uint64_t n_slots) {
    if (tile == 0u) return 0u;
    if (tile >= n_tiles) return n_slots;
    const uint64_t p = (uint64_t)tile * kSlotBlock;
    return p + pcs[p].tag;
}
// The tile of tag i's tail slot: the tile of the last piece of tags 0..i.
__device__ __forceinline__ uint64_t tail_tile(const uint64_t* base, uint32_t i) {
    const uint64_t p = base[i + 1] - (uint64_t)(i + 1);  // pieces of tags 0..i
    return p ? (p - 1u) / kSlotBlock : 0u;
}

// One thread per piece: its Euler spiral and parallel curves as emission
// items (records relative to the slot) and the slot's record count.  A
// workgroup takes kPieceGroup consecutive piece tiles at a time and orders
// their pieces by work class (curve pieces, then line pieces), so a wave runs
// pieces of one kind and only one wave of the group mixes the two; it then
// runs the order in passes of kSlotBlock pieces, each piece's items going to
// its own tile's region.  The tails are done by tail_kernel.  Every side has
// one range, a few have a second one past a
// parallel-curve cusp: the counts of the first ranges run on the piece's own
// thread, the second ranges of each wave are packed onto its first lanes
// (the piece's k0, k1, L, width and cusp go through the wave's part of LDS,
// so no block barrier is needed), and then each thread writes its piece's
// items in canonical order.
template <int MinWaves, bool Stats, bool Newton>
__global__ __launch_bounds__(kSlotBlock, MinWaves) void slot_kernel(SceneView sv, Cfg cfg, ItemWs ws,
                                                                    const Slot* __restrict__ pcs,
                                                                    const uint64_t* __restrict__ n_slots_dev,
                                                                    uint64_t slot_cap, uint32_t* __restrict__ rc,
                                                                    unsigned long long* __restrict__ stats) {
    __shared__ uint32_t s_n[kPieceGroup];  // units taken in each tile of the group
    __shared__ uint32_t s_order[kPieceGroup * kSlotBlock];  // group ordinal at each position of the class order
    __shared__ uint32_t s_hist[kPieceGroup][kSlotBlock / 64][2];
    __shared__ uint32_t s_task[2 * kSlotBlock];     // owner thread << 2 | side << 1 | reversed
    __shared__ double s_own[kSlotBlock][4];        // k0, k1, L, w of the owner's piece
    __shared__ double s_tc[kSlotBlock][2];         // cusp u of each side
    __shared__ RangeRes s_res[2 * kSlotBlock];
    __shared__ RangeRes s_first[2][kSlotBlock];    // each side's first range
    const uint64_t n_slots = *n_slots_dev;
    if (n_slots > slot_cap) return;  // reported by the finish kernel
    const uint64_t n_pieces = n_slots - sv.n_tags;
    const uint32_t n_tiles = piece_tile_count(n_pieces);
    // groups of kPieceGroup tiles, then the last kSingleTiles tiles one at a
    // time, so that the launch's last round is short
    const uint32_t n_multi = n_tiles > kSingleTiles ? (n_tiles - kSingleTiles) / kPieceGroup : 0u;
    const uint32_t n_groups = n_multi + (n_tiles - n_multi * kPieceGroup);
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t st[kStN] = {0, 0, 0, 0, 0, 0};
    for (uint32_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
        const uint32_t tile0 = grp < n_multi ? grp * kPieceGroup : n_multi * kPieceGroup + (grp - n_multi);
        const uint32_t n_gt = grp < n_multi ? kPieceGroup : 1u;  // tiles of this group
        const uint64_t gfirst = (uint64_t)tile0 * kSlotBlock;
        if (t < kPieceGroup) s_n[t] = 0u;
        // the group's work-class order (curve pieces, then line pieces): each
        // thread ranks its piece of every tile among its wave's pieces of that
        // class, and the waves' class counts go to s_hist
        uint32_t cls[kPieceGroup], rank[kPieceGroup];
#pragma unroll
        for (uint32_t g = 0; g < kPieceGroup; g++) {
            const uint64_t p = gfirst + g * kSlotBlock + t;
            cls[g] = (g < n_gt && p < n_pieces) ? (code_line(pcs[p].code) ? 1u : 0u) : 2u;
            rank[g] = 0u;
#pragma unroll
            for (uint32_t c = 0; c < 2; c++) {
                const uint64_t m = __ballot(cls[g] == c);
                if (cls[g] == c) rank[g] = (uint32_t)__popcll(m & below);
                if (lane == 0) s_hist[g][wv][c] = (uint32_t)__popcll(m);
            }
        }
        __syncthreads();
        uint32_t n_curve = 0, n_valid = 0;
        for (uint32_t g = 0; g < kPieceGroup; g++)
            for (uint32_t w = 0; w < kSlotBlock / 64; w++) {
                n_curve += s_hist[g][w][0];
                n_valid += s_hist[g][w][0] + s_hist[g][w][1];
            }
#pragma unroll
        for (uint32_t g = 0; g < kPieceGroup; g++) {
            if (cls[g] < 2u) {
                uint32_t pos = rank[g] + (cls[g] ? n_curve : 0u);
                for (uint32_t g2 = 0; g2 < kPieceGroup; g2++)
                    for (uint32_t w = 0; w < kSlotBlock / 64; w++)
                        if (g2 < g || (g2 == g && w < wv)) pos += s_hist[g2][w][cls[g]];
                s_order[pos] = g * kSlotBlock + t;
            }
        }
        __syncthreads();
        for (uint32_t pass = 0; pass < kPieceGroup && pass * kSlotBlock < n_valid; pass++) {
            const uint32_t qo = pass * kSlotBlock + t;  // this thread's position in the class order
            // phase 1: the piece's spiral, its sides and the first range of each
            const bool act = qo < n_valid;
            uint64_t j = 0;  // the piece's slot
            uint32_t kt = 0;  // its tile within the group
            Slot sl{0u, kSlotTail};
            if (act) {
                const uint32_t o = s_order[qo];
                kt = o / kSlotBlock;
                sl = pcs[gfirst + o];
                j = gfirst + o + sl.tag;
            }
            ItemSink<LaneAlloc, Stats> k;
            k.units = ws.units;
            k.es_tab = ws.es_tab;
            k.al.next = ~0ull;
            k.path = 0xffffffffu;
            k.slot = (uint32_t)j;
            k.n = 0;
            if (Stats)
                for (int q = 0; q < kStN; q++) k.st[q] = 0;
            bool have = false;
            ES es;
            SideGeo g0, g1;
            uint32_t qa = 0, qb = 0;
            bool side1 = false;  // a stroke's second side (a fill has one)
            if (act && sl.tag < sv.n_tags) {
                k.path = path_of(sv, sl.tag);
                TagInfo ti;
                Seg sg;
                fetch_tag(sv, sl.tag, ti, sg);
                if (ti.kind == kTagSegment) {
                    have = true;
                    piece_es(k, cfg, sg, ti.line, code_t0u(sl.code), code_depth(sl.code), code_pivot(sl.code), es);
                    side1 = !sg.fill;
                    g0 = side_geo(es, sg.w, 0);
                    g1 = side_geo(es, sg.w, 1);
                    g1.split = g1.split && side1;
                    s_first[0][t] = range_count<Newton>(cfg, es.k0, es.k1, es.L, g0.h, 0.0, g0.tc, g0.rev1);
                    if (side1) s_first[1][t] = range_count<Newton>(cfg, es.k0, es.k1, es.L, g1.h, 0.0, g1.tc, g1.rev1);
                    if (g0.split || g1.split) {
                        s_own[t][0] = es.k0;
                        s_own[t][1] = es.k1;
                        s_own[t][2] = es.L;
                        s_own[t][3] = sg.w;
                        s_tc[t][0] = g0.tc;
                        s_tc[t][1] = g1.tc;
                    }
                }
            }
            // phase 2: the second ranges of the wave, packed onto its first lanes
            // (wave-private LDS: no block barrier)
            const bool sp0 = have && g0.split, sp1 = have && g1.split;
            const uint64_t m0 = __ballot(sp0), m1 = __ballot(sp1);
            const uint32_t n0 = (uint32_t)__popcll(m0), n_task = n0 + (uint32_t)__popcll(m1);
            uint32_t* w_task = s_task + wv * 128u;
            RangeRes* w_res = s_res + wv * 128u;
            if (sp0) {
                qa = (uint32_t)__popcll(m0 & below);
                w_task[qa] = (t << 2) | (g0.rev2 ? 1u : 0u);
            }
            if (sp1) {
                qb = n0 + (uint32_t)__popcll(m1 & below);
                w_task[qb] = (t << 2) | 2u | (g1.rev2 ? 1u : 0u);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (uint32_t q = lane; q < n_task; q += 64u) {
                const uint32_t task = w_task[q], own = task >> 2, side = (task >> 1) & 1u;
                const double w = s_own[own][3];
                w_res[q] = range_count<Newton>(cfg, s_own[own][0], s_own[own][1], s_own[own][2], side ? -w : w,
                                               s_tc[own][side], 1.0, (task & 1u) != 0u);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // phase 3: the items of each piece in canonical order, into units
            // reserved for the whole wave at once
            auto put_all = [&](auto& sink) {
                range_put(sink, cfg, es, g0.h, 0.0, g0.tc, g0.rev1, true, !g0.split, g0.P0, g0.Pc, s_first[0][t]);
                if (g0.split) range_put(sink, cfg, es, g0.h, g0.tc, 1.0, g0.rev2, false, true, g0.Pc, g0.P1, w_res[qa]);
                if (side1) {
                    range_put(sink, cfg, es, g1.h, 0.0, g1.tc, g1.rev1, true, !g1.split, g1.P0, g1.Pc, s_first[1][t]);
                    if (g1.split)
                        range_put(sink, cfg, es, g1.h, g1.tc, 1.0, g1.rev2, false, true, g1.Pc, g1.P1, w_res[qb]);
                }
            };
            uint32_t need = 0;
            if (have) {
                ItemSink<CountAlloc, false> dry;
                dry.units = ws.units;
                dry.es_tab = ws.es_tab;
                dry.al.n = 0;
                dry.path = 0;
                dry.slot = 0;
                dry.n = 0;
                put_all(dry);
                need = dry.al.n;
            }
            if (need) {
                // one LDS atomic per lane on its tile's counter (lanes of a wave
                // can belong to different tiles of the group)
                const uint32_t at = atomicAdd(&s_n[kt], need);
                const uint64_t region = ((uint64_t)tile0 + kt) * ws.region_cap;
                if (at + need <= ws.region_cap) {
                    k.al.next = region + at;
                } else {
                    for (uint32_t u = at; u < ws.region_cap; u++) ws.units[region + u].w[0] = 0u;
                    const unsigned long long o = atomicAdd(&ws.ctl->ovf_n, (unsigned long long)need);
                    k.al.next = (o + need <= ws.ovf_cap) ? ws.ovf_base + o : ~0ull;
                }
            }
            if (have) put_all(k);
            if (act) {
                rc[j] = k.n;
                if (Stats)
                    for (int q = 0; q < kStN; q++) st[q] += k.st[q];
            }
        }
        __syncthreads();
        if (t < n_gt) {
            ws.tile_n[tile0 + t] = s_n[t];
            atomicAdd(&ws.ctl->items_total, (unsigned long long)s_n[t]);
        }
    }
    if (Stats) {
        for (int q = kStPieces; q <= kStEvolutes; q++)
            if (st[q]) atomicAdd(&stats[q], (unsigned long long)st[q]);
    }
}

// Sink of a tail: a join or cap is one item (or none), held in registers
// until the block has placed it.
template <bool Stats>
struct TailSink {
    static constexpr bool kStats = Stats;
    uint32_t hdr, nrec, n;
    JoinP p;
    uint32_t st[Stats ? kStN : 1];
    __device__ void put(uint32_t h, uint32_t nr, uint32_t, const JoinP& q) {
        if constexpr (Stats) st[kStJoins]++;
        hdr = h;
        nrec = nr;
        p = q;
        n += nr;
    }
};

// One thread per tag: its tail slot (the last of its slots, at
// base[tag + 1] - 1) holds the join with the next segment or the cap
// (Algorithm 1).  The items continue the regions of the tails' piece tiles
// after the piece launch's items: a block's consecutive tags have increasing
// tail tiles spanning a few tiles, so it counts its units per tile in LDS and
// takes them from each tile's counter with one global atomic (per lane only
// when the block spans more than kTailWin tiles).
template <bool Stats>
__global__ __launch_bounds__(kTailBlock, 3) void tail_kernel(SceneView sv, Cfg cfg, ItemWs ws,
                                                            const uint64_t* __restrict__ base, uint64_t slot_cap,
                                                            uint32_t* __restrict__ rc,
                                                            unsigned long long* __restrict__ stats) {
    __shared__ uint32_t s_cnt[kTailWin];
    __shared__ uint32_t s_at[kTailWin];
    __shared__ uint32_t s_asked;
    const uint32_t n = sv.n_tags;
    if (base[n] > slot_cap) return;  // reported by the finish kernel
    const uint32_t t = threadIdx.x;
    if (t == 0) s_asked = 0u;
    uint32_t asked = 0, joins = 0;
    for (uint32_t i0 = blockIdx.x * kTailBlock; i0 < n; i0 += gridDim.x * kTailBlock) {
        const uint32_t i = i0 + t;
        const uint32_t ilast = min(n, i0 + kTailBlock) - 1u;
        const uint64_t tile_lo = tail_tile(base, i0);
        const uint64_t span = tail_tile(base, ilast) - tile_lo + 1u;
        const bool win = span <= (uint64_t)kTailWin;
        if (t < kTailWin) s_cnt[t] = 0u;
        __syncthreads();
        TailSink<Stats> k;
        k.nrec = 0;
        k.n = 0;
        if (Stats) k.st[kStJoins] = 0;
        uint64_t slot = 0, tile = 0;
        uint32_t need = 0, local = 0;
        if (i < n) {
            slot = base[i + 1] - 1u;
            tile = tail_tile(base, i);
            TagInfo ti;
            Seg sg;
            fetch_tag(sv, i, ti, sg);
            emit_tail(k, cfg, sv, i, ti, sg);
            need = k.nrec ? chunks(k.nrec, cfg.K) * Units<JoinP>::n : 0u;
            if (win && need) local = atomicAdd(&s_cnt[tile - tile_lo], need);
        }
        __syncthreads();
        if (win && t < span && s_cnt[t]) s_at[t] = atomicAdd(&ws.tile_n[tile_lo + t], s_cnt[t]);
        __syncthreads();
        if (i < n) {
            if (need) {
                const uint32_t at = win ? s_at[tile - tile_lo] + local : atomicAdd(&ws.tile_n[tile], need);
                uint64_t u = tile * ws.region_cap + at;
                if (at + need > ws.region_cap) {
                    // the part inside the region is left empty; the item goes to the overflow area
                    for (uint32_t j = at; j < ws.region_cap; j++) ws.units[tile * ws.region_cap + j].w[0] = 0u;
                    const unsigned long long o = atomicAdd(&ws.ctl->ovf_n, (unsigned long long)need);
                    u = (o + need <= ws.ovf_cap) ? ws.ovf_base + o : ~0ull;
                }
                if (u != ~0ull) write_item(ws.units, u, k.hdr, path_of(sv, i), (uint32_t)slot, 0u, k.nrec, cfg.K, k.p);
            }
            rc[slot] = k.n;
            asked += need;
            if (Stats) joins += k.st[kStJoins];
        }
        __syncthreads();  // s_cnt and s_at are reused
    }
    atomicAdd(&s_asked, asked);
    __syncthreads();
    if (t == 0 && s_asked) atomicAdd(&ws.ctl->items_total, (unsigned long long)s_asked);
    if (Stats && joins) atomicAdd(&stats[kStJoins], (unsigned long long)joins);
}

// One item chunk starting at unit u: loads its one or two units and writes
// its records.
template <bool Newton>
__device__ __forceinline__ void record_item(const SceneView& sv, const ItemWs& ws, const Unit* u,
                                            const uint64_t* roff, uint64_t n_slots, float* out, uint64_t cap,
                                            int arcs, const XIncF& xi, float* stage = nullptr, uint64_t lo = 0,
                                            uint64_t hi = 0) {
    uint32_t w[2 * kUnitWords];
    const uint4* src = reinterpret_cast<const uint4*>(u);
#pragma unroll
    for (int j = 0; j < 4; j++) reinterpret_cast<uint4*>(w)[j] = src[j];
    const uint32_t kind = w[0] & 15u;
    if (kind == 0u) return;
    if (kind != kItemOffset) {
#pragma unroll
        for (int j = 4; j < 8; j++) reinterpret_cast<uint4*>(w)[j] = src[j];
    }
    const uint32_t path = w[1], slot = w[2];
    if (slot >= n_slots) return;
    const uint64_t end = roff[slot + 1] < cap ? roff[slot + 1] : cap;
    RecOut o{out, roff[slot] + w[3], end, path, arcs, stage, lo, hi};
    emit_item<Newton>(w, ws.es_tab + 8 * (size_t)slot, xi, o);
}

// Per item chunk, the FP32 per-point work: records at
// roff[slot] + the chunk's position within its slot.
template <bool Newton>
__global__ __launch_bounds__(kRecBlock, Newton ? 3 : 6) void record_kernel(SceneView sv, ItemWs ws, int arcs,
                                                           const uint64_t* __restrict__ roff,
                                                           const Slot* __restrict__ pcs,
                                                           const uint64_t* __restrict__ n_slots_dev, uint64_t slot_cap,
                                                           float* __restrict__ out, uint64_t cap_records, XIncF xi) {
    const uint64_t n_slots = *n_slots_dev;
    // nothing is written when the records exceed the capacity, or slots or items were dropped
    if (n_slots > slot_cap || roff[n_slots] > cap_records || ws.ctl->ovf_n > ws.ovf_cap) return;
    const uint32_t n_tiles = piece_tile_count(n_slots - sv.n_tags);
    const uint32_t b = blockIdx.x;
    if (b < kRecGrid) {
        // a tile's units, one per thread (units in any order: every record's
        // position comes from the scans)
        // the tile's slots own one contiguous output range: records in its
        // first kStageWords words are staged in LDS and copied out with
        // coalesced stores once the tile is done
        __shared__ float s_stage[kStageWords];
        const uint32_t words = arcs ? 6u : 5u;
        for (uint32_t tile = b; tile < n_tiles; tile += kRecGrid) {
            const uint32_t cnt = ws.tile_n[tile] < ws.region_cap ? ws.tile_n[tile] : ws.region_cap;
            const Unit* base = ws.units + (uint64_t)tile * ws.region_cap;
            const uint64_t s_lo = tile_first_slot(pcs, tile, n_tiles, n_slots);
            const uint64_t s_hi = tile_first_slot(pcs, tile + 1u, n_tiles, n_slots);
            const uint64_t lo = roff[s_lo];
            const uint64_t n_rec = roff[s_hi] - lo;
            // (a tile whose items spilled into the overflow area is not
            // staged: those records are written by the overflow blocks)
            const uint64_t n_st = ws.tile_n[tile] > ws.region_cap ? 0u
                                  : (n_rec < kStageWords / words ? n_rec : kStageWords / words);
            for (uint32_t s2 = threadIdx.x; s2 < cnt; s2 += kRecBlock)
                record_item<Newton>(sv, ws, base + s2, roff, n_slots, out, cap_records, arcs, xi, s_stage, lo,
                                    lo + n_st);
            __syncthreads();
            uint32_t* dst = reinterpret_cast<uint32_t*>(out) + lo * words;
            const uint32_t* src = reinterpret_cast<const uint32_t*>(s_stage);
            for (uint32_t d = threadIdx.x; d < (uint32_t)n_st * words; d += kRecBlock) dst[d] = src[d];
            __syncthreads();
        }
    } else {
        const uint64_t cnt = ws.ctl->ovf_n;
        const Unit* base = ws.units + ws.ovf_base;
        for (uint64_t s = (uint64_t)(b - kRecGrid) * kRecBlock + threadIdx.x; s < cnt;
             s += (uint64_t)kOvfBlocks * kRecBlock)
            record_item<Newton>(sv, ws, base + s, roff, n_slots, out, cap_records, arcs, xi);
    }
}

// ----------------------------------------------------- single pass
// The paper's own organisation (Section 8.1), kept as an ablation of the
// count / scan / write pipeline: one thread per tag runs its bisection, its
// pieces' sides and its join or cap in sequence, and every item's records
// are reserved with one atomic add on a global counter and written at once
// (a line soup: records of a range stay together, ranges land in any order).
struct SoupSink {
    static constexpr bool kStats = false;
    float* out;
    uint64_t cap;
    unsigned long long* counter;
    float* es_tab;  // the current piece's FP32 spiral (8 floats, slot 0)
    XIncF xi;
    uint32_t path, slot, n, arcs, newton;
    uint32_t st[1];
    template <class P>
    __device__ void put(uint32_t hdr, uint32_t nrec, uint32_t K, const P& p) {
        n += nrec;
        if (nrec == 0u) return;
        const uint64_t base = atomicAdd(counter, (unsigned long long)nrec);
        if (base + nrec > cap) return;  // counted only: the caller sees the total
        uint32_t w[2 * kUnitWords];
        *reinterpret_cast<P*>(w + kHdrWords) = p;
        const uint32_t nc = chunks(nrec, K);
        for (uint32_t c = 0; c < nc; c++) {
            const uint32_t nchunk = (c + 1 < nc) ? K : nrec - c * K;
            w[0] = hdr | (nchunk << 24);
            w[1] = path;
            w[2] = 0u;
            w[3] = c * K;
            w[4] = c * K;
            w[5] = nrec;
            RecOut o{out, base + (uint64_t)c * K, base + nrec, path, (int)arcs, nullptr, 0, 0};
            if (newton) emit_item<true>(w, es_tab, xi, o);
            else emit_item<false>(w, es_tab, xi, o);
        }
    }
};

__global__ __launch_bounds__(256) void soup_kernel(SceneView sv, Cfg cfg, XIncF xi, float* __restrict__ out,
                                                   uint64_t cap, unsigned long long* __restrict__ counter) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sv.n_tags; i += stride) {
        float es_loc[8];
        SoupSink k{out, cap, counter, es_loc, xi, path_of(sv, i), 0u, 0u, (uint32_t)cfg.arcs,
                   (uint32_t)(cfg.newton && !cfg.arcs), {0u}};
        soup_tag(k, cfg, sv, i);
    }
}

hipError_t launch_soup(const SceneView& sv, const Cfg& cfg, void* out, uint64_t cap_records,
                       unsigned long long* counter, hipStream_t s) {
    if (sv.n_tags == 0) return hipSuccess;
    XIncF xi;
    for (int k = 0; k < 5; k++) xi.v[k] = (float)cfg.xinc[k];
    const uint32_t blocks = (sv.n_tags + 255u) / 256u;
    soup_kernel<<<blocks < 16384u ? blocks : 16384u, 256, 0, s>>>(sv, cfg, xi, (float*)out, cap_records, counter);
    return hipGetLastError();
}

// dst[0] = records, dst[1] = 0 when everything fit, else 1 (slots or items
// were dropped: the workspace must grow); the counters stay in ws.ctl.
__global__ void finish_kernel(const uint64_t* __restrict__ roff, const uint64_t* __restrict__ n_slots_dev,
                              uint64_t slot_cap, uint32_t n_tags, const ItemWs ws, uint64_t* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (n_tags == 0) {
            dst[0] = 0;
            dst[1] = 0;
            return;
        }
        const uint64_t ns = *n_slots_dev;
        const bool slots_ok = ns <= slot_cap;
        dst[0] = slots_ok ? roff[ns] : 0ull;
        dst[1] = (!slots_ok || ws.ctl->ovf_n > ws.ovf_cap) ? 1ull : 0ull;
        ws.ctl->slots_total = ns;
    }
}

// Per-tag record counts and offsets (verification exports):
// offs[t] = roff[base[t]], counts[t] = offs[t + 1] - offs[t].
__global__ void tag_records_kernel(const uint64_t* __restrict__ base, const uint64_t* __restrict__ roff,
                                   uint64_t slot_cap, uint32_t n_tags, uint32_t* __restrict__ counts,
                                   uint64_t* __restrict__ offs) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n_tags) return;
    const bool fit = base[n_tags] <= slot_cap;  // else the slots were dropped: report zeros
    const uint64_t o = fit ? roff[base[i]] : 0ull;
    if (offs) offs[i] = o;
    if (counts && i < n_tags) counts[i] = fit ? (uint32_t)(roff[base[i + 1]] - o) : 0u;
}

// ------------------------------------------------------------- batches
// Concatenate scenes into one arena: block (x, s) copies a strided share of
// scene s's streams.  Concatenation needs no index fix-ups: every scene
// starts a path, a style and a transform, so the tag-monoid scan of the
// arena gives global stream indices, and the path map keeps each scene's own
// input path numbers.
constexpr int kGatherBlock = 256;
constexpr int kGatherBlocksPerScene = 32;

__global__ __launch_bounds__(kGatherBlock) void gather_kernel(const GatherDesc* __restrict__ descs,
                                                              uint8_t* __restrict__ tags, float2* __restrict__ pts,
                                                              StyleD* __restrict__ styles, float* __restrict__ xforms,
                                                              uint32_t* __restrict__ path_map) {
    const GatherDesc d = descs[blockIdx.y];
    const uint32_t stride = kGatherBlock * kGatherBlocksPerScene;
    const uint32_t t0 = blockIdx.x * kGatherBlock + threadIdx.x;
    for (uint32_t i = t0; i < d.n_tags; i += stride) tags[d.tag_base + i] = d.tags[i];
    for (uint32_t i = t0; i < d.n_pts; i += stride) pts[d.pt_base + i] = d.pts[i];
    for (uint32_t i = t0; i < d.n_styles; i += stride) styles[d.style_base + i] = d.styles[i];
    for (uint32_t i = t0; i < 6 * d.n_xforms; i += stride) xforms[6 * (size_t)d.xform_base + i] = d.xforms[i];
    for (uint32_t i = t0; i < d.n_paths; i += stride) path_map[d.path_base + i] = d.path_map[i];
}

// scene_offsets[s] = first record of scene s; scene_offsets[n] = total
// (slot base of the scene's first tag, then that slot's record offset)
__global__ void scene_offsets_kernel(const uint64_t* __restrict__ base, const uint64_t* __restrict__ roff,
                                     uint64_t slot_cap, const GatherDesc* __restrict__ descs, uint32_t n_scenes,
                                     uint32_t n_tags, uint64_t* __restrict__ out) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    // zeros when empty or when the slots were dropped (the status word says so)
    const bool fit = n_tags && base[n_tags] <= slot_cap;
    if (s < n_scenes) out[s] = fit ? roff[base[descs[s].tag_base]] : 0ull;
    if (s == n_scenes) out[s] = fit ? roff[base[n_tags]] : 0ull;
}

// ------------------------------------------------------------- launches
int scan_tiles(uint32_t n) { return (int)((n + kScanBlock * kTagItems - 1) / (kScanBlock * kTagItems)); }
static int count_scan_tiles(uint32_t n, int items = kCountItems) {
    return (int)((n + (uint32_t)(kScanBlock * items) - 1) / (uint32_t)(kScanBlock * items));
}

uint32_t piece_tiles(uint32_t n, uint32_t tile) { return (n + tile - 1) / tile; }
uint32_t slot_tiles(uint64_t n_slots) { return (uint32_t)((n_slots + kSlotBlock - 1) / kSlotBlock); }
uint32_t slot_block() { return kSlotBlock; }

hipError_t launch_scan_tags(const uint8_t* tags, uint32_t n, uint32_t* mon, void* ctl, void* st, WsCtl* ws_reset,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    scan_tags_kernel<<<scan_tiles(n), kScanBlock, 0, s>>>(tags, n, mon, (ScanCtl*)ctl, (TileStatus*)st, ws_reset);
    return hipGetLastError();
}
hipError_t launch_scan_counts(const uint32_t* in, uint32_t n, uint64_t* out, void* ctl, void* st, hipStream_t s) {
    if (n == 0) return hipSuccess;
    scan_counts_kernel<<<count_scan_tiles(n), kScanBlock, 0, s>>>(in, n, out, (ScanCtl*)ctl, (TileStatus*)st);
    return hipGetLastError();
}
__global__ void zero_u64_kernel(uint64_t* out) {
    if (threadIdx.x == 0) out[0] = 0ull;
}
hipError_t launch_zero_u64(uint64_t* out, hipStream_t s) {
    zero_u64_kernel<<<1, 64, 0, s>>>(out);
    return hipGetLastError();
}
hipError_t launch_scan_counts_dev(const uint32_t* in, const uint64_t* n_dev, uint32_t cap, uint64_t* out, void* ctl,
                                  void* st, hipStream_t s) {
    const int g = count_scan_tiles(cap > 0 ? cap : 1, kRecCountItems);
    scan_counts_dev_kernel<<<g, kScanBlock, 0, s>>>(in, n_dev, cap, out, (ScanCtl*)ctl, (TileStatus*)st);
    return hipGetLastError();
}

template <bool Write, bool Stats>
static void bisect_launch(uint32_t g, hipStream_t s, int waves, const SceneView& sv, const Cfg& cfg, uint32_t range,
                          uint32_t keep, uint32_t* nslots, uint32_t* codes, const uint64_t* base, Slot* pcs,
                          uint64_t cap, unsigned long long* stats) {
    if (waves <= 2)
        bisect_kernel<Write, Stats, 2><<<g, kBisectBlock, 0, s>>>(sv, cfg, range, keep, nslots, codes, base, pcs, cap,
                                                                stats);
    else if (waves == 3)
        bisect_kernel<Write, Stats, 3><<<g, kBisectBlock, 0, s>>>(sv, cfg, range, keep, nslots, codes, base, pcs, cap,
                                                                stats);
    else
        bisect_kernel<Write, Stats, 4><<<g, kBisectBlock, 0, s>>>(sv, cfg, range, keep, nslots, codes, base, pcs, cap,
                                                                stats);
}
hipError_t launch_bisect(const SceneView& sv, const Cfg& cfg, uint32_t range, uint32_t keep, int waves, bool write,
                         uint32_t* nslots, uint32_t* codes, const uint64_t* base, Slot* pcs, uint64_t slot_cap,
                         unsigned long long* stats, hipStream_t s) {
    if (sv.n_tags == 0) return hipSuccess;
    if (range == 0 || range % 64u || range > kBisectMaxRange || keep < (uint32_t)kKeepCodes)
        return hipErrorInvalidValue;
    // a scene too small to give every SIMD a wave at this range takes
    // shorter ranges (down to one tag per lane)
    const uint32_t fill = ((sv.n_tags / 4096u + 63u) / 64u) * 64u;
    if (fill < range) range = fill < 64u ? 64u : fill;
    const uint32_t g = (sv.n_tags + range - 1) / range;
    if (write)
        bisect_launch<true, false>(g, s, waves, sv, cfg, range, keep, nslots, codes, base, pcs, slot_cap, stats);
    else if (stats)
        bisect_launch<false, true>(g, s, waves, sv, cfg, range, keep, nslots, codes, base, pcs, slot_cap, stats);
    else
        bisect_launch<false, false>(g, s, waves, sv, cfg, range, keep, nslots, codes, base, pcs, slot_cap, stats);
    return hipGetLastError();
}
template <bool Newton>
static void slot_launch(uint32_t g, hipStream_t s, int waves, const SceneView& sv, const Cfg& cfg, const ItemWs& ws,
                        const Slot* pcs, const uint64_t* n_slots_dev, uint64_t slot_cap, uint32_t* rc,
                        unsigned long long* stats) {
    if (stats)
        slot_kernel<1, true, Newton><<<g, kSlotBlock, 0, s>>>(sv, cfg, ws, pcs, n_slots_dev, slot_cap, rc, stats);
    else if (waves <= 1)
        slot_kernel<1, false, Newton><<<g, kSlotBlock, 0, s>>>(sv, cfg, ws, pcs, n_slots_dev, slot_cap, rc, stats);
    else if (waves == 2)
        slot_kernel<2, false, Newton><<<g, kSlotBlock, 0, s>>>(sv, cfg, ws, pcs, n_slots_dev, slot_cap, rc, stats);
    else
        slot_kernel<3, false, Newton><<<g, kSlotBlock, 0, s>>>(sv, cfg, ws, pcs, n_slots_dev, slot_cap, rc, stats);
}
hipError_t launch_slots(const SceneView& sv, const Cfg& cfg, const ItemWs& ws, const Slot* pcs,
                        const uint64_t* n_slots_dev, uint64_t slot_cap, uint32_t* rc, int waves,
                        unsigned long long* stats, hipStream_t s) {
    if (sv.n_tags == 0) return hipSuccess;
    const uint32_t g = std::min<uint32_t>(kSlotGrid, std::max<uint32_t>(1u, slot_tiles(slot_cap)));
    // the exact-integral counts apply to line output only
    if (cfg.newton && !cfg.arcs)
        slot_launch<true>(g, s, waves, sv, cfg, ws, pcs, n_slots_dev, slot_cap, rc, stats);
    else
        slot_launch<false>(g, s, waves, sv, cfg, ws, pcs, n_slots_dev, slot_cap, rc, stats);
    return hipGetLastError();
}
hipError_t launch_tails(const SceneView& sv, const Cfg& cfg, const ItemWs& ws, const uint64_t* base,
                        uint64_t slot_cap, uint32_t* rc, unsigned long long* stats, hipStream_t s) {
    if (sv.n_tags == 0) return hipSuccess;
    const uint32_t g = std::min<uint32_t>(kTailGrid, (sv.n_tags + kTailBlock - 1) / kTailBlock);
    if (stats) tail_kernel<true><<<g, kTailBlock, 0, s>>>(sv, cfg, ws, base, slot_cap, rc, stats);
    else tail_kernel<false><<<g, kTailBlock, 0, s>>>(sv, cfg, ws, base, slot_cap, rc, stats);
    return hipGetLastError();
}
hipError_t launch_records(const SceneView& sv, const ItemWs& ws, const Cfg& cfg, const uint64_t* roff, const Slot* pcs,
                          const uint64_t* n_slots_dev, uint64_t slot_cap, void* out, uint64_t cap, hipStream_t s) {
    if (sv.n_tags == 0) return hipSuccess;
    XIncF xi;
    for (int k = 0; k < 5; k++) xi.v[k] = (float)cfg.xinc[k];
    // exact-density items exist only with line output in the Newton mode
    if (cfg.newton && !cfg.arcs)
        record_kernel<true><<<kRecGrid + kOvfBlocks, kRecBlock, 0, s>>>(sv, ws, cfg.arcs, roff, pcs, n_slots_dev,
                                                                        slot_cap, (float*)out, cap, xi);
    else
        record_kernel<false><<<kRecGrid + kOvfBlocks, kRecBlock, 0, s>>>(sv, ws, cfg.arcs, roff, pcs, n_slots_dev,
                                                                         slot_cap, (float*)out, cap, xi);
    return hipGetLastError();
}
hipError_t launch_gather(const GatherDesc* descs, uint32_t n_scenes, uint8_t* tags, float2* pts, StyleD* styles,
                         float* xforms, uint32_t* path_map, hipStream_t s) {
    if (n_scenes == 0) return hipSuccess;
    gather_kernel<<<dim3(kGatherBlocksPerScene, n_scenes), kGatherBlock, 0, s>>>(descs, tags, pts, styles, xforms,
                                                                                 path_map);
    return hipGetLastError();
}
hipError_t launch_scene_offsets(const uint64_t* base, const uint64_t* roff, uint64_t slot_cap, const GatherDesc* descs,
                                uint32_t n_scenes, uint32_t n_tags, uint64_t* scene_offsets, hipStream_t s) {
    scene_offsets_kernel<<<(n_scenes + 1 + 255) / 256, 256, 0, s>>>(base, roff, slot_cap, descs, n_scenes, n_tags,
                                                                    scene_offsets);
    return hipGetLastError();
}
hipError_t launch_finish(const uint64_t* roff, const uint64_t* n_slots_dev, uint64_t slot_cap, uint32_t n_tags,
                         const ItemWs& ws, uint64_t* dst, hipStream_t s) {
    finish_kernel<<<1, 64, 0, s>>>(roff, n_slots_dev, slot_cap, n_tags, ws, dst);
    return hipGetLastError();
}
hipError_t launch_tag_records(const uint64_t* base, const uint64_t* roff, uint64_t slot_cap, uint32_t n_tags,
                              uint32_t* counts, uint64_t* offs, hipStream_t s) {
    tag_records_kernel<<<(n_tags + 1 + 255) / 256, 256, 0, s>>>(base, roff, slot_cap, n_tags, counts, offs);
    return hipGetLastError();
}
size_t scan_status_bytes(uint32_t n) { return (size_t)scan_tiles(n > 0 ? n : 1) * sizeof(TileStatus); }
size_t scan_ctl_bytes() { return sizeof(ScanCtl); }


// ------------------------------------------------------------- dashing
// The dashed encoding of a scene (dash patterns of Sections 1 and 9.3), in
// five passes over the source tags: the grid length of every dashed segment;
// an exclusive scan of (length, subpath ends) giving each tag its position
// along the scene and its subpath; each subpath's start position; per tag
// the tags and points it contributes to the dashed encoding; a scan of
// those counts; and the write pass.  Every path of the result opens with an
// empty closed subpath carrying its style and transform bits and ends with
// one carrying its path end bit; each dash is an open subpath ([start point]
// [parts of segments][stroke cap marker]); solid strokes and fills are
// copied.
__global__ __launch_bounds__(256) void dash_measure_kernel(SceneView sv, const DashDesc* __restrict__ desc,
                                                           uint64_t* __restrict__ len, double* __restrict__ panels) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sv.n_tags) return;
    const uint32_t tag = sv.tags[i];
    uint64_t q = 0;
    if (!(tag & kTagEnd)) {
        const uint32_t sty = sv.mon[2 * (size_t)sv.mon_stride + i];
        if (sty < sv.n_styles && desc[sty].n) {
            const int c = (int)(tag & kTagCount);
            const float2* D = sv.pts + sv.mon[i];
            D2 P[4];
            for (int j = 0; j <= c; j++) P[j] = d2((double)D[j].x, (double)D[j].y);
            double panel[kDashPanels];
            q = (uint64_t)dash_fix(dash_len_d(P, c, panel));
            // kept for the count and write passes (panel k of every tag together)
            for (int k = 0; k < kDashPanels; k++) panels[(size_t)k * sv.n_tags + i] = panel[k];
        }
    }
    len[i] = q;
}

// exclusive scan of (len, subpath end) over the tags; cum[n], subix[n] = totals
__global__ __launch_bounds__(kScanBlock) void dash_scan_kernel(const uint8_t* __restrict__ tags,
                                                               const uint64_t* __restrict__ len, uint32_t n,
                                                               uint64_t* __restrict__ cum,
                                                               uint32_t* __restrict__ subix, ScanCtl* ctl,
                                                               TileStatus* st) {
    auto load = [&](uint64_t base, Pair* item) {
#pragma unroll
        for (int j = 0; j < kTagItems; j++)
            item[j] = (base + j < n) ? Pair{len[base + j], (tags[base + j] & kTagEnd) ? 1ull : 0ull} : Pair{0, 0};
    };
    auto store = [&](uint64_t base, const Pair* incl, Pair pre) {
#pragma unroll
        for (int j = 0; j < kTagItems; j++) {
            const Pair ex = j > 0 ? pre + incl[j - 1] : pre;
            if (base + j < n) {
                cum[base + j] = ex.a;
                subix[base + j] = (uint32_t)ex.b;
            }
            if (base + j == (uint64_t)n - 1u) {
                cum[n] = pre.a + incl[j].a;
                subix[n] = (uint32_t)(pre.b + incl[j].b);
            }
        }
    };
    scan_tile<kTagItems>(load, store, n, ctl, st);
}

__global__ __launch_bounds__(256) void dash_sub_start_kernel(const uint8_t* __restrict__ tags,
                                                             const uint64_t* __restrict__ cum,
                                                             const uint32_t* __restrict__ subix, uint32_t n,
                                                             uint64_t* __restrict__ sub_start) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0) sub_start[0] = 0;
    if (tags[i] & kTagEnd) sub_start[subix[i] + 1u] = cum[i];
}

// chunks of each tag (at most kDashMaxChunks; more sets the flag)
__global__ __launch_bounds__(256) void dash_nch_kernel(DashIn in, uint32_t* __restrict__ nch,
                                                       uint32_t* __restrict__ flag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= in.sv.n_tags) return;
    uint32_t q = dash_chunks(in, i);
    if (q > kDashMaxChunks) {
        atomicOr(flag, 1u);
        q = 1u;
    }
    nch[i] = q;
}

// the owner tag of every chunk
__global__ __launch_bounds__(256) void dash_chunk_tag_kernel(const uint32_t* __restrict__ nch,
                                                             const uint64_t* __restrict__ chb, uint32_t n,
                                                             uint32_t* __restrict__ ch_tag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t at = chb[i];
    for (uint32_t q = 0; q < nch[i]; q++) ch_tag[at + q] = i;
}

// The chunk a thread of a 256-thread block takes: the block's chunks
// ordered by kind (dashed lines, quadratics, cubics, the rest), so that a
// wave mostly runs one degree's code (the per-degree dash code would
// otherwise run three times over in a mixed wave).  ~0u: none.
__device__ uint32_t dash_chunk_of_thread(const DashIn& in, const uint32_t* __restrict__ ch_tag, uint32_t n_ch,
                                         uint32_t* s_ord, uint32_t (*s_hist)[4]) {
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    const uint32_t k = blockIdx.x * 256u + t;
    uint32_t cls = 4u;
    if (k < n_ch) {
        const uint32_t i = ch_tag[k];
        const uint32_t tag = in.sv.tags[i];
        cls = (!(tag & kTagEnd) && dash_desc_of(in, i).n) ? (tag & kTagCount) - 1u : 3u;
    }
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t rank = 0;
#pragma unroll
    for (uint32_t c = 0; c < 4; c++) {
        const uint64_t m = __ballot(cls == c);
        if (cls == c) rank = (uint32_t)__popcll(m & below);
        if (lane == 0) s_hist[wv][c] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    uint32_t pos = rank, n_valid = 0;
    for (uint32_t c = 0; c < 4; c++)
        for (uint32_t w = 0; w < 4; w++) {
            if (c < cls || (c == cls && w < wv)) pos += s_hist[w][c];
            n_valid += s_hist[w][c];
        }
    if (cls < 4u) s_ord[pos] = t;
    __syncthreads();
    return t < n_valid ? blockIdx.x * 256u + s_ord[t] : ~0u;
}

__global__ __launch_bounds__(256) void dash_count_kernel(DashIn in, const uint32_t* __restrict__ ch_tag,
                                                         const uint64_t* __restrict__ chb, uint32_t n_ch,
                                                         uint2* __restrict__ cnt) {
    __shared__ uint32_t s_ord[256];
    __shared__ uint32_t s_hist[4][4];
    const uint32_t k = dash_chunk_of_thread(in, ch_tag, n_ch, s_ord, s_hist);
    if (k == ~0u) return;
    const uint32_t i = ch_tag[k];
    uint32_t nt = 0, np = 0;
    dash_tag<false>(in, i, (uint32_t)(k - chb[i]), nullptr, nullptr, 0, 0, nt, np);
    cnt[k] = make_uint2(nt, np);
}

// exclusive scan of (tags, points) counts; otag[n], opt[n] = totals
__global__ __launch_bounds__(kScanBlock) void dash_off_scan_kernel(const uint2* __restrict__ cnt, uint32_t n,
                                                                   uint64_t* __restrict__ otag,
                                                                   uint64_t* __restrict__ opt, ScanCtl* ctl,
                                                                   TileStatus* st) {
    auto load = [&](uint64_t base, Pair* item) {
#pragma unroll
        for (int j = 0; j < kTagItems; j++) {
            const uint2 v = (base + j < n) ? cnt[base + j] : make_uint2(0u, 0u);
            item[j] = Pair{v.x, v.y};
        }
    };
    auto store = [&](uint64_t base, const Pair* incl, Pair pre) {
#pragma unroll
        for (int j = 0; j < kTagItems; j++) {
            const Pair ex = j > 0 ? pre + incl[j - 1] : pre;
            if (base + j < n) {
                otag[base + j] = ex.a;
                opt[base + j] = ex.b;
            }
            if (base + j == (uint64_t)n - 1u) {
                otag[n] = pre.a + incl[j].a;
                opt[n] = pre.b + incl[j].b;
            }
        }
    };
    scan_tile<kTagItems>(load, store, n, ctl, st);
}

__global__ __launch_bounds__(256) void dash_write_kernel(DashIn in, const uint32_t* __restrict__ ch_tag,
                                                         const uint64_t* __restrict__ chb, uint32_t n_ch,
                                                         const uint64_t* __restrict__ otag,
                                                         const uint64_t* __restrict__ opt,
                                                         uint8_t* __restrict__ tags_out, float2* __restrict__ pts_out) {
    __shared__ uint32_t s_ord[256];
    __shared__ uint32_t s_hist[4][4];
    const uint32_t k = dash_chunk_of_thread(in, ch_tag, n_ch, s_ord, s_hist);
    if (k == ~0u) return;
    const uint32_t i = ch_tag[k];
    uint32_t nt = 0, np = 0;
    dash_tag<true>(in, i, (uint32_t)(k - chb[i]), tags_out, pts_out, otag[k], opt[k], nt, np);
}

hipError_t launch_dash(const SceneView& sv, const DashBufs& b, int phase, uint8_t* tags_out, float2* pts_out,
                       hipStream_t s) {
    const uint32_t n = sv.n_tags;
    if (n == 0) return hipSuccess;
    const uint32_t g = (n + 255u) / 256u;
    DashIn in{sv, b.desc, b.pat, b.panels, b.len, b.cum, b.subix, b.sub_start};
    if (phase == 0) {
        dash_measure_kernel<<<g, 256, 0, s>>>(sv, b.desc, b.len, b.panels);
        dash_scan_kernel<<<scan_tiles(n), kScanBlock, 0, s>>>(sv.tags, b.len, n, b.cum, b.subix, (ScanCtl*)b.ctl0,
                                                               (TileStatus*)b.st0);
        dash_sub_start_kernel<<<g, 256, 0, s>>>(sv.tags, b.cum, b.subix, n, b.sub_start);
        dash_nch_kernel<<<g, 256, 0, s>>>(in, b.nch, b.flag);
        return launch_scan_counts(b.nch, n, b.chb, b.ctl1, b.st1, s);
    }
    if (b.n_ch == 0) return hipSuccess;
    const uint32_t gc = (b.n_ch + 255u) / 256u;
    if (phase == 1) {
        dash_chunk_tag_kernel<<<g, 256, 0, s>>>(b.nch, b.chb, n, b.ch_tag);
        dash_count_kernel<<<gc, 256, 0, s>>>(in, b.ch_tag, b.chb, b.n_ch, b.cnt);
        dash_off_scan_kernel<<<scan_tiles(b.n_ch), kScanBlock, 0, s>>>(b.cnt, b.n_ch, b.otag, b.opt,
                                                                        (ScanCtl*)b.ctl2, (TileStatus*)b.st2);
    } else {
        dash_write_kernel<<<gc, 256, 0, s>>>(in, b.ch_tag, b.chb, b.n_ch, b.otag, b.opt, tags_out, pts_out);
    }
    return hipGetLastError();
}

}  // namespace sx
