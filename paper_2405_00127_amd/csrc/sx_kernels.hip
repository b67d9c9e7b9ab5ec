// HIP kernels of the stroke-expansion hot path for gfx950 (wave64).
//
//  scan_tags_kernel   tag-monoid prefix scan (Section 8.2): single pass,
//                     wave64 shuffle scan + LDS block scan + decoupled
//                     look-back over dynamically numbered tiles.
//  piece_kernel       per tag, the per-segment decisions (Algorithm 1 /
//                     Algorithm 2) in FP64; writes emission items into the
//                     workspace (slots handed out per tile by LDS atomics,
//                     overflow through one global counter) and the tag's
//                     record count.
//  scan_counts_kernel exclusive scan of the counts into u64 output offsets
//                     (replaces the paper's atomic bump allocation, so the
//                     output order is canonical and deterministic).
//  record_kernel      per item chunk, the FP32 per-point work: records at
//                     offsets[tag] + the chunk's position within the tag.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sx_device.h"
#include "sx_kernels.h"

namespace sx {

// ------------------------------------------------------ look-back scan
// Per-tile status word: (epoch << 2) | state, state 1 = aggregate ready,
// 2 = inclusive prefix ready.  The epoch (kept in device memory and bumped
// by the last tile of every launch) makes stale flags of earlier launches
// read as "not ready", so nothing has to be cleared between launches and the
// kernels can be replayed inside a HIP graph.
// The aggregate and the inclusive prefix live in separate words: a reader
// that saw "aggregate ready" must never pick up a later inclusive value.
struct TileStatus {
    uint32_t flag;
    uint32_t pad;
    uint64_t agg_a, agg_b;
    uint64_t inc_a, inc_b;
    uint64_t pad2[3];
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

__device__ __forceinline__ uint32_t load_acquire(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_release(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish a tile's value with its state (data first, then the flag).
__device__ __forceinline__ void publish(TileStatus* st, uint32_t tile, uint32_t epoch, uint32_t state, Pair v) {
    if (state == 1) {
        st[tile].agg_a = v.a;
        st[tile].agg_b = v.b;
    } else {
        st[tile].inc_a = v.a;
        st[tile].inc_b = v.b;
    }
    __threadfence();
    store_release(&st[tile].flag, (epoch << 2) | state);
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
        int64_t idx = pos - lane;
        uint32_t state;
        Pair v{0, 0};
        for (uint32_t spins = 0;; spins++) {
            state = 3;  // lanes past tile 0 count as "inclusive zero"
            if (idx >= 0) {
                uint32_t f = load_acquire(&st[idx].flag);
                state = ((f >> 2) == (epoch & 0x3fffffffu)) ? (f & 3u) : 0u;
            }
            if (__ballot(state == 0u) == 0ull) break;
            if (spins >= kSpinLimit) {
                if (lane == 0) atomicOr(err, 1u);
                state = 3;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (idx >= 0 && state == 1u) {
            v.a = __hip_atomic_load(&st[idx].agg_a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            v.b = __hip_atomic_load(&st[idx].agg_b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (idx >= 0 && state == 2u) {
            v.a = __hip_atomic_load(&st[idx].inc_a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            v.b = __hip_atomic_load(&st[idx].inc_b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        uint64_t incl_mask = __ballot(state >= 2u);
        if (incl_mask) {
            int first = __builtin_ctzll(incl_mask);  // nearest tile with a full prefix
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
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ Pair tag_inc(uint32_t t) {
    uint64_t pts = (t & kTagCount) + ((t & kTagEnd) ? 1u : 0u);
    uint64_t pth = (t & kTagPath) ? 1u : 0u;
    uint64_t sty = (t & kTagStyle) ? 1u : 0u;
    uint64_t xf = (t & kTagXform) ? 1u : 0u;
    return Pair{pts | (pth << 32), sty | (xf << 32)};
}

template <class Load, class Store>
__device__ void scan_tile(Load load, Store store, uint32_t n, ScanCtl* ctl, TileStatus* st) {
    __shared__ uint32_t s_tile, s_epoch;
    __shared__ Pair s_wave[kScanBlock / 64];
    __shared__ Pair s_excl;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) {
        s_tile = atomicAdd(&ctl->ticket, 1u);
        s_epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t tile = s_tile, epoch = s_epoch & 0x3fffffffu;
    const uint64_t base = (uint64_t)tile * kScanTile + (uint64_t)tid * kScanItems;
    Pair item[kScanItems];
    load(base, item);
    Pair run{0, 0};
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
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
            if (lane == 0) publish(st, tile, epoch, 2, agg);
        } else {
            if (lane == 0) publish(st, tile, epoch, 1, agg);
            excl = look_back(st, tile, epoch, lane, &ctl->err);
            if (lane == 0) publish(st, tile, epoch, 2, excl + agg);
        }
        if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    Pair pre = s_excl + texcl;
    store(base, item, pre);
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
        if (atomicAdd(&ctl->done, 1u) == ntiles - 1) {
            ctl->ticket = 0;
            ctl->done = 0;
            __threadfence();
            __hip_atomic_store(&ctl->epoch, (s_epoch + 1u) & 0x3fffffffu, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
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
        if (base + kScanItems <= n) {
            uint4 raw = *reinterpret_cast<const uint4*>(tags + base);
            uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
            for (int j = 0; j < kScanItems; j++) item[j] = tag_inc((w[j >> 2] >> (8 * (j & 3))) & 0xffu);
        } else {
#pragma unroll
            for (int j = 0; j < kScanItems; j++) item[j] = (base + j < n) ? tag_inc(tags[base + j]) : Pair{0, 0};
        }
    };
    auto store = [&](uint64_t base, const Pair* incl, Pair pre) {
        // item j: exclusive = pre + incl[j-1]; style/xform stored inclusive - 1
        uint32_t o_off[kScanItems], o_pth[kScanItems], o_sty[kScanItems], o_xf[kScanItems];
#pragma unroll
        for (int j = 0; j < kScanItems; j++) {
            Pair ex = pre;
            if (j > 0) ex = ex + incl[j - 1];
            Pair in = pre + incl[j];
            o_off[j] = (uint32_t)ex.a;
            o_pth[j] = (uint32_t)(ex.a >> 32);
            o_sty[j] = (uint32_t)in.b - 1u;
            o_xf[j] = (uint32_t)(in.b >> 32) - 1u;
        }
        uint32_t* m0 = mon;
        uint32_t* m1 = mon + n;
        uint32_t* m2 = mon + 2 * (size_t)n;
        uint32_t* m3 = mon + 3 * (size_t)n;
        if (base + kScanItems <= n && (n & 3u) == 0u) {
#pragma unroll
            for (int j = 0; j < kScanItems; j += 4) {
                *reinterpret_cast<uint4*>(m0 + base + j) = make_uint4(o_off[j], o_off[j + 1], o_off[j + 2], o_off[j + 3]);
                *reinterpret_cast<uint4*>(m1 + base + j) = make_uint4(o_pth[j], o_pth[j + 1], o_pth[j + 2], o_pth[j + 3]);
                *reinterpret_cast<uint4*>(m2 + base + j) = make_uint4(o_sty[j], o_sty[j + 1], o_sty[j + 2], o_sty[j + 3]);
                *reinterpret_cast<uint4*>(m3 + base + j) = make_uint4(o_xf[j], o_xf[j + 1], o_xf[j + 2], o_xf[j + 3]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < kScanItems; j++) {
                if (base + j < n) {
                    m0[base + j] = o_off[j];
                    m1[base + j] = o_pth[j];
                    m2[base + j] = o_sty[j];
                    m3[base + j] = o_xf[j];
                }
            }
        }
    };
    scan_tile(load, store, n, ctl, st);
}

// exclusive scan of u32 counts into u64 offsets; out[n] = total
__global__ __launch_bounds__(kScanBlock) void scan_counts_kernel(const uint32_t* __restrict__ in, uint32_t n,
                                                                 uint64_t* __restrict__ out, ScanCtl* ctl,
                                                                 TileStatus* st) {
    auto load = [&](uint64_t base, Pair* item) {
        if (base + kScanItems <= n) {
#pragma unroll
            for (int j = 0; j < kScanItems; j += 4) {
                uint4 v = *reinterpret_cast<const uint4*>(in + base + j);
                item[j] = Pair{v.x, 0};
                item[j + 1] = Pair{v.y, 0};
                item[j + 2] = Pair{v.z, 0};
                item[j + 3] = Pair{v.w, 0};
            }
        } else {
#pragma unroll
            for (int j = 0; j < kScanItems; j++) item[j] = Pair{(base + j < n) ? (uint64_t)in[base + j] : 0ull, 0};
        }
    };
    auto store = [&](uint64_t base, const Pair* incl, Pair pre) {
#pragma unroll
        for (int j = 0; j < kScanItems; j++) {
            uint64_t ex = pre.a + (j > 0 ? incl[j - 1].a : 0ull);
            if (base + j < n) out[base + j] = ex;
            if (base + j == (uint64_t)n - 1u) out[n] = pre.a + incl[j].a;
        }
    };
    scan_tile(load, store, n, ctl, st);
}

// ------------------------------------------------------ pieces / records
constexpr int kTagBlock = 256;
constexpr int kRecBlock = 256;
constexpr int kOvfBlocks = 512;  // record-kernel blocks striding over the overflow slots

// Slot allocator of one piece-kernel tile: the tile's own region first (LDS
// counter), then the shared overflow region (global counter).
struct TileAlloc {
    Item* items;
    uint32_t* lds_n;
    uint64_t region;
    uint32_t region_cap;
    unsigned long long* ovf_n;
    uint64_t ovf_base, ovf_cap;
    __device__ uint64_t alloc(uint32_t nc) {
        uint32_t s = atomicAdd(lds_n, nc);
        if (s + nc <= region_cap) return region + s;
        // the part of the request inside the region is left empty
        for (uint32_t j = s; j < region_cap; j++) items[region + j].hdr = 0u;
        unsigned long long o = atomicAdd(ovf_n, (unsigned long long)nc);
        if (o + nc <= ovf_cap) return ovf_base + o;
        return ~0ull;
    }
};

// Work class of a tag for the in-block ordering: cubics (longest bisection),
// quadratics, then lines and stroke cap markers (no bisection).
__device__ __forceinline__ uint32_t work_class(uint32_t tag) {
    if (tag & kTagEnd) return 2u;
    const uint32_t c = tag & kTagCount;
    return c == 3u ? 0u : (c == 2u ? 1u : 2u);
}

// MinWaves: waves per SIMD the register allocation must allow (1, 2 or 3):
// more waves hide more latency, at the price of spills to scratch.
// Block: tags per workgroup and per workspace tile (64 or 256).  With one
// wave per block a SIMD takes new work as soon as its own wave finishes;
// with several, the block first orders its tags by work class (a stable
// counting sort in LDS) so that each wave runs tags of one kind: a wave of
// lines no longer waits for one lane's cubic bisection.
template <int MinWaves, int Block>
__global__ __launch_bounds__(Block, MinWaves) void piece_kernel(SceneView sv, Cfg cfg, ItemWs ws,
                                                                uint32_t* __restrict__ counts) {
    __shared__ uint32_t s_n;
    __shared__ uint32_t s_order[Block];
    __shared__ uint32_t s_hist[Block / 64][3];
    const uint32_t t = threadIdx.x;
    const uint32_t first = blockIdx.x * Block;
    if (t == 0) s_n = 0;
    uint32_t i = first + t;
    if constexpr (Block > 64) {
        const uint32_t lane = t & 63u, wv = t >> 6;
        const uint32_t cls = i < sv.n_tags ? work_class(sv.tags[i]) : 2u;
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        uint64_t m[3];
        uint32_t rank = 0;
#pragma unroll
        for (uint32_t c = 0; c < 3; c++) {
            m[c] = __ballot(cls == c);
            if (cls == c) rank = (uint32_t)__popcll(m[c] & below);
        }
        if (lane == 0) {
#pragma unroll
            for (uint32_t c = 0; c < 3; c++) s_hist[wv][c] = (uint32_t)__popcll(m[c]);
        }
        __syncthreads();
        // destination = tags of lower classes + same class in earlier waves + rank
        uint32_t pos = rank;
        for (uint32_t c = 0; c < 3; c++)
            for (uint32_t w = 0; w < Block / 64; w++)
                if (c < cls || (c == cls && w < wv)) pos += s_hist[w][c];
        s_order[pos] = t;
        __syncthreads();
        i = first + s_order[t];
    } else {
        __syncthreads();
    }
    if (i < sv.n_tags) {
        TileAlloc al{ws.items, &s_n, (uint64_t)blockIdx.x * ws.region_cap, ws.region_cap, &ws.ctl->ovf_n,
                     ws.ovf_base, ws.ovf_cap};
        ItemSink<TileAlloc> k{ws.items, al, i, 0};
        process_tag(k, cfg, sv, i);
        counts[i] = k.n;
    }
    __syncthreads();
    if (t == 0) {
        ws.tile_n[blockIdx.x] = s_n;
        atomicAdd(&ws.ctl->items_total, (unsigned long long)s_n);
    }
}

// The piece kernel with work counters (one configuration; not timed):
// stats[j] += per-tag counts j (fit trials, pieces, ranges, evolutes,
// joins and caps, lines).  Items and counts are written as by piece_kernel.
__global__ __launch_bounds__(kTagBlock) void piece_stats_kernel(SceneView sv, Cfg cfg, ItemWs ws,
                                                                uint32_t* __restrict__ counts,
                                                                unsigned long long* __restrict__ stats) {
    __shared__ uint32_t s_n;
    __shared__ unsigned long long s_st[kStN];
    if (threadIdx.x == 0) s_n = 0;
    if (threadIdx.x < kStN) s_st[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t i = blockIdx.x * kTagBlock + threadIdx.x;
    if (i < sv.n_tags) {
        TileAlloc al{ws.items, &s_n, (uint64_t)blockIdx.x * ws.region_cap, ws.region_cap, &ws.ctl->ovf_n,
                     ws.ovf_base, ws.ovf_cap};
        ItemSink<TileAlloc, true> k{ws.items, al, i, 0, {0, 0, 0, 0, 0, 0}};
        process_tag(k, cfg, sv, i);
        counts[i] = k.n;
        for (int j = 0; j < kStN; j++)
            if (k.st[j]) atomicAdd(&s_st[j], (unsigned long long)k.st[j]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ws.tile_n[blockIdx.x] = s_n;
        atomicAdd(&ws.ctl->items_total, (unsigned long long)s_n);
    }
    if (threadIdx.x < kStN) atomicAdd(&stats[threadIdx.x], s_st[threadIdx.x]);
}

// Record-kernel item classes: offset ranges placed by the density inverse,
// other offset ranges, evolute bundles, joins and caps (and empty slots).
constexpr uint32_t kItemClasses = 4;
__device__ __forceinline__ uint32_t item_class(uint32_t hdr) {
    const uint32_t kind = hdr & 15u;
    if (kind == kItemOffset) return (hdr & kIfPlaceF) ? 0u : 1u;
    return kind == kItemEvolute ? 2u : 3u;
}

__device__ __forceinline__ void record_item(const SceneView& sv, const Item* slot, const uint64_t* offsets,
                                            float* out, uint64_t cap, int arcs) {
    Item it;
    load_item(it, slot);
    if ((it.hdr & 15u) == 0u || it.tag >= sv.n_tags) return;
    const uint32_t pi = sv.mon[(size_t)sv.n_tags + it.tag];
    const uint32_t path = pi < sv.n_paths ? sv.path_map[pi] : 0xffffffffu;
    const uint64_t end = offsets[it.tag + 1] < cap ? offsets[it.tag + 1] : cap;
    RecOut o{out, offsets[it.tag] + it.local, end, path, arcs};
    emit_item(it, o);
}

__global__ __launch_bounds__(kRecBlock) void record_kernel(SceneView sv, ItemWs ws, int arcs,
                                                           const uint64_t* __restrict__ offsets,
                                                           float* __restrict__ out, uint64_t cap_records,
                                                           uint32_t n_tiles) {
    // nothing is written when the records exceed the capacity or items were dropped
    if (offsets[sv.n_tags] > cap_records || ws.ctl->ovf_n > ws.ovf_cap) return;
    const uint32_t b = blockIdx.x;
    if (b < n_tiles) {
        // a tile's items, kRecBlock at a time, each round ordered by item
        // class so that a wave runs items of one kind
        __shared__ uint32_t s_order[kRecBlock];
        __shared__ uint32_t s_hist[kRecBlock / 64][kItemClasses];
        const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
        const uint32_t cnt = ws.tile_n[b] < ws.region_cap ? ws.tile_n[b] : ws.region_cap;
        const Item* base = ws.items + (uint64_t)b * ws.region_cap;
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        for (uint32_t r0 = 0; r0 < cnt; r0 += kRecBlock) {
            const uint32_t cls = (r0 + t < cnt) ? item_class(base[r0 + t].hdr) : kItemClasses - 1;
            uint32_t rank = 0;
#pragma unroll
            for (uint32_t c = 0; c < kItemClasses; c++) {
                const uint64_t m = __ballot(cls == c);
                if (cls == c) rank = (uint32_t)__popcll(m & below);
                if (lane == 0) s_hist[wv][c] = (uint32_t)__popcll(m);
            }
            __syncthreads();
            uint32_t pos = rank;
            for (uint32_t c = 0; c < kItemClasses; c++)
                for (uint32_t w = 0; w < kRecBlock / 64; w++)
                    if (c < cls || (c == cls && w < wv)) pos += s_hist[w][c];
            s_order[pos] = t;
            __syncthreads();
            const uint32_t s2 = r0 + s_order[t];
            if (s2 < cnt) record_item(sv, base + s2, offsets, out, cap_records, arcs);
            __syncthreads();
        }
    } else {
        const uint64_t cnt = ws.ctl->ovf_n;
        const Item* base = ws.items + ws.ovf_base;
        for (uint64_t s = (uint64_t)(b - n_tiles) * kRecBlock + threadIdx.x; s < cnt; s += (uint64_t)kOvfBlocks * kRecBlock)
            record_item(sv, base + s, offsets, out, cap_records, arcs);
    }
}

// out[0] = records, out[1] = 0, or the item count the workspace must hold
// when items were dropped
__global__ void finish_kernel(const uint64_t* __restrict__ offsets, uint32_t n, const ItemWs ws,
                              uint64_t* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        dst[0] = n ? offsets[n] : 0ull;
        dst[1] = (n && ws.ctl->ovf_n > ws.ovf_cap) ? ws.ctl->items_total : 0ull;
    }
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
__global__ void scene_offsets_kernel(const uint64_t* __restrict__ offsets, const GatherDesc* __restrict__ descs,
                                     uint32_t n_scenes, uint32_t n_tags, uint64_t* __restrict__ out) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_scenes) out[s] = n_tags ? offsets[descs[s].tag_base] : 0ull;
    if (s == n_scenes) out[s] = n_tags ? offsets[n_tags] : 0ull;
}

// ------------------------------------------------------------- launches
int scan_tiles(uint32_t n) { return (int)((n + kScanTile - 1) / kScanTile); }

uint32_t piece_tiles(uint32_t n, uint32_t tile) { return (n + tile - 1) / tile; }

hipError_t launch_scan_tags(const uint8_t* tags, uint32_t n, uint32_t* mon, void* ctl, void* st, WsCtl* ws_reset,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    scan_tags_kernel<<<scan_tiles(n), kScanBlock, 0, s>>>(tags, n, mon, (ScanCtl*)ctl, (TileStatus*)st, ws_reset);
    return hipGetLastError();
}
hipError_t launch_scan_counts(const uint32_t* in, uint32_t n, uint64_t* out, void* ctl, void* st, hipStream_t s) {
    if (n == 0) return hipSuccess;
    scan_counts_kernel<<<scan_tiles(n), kScanBlock, 0, s>>>(in, n, out, (ScanCtl*)ctl, (TileStatus*)st);
    return hipGetLastError();
}
hipError_t launch_pieces(const SceneView& sv, const Cfg& cfg, const ItemWs& ws, uint32_t* counts, int waves,
                         hipStream_t s) {
    if (sv.n_tags == 0) return hipSuccess;
    const uint32_t g = piece_tiles(sv.n_tags, ws.tile);
    if (ws.tile == 64) {
        if (waves <= 1) piece_kernel<1, 64><<<g, 64, 0, s>>>(sv, cfg, ws, counts);
        else if (waves == 2) piece_kernel<2, 64><<<g, 64, 0, s>>>(sv, cfg, ws, counts);
        else piece_kernel<3, 64><<<g, 64, 0, s>>>(sv, cfg, ws, counts);
    } else {
        if (waves <= 1) piece_kernel<1, 256><<<g, 256, 0, s>>>(sv, cfg, ws, counts);
        else if (waves == 2) piece_kernel<2, 256><<<g, 256, 0, s>>>(sv, cfg, ws, counts);
        else piece_kernel<3, 256><<<g, 256, 0, s>>>(sv, cfg, ws, counts);
    }
    return hipGetLastError();
}
hipError_t launch_piece_stats(const SceneView& sv, const Cfg& cfg, const ItemWs& ws, uint32_t* counts,
                              unsigned long long* stats, hipStream_t s) {
    if (sv.n_tags == 0) return hipSuccess;
    if (ws.tile != (uint32_t)kTagBlock) return hipErrorInvalidValue;
    piece_stats_kernel<<<piece_tiles(sv.n_tags, kTagBlock), kTagBlock, 0, s>>>(sv, cfg, ws, counts, stats);
    return hipGetLastError();
}
hipError_t launch_records(const SceneView& sv, const ItemWs& ws, int arcs, const uint64_t* offsets, void* out,
                          uint64_t cap, hipStream_t s) {
    if (sv.n_tags == 0) return hipSuccess;
    const uint32_t nt = piece_tiles(sv.n_tags, ws.tile);
    record_kernel<<<nt + kOvfBlocks, kRecBlock, 0, s>>>(sv, ws, arcs, offsets, (float*)out, cap, nt);
    return hipGetLastError();
}
hipError_t launch_gather(const GatherDesc* descs, uint32_t n_scenes, uint8_t* tags, float2* pts, StyleD* styles,
                         float* xforms, uint32_t* path_map, hipStream_t s) {
    if (n_scenes == 0) return hipSuccess;
    gather_kernel<<<dim3(kGatherBlocksPerScene, n_scenes), kGatherBlock, 0, s>>>(descs, tags, pts, styles, xforms,
                                                                                 path_map);
    return hipGetLastError();
}
hipError_t launch_scene_offsets(const uint64_t* offsets, const GatherDesc* descs, uint32_t n_scenes, uint32_t n_tags,
                                uint64_t* scene_offsets, hipStream_t s) {
    scene_offsets_kernel<<<(n_scenes + 1 + 255) / 256, 256, 0, s>>>(offsets, descs, n_scenes, n_tags, scene_offsets);
    return hipGetLastError();
}
hipError_t launch_finish(const uint64_t* offsets, uint32_t n, const ItemWs& ws, uint64_t* dst, hipStream_t s) {
    finish_kernel<<<1, 64, 0, s>>>(offsets, n, ws, dst);
    return hipGetLastError();
}
size_t scan_status_bytes(uint32_t n) { return (size_t)scan_tiles(n > 0 ? n : 1) * sizeof(TileStatus); }
size_t scan_ctl_bytes() { return sizeof(ScanCtl); }

}  // namespace sx
