// Test shim: the device code of the expansion (sx_device.h) compiled for the
// host and driven through the same steps as the GPU pipeline -- tag monoids,
// the bisection of every segment into slots, each slot's items, the scan of
// the slots' record counts, each item's records -- so the CPU suite can check
// the kernels' arithmetic against the oracle without a GPU.  Serial, test
// infrastructure only.
#include <vector>
#include <cstring>
#include "sx_device.h"
#include "sx_encode.h"
using namespace sx;
static uint32_t g_K = 16;
extern "C" void dh_set_k(uint32_t k) { g_K = k; }
// counts: per-tag record counts (cap_tags entries); recs: records (cap_recs,
// or null to count only).  Returns 0, or < 0 on invalid input / short buffers.
extern "C" int dh_expand(const sx_paths* paths, const sx_style* styles, uint32_t ns, const sx_affine* xf, uint32_t nx,
                     float tol, int mode, uint32_t* counts, uint32_t cap_tags, float* recs, uint64_t cap_recs,
                     uint32_t* n_tags_out, uint64_t* n_recs_out, int paper_fit) {
    HostEncoding enc; std::string err;
    if (!encode_paths(*paths, styles, ns, nx, enc, err)) return -1;
    uint32_t n = enc.tags.size();
    *n_tags_out = n;
    if (n > cap_tags) return -4;
    const uint32_t ms = mon_stride_of(n);
    std::vector<uint32_t> mon(4 * (size_t)ms + 4);
    uint32_t off = 0, pth = 0, sty = 0, xfi = 0;
    for (uint32_t i = 0; i < n; i++) {
        uint32_t t = enc.tags[i];
        mon[i] = off; mon[ms + i] = pth;
        sty += (t & kTagStyle) ? 1 : 0; xfi += (t & kTagXform) ? 1 : 0;
        mon[2 * ms + i] = sty - 1; mon[3 * ms + i] = xfi - 1;
        off += (t & kTagCount) + ((t & kTagEnd) ? 1 : 0);
        pth += (t & kTagPath) ? 1 : 0;
    }
    std::vector<StyleD> sd;
    for (auto k : enc.style_stream) { const sx_style& s = styles[k]; sd.push_back(((s.flags & 1) ? StyleD{0.0f, 1.0f, kStyleFill} : StyleD{s.half_width, s.miter_limit, (uint32_t)s.join | ((uint32_t)s.start_cap << 8) | ((uint32_t)s.end_cap << 16)})); }
    std::vector<float> xd;
    for (auto k : enc.xform_stream) { const sx_affine& X = xf[k]; float v[6] = {X.a, X.b, X.c, X.d, X.e, X.f}; xd.insert(xd.end(), v, v + 6); }
    SceneView sv;
    sv.tags = enc.tags.data(); sv.pts = (const float2*)enc.data.data(); sv.styles = sd.data(); sv.xforms = xd.data();
    sv.path_map = enc.path_map.data(); sv.mon = mon.data(); sv.n_tags = n; sv.n_pts = enc.data.size()/2; sv.n_styles = sd.size(); sv.n_xforms = xd.size()/6; sv.n_paths = enc.path_map.size(); sv.mon_stride = ms;
    Cfg cfg; double tf = kFlatFrac * (double)tol;
    cfg.tau_fit = kFitFrac * (double)tol; cfg.tau_flat = tf; cfg.inv_sqrt8tf = std::sqrt(1.0 / (8.0 * tf));
    cfg.cbrt_inv120tf = std::cbrt(1.0 / (120.0 * tf)); cfg.arcs = mode; cfg.paper_fit = paper_fit & 1; cfg.newton = (paper_fit >> 1) & 1;
    cfg.K = g_K;
    set_break_increments(cfg.xinc);
    // slot pipeline on the host: bisection -> slots, slots -> items, scan, records
    struct Fix {
        uint64_t next, cap;
        SX_HD uint64_t alloc(uint32_t nc) { if (next + nc > cap) { next += nc; return ~0ull; } uint64_t b = next; next += nc; return b; }
    };
    std::vector<Slot> slots;
    std::vector<uint64_t> tag_first(n + 1);
    for (uint32_t i = 0; i < n; i++) {
        tag_first[i] = slots.size();
        TagInfo ti; Seg sg;
        fetch_tag(sv, i, ti, sg);
        if (ti.kind == kTagSegment) {
            Bisect bs; bisect_init(bs, sg);
            for (;;) {
                uint32_t t0u, depth; bool done, pivot;
                if (bisect_step(bs, sg, cfg, ti.line, t0u, depth, pivot, done)) {
                    slots.push_back(Slot{i, slot_code(t0u, depth, pivot)});
                    if (done) break;
                }
            }
        }
        slots.push_back(Slot{i, kSlotTail});
    }
    tag_first[n] = slots.size();
    std::vector<Unit> items, st(1024);
    std::vector<float> es_tab(8 * slots.size() + 8);
    std::vector<uint32_t> rc(slots.size());
    for (size_t j = 0; j < slots.size(); j++) {
        const Slot sl = slots[j];
        for (;;) {
            ItemSink<Fix> kw{st.data(), es_tab.data(), Fix{0, st.size()}, enc.path_map[mon[ms + sl.tag]], (uint32_t)j, 0};
            TagInfo ti; Seg sg;
            fetch_tag(sv, sl.tag, ti, sg);
            if (sl.code == kSlotTail) emit_tail(kw, cfg, sv, sl.tag, ti, sg);
            else emit_piece(kw, cfg, sg, ti.line, code_t0u(sl.code), code_depth(sl.code), code_pivot(sl.code));
            if (kw.al.next > st.size()) { st.resize(kw.al.next); continue; }
            items.insert(items.end(), st.begin(), st.begin() + kw.al.next);
            rc[j] = kw.n;
            break;
        }
    }
    std::vector<uint64_t> roff(slots.size() + 1);
    uint64_t acc = 0;
    for (size_t j = 0; j < slots.size(); j++) { roff[j] = acc; acc += rc[j]; }
    roff[slots.size()] = acc;
    uint64_t total = acc;
    std::vector<uint64_t> offs(n + 1);
    for (uint32_t i = 0; i <= n; i++) offs[i] = roff[tag_first[i]];
    for (uint32_t i = 0; i < n; i++) counts[i] = (uint32_t)(offs[i + 1] - offs[i]);
    *n_recs_out = total;
    if (!recs || total > cap_recs) return 0;
    for (size_t u = 0; u < items.size(); u++) {
        const uint32_t* w = items[u].w;
        const uint32_t kind = w[0] & 15u;
        if (kind == 0) continue;
        uint32_t buf[32];
        memcpy(buf, w, 64);
        if (kind != kItemOffset) memcpy(buf + 16, items[u + 1].w, 64);
        const uint32_t path = w[1], slot = w[2];
        RecOut o{recs, roff[slot] + w[3], roff[slot + 1], path, cfg.arcs};
        XIncF xi;
        for (int q = 0; q < 5; q++) xi.v[q] = (float)cfg.xinc[q];
        if (cfg.newton) emit_item<true>(buf, es_tab.data() + 8 * (size_t)slot, xi, o);
        else emit_item<false>(buf, es_tab.data() + 8 * (size_t)slot, xi, o);
        if (o.idx != roff[slot] + w[3] + item_n(w[0])) return -10;
    }
    return 0;
}
