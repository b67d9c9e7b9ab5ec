// Test shim: the single-pass kernel's per-tag body (soup_tag, the same code
// the kernel runs) built for the host, with a sink that reserves records on
// a plain counter (the kernel's atomic add) and checks every record index
// against the output buffer.  Built with the host sanitizers (address,
// undefined behaviour) by the CPU test.  Test infrastructure only.
#include <cstdio>
#include <cstring>
#include <vector>
#include "sx_device.h"
#include "sx_encode.h"
using namespace sx;

struct HostSoupSink {
    static constexpr bool kStats = false;
    float* out;
    uint64_t cap;
    uint64_t* counter;
    float* es_tab;
    XIncF xi;
    uint32_t path, slot, n, arcs, newton;
    uint32_t st[1];
    uint64_t bad;  // records written outside their reservation
    template <class P>
    void put(uint32_t hdr, uint32_t nrec, uint32_t K, const P& p) {
        n += nrec;
        if (nrec == 0u) return;
        const uint64_t base = *counter;
        *counter += nrec;
        if (base + nrec > cap) return;
        uint32_t w[2 * kUnitWords] = {};
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
            if (o.idx != base + (uint64_t)c * K + nchunk) bad++;
        }
    }
};

// Returns 0; *n_out: records the scene needs; recs (cap records) receives them
// when they fit.  flags: bit 1 the exact-density mode.
extern "C" int soup_expand(const sx_paths* paths, const sx_style* styles, uint32_t ns, const sx_affine* xf,
                           uint32_t nx, float tol, int mode, uint32_t K, int flags, float* recs, uint64_t cap,
                           uint64_t* n_out, uint64_t* bad_out) {
    HostEncoding enc;
    std::string err;
    if (!encode_paths(*paths, styles, ns, nx, enc, err)) return -1;
    const uint32_t n = (uint32_t)enc.tags.size();
    const uint32_t ms = mon_stride_of(n);
    std::vector<uint32_t> mon(4 * (size_t)ms + 4);
    uint32_t off = 0, pth = 0, sty = 0, xfi = 0;
    for (uint32_t i = 0; i < n; i++) {
        const uint32_t t = enc.tags[i];
        mon[i] = off;
        mon[ms + i] = pth;
        sty += (t & kTagStyle) ? 1 : 0;
        xfi += (t & kTagXform) ? 1 : 0;
        mon[2 * ms + i] = sty - 1;
        mon[3 * ms + i] = xfi - 1;
        off += (t & kTagCount) + ((t & kTagEnd) ? 1 : 0);
        pth += (t & kTagPath) ? 1 : 0;
    }
    std::vector<StyleD> sd;
    for (auto k : enc.style_stream) {
        const sx_style& s = styles[k];
        sd.push_back((s.flags & 1) ? StyleD{0.0f, 1.0f, kStyleFill}
                                   : StyleD{s.half_width, s.miter_limit,
                                            (uint32_t)s.join | ((uint32_t)s.start_cap << 8) |
                                                ((uint32_t)s.end_cap << 16)});
    }
    std::vector<float> xd;
    for (auto k : enc.xform_stream) {
        const sx_affine& X = xf[k];
        const float v[6] = {X.a, X.b, X.c, X.d, X.e, X.f};
        xd.insert(xd.end(), v, v + 6);
    }
    SceneView sv;
    sv.tags = enc.tags.data();
    sv.pts = (const float2*)enc.data.data();
    sv.styles = sd.data();
    sv.xforms = xd.data();
    sv.path_map = enc.path_map.data();
    sv.mon = mon.data();
    sv.n_tags = n;
    sv.n_pts = (uint32_t)(enc.data.size() / 2);
    sv.n_styles = (uint32_t)sd.size();
    sv.n_xforms = (uint32_t)(xd.size() / 6);
    sv.n_paths = (uint32_t)enc.path_map.size();
    sv.mon_stride = ms;
    Cfg cfg;
    const double tf = kFlatFrac * (double)tol;
    cfg.tau_fit = kFitFrac * (double)tol;
    cfg.tau_flat = tf;
    cfg.inv_sqrt8tf = std::sqrt(1.0 / (8.0 * tf));
    cfg.cbrt_inv120tf = std::cbrt(1.0 / (120.0 * tf));
    cfg.arcs = mode;
    cfg.paper_fit = 0;
    cfg.newton = (flags >> 1) & 1;
    cfg.K = K;
    set_break_increments(cfg.xinc);
    XIncF xi;
    for (int q = 0; q < 5; q++) xi.v[q] = (float)cfg.xinc[q];
    uint64_t counter = 0, bad = 0;
    for (uint32_t i = 0; i < n; i++) {
        float es_loc[8];
        HostSoupSink k{recs, cap, &counter, es_loc, xi, 0u, 0u, 0u, (uint32_t)mode,
                       (uint32_t)(cfg.newton && !mode), {0u}, 0u};
        const uint32_t pi = sv.mon[(size_t)ms + i];
        k.path = pi < sv.n_paths ? sv.path_map[pi] : 0xffffffffu;
        soup_tag(k, cfg, sv, i);
        bad += k.bad;
    }
    *n_out = counter;
    *bad_out = bad;
    return 0;
}
