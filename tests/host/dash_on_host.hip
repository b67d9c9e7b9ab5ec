// Test shim: the dashing passes' per-tag code (dash_len_d, dash_chunks,
// dash_tag in sx_device.h, the code the kernels run) built for the host and
// driven serially: grid lengths, their exclusive prefix with the subpath
// index, subpath starts, the work chunks, per-chunk counts, their prefix,
// the write pass.  Returns the
// dashed encoding for comparison with the oracle's.  Test infrastructure only.
#include <cstring>
#include <vector>
#include "sx_device.h"
#include "sx_encode.h"
using namespace sx;

// dash tables per user style as in sx_scene_encode_dashed; returns 0, -1 on
// invalid input, -4 when the output buffers are short (*nt, *np: the need)
extern "C" int dh_dash(const sx_paths* paths, const sx_style* styles, uint32_t ns, const float* dash_arr,
                       const uint32_t* dash_off, const float* dash_phase, uint32_t nx, uint8_t* tags_out,
                       float* pts_out, uint64_t cap_tags, uint64_t cap_pts, uint64_t* nt_out, uint64_t* np_out) {
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
    // patterns per style entry
    std::vector<DashDesc> desc;
    std::vector<int64_t> pat;
    for (auto k : enc.style_stream) {
        DashDesc d{(uint32_t)pat.size(), 0, 0, 0};
        const uint32_t cnt = dash_off[k + 1] - dash_off[k];
        if (!(styles[k].flags & 1) && cnt) {
            const uint32_t m = (cnt & 1u) ? 2 * cnt : cnt;
            int64_t period = 0;
            for (uint32_t j = 0; j < m; j++) {
                pat.push_back(dash_fix((double)dash_arr[dash_off[k] + j % cnt]));
                period += pat.back();
            }
            if (period > 0) {
                int64_t ph = dash_fix((double)dash_phase[k]) % period;
                d.n = m;
                d.period = period;
                d.phase = ph < 0 ? ph + period : ph;
            } else {
                pat.resize(d.off);
            }
        }
        desc.push_back(d);
    }
    SceneView sv;
    sv.tags = enc.tags.data();
    sv.pts = (const float2*)enc.data.data();
    sv.styles = nullptr;
    sv.xforms = nullptr;
    sv.path_map = enc.path_map.data();
    sv.mon = mon.data();
    sv.n_tags = n;
    sv.n_pts = (uint32_t)(enc.data.size() / 2);
    sv.n_styles = (uint32_t)desc.size();
    sv.n_xforms = 0;
    sv.n_paths = (uint32_t)enc.path_map.size();
    sv.mon_stride = ms;
    std::vector<uint64_t> len(n + 1, 0), cum(n + 1, 0), sub(n + 2, 0);
    std::vector<double> panels((size_t)n * kDashPanels + 1, 0.0);
    std::vector<uint32_t> subix(n + 1, 0);
    for (uint32_t i = 0; i < n; i++) {
        const uint32_t tag = enc.tags[i];
        const uint32_t s = mon[2 * ms + i];
        if (!(tag & kTagEnd) && desc[s].n) {
            const int c = (int)(tag & kTagCount);
            const float2* D = sv.pts + mon[i];
            D2 P[4];
            for (int j = 0; j <= c; j++) P[j] = d2((double)D[j].x, (double)D[j].y);
            double panel[kDashPanels];
            len[i] = (uint64_t)dash_fix(dash_len_d(P, c, panel));
            for (int k = 0; k < kDashPanels; k++) panels[(size_t)k * n + i] = panel[k];
        }
    }
    for (uint32_t i = 0; i < n; i++) {
        cum[i + 1] = cum[i] + len[i];
        subix[i + 1] = subix[i] + ((enc.tags[i] & kTagEnd) ? 1u : 0u);
    }
    for (uint32_t i = 0; i < n; i++)
        if (enc.tags[i] & kTagEnd) sub[subix[i] + 1] = cum[i];
    DashIn in{sv, desc.data(), pat.data(), panels.data(), len.data(), cum.data(), subix.data(), sub.data()};
    // work chunks as the kernels take them: (tag, chunk index)
    std::vector<std::pair<uint32_t, uint32_t>> chunks;
    for (uint32_t i = 0; i < n; i++)
        for (uint32_t q = 0, nq = dash_chunks(in, i); q < nq; q++) chunks.push_back({i, q});
    const size_t nc = chunks.size();
    std::vector<uint64_t> ot(nc + 1, 0), op(nc + 1, 0);
    for (size_t k = 0; k < nc; k++) {
        uint32_t a = 0, b = 0;
        dash_tag<false>(in, chunks[k].first, chunks[k].second, nullptr, nullptr, 0, 0, a, b);
        ot[k + 1] = ot[k] + a;
        op[k + 1] = op[k] + b;
    }
    *nt_out = ot[nc];
    *np_out = op[nc];
    if (!tags_out || ot[nc] > cap_tags || op[nc] > cap_pts) return tags_out ? -4 : 0;
    for (size_t k = 0; k < nc; k++) {
        uint32_t a = 0, b = 0;
        dash_tag<true>(in, chunks[k].first, chunks[k].second, tags_out, (float2*)pts_out, ot[k], op[k], a, b);
        if (a != ot[k + 1] - ot[k] || b != op[k + 1] - op[k]) return -5;  // the passes disagree
    }
    return 0;
}
