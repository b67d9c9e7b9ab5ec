// Host path encoder (Section 8.2, Table 1).
//
// Produces the tag stream (one byte per segment plus one stroke cap marker
// per subpath), the overlapping point stream (each segment's first point is
// the previous segment's last, except at subpath starts), the style and
// transform streams (one entry per change between consecutive paths, the
// tag's style / transform bit marking the change) and the encoded-path ->
// input-path map.  A fill's subpaths all end closed: a line back to the start
// point is added where a subpath ends elsewhere without a closepath.
#include "sx_encode.h"

#include <cmath>
#include <cstring>

namespace sx {

namespace {
constexpr uint8_t kCount = 0x03, kEnd = 0x04, kF32 = 0x08, kPathBit = 0x10, kXfBit = 0x20, kStyleBit = 0x40,
                  kClosedBit = 0x80;

struct SubpathState {
    bool open = false;     // a moveto (or closepath) established a current point
    uint32_t nseg = 0;     // drawing segments emitted so far
    bool closed = false;
    float sx = 0, sy = 0;  // subpath start
    float cx = 0, cy = 0;  // current point
    bool has_dir = false;  // start-tangent point found
    float dx = 0, dy = 0;
};

inline bool same(float ax, float ay, float bx, float by) { return ax == bx && ay == by; }
}  // namespace

bool encode_paths(const sx_paths& in, const sx_style* styles, uint32_t n_styles, uint32_t n_xforms,
                  HostEncoding& out, std::string& err) {
    out = HostEncoding{};
    out.tags.reserve(in.verb_off ? in.verb_off[in.n_paths] + in.n_paths : 0);
    int64_t prev_style = -1, prev_xf = -1;
    auto put_pt = [&](float x, float y) {
        out.data.push_back(x);
        out.data.push_back(y);
    };
    for (uint32_t k = 0; k < in.n_paths; k++) {
        if (in.style_ix[k] >= n_styles) { err = "style index out of range"; return false; }
        if (in.xform_ix[k] >= n_xforms) { err = "transform index out of range"; return false; }
        if (in.verb_off[k + 1] < in.verb_off[k] || in.pt_off[k + 1] < in.pt_off[k]) {
            err = "offsets not increasing";
            return false;
        }
        const size_t first_tag = out.tags.size();
        const bool fill = (styles[in.style_ix[k]].flags & SX_STYLE_FILL) != 0;
        const float* P = in.pts + 2 * (size_t)in.pt_off[k];
        const uint32_t np = in.pt_off[k + 1] - in.pt_off[k];
        uint32_t pi = 0;
        SubpathState sp;
        auto close_line = [&]() {
            if (!same(sp.cx, sp.cy, sp.sx, sp.sy)) {
                out.tags.push_back((uint8_t)(1u | kF32));
                put_pt(sp.sx, sp.sy);
                sp.cx = sp.sx;
                sp.cy = sp.sy;
            }
        };
        auto finish = [&]() {
            if (sp.open && sp.nseg > 0) {
                if (fill && !sp.closed) {
                    close_line();
                    sp.closed = true;
                }
                out.tags.push_back((uint8_t)(2u | kEnd | kF32 | (sp.closed ? kClosedBit : 0u)));
                if (!sp.has_dir) { sp.dx = sp.sx + 1.0f; sp.dy = sp.sy; }
                put_pt(sp.sx, sp.sy);
                put_pt(sp.dx, sp.dy);
            }
        };
        for (uint32_t vi = in.verb_off[k]; vi < in.verb_off[k + 1]; vi++) {
            const uint8_t v = in.verbs[vi];
            if (v == SX_MOVE) {
                finish();
                if (pi + 1 > np) { err = "point count mismatch"; return false; }
                float x = P[2 * pi], y = P[2 * pi + 1];
                if (!std::isfinite(x) || !std::isfinite(y)) { err = "non-finite coordinate"; return false; }
                sp = SubpathState{};
                sp.open = true;
                sp.sx = sp.cx = x;
                sp.sy = sp.cy = y;
                pi++;
            } else if (v == SX_CLOSE) {
                if (!sp.open) continue;
                if (sp.nseg > 0) close_line();
                sp.closed = true;
                finish();
                // the current point returns to the start; a following drawing
                // verb opens a new subpath there
                float x = sp.sx, y = sp.sy;
                sp = SubpathState{};
                sp.open = true;
                sp.sx = sp.cx = x;
                sp.sy = sp.cy = y;
            } else if (v == SX_LINE || v == SX_QUAD || v == SX_CUBIC) {
                if (!sp.open) { err = "path must start with SX_MOVE"; return false; }
                const uint32_t c = v;
                if (pi + c > np) { err = "point count mismatch"; return false; }
                bool moves = false;
                for (uint32_t j = 0; j < c; j++) {
                    float x = P[2 * (pi + j)], y = P[2 * (pi + j) + 1];
                    if (!std::isfinite(x) || !std::isfinite(y)) { err = "non-finite coordinate"; return false; }
                    if (!same(x, y, sp.cx, sp.cy)) moves = true;
                }
                if (!moves) { pi += c; continue; }  // zero-length segment
                if (sp.nseg == 0) put_pt(sp.cx, sp.cy);
                if (!sp.has_dir) {
                    for (uint32_t j = 0; j < c; j++) {
                        float x = P[2 * (pi + j)], y = P[2 * (pi + j) + 1];
                        if (!same(x, y, sp.sx, sp.sy)) {
                            sp.dx = x;
                            sp.dy = y;
                            sp.has_dir = true;
                            break;
                        }
                    }
                }
                for (uint32_t j = 0; j < c; j++) put_pt(P[2 * (pi + j)], P[2 * (pi + j) + 1]);
                out.tags.push_back((uint8_t)(c | kF32));
                sp.cx = P[2 * (pi + c - 1)];
                sp.cy = P[2 * (pi + c - 1) + 1];
                pi += c;
                sp.nseg++;
            } else {
                err = "unknown verb";
                return false;
            }
        }
        finish();
        if (pi != np) { err = "point count mismatch"; return false; }
        if (out.tags.size() > first_tag) {
            out.tags.back() |= kPathBit;
            if ((int64_t)in.style_ix[k] != prev_style) {
                out.tags[first_tag] |= kStyleBit;
                out.style_stream.push_back(in.style_ix[k]);
                prev_style = in.style_ix[k];
            }
            if ((int64_t)in.xform_ix[k] != prev_xf) {
                out.tags[first_tag] |= kXfBit;
                out.xform_stream.push_back(in.xform_ix[k]);
                prev_xf = in.xform_ix[k];
            }
            out.path_map.push_back(k);
        }
        if (out.tags.size() > 0xF0000000ull) { err = "scene too large"; return false; }
    }
    return true;
}

}  // namespace sx
