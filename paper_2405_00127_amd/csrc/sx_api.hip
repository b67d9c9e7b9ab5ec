// C ABI of the strokex library (declared in include/strokex.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "strokex.h"
#include "sx_device.h"
#include "sx_encode.h"
#include "sx_kernels.h"

struct sx_ctx {
    int device = 0;
    std::string err;
    uint64_t* pinned_total = nullptr;  // host-pinned 2 x u64: record count, items needed
};

struct sx_scene {
    sx_ctx* ctx = nullptr;
    uint32_t n_tags = 0, n_pts = 0, n_paths = 0, n_styles = 0, n_xforms = 0;
    uint8_t* d_tags = nullptr;
    float2* d_pts = nullptr;
    sx::StyleD* d_styles = nullptr;
    float* d_xforms = nullptr;
    uint32_t* d_path_map = nullptr;
    uint32_t* d_mon = nullptr;
    uint32_t* d_counts = nullptr;
    uint64_t* d_offsets = nullptr;
    void* d_scan_ctl = nullptr;  // two control blocks (tags, counts)
    void* d_status_tags = nullptr;
    void* d_status_counts = nullptr;
    // item workspace of the piece / record kernels
    sx::Item* d_items = nullptr;
    uint32_t* d_tile_n = nullptr;
    sx::WsCtl* d_ws_ctl = nullptr;
    uint32_t region_cap = 0;  // slots per piece tile
    uint64_t ovf_cap = 0;     // shared overflow slots
    uint32_t chunk_k = 16;    // records per item chunk
    hipStream_t last_stream = nullptr;
};

namespace {

constexpr uint32_t kRegionPerTag = 8;      // initial item slots per tag
constexpr uint64_t kMinOverflow = 65536;   // initial shared overflow slots (minimum)

int fail(sx_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}
int hip_fail(sx_ctx* ctx, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? SX_ENOMEM : SX_EDEVICE, m);
}

template <class T>
hipError_t dalloc(T** p, size_t bytes) {
    return hipMalloc((void**)p, bytes ? bytes : 16);
}

void free_scene(sx_scene* s) {
    if (!s) return;
    void* bufs[] = {s->d_tags,     s->d_pts,           s->d_styles,        s->d_xforms, s->d_path_map,
                    s->d_mon,      s->d_counts,        s->d_offsets,       s->d_scan_ctl, s->d_status_tags,
                    s->d_status_counts, s->d_items,    s->d_tile_n,        s->d_ws_ctl};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete s;
}

bool similarity(const sx_affine& X) {
    bool rot = (X.a == X.d) && (X.b == -X.c);
    bool refl = (X.a == -X.d) && (X.b == X.c);
    double det = (double)X.a * X.d - (double)X.b * X.c;
    bool fin = std::isfinite(X.a) && std::isfinite(X.b) && std::isfinite(X.c) && std::isfinite(X.d) &&
               std::isfinite(X.e) && std::isfinite(X.f);
    return fin && (rot || refl) && det != 0.0;
}

sx::SceneView view(const sx_scene* s) {
    sx::SceneView v;
    v.tags = s->d_tags;
    v.pts = s->d_pts;
    v.styles = s->d_styles;
    v.xforms = s->d_xforms;
    v.path_map = s->d_path_map;
    v.mon = s->d_mon;
    v.n_tags = s->n_tags;
    v.n_pts = s->n_pts;
    v.n_styles = s->n_styles;
    v.n_xforms = s->n_xforms;
    v.n_paths = s->n_paths;
    return v;
}

sx::ItemWs workspace(const sx_scene* s) {
    sx::ItemWs w;
    w.items = s->d_items;
    w.tile_n = s->d_tile_n;
    w.ctl = s->d_ws_ctl;
    w.region_cap = s->region_cap;
    w.ovf_base = (uint64_t)sx::piece_tiles(s->n_tags) * s->region_cap;
    w.ovf_cap = s->ovf_cap;
    return w;
}

// (Re)allocate the item workspace: region_per_tag slots per tag in each
// piece tile's region plus ovf shared slots.  The caller has synchronised.
hipError_t size_workspace(sx_scene* s, uint32_t region_per_tag, uint64_t ovf) {
    if (s->d_items) (void)hipFree(s->d_items);
    s->d_items = nullptr;
    s->region_cap = region_per_tag * sx::tag_block();
    s->ovf_cap = ovf;
    const uint64_t slots = (uint64_t)sx::piece_tiles(s->n_tags) * s->region_cap + ovf;
    return dalloc(&s->d_items, slots * sizeof(sx::Item));
}

bool make_cfg(float tol, int mode, sx::Cfg& cfg) {
    if (!(tol > 0.0f) || !std::isfinite(tol)) return false;
    if (mode != SX_OUT_LINES && mode != SX_OUT_ARCS) return false;
    double tf = sx::kFlatFrac * (double)tol;
    cfg.tau_fit = sx::kFitFrac * (double)tol;
    cfg.tau_flat = tf;
    cfg.inv_sqrt8tf = std::sqrt(1.0 / (8.0 * tf));
    cfg.cbrt_inv120tf = std::cbrt(1.0 / (120.0 * tf));
    cfg.arcs = mode == SX_OUT_ARCS;
    cfg.paper_fit = 0;
    cfg.K = 16;
    return true;
}

// tag scan + pieces + count scan
int run_counts(sx_ctx* ctx, const sx_scene* s, const sx::Cfg& cfg, hipStream_t st) {
    hipError_t e;
    char* ctl = (char*)s->d_scan_ctl;
    if ((e = sx::launch_scan_tags(s->d_tags, s->n_tags, s->d_mon, ctl, s->d_status_tags, s->d_ws_ctl, st)) !=
        hipSuccess)
        return hip_fail(ctx, e, "scan_tags launch");
    if ((e = sx::launch_pieces(view(s), cfg, workspace(s), s->d_counts, st)) != hipSuccess)
        return hip_fail(ctx, e, "pieces launch");
    if ((e = sx::launch_scan_counts(s->d_counts, s->n_tags, s->d_offsets, ctl + sx::scan_ctl_bytes(),
                                    s->d_status_counts, st)) != hipSuccess)
        return hip_fail(ctx, e, "scan_counts launch");
    return SX_OK;
}

// the whole pipeline; dst (device) receives {records, items needed or 0}
int run_all(sx_ctx* ctx, const sx_scene* s, const sx::Cfg& cfg, void* out, uint64_t cap_records, uint64_t* dst,
            hipStream_t st) {
    int r = run_counts(ctx, s, cfg, st);
    if (r != SX_OK) return r;
    hipError_t e = sx::launch_records(view(s), workspace(s), cfg.arcs, s->d_offsets, out, cap_records, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "records launch");
    e = sx::launch_finish(s->d_offsets, s->n_tags, workspace(s), dst, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "finish launch");
    return SX_OK;
}

}  // namespace

extern "C" {

const char* sx_version(void) { return "strokex 0.1 (gfx950)"; }

int sx_ctx_create(int device, sx_ctx** out) {
    if (!out) return SX_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SX_EDEVICE;
    sx_ctx* c = new (std::nothrow) sx_ctx();
    if (!c) return SX_ENOMEM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete c; return SX_EDEVICE; }
    if (hipHostMalloc((void**)&c->pinned_total, 2 * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return SX_ENOMEM;
    }
    *out = c;
    return SX_OK;
}

int sx_ctx_destroy(sx_ctx* ctx) {
    if (!ctx) return SX_OK;
    if (ctx->pinned_total) (void)hipHostFree(ctx->pinned_total);
    delete ctx;
    return SX_OK;
}

const char* sx_last_error(const sx_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sx_scene_encode(sx_ctx* ctx, const sx_paths* paths, const sx_style* styles, uint32_t n_styles,
                    const sx_affine* xforms, uint32_t n_xforms, void* stream, sx_scene** out) {
    if (!ctx || !out) return SX_EINVAL;
    *out = nullptr;
    if (!paths || (paths->n_paths && (!paths->verbs || !paths->verb_off || !paths->pts || !paths->pt_off ||
                                      !paths->style_ix || !paths->xform_ix)))
        return fail(ctx, SX_EINVAL, "null path arrays");
    if ((n_styles && !styles) || (n_xforms && !xforms)) return fail(ctx, SX_EINVAL, "null style/transform table");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SX_EDEVICE, "hipSetDevice");
    sx::HostEncoding enc;
    std::string err;
    if (!sx::encode_paths(*paths, n_styles, n_xforms, enc, err)) return fail(ctx, SX_EINVAL, err);
    // validate the styles and transforms that are actually used
    std::vector<sx::StyleD> sd(enc.style_stream.size());
    for (size_t i = 0; i < enc.style_stream.size(); i++) {
        const sx_style& st = styles[enc.style_stream[i]];
        if (!(st.half_width >= 0.0f) || !std::isfinite(st.half_width)) return fail(ctx, SX_EINVAL, "half_width < 0");
        if (!(st.miter_limit >= 1.0f) || !std::isfinite(st.miter_limit)) return fail(ctx, SX_EINVAL, "miter_limit < 1");
        if (st.join > 2 || st.start_cap > 2 || st.end_cap > 2) return fail(ctx, SX_EINVAL, "bad join/cap");
        if (st.flags != 0) return fail(ctx, SX_EINVAL, "style flags are reserved");
        sd[i] = sx::StyleD{st.half_width, st.miter_limit,
                           (uint32_t)st.join | ((uint32_t)st.start_cap << 8) | ((uint32_t)st.end_cap << 16)};
    }
    std::vector<float> xd(6 * enc.xform_stream.size());
    for (size_t i = 0; i < enc.xform_stream.size(); i++) {
        const sx_affine& X = xforms[enc.xform_stream[i]];
        if (!similarity(X)) return fail(ctx, SX_EINVAL, "stroke transforms must be similarities");
        const float v[6] = {X.a, X.b, X.c, X.d, X.e, X.f};
        memcpy(&xd[6 * i], v, sizeof(v));
    }
    sx_scene* s = new (std::nothrow) sx_scene();
    if (!s) return fail(ctx, SX_ENOMEM, "scene alloc");
    s->ctx = ctx;
    s->n_tags = (uint32_t)enc.tags.size();
    s->n_pts = (uint32_t)(enc.data.size() / 2);
    s->n_paths = (uint32_t)enc.path_map.size();
    s->n_styles = (uint32_t)sd.size();
    s->n_xforms = (uint32_t)enc.xform_stream.size();
    hipStream_t st = (hipStream_t)stream;
    const size_t ntag_pad = ((size_t)s->n_tags + 16 + 15) & ~(size_t)15;
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    A(dalloc(&s->d_tags, ntag_pad));
    A(dalloc(&s->d_pts, (size_t)s->n_pts * sizeof(float2)));
    A(dalloc(&s->d_styles, sd.size() * sizeof(sx::StyleD)));
    A(dalloc(&s->d_xforms, xd.size() * sizeof(float)));
    A(dalloc(&s->d_path_map, enc.path_map.size() * sizeof(uint32_t)));
    A(dalloc(&s->d_mon, 4 * (size_t)s->n_tags * sizeof(uint32_t)));
    A(dalloc(&s->d_counts, ((size_t)s->n_tags + 16) * sizeof(uint32_t)));
    A(dalloc(&s->d_offsets, ((size_t)s->n_tags + 1) * sizeof(uint64_t)));
    A(dalloc(&s->d_scan_ctl, 2 * sx::scan_ctl_bytes()));
    A(dalloc(&s->d_status_tags, sx::scan_status_bytes(s->n_tags)));
    A(dalloc(&s->d_status_counts, sx::scan_status_bytes(s->n_tags)));
    A(dalloc(&s->d_tile_n, (size_t)sx::piece_tiles(s->n_tags) * sizeof(uint32_t)));
    A(dalloc(&s->d_ws_ctl, sizeof(sx::WsCtl)));
    A(size_workspace(s, kRegionPerTag, std::max<uint64_t>(s->n_tags, kMinOverflow)));
    if (e != hipSuccess) {
        free_scene(s);
        return hip_fail(ctx, e, "scene allocation");
    }
    A(hipMemsetAsync(s->d_tags, 0, ntag_pad, st));
    A(hipMemsetAsync(s->d_scan_ctl, 0, 2 * sx::scan_ctl_bytes(), st));
    A(hipMemsetAsync(s->d_status_tags, 0, sx::scan_status_bytes(s->n_tags), st));
    A(hipMemsetAsync(s->d_status_counts, 0, sx::scan_status_bytes(s->n_tags), st));
    A(hipMemsetAsync(s->d_ws_ctl, 0, sizeof(sx::WsCtl), st));
    if (s->n_tags) A(hipMemcpyAsync(s->d_tags, enc.tags.data(), s->n_tags, hipMemcpyHostToDevice, st));
    if (s->n_pts)
        A(hipMemcpyAsync(s->d_pts, enc.data.data(), enc.data.size() * sizeof(float), hipMemcpyHostToDevice, st));
    if (!sd.empty()) A(hipMemcpyAsync(s->d_styles, sd.data(), sd.size() * sizeof(sx::StyleD), hipMemcpyHostToDevice, st));
    if (!xd.empty()) A(hipMemcpyAsync(s->d_xforms, xd.data(), xd.size() * sizeof(float), hipMemcpyHostToDevice, st));
    if (!enc.path_map.empty())
        A(hipMemcpyAsync(s->d_path_map, enc.path_map.data(), enc.path_map.size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice, st));
    // host vectors die with this call: finish the uploads before returning
    A(hipStreamSynchronize(st));
    if (e != hipSuccess) {
        free_scene(s);
        return hip_fail(ctx, e, "scene upload");
    }
    s->last_stream = st;
    *out = s;
    return SX_OK;
}

int sx_scene_release(sx_ctx* ctx, sx_scene* scene) {
    if (!scene) return SX_OK;
    if (ctx && scene->ctx != ctx) return fail(ctx, SX_EINVAL, "scene belongs to another context");
    (void)hipStreamSynchronize(scene->last_stream);
    free_scene(scene);
    return SX_OK;
}

int sx_scene_info(const sx_scene* s, uint32_t* n_tags, uint32_t* n_pts, uint32_t* n_paths, uint32_t* n_styles,
                  uint32_t* n_xforms) {
    if (!s) return SX_EINVAL;
    if (n_tags) *n_tags = s->n_tags;
    if (n_pts) *n_pts = s->n_pts;
    if (n_paths) *n_paths = s->n_paths;
    if (n_styles) *n_styles = s->n_styles;
    if (n_xforms) *n_xforms = s->n_xforms;
    return SX_OK;
}

int sx_scene_download(const sx_scene* s, uint8_t* tags, float* data, uint32_t* path_map) {
    if (!s) return SX_EINVAL;
    hipError_t e = hipSuccess;
    if (tags && s->n_tags) e = hipMemcpy(tags, s->d_tags, s->n_tags, hipMemcpyDeviceToHost);
    if (e == hipSuccess && data && s->n_pts)
        e = hipMemcpy(data, s->d_pts, (size_t)s->n_pts * sizeof(float2), hipMemcpyDeviceToHost);
    if (e == hipSuccess && path_map && s->n_paths)
        e = hipMemcpy(path_map, s->d_path_map, (size_t)s->n_paths * sizeof(uint32_t), hipMemcpyDeviceToHost);
    return e == hipSuccess ? SX_OK : SX_EDEVICE;
}

int sx_expand_async(sx_ctx* ctx, const sx_scene* scene, float tolerance, int output_mode, void* out_dev,
                    uint64_t out_capacity_bytes, uint64_t* out_count_dev, void* stream) {
    if (!ctx || !scene) return SX_EINVAL;
    sx::Cfg cfg;
    if (!make_cfg(tolerance, output_mode, cfg)) return fail(ctx, SX_EINVAL, "bad tolerance or output mode");
    if (!out_count_dev) return fail(ctx, SX_EINVAL, "null count pointer");
    if (out_capacity_bytes && !out_dev) return fail(ctx, SX_EINVAL, "null output buffer");
    hipStream_t st = (hipStream_t)stream;
    const_cast<sx_scene*>(scene)->last_stream = st;
    cfg.K = scene->chunk_k;
    const uint64_t rec = output_mode == SX_OUT_ARCS ? sizeof(sx_arc) : sizeof(sx_line);
    if (scene->n_tags == 0) {
        hipError_t e = hipMemsetAsync(out_count_dev, 0, 2 * sizeof(uint64_t), st);
        return e == hipSuccess ? SX_OK : hip_fail(ctx, e, "memset");
    }
    return run_all(ctx, scene, cfg, out_dev, out_capacity_bytes / rec, out_count_dev, st);
}

int sx_expand(sx_ctx* ctx, const sx_scene* scene, float tolerance, int output_mode, void* out_dev,
              uint64_t out_capacity_bytes, uint64_t* out_count, void* stream) {
    if (!ctx || !scene || !out_count) return SX_EINVAL;
    sx::Cfg cfg;
    if (!make_cfg(tolerance, output_mode, cfg)) return fail(ctx, SX_EINVAL, "bad tolerance or output mode");
    if (out_capacity_bytes && !out_dev) return fail(ctx, SX_EINVAL, "null output buffer");
    hipStream_t st = (hipStream_t)stream;
    sx_scene* s = const_cast<sx_scene*>(scene);
    s->last_stream = st;
    cfg.K = s->chunk_k;
    const uint64_t rec = output_mode == SX_OUT_ARCS ? sizeof(sx_arc) : sizeof(sx_line);
    *out_count = 0;
    if (s->n_tags == 0) return SX_OK;
    // the second attempt has a workspace sized from the first one's request
    // and cannot overflow (the item count is a deterministic function of the
    // scene, tolerance and mode)
    for (int attempt = 0; attempt < 2; attempt++) {
        uint64_t* dev2 = (uint64_t*)s->d_ws_ctl->result;
        int r = run_all(ctx, s, cfg, out_dev, out_capacity_bytes / rec, dev2, st);
        if (r != SX_OK) return r;
        hipError_t e = hipMemcpyAsync(ctx->pinned_total, dev2, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(ctx, e, "count readback");
        const uint64_t need = ctx->pinned_total[1];
        *out_count = ctx->pinned_total[0];
        if (need == 0) break;
        if (attempt == 1) return fail(ctx, SX_EDEVICE, "item workspace overflow after resizing");
        const uint64_t per_tag = (need * 5 / 4 + s->n_tags - 1) / s->n_tags;
        const uint32_t region = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(per_tag, kRegionPerTag), 256);
        e = size_workspace(s, region, need);
        if (e != hipSuccess) return hip_fail(ctx, e, "item workspace allocation");
    }
    if (*out_count > out_capacity_bytes / rec) return fail(ctx, SX_ETOOSMALL, "output buffer too small");
    return SX_OK;
}

int sx_run_phase(sx_ctx* ctx, const sx_scene* s, int phase, float tolerance, int output_mode, void* out_dev,
                 uint64_t out_capacity_bytes, void* stream) {
    if (!ctx || !s) return SX_EINVAL;
    sx::Cfg cfg;
    if (!make_cfg(tolerance, output_mode, cfg)) return fail(ctx, SX_EINVAL, "bad tolerance or output mode");
    if (s->n_tags == 0) return SX_OK;
    cfg.K = s->chunk_k;
    hipStream_t st = (hipStream_t)stream;
    const_cast<sx_scene*>(s)->last_stream = st;
    char* ctl = (char*)s->d_scan_ctl;
    const uint64_t rec = output_mode == SX_OUT_ARCS ? sizeof(sx_arc) : sizeof(sx_line);
    hipError_t e;
    switch (phase) {
        case SX_PHASE_SCAN_TAGS:
            e = sx::launch_scan_tags(s->d_tags, s->n_tags, s->d_mon, ctl, s->d_status_tags, s->d_ws_ctl, st);
            break;
        case SX_PHASE_PIECES:
            e = sx::launch_pieces(view(s), cfg, workspace(s), s->d_counts, st);
            break;
        case SX_PHASE_SCAN_COUNTS:
            e = sx::launch_scan_counts(s->d_counts, s->n_tags, s->d_offsets, ctl + sx::scan_ctl_bytes(),
                                       s->d_status_counts, st);
            break;
        case SX_PHASE_RECORDS:
            if (out_capacity_bytes && !out_dev) return fail(ctx, SX_EINVAL, "null output buffer");
            e = sx::launch_records(view(s), workspace(s), cfg.arcs, s->d_offsets, out_dev, out_capacity_bytes / rec,
                                   st);
            break;
        default:
            return fail(ctx, SX_EINVAL, "bad phase");
    }
    return e == hipSuccess ? SX_OK : hip_fail(ctx, e, "phase launch");
}

int sx_debug_monoids(sx_ctx* ctx, const sx_scene* s, uint32_t* out4xn_dev, void* stream) {
    if (!ctx || !s || (!out4xn_dev && s->n_tags)) return SX_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    char* ctl = (char*)s->d_scan_ctl;
    hipError_t e = sx::launch_scan_tags(s->d_tags, s->n_tags, s->d_mon, ctl, s->d_status_tags, nullptr, st);
    if (e == hipSuccess && s->n_tags)
        e = hipMemcpyAsync(out4xn_dev, s->d_mon, 4 * (size_t)s->n_tags * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? SX_OK : hip_fail(ctx, e, "monoids");
}

int sx_debug_counts(sx_ctx* ctx, const sx_scene* s, float tolerance, int output_mode, uint32_t* counts_dev,
                    void* stream) {
    if (!ctx || !s || (!counts_dev && s->n_tags)) return SX_EINVAL;
    sx::Cfg cfg;
    if (!make_cfg(tolerance, output_mode, cfg)) return fail(ctx, SX_EINVAL, "bad tolerance or output mode");
    if (s->n_tags == 0) return SX_OK;
    cfg.K = s->chunk_k;
    hipStream_t st = (hipStream_t)stream;
    int r = run_counts(ctx, s, cfg, st);
    if (r != SX_OK) return r;
    hipError_t e = hipMemcpyAsync(counts_dev, s->d_counts, (size_t)s->n_tags * sizeof(uint32_t),
                                  hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? SX_OK : hip_fail(ctx, e, "counts copy");
}

int sx_debug_offsets(sx_ctx* ctx, const sx_scene* s, float tolerance, int output_mode, uint64_t* offsets_dev,
                     void* stream) {
    if (!ctx || !s || !offsets_dev) return SX_EINVAL;
    sx::Cfg cfg;
    if (!make_cfg(tolerance, output_mode, cfg)) return fail(ctx, SX_EINVAL, "bad tolerance or output mode");
    hipStream_t st = (hipStream_t)stream;
    if (s->n_tags == 0) {
        hipError_t e = hipMemsetAsync(offsets_dev, 0, sizeof(uint64_t), st);
        return e == hipSuccess ? SX_OK : hip_fail(ctx, e, "memset");
    }
    cfg.K = s->chunk_k;
    int r = run_counts(ctx, s, cfg, st);
    if (r != SX_OK) return r;
    hipError_t e = hipMemcpyAsync(offsets_dev, s->d_offsets, ((size_t)s->n_tags + 1) * sizeof(uint64_t),
                                  hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? SX_OK : hip_fail(ctx, e, "offsets copy");
}

int sx_scan_u32(sx_ctx* ctx, const uint32_t* in_dev, uint64_t* out_dev, uint32_t n, void* stream) {
    if (!ctx || !out_dev || (n && !in_dev)) return SX_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        hipError_t e = hipMemsetAsync(out_dev, 0, sizeof(uint64_t), st);
        return e == hipSuccess ? SX_OK : hip_fail(ctx, e, "memset");
    }
    void *ctl = nullptr, *status = nullptr;
    hipError_t e = hipMalloc(&ctl, sx::scan_ctl_bytes());
    if (e == hipSuccess) e = hipMalloc(&status, sx::scan_status_bytes(n));
    if (e == hipSuccess) e = hipMemsetAsync(ctl, 0, sx::scan_ctl_bytes(), st);
    if (e == hipSuccess) e = hipMemsetAsync(status, 0, sx::scan_status_bytes(n), st);
    if (e == hipSuccess) e = sx::launch_scan_counts(in_dev, n, out_dev, ctl, status, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (ctl) (void)hipFree(ctl);
    if (status) (void)hipFree(status);
    return e == hipSuccess ? SX_OK : hip_fail(ctx, e, "scan_u32");
}

}  // extern "C"
