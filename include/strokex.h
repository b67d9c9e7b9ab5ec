/*
 * strokex -- GPU stroke expansion for AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library that turns stroked vector paths (lines, quadratic and
 * cubic Beziers with SVG joins and caps) into strongly correct outlines made
 * of line or circular-arc segments, following Levien & Uguray, "GPU-friendly
 * Stroke Expansion" (arXiv:2405.00127):
 *   - path encoding: tag stream + overlapping point stream, one stroke cap
 *     marker per subpath (Section 8.2, Table 1);
 *   - tag-monoid prefix scan giving each segment its path, style, transform
 *     and point offset (Section 8.2);
 *   - per segment, cubic -> Euler spiral subdivision driven by the error
 *     estimate of Section 7.1 (Algorithm 2), parallel curves flattened to lines
 *     with the density integral of Section 4 or to arcs with the metric of
 *     Section 5, evolutes for strong correctness (Section 6);
 *   - joins and caps from each segment's neighbour (Algorithm 1).
 *
 * All pointers are plain host or device pointers as stated per argument; no
 * framework types cross this boundary.  Calls are ordered on the given HIP
 * stream (hipStream_t passed as void*; NULL = the null stream).  A context is
 * not thread-safe: use one per host thread.
 *
 * Every entry point returns an sx_status.  On failure sx_last_error(ctx)
 * describes it; the context stays usable.
 */
#ifndef STROKEX_H
#define STROKEX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SX_OK = 0,
    SX_EINVAL = -1,    /* invalid argument or input geometry */
    SX_ENOMEM = -2,    /* device or host allocation failed */
    SX_EDEVICE = -3,   /* a HIP call failed */
    SX_ETOOSMALL = -4, /* output buffer too small; required count reported */
    SX_EBUSY = -5
} sx_status;

/* Path verbs (SVG moveto / lineto / quadto / curveto / closepath, Section 8.1). */
enum { SX_MOVE = 0, SX_LINE = 1, SX_QUAD = 2, SX_CUBIC = 3, SX_CLOSE = 4 };
/* Join and cap styles (SVG, criteria list of Section 8). */
enum { SX_JOIN_BEVEL = 0, SX_JOIN_MITER = 1, SX_JOIN_ROUND = 2 };
enum { SX_CAP_BUTT = 0, SX_CAP_SQUARE = 1, SX_CAP_ROUND = 2 };
/* Output primitive (Section 8.1: line soup, or arcs storing curvature). */
enum { SX_OUT_LINES = 0, SX_OUT_ARCS = 1 };

/* Style flags.  SX_STYLE_FILL: the path is filled, not stroked: it is
 * flattened at offset 0 (the h = 0 regime of Section 4), one output run per
 * Euler spiral piece along the path itself, every subpath closed by a line
 * back to its start, no joins or caps; half_width, miter_limit, join and
 * caps are ignored. */
enum { SX_STYLE_FILL = 1 };

/* Stroke style, one per path (Section 8.2: style stream).  half_width >= 0
 * in the path's local units (scaled by sqrt|det| of the transform);
 * miter_limit >= 1 (SVG ratio of miter length to stroke width). 12 bytes. */
typedef struct {
    float half_width;
    float miter_limit;
    uint8_t join, start_cap, end_cap, flags; /* flags: 0 (stroke) or SX_STYLE_FILL; other bits reserved */
} sx_style;

/* Affine transform, one per path (Section 8.2: transform stream):
 * x' = a x + c y + e,  y' = b x + d y + f.  Strokes need a similarity
 * (rotation or reflection with uniform scale): a == d && b == -c, or
 * a == -d && b == c, exactly. */
typedef struct {
    float a, b, c, d, e, f;
} sx_affine;

/* Input paths, all host memory, owned by the caller and read only during
 * sx_scene_encode.  Path k owns verbs[verb_off[k] .. verb_off[k+1]) and points
 * pts[2*pt_off[k] .. 2*pt_off[k+1]) (x, y pairs); every path starts with
 * SX_MOVE.  MOVE / LINE take 1 point, QUAD 2, CUBIC 3, CLOSE none. */
typedef struct {
    const uint8_t *verbs;
    const uint32_t *verb_off; /* n_paths + 1 */
    const float *pts;
    const uint32_t *pt_off;   /* n_paths + 1 */
    const uint32_t *style_ix; /* n_paths, index into the style table */
    const uint32_t *xform_ix; /* n_paths, index into the transform table */
    uint32_t n_paths;
} sx_paths;

/* Output records (Section 8.1).  path_ix is the input path index.
 * Arcs: signed curvature of the circular arc from (x0,y0) to (x1,y1),
 * positive when it turns counter-clockwise (y up); 0 for a straight line. */
typedef struct {
    float x0, y0, x1, y1;
    uint32_t path_ix;
} sx_line; /* 20 bytes */

typedef struct {
    float x0, y0, x1, y1, curvature;
    uint32_t path_ix;
} sx_arc; /* 24 bytes */

typedef struct sx_ctx sx_ctx;
typedef struct sx_scene sx_scene;

/* Context configuration, fixed for the context's life (NULL = all fields 0,
 * the defaults).
 *   fit_mode  the error the cubic -> Euler spiral bisection compares with
 *             its share of the tolerance (Algorithm 2, Section 7.1):
 *             SX_FIT_OFFSET (default) est x (chord + 9 |h|) x 1.6, where est
 *             is the chord-normalised estimate of Section 7.1 and h the
 *             half-width, so that the parallel curves stay within tolerance;
 *             SX_FIT_PAPER est x chord, the positional estimate alone (it
 *             lets wide strokes leave the tolerance; kept for comparison).
 *   density   how offset lines are counted and placed (Section 4.2):
 *             SX_DENSITY_APPROX (default) with the piecewise approximation
 *             f_approx of the subdivision density integral and its closed
 *             inverse; SX_DENSITY_NEWTON with the exact integral f, points
 *             placed by the approximate inverse refined by two Newton steps
 *             on f (the higher-quality option the section describes).
 *   constants_version  0 or SX_CONSTANTS_VERSION: the version of the
 *             printed constants (Section 4.2 c1..c3, Section 7.1
 *             coefficients, Appendix A polynomials) the caller expects.
 *   reserved  0.
 * The outline depends on fit_mode and density; sx_set_tuning never changes
 * it. */
enum { SX_FIT_OFFSET = 0, SX_FIT_PAPER = 1 };
enum { SX_DENSITY_APPROX = 0, SX_DENSITY_NEWTON = 1 };
#define SX_CONSTANTS_VERSION 1u
typedef struct {
    uint32_t fit_mode;
    uint32_t density;
    uint32_t constants_version;
    uint32_t reserved;
} sx_config;

/* Create a context on HIP device `device` with configuration *cfg (NULL:
 * defaults).  *out receives the handle.  Errors: SX_EINVAL (null out, a
 * field out of range, an unknown constants version, reserved != 0),
 * SX_EDEVICE (no such device), SX_ENOMEM. */
int sx_ctx_create(int device, const sx_config *cfg, sx_ctx **out);
/* The configuration the context was created with. */
int sx_get_config(const sx_ctx *ctx, sx_config *cfg);
/* Destroy a context and every scene it still owns.  NULL is a no-op. */
int sx_ctx_destroy(sx_ctx *ctx);
/* Text of the last error on this context (never NULL; "" when none). */
const char *sx_last_error(const sx_ctx *ctx);
/* Library version string. */
const char *sx_version(void);

/* Encode paths into a device-resident scene (Section 8.2): tags, the
 * overlapping point stream, style / transform streams and the encoded-path to
 * input-path map; closing lines are inserted for closed subpaths whose end
 * differs from their start (every subpath of a fill is closed), one stroke
 * cap marker is appended per subpath, zero-length segments and empty
 * subpaths are dropped.  The upload is ordered on `stream`; the host inputs
 * may be reused when this returns.
 * Errors: SX_EINVAL (path not starting with MOVE, unknown verb, point count
 * mismatch, non-finite coordinate, style or transform index out of range,
 * reserved style flags, for strokes half_width < 0, miter_limit < 1, bad
 * join or cap, or a transform that is not a similarity; for fills a
 * transform that is not an invertible finite affine map),
 * SX_ENOMEM, SX_EDEVICE.  The scene is owned by ctx. */
int sx_scene_encode(sx_ctx *ctx, const sx_paths *paths, const sx_style *styles, uint32_t n_styles,
                    const sx_affine *xforms, uint32_t n_xforms, void *stream, sx_scene **out);
/* Dash pattern of a stroke style (SVG stroke-dasharray / stroke-dashoffset,
 * in the path's own units): array[0 .. count) alternate dash and gap
 * lengths (an odd count repeats once), offset shifts the pattern's start.
 * count 0, or a pattern of total length 0, leaves the stroke solid. */
typedef struct {
    const float *array;
    uint32_t count;  /* <= 32 */
    float offset;
} sx_dash;

/* Encode paths with dash patterns (dashes[k] for styles[k]; fills are never
 * dashed): as sx_scene_encode, then the GPU cuts every dashed subpath into
 * dashes, each an open subpath stroked with the style's joins and caps
 * (the dash patterns of Sections 1 and 9.3, done as prefix sums of segment
 * arc lengths).  The pattern restarts at every subpath; a closed subpath is
 * dashed along its closing line and no dash continues across its start
 * point; zero-length dashes draw nothing.  Arc length: 16 parameter panels
 * of 8-node Gauss-Legendre of |B'(t)| per segment, on a grid of 2^-24
 * units; a dash ends inside a segment at the parameter where that integral
 * reaches it, and its part of the segment is the segment restricted there
 * (control points rounded to FP32); a part whose rounded control points all
 * coincide is left out, like a zero-length input segment, and a dash left
 * without parts draws nothing.  Every path of the result opens and
 * ends with an empty closed subpath (they draw nothing).  The returned
 * scene expands like any other; sx_scene_dash_ms gives the device time of
 * the dashing passes.  Synchronous.  Errors: those of sx_scene_encode, and
 * SX_EINVAL for a null table, count > 32, a negative or non-finite value, a
 * non-finite offset, or a pattern whose total length is positive but below
 * 2^-10 units. */
int sx_scene_encode_dashed(sx_ctx *ctx, const sx_paths *paths, const sx_style *styles, const sx_dash *dashes,
                           uint32_t n_styles, const sx_affine *xforms, uint32_t n_xforms, void *stream,
                           sx_scene **out);
/* Device milliseconds of the dashing passes of a dashed scene (0 otherwise). */
int sx_scene_dash_ms(const sx_scene *scene, float *ms);

/* Release a scene (waits for work queued on the scene's last stream). */
int sx_scene_release(sx_ctx *ctx, sx_scene *scene);
/* Sizes of an encoded scene (any pointer may be NULL). */
int sx_scene_info(const sx_scene *scene, uint32_t *n_tags, uint32_t *n_pts, uint32_t *n_paths,
                  uint32_t *n_styles, uint32_t *n_xforms);
/* Copy the encoded streams back to host memory (for verification):
 * tags n_tags bytes, data 2*n_pts floats, path_map n_paths u32.  NULL skips.
 * Synchronous. */
int sx_scene_download(const sx_scene *scene, uint8_t *tags, float *data, uint32_t *path_map);

/* Expand a scene: tag-monoid scan, per-segment decisions writing emission
 * items and per-tag record counts, exclusive scan of the counts (output
 * offsets), records written at their offsets in canonical order (by tag;
 * within a tag: Euler spiral pieces in parameter order, side A (right,
 * p + wN) then side B, then the join or cap; a fill's piece has one run along
 * the path and its tags no join or cap).
 *   tolerance  > 0, in output units (pixels), Frechet-style bound;
 *   output_mode SX_OUT_LINES (sx_line records) or SX_OUT_ARCS (sx_arc);
 *   out_dev    device memory, out_capacity_bytes bytes, caller-owned;
 *   out_count  host pointer, receives the number of records.
 * If the outline needs more than out_capacity_bytes, nothing is written,
 * *out_count holds the required record count and SX_ETOOSMALL is returned
 * (retry with a larger buffer).  The scene's item workspace (device memory
 * owned by the scene) grows here when a scene needs more items than it
 * holds.  Blocks the host until the count is known.
 * Errors: SX_EINVAL (tolerance not finite and > 0, bad mode), SX_ENOMEM,
 * SX_EDEVICE. */
int sx_expand(sx_ctx *ctx, const sx_scene *scene, float tolerance, int output_mode, void *out_dev,
              uint64_t out_capacity_bytes, uint64_t *out_count, void *stream);

/* Single-pass expansion, the paper's own organisation (Section 8.1), kept as
 * an ablation of the count / scan / write pipeline: after the tag-monoid
 * scan, one thread per tag runs its bisection, its pieces' parallel curves
 * and its join or cap, reserving each range's (or join's) records with an
 * atomic add on one counter.  The records are the same as sx_expand's but in
 * no defined order across ranges (a line soup; within a range they keep
 * their order).  out_dev: device memory of out_capacity_bytes, caller-owned;
 * *out_count (host) receives the number of records the scene needs.  If it
 * exceeds the capacity, the records past it are dropped (those before it are
 * written, in no defined selection) and SX_ETOOSMALL is returned: size the
 * buffer with *out_count and call again.  Blocks the host until the count is
 * known.  Errors: SX_EINVAL (tolerance, mode, null pointers), SX_ETOOSMALL,
 * SX_EDEVICE.  Currently switched off: returns SX_EDEVICE without launching
 * anything for a non-empty scene (its kernel has been seen not to finish and
 * the cause is not yet known). */
int sx_expand_soup(sx_ctx *ctx, sx_scene *scene, float tolerance, int output_mode, void *out_dev,
                   uint64_t out_capacity_bytes, uint64_t *out_count, void *stream);

/* Host-side estimate of the records a scene needs, for sizing the
 * single-pass output before any GPU work (Section 8.1 sizes its buffer with
 * Wang's formula): per curve, Wang's count sqrt(d (d - 1) M / (8 t)) at the
 * flattening tolerance t (M the largest second difference of the world
 * control polygon), times sqrt(1 + w d (d - 1) M / chord^2) per stroke side,
 * plus evolute room, plus a bound per join or cap.  A heuristic, not a bound
 * (parallel curves near cusps can need more): sx_expand_soup reports the
 * exact need when it is short.  Scenes from sx_scene_encode only (0 for a
 * batch arena).  Errors: SX_EINVAL. */
int sx_scene_estimate(const sx_scene *scene, float tolerance, int output_mode, uint64_t *out_records);

/* Same pipeline without any host synchronisation or allocation (capturable
 * in a HIP graph).  out_count_dev: device memory, two uint64_t:
 *   [0] the record count (always written when the workspace sufficed);
 *   [1] 0 on success, else 1: the scene's slot or item workspace was too
 *       small and nothing was emitted; one sx_expand call with the same
 *       tolerance and mode resizes it.
 * When [0] exceeds the capacity nothing is emitted either; the caller
 * compares it with the capacity afterwards. */
int sx_expand_async(sx_ctx *ctx, const sx_scene *scene, float tolerance, int output_mode, void *out_dev,
                    uint64_t out_capacity_bytes, uint64_t *out_count_dev, void *stream);

/* Verification exports, running the same kernels as sx_expand:
 * monoids: 4 x n_tags uint32 in device memory (SoA: point offset, path index,
 * style index, transform index), exclusive for offset / path and inclusive-1
 * for style / transform (Section 8.2). */
int sx_debug_monoids(sx_ctx *ctx, const sx_scene *scene, uint32_t *out4xn_dev, void *stream);
/* counts: n_tags uint32 (device) = records each tag emits. */
int sx_debug_counts(sx_ctx *ctx, const sx_scene *scene, float tolerance, int output_mode,
                    uint32_t *counts_dev, void *stream);
/* offsets: n_tags + 1 uint64 (device) = exclusive scan of the counts. */
int sx_debug_offsets(sx_ctx *ctx, const sx_scene *scene, float tolerance, int output_mode,
                     uint64_t *offsets_dev, void *stream);

/* Work done by the piece phase (Algorithms 1-2) on a scene, counted by an
 * instrumented run of the same computation (synchronous; host output):
 *   stats6[0] fit trials of the cubic bisection (Algorithm 2; lines excluded)
 *   stats6[1] accepted Euler spiral pieces (lines included)
 *   stats6[2] parallel-curve ranges (Sections 4-5)
 *   stats6[3] evolute bundles (Section 6)
 *   stats6[4] joins and caps (Algorithm 1)
 *   stats6[5] line segments (straight pieces)
 * Errors: SX_EINVAL, SX_EDEVICE. */
int sx_debug_piece_stats(sx_ctx *ctx, const sx_scene *scene, float tolerance, int output_mode, uint64_t *stats6,
                         void *stream);

/* The phases of sx_expand_async, one kernel each, for per-kernel timing:
 *   SX_PHASE_SCAN_TAGS     tag-monoid scan (Section 8.2)
 *   SX_PHASE_BISECT_COUNT  Algorithm 2 per segment: slots per tag (pieces + 1)
 *   SX_PHASE_SCAN_SLOTS    exclusive scan of the slot counts (slot bases)
 *   SX_PHASE_BISECT_WRITE  Algorithm 2 again: each piece's slot at its base
 *   SX_PHASE_PIECES        per piece slot: Euler spiral, parallel curves and
 *                          counts (Sections 4-6) as emission items, and the
 *                          slot's record count
 *   SX_PHASE_TAILS         per tail slot: the join or cap (Algorithm 1)
 *   SX_PHASE_SCAN_RECORDS  exclusive scan of the record counts (offsets)
 *   SX_PHASE_RECORDS       per item, records written at their offsets
 * Run in this order on one stream they equal sx_expand_async without the
 * final count copy.  out_dev / out_capacity_bytes are used by
 * SX_PHASE_RECORDS only (nothing is written when the total exceeds the
 * capacity).  Errors: SX_EINVAL (bad phase, tolerance or mode), SX_EDEVICE. */
enum {
    SX_PHASE_SCAN_TAGS = 0,
    SX_PHASE_BISECT_COUNT = 1,
    SX_PHASE_SCAN_SLOTS = 2,
    SX_PHASE_BISECT_WRITE = 3,
    SX_PHASE_PIECES = 4,
    SX_PHASE_TAILS = 5,
    SX_PHASE_SCAN_RECORDS = 6,
    SX_PHASE_RECORDS = 7
};
int sx_run_phase(sx_ctx *ctx, const sx_scene *scene, int phase, float tolerance, int output_mode, void *out_dev,
                 uint64_t out_capacity_bytes, void *stream);

/* ---- Batches: many scenes in one pipeline launch -------------------------
 * A batch owns a device arena into which sx_batch_set concatenates the
 * streams of n already encoded scenes (tags, points, styles, transforms, path
 * maps; Section 8.2).  Every scene starts a new path, style and transform, so
 * the tag-monoid scan of the concatenation gives each segment the same path,
 * style, transform and neighbours it has in its own scene: the outline of a
 * scene is the same alone and in a batch, bit for bit, and its records keep
 * the scene's own input path indices. */
typedef struct sx_batch sx_batch;
int sx_batch_create(sx_ctx *ctx, sx_batch **out);
/* Waits for the batch's streams, then frees it and its arena. */
int sx_batch_destroy(sx_ctx *ctx, sx_batch *batch);
/* Gather scenes[0..n) (n <= 65535, all of ctx) into the arena, ordered on
 * `stream`: one descriptor upload and one gather kernel.  The arena grows
 * (synchronous allocation) when the scenes need more room than it has; it
 * never shrinks.  The scenes must stay alive until the gather has run on
 * `stream`; after that the batch does not read them.
 * Errors: SX_EINVAL (null or foreign scene, n too large, sizes over 2^32),
 * SX_ENOMEM, SX_EDEVICE. */
int sx_batch_set(sx_ctx *ctx, sx_batch *batch, const sx_scene *const *scenes, uint32_t n, void *stream);
/* Number of scenes set and the arena as a scene (owned by the batch: it may
 * be passed to sx_expand, e.g. to size the output and the item workspace,
 * but not to sx_scene_release or sx_batch_set). */
int sx_batch_info(const sx_batch *batch, uint32_t *n_scenes, sx_scene **arena);
/* Expand every scene of the batch in one pipeline (the kernels of
 * sx_expand_async over the arena, then one kernel for the per-scene
 * offsets); no host synchronisation or allocation, capturable in a HIP graph.
 *   out_dev / out_capacity_bytes  device output, records of scene s at
 *                                 [scene_offsets[s], scene_offsets[s+1]);
 *   scene_offsets_dev             device, n_scenes + 1 uint64_t;
 *   status_dev                    device, 2 uint64_t as out_count_dev of
 *                                 sx_expand_async (total records; 0 or the
 *                                 item workspace needed).
 * Nothing is emitted when the total exceeds the capacity or the workspace is
 * too small (one sx_expand on the arena resizes it).
 * Errors: SX_EINVAL (bad tolerance or mode, null pointers), SX_EDEVICE. */
int sx_batch_expand(sx_ctx *ctx, sx_batch *batch, float tolerance, int output_mode, void *out_dev,
                    uint64_t out_capacity_bytes, uint64_t *scene_offsets_dev, uint64_t *status_dev, void *stream);

/* Launch parameters of a context (used by every later call on it; the
 * outline does not depend on them):
 *   piece_waves   1..3: waves per SIMD the slot kernel's register
 *                 allocation allows (more waves hide more latency but spill);
 *   chunk_k       1..255: records per emission item chunk (work per thread
 *                 of the record kernel);
 *   bisect_range  tags per bisection wave, a multiple of 64 up to 1024
 *                 (0 = 256): longer ranges keep lanes refilled longer;
 *   bisect_waves  2, 3 or 4 (0 = 2): waves per SIMD of the bisection kernels.
 * Defaults {2, 16, 256, 2}.  Errors: SX_EINVAL (out of range). */
typedef struct {
    uint32_t piece_waves;
    uint32_t chunk_k;
    uint32_t bisect_range;
    uint32_t bisect_waves;
} sx_tuning;
int sx_set_tuning(sx_ctx *ctx, const sx_tuning *tuning);
int sx_get_tuning(const sx_ctx *ctx, sx_tuning *tuning);

/* Scan primitive on its own: exclusive prefix sum of n uint32 values into
 * n + 1 uint64 (device pointers), single-pass decoupled look-back. */
int sx_scan_u32(sx_ctx *ctx, const uint32_t *in_dev, uint64_t *out_dev, uint32_t n, void *stream);

/* The same scan for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): no
 * allocation and no host synchronisation.  The scan's control block and
 * per-tile status words live in a static device array of the library
 * (SX_SCAN_NOALLOC_BYTES bytes per GPU, held until the process ends; its
 * device address is looked up once per device when a context is created).
 * n <= SX_SCAN_NOALLOC_MAX, else SX_EINVAL and nothing is launched.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one device
 * (other streams, other contexts, other host threads) race and give wrong
 * sums; serialise them.  Ordered on `stream`; in_dev, out_dev as for
 * sx_scan_u32.  Errors: SX_EINVAL, SX_EDEVICE. */
#define SX_SCAN_NOALLOC_MAX (1u << 24)
#define SX_SCAN_NOALLOC_BYTES (256u + 262144u)
int sx_scan_u32_noalloc(sx_ctx *ctx, const uint32_t *in_dev, uint64_t *out_dev, uint32_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* STROKEX_H */
