/*
 * strokex oracle -- plain, slow FP64 CPU reference for GPU-friendly stroke
 * expansion (Levien & Uguray, "GPU-friendly Stroke Expansion",
 * arXiv:2405.00127).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the HIP library; every constant below is
 * typed in from the paper (or from a reading of it, listed in the design
 * notes) independently of the GPU source.
 *
 * Everything is computed in double precision.  FP32 inputs are widened
 * exactly.  The code follows the paper's steps in the paper's order:
 *
 *   encode            Section 8.2, Table 1 (path tags, overlapping point stream,
 *                     stroke cap marker per subpath)
 *   tag monoid        Section 8.2 (prefix sums of the per-tag increments)
 *   segment fetch     Section 8.1 (degree elevation of lines and quads)
 *   cubic -> ES       Algorithm 2, Section 7 (adaptive bisection with the
 *                     error estimate of Section 7.1, two-word stack, cusp
 *                     perturbation of Section 7.3)
 *   ES parameters     Appendix A (k1 and chord/arc-length polynomials)
 *   offset flattening Sections 4.1 / 4.2 (subdivision density integral of
 *                     the ES parallel curve and its piecewise approximation)
 *   arc output        Section 5 (cube-root arc metric with the 0.4|h s k'| term)
 *   evolutes          Section 6 (density |s|^-1/2; emitted twice with the
 *                     connecting lines, reversed parallel section)
 *   joins / caps      Algorithm 1 and the SVG styles named in Section 8
 *
 * Where the paper is silent the readings are named G1..G27 in comments.
 *
 * Pins: every function here is checked by the CPU test suite against closed
 * forms, library quadrature, brute force on tiny inputs and FP64 dense
 * sampling of the exact offset curve (see tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- tags -- */
/* Table 1 (Section 8.2): bits 0-1 coordinate count, 2 subpath end, 3 f32,
 * 4 path end, 5 transform, 6 style.  Bit 7 is unused in the paper; reading
 * G13 stores "subpath closed" there, on the stroke cap marker. */
#define OX_TAG_COUNT 0x03u
#define OX_TAG_SUBPATH_END 0x04u
#define OX_TAG_F32 0x08u
#define OX_TAG_PATH 0x10u
#define OX_TAG_XFORM 0x20u
#define OX_TAG_STYLE 0x40u
#define OX_TAG_CLOSED 0x80u

enum { OX_MOVE = 0, OX_LINE = 1, OX_QUAD = 2, OX_CUBIC = 3, OX_CLOSE = 4 };
enum { OX_JOIN_BEVEL = 0, OX_JOIN_MITER = 1, OX_JOIN_ROUND = 2 };
enum { OX_CAP_BUTT = 0, OX_CAP_SQUARE = 1, OX_CAP_ROUND = 2 };
/* style flag: the path is filled, not stroked (reading G33) */
#define OX_STYLE_FILL 0x01u
enum { OX_OUT_LINES = 0, OX_OUT_ARCS = 1 };
enum { OX_FIT_OFFSET = 0, OX_FIT_PAPER = 1 };
/* fit-mode bit: leave out the hodograph test of reading G29 (Algorithm 2 as
 * printed; kept only so the tests can show what the reading prevents) */
#define OX_FIT_NO_HODO 2
/* mode bit: count offset lines with the exact subdivision density integral f
 * and place their points by the f_approx inverse refined by two Newton steps
 * on f (the higher-quality option of Section 4.2) */
#define OX_DENSITY_NEWTON 4

/* kinds recorded per output (for the tests' geometric checks only) */
enum { OX_K_OFFSET = 0, OX_K_EVOLUTE = 1, OX_K_CONNECT = 2, OX_K_JOIN_OUTER = 3,
       OX_K_JOIN_INNER = 4, OX_K_CAP = 5 };

typedef struct {
    float half_width, miter_limit;
    uint8_t join, start_cap, end_cap, flags;
} ox_style; /* 12 bytes, same memory layout as the public style record */

/* --------------------------------------------------------- readings ------ */
/* G1: the paper gives no value for the ES fit tolerance.  The total
 * tolerance tau is split between the cubic->ES fit and the flattening of
 * the parallel curve. */
#ifndef OX_FIT_FRAC
#define OX_FIT_FRAC 0.15
#endif
#ifndef OX_FLAT_FRAC
#define OX_FLAT_FRAC 0.65
#endif
/* G2: the error estimate of Section 7.1 is positional; a parallel curve at
 * distance h also inherits the ES's tangent error times h.  err_px =
 * est * (chord + K |h|) * S. */
#ifndef OX_FIT_K
#define OX_FIT_K 9.0
#endif
#ifndef OX_FIT_S
#define OX_FIT_S 1.6
#endif
/* G10: near-zero derivative threshold (relative to the control polygon
 * length) and the parameter perturbation (Section 7.3). */
#ifndef OX_EPS_Q
#define OX_EPS_Q 1e-5
#endif
#ifndef OX_DELTA_T
#define OX_DELTA_T (1.0 / 4096.0)
#endif
/* G11: bisection depth cap. */
#ifndef OX_MAX_DEPTH
#define OX_MAX_DEPTH 16
#endif
/* G28: lower clamp for the Appendix A chord/arc ratio (only reached by
 * pieces accepted at the depth cap with near-reversed tangents). */
/* G31: nearly tangent-continuous joins */
#ifndef OX_SMOOTH_JOIN
#define OX_SMOOTH_JOIN 1e-5
#endif
#ifndef OX_C_MIN
#define OX_C_MIN 0.1
#endif
/* G33: fill flattening is the same expansion at offset 0 (Section 4, the
 * h = 0 regime): the fit error without the width term, one side (the path
 * itself, forward in u), no joins or caps, and every subpath closed by a
 * line back to its start.  Pieces accepted at the depth cap draw their
 * chord.  Without a width, any invertible affine transform is allowed. */

/* ----------------------------------------------------- result records -- */
typedef struct {
    double x0, y0, x1, y1, curv;
    uint32_t path;
    uint32_t kind;
    uint32_t tag;
} ox_out;

/* per-tag decision margins (relative distances to each threshold) */
typedef struct {
    double fit;    /* min |err/tau_fit - 1| over non-forced fit decisions */
    double count;  /* min distance of a count estimate to an integer      */
    double rho;    /* min |rho| at piece ends                              */
    double q;      /* min ||q|/(eps L) - 1| perturbation decisions         */
    double len;    /* min |hodograph turning test| / scale (reading G29)   */
    double join;   /* join decisions: |cr| distance to its thresholds (abs.) */
    uint32_t n_pieces;
    uint32_t max_depth_hits;
} ox_margin;

typedef struct {
    double t0, t1, k0, k1, chord, L, th0, th1;
    uint32_t tag;
    uint32_t forced;
} ox_piece;

typedef struct ox_enc {
    uint8_t *tags;
    float *data; /* x,y pairs */
    uint32_t *style_stream; /* index into caller's style table, per style entry */
    uint32_t *xform_stream;
    uint32_t *path_map;     /* encoded path -> input path index */
    uint32_t n_tags, n_pts, n_styles, n_xforms, n_paths;
    uint32_t cap_tags, cap_pts, cap_styles, cap_xforms, cap_paths;
    int status;
} ox_enc;

typedef struct ox_res {
    ox_out *out;
    uint64_t n_out, cap_out;
    uint32_t *counts; /* per tag */
    ox_margin *margins;
    ox_piece *pieces;
    uint64_t n_pieces, cap_pieces;
    uint32_t n_tags;
    int status;
} ox_res;

/* ----------------------------------------------------------- vectors ---- */
typedef struct { double x, y; } v2;
static v2 v2m(double x, double y) { v2 r = {x, y}; return r; }
static v2 vadd(v2 a, v2 b) { return v2m(a.x + b.x, a.y + b.y); }
static v2 vsub(v2 a, v2 b) { return v2m(a.x - b.x, a.y - b.y); }
static v2 vscale(v2 a, double s) { return v2m(a.x * s, a.y * s); }
static double vdot(v2 a, v2 b) { return a.x * b.x + a.y * b.y; }
static double vcross(v2 a, v2 b) { return a.x * b.y - a.y * b.x; }
static double vlen(v2 a) { return hypot(a.x, a.y); }
static int vzero(v2 a) { return a.x == 0.0 && a.y == 0.0; }
static int veq(v2 a, v2 b) { return a.x == b.x && a.y == b.y; }
static v2 vunit(v2 a) { double l = vlen(a); return v2m(a.x / l, a.y / l); }
/* right normal of a unit tangent: N = (T_y, -T_x), so that N' = kappa T */
static v2 vnormal(v2 t) { return v2m(t.y, -t.x); }
/* complex product / quotient (points as complex numbers) */
static v2 cmul(v2 a, v2 b) { return v2m(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
static v2 cdiv(v2 a, v2 b) {
    double d = b.x * b.x + b.y * b.y;
    return v2m((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

/* ===================================================== 1. encoding ====== */
/* Section 8.2: tag stream + overlapping point stream.  Subpath boundaries
 * move from the moveto to the end of the subpath; a closing line is
 * inserted when a closed subpath does not end at its start point; one stroke
 * cap marker (count 2, subpath end) is appended per subpath carrying the
 * start point and a second point giving the start tangent (reading G14: the
 * first control point of the first segment that differs from the start).
 * Zero-length segments (all points equal to the current point) are dropped;
 * subpaths left without segments are dropped (reading G22). */

static int enc_reserve(ox_enc *e, uint32_t ntag, uint32_t npt) {
    if (e->n_tags + ntag > e->cap_tags) {
        uint32_t c = e->cap_tags ? e->cap_tags : 64;
        while (c < e->n_tags + ntag) c *= 2;
        uint8_t *p = (uint8_t *)realloc(e->tags, c);
        if (!p) return -1;
        e->tags = p; e->cap_tags = c;
    }
    if (e->n_pts + npt > e->cap_pts) {
        uint32_t c = e->cap_pts ? e->cap_pts : 64;
        while (c < e->n_pts + npt) c *= 2;
        float *p = (float *)realloc(e->data, (size_t)c * 2 * sizeof(float));
        if (!p) return -1;
        e->data = p; e->cap_pts = c;
    }
    return 0;
}

static int enc_push_u32(uint32_t **arr, uint32_t *n, uint32_t *cap, uint32_t v) {
    if (*n + 1 > *cap) {
        uint32_t c = *cap ? *cap * 2 : 16;
        uint32_t *p = (uint32_t *)realloc(*arr, (size_t)c * sizeof(uint32_t));
        if (!p) return -1;
        *arr = p; *cap = c;
    }
    (*arr)[(*n)++] = v;
    return 0;
}

static void enc_pt(ox_enc *e, float x, float y) {
    e->data[2 * e->n_pts] = x;
    e->data[2 * e->n_pts + 1] = y;
    e->n_pts++;
}

/* closing line from the current point back to the subpath's start point
 * (none when the current point is already there) */
static int enc_closing_line(ox_enc *e, float sx, float sy, float *cx, float *cy) {
    if (*cx == sx && *cy == sy) return 0;
    if (enc_reserve(e, 1, 1)) return -2;
    e->tags[e->n_tags++] = (uint8_t)(1u | OX_TAG_F32);
    enc_pt(e, sx, sy);
    *cx = sx; *cy = sy;
    return 0;
}

/* Status codes match the public ABI's meaning: 0 ok, -1 invalid input.
 * path_fill (may be NULL: all strokes) marks the paths drawn as fills, whose
 * subpaths are all closed (reading G33). */
ox_enc *ox_encode(const uint8_t *verbs, const uint32_t *verb_off, const float *pts,
                  const uint32_t *pt_off, const uint32_t *style_ix, const uint32_t *xform_ix,
                  uint32_t n_paths, uint32_t n_styles, uint32_t n_xforms, const uint8_t *path_fill) {
    ox_enc *e = (ox_enc *)calloc(1, sizeof(ox_enc));
    if (!e) return NULL;
    int32_t prev_style = -1, prev_xf = -1;
    for (uint32_t k = 0; k < n_paths; k++) {
        if (style_ix[k] >= n_styles || xform_ix[k] >= n_xforms) { e->status = -1; return e; }
        uint32_t first_tag = e->n_tags;
        const float *P = pts + 2 * (size_t)pt_off[k];
        uint32_t np = pt_off[k + 1] - pt_off[k];
        uint32_t pi = 0;
        int in_sub = 0, sub_nseg = 0, closed = 0;
        const int fill = path_fill ? (path_fill[k] != 0) : 0;
        float sx = 0, sy = 0, cx = 0, cy = 0;      /* subpath start / current */
        float dirx = 0, diry = 0; int have_dir = 0; /* G14 tangent point */
        for (uint32_t vi = verb_off[k]; vi < verb_off[k + 1]; vi++) {
            uint8_t v = verbs[vi];
            if (v == OX_MOVE || v == OX_CLOSE) {
                if (v == OX_CLOSE) {
                    if (!in_sub) continue;
                    if (sub_nseg > 0 && enc_closing_line(e, sx, sy, &cx, &cy)) { e->status = -2; return e; }
                    closed = 1;
                } else if (fill && in_sub && sub_nseg > 0 && !closed) {
                    /* a fill's subpath ends closed */
                    if (enc_closing_line(e, sx, sy, &cx, &cy)) { e->status = -2; return e; }
                    closed = 1;
                }
                if (in_sub && sub_nseg > 0) {
                    /* stroke cap marker: count 2 + subpath end, points (start, dir) */
                    if (enc_reserve(e, 1, 2)) { e->status = -2; return e; }
                    e->tags[e->n_tags++] = (uint8_t)(2u | OX_TAG_SUBPATH_END | OX_TAG_F32 |
                                                     (closed ? OX_TAG_CLOSED : 0u));
                    if (!have_dir) { dirx = sx + 1.0f; diry = sy; }
                    enc_pt(e, sx, sy);
                    enc_pt(e, dirx, diry);
                }
                if (v == OX_MOVE) {
                    if (pi + 1 > np) { e->status = -1; return e; }
                    sx = cx = P[2 * pi]; sy = cy = P[2 * pi + 1];
                    pi += 1;
                    in_sub = 1;
                } else {
                    /* after closepath the current point is the start point and
                     * a following drawing verb opens a new subpath there */
                    cx = sx; cy = sy;
                    in_sub = 1;
                }
                sub_nseg = 0; closed = 0; have_dir = 0;
                continue;
            }
            if (v < OX_LINE || v > OX_CUBIC) { e->status = -1; return e; }
            if (!in_sub) { e->status = -1; return e; } /* path must start with moveto */
            uint32_t c = v;
            if (pi + c > np) { e->status = -1; return e; }
            int nonzero = 0;
            for (uint32_t j = 0; j < c; j++) {
                float x = P[2 * (pi + j)], y = P[2 * (pi + j) + 1];
                if (!isfinite(x) || !isfinite(y)) { e->status = -1; return e; }
                if (!(x == cx && y == cy)) nonzero = 1;
            }
            if (!nonzero) { pi += c; continue; } /* zero-length segment */
            if (enc_reserve(e, 1, c + 1)) { e->status = -2; return e; }
            if (sub_nseg == 0) enc_pt(e, cx, cy); /* subpath start point */
            if (!have_dir) {
                for (uint32_t j = 0; j < c; j++) {
                    float x = P[2 * (pi + j)], y = P[2 * (pi + j) + 1];
                    if (!(x == sx && y == sy)) { dirx = x; diry = y; have_dir = 1; break; }
                }
            }
            for (uint32_t j = 0; j < c; j++) enc_pt(e, P[2 * (pi + j)], P[2 * (pi + j) + 1]);
            e->tags[e->n_tags++] = (uint8_t)(c | OX_TAG_F32);
            cx = P[2 * (pi + c - 1)]; cy = P[2 * (pi + c - 1) + 1];
            pi += c;
            sub_nseg++;
        }
        /* a path's verbs consume exactly the points it owns */
        if (pi != np) { e->status = -1; return e; }
        if (fill && in_sub && sub_nseg > 0 && !closed) {
            if (enc_closing_line(e, sx, sy, &cx, &cy)) { e->status = -2; return e; }
            closed = 1;
        }
        if (in_sub && sub_nseg > 0) {
            if (enc_reserve(e, 1, 2)) { e->status = -2; return e; }
            e->tags[e->n_tags++] = (uint8_t)(2u | OX_TAG_SUBPATH_END | OX_TAG_F32 |
                                             (closed ? OX_TAG_CLOSED : 0u));
            if (!have_dir) { dirx = sx + 1.0f; diry = sy; }
            enc_pt(e, sx, sy);
            enc_pt(e, dirx, diry);
        }
        if (e->n_tags > first_tag) {
            e->tags[e->n_tags - 1] |= OX_TAG_PATH;
            if ((int32_t)style_ix[k] != prev_style) {
                e->tags[first_tag] |= OX_TAG_STYLE;
                if (enc_push_u32(&e->style_stream, &e->n_styles, &e->cap_styles, style_ix[k])) { e->status = -2; return e; }
                prev_style = (int32_t)style_ix[k];
            }
            if ((int32_t)xform_ix[k] != prev_xf) {
                e->tags[first_tag] |= OX_TAG_XFORM;
                if (enc_push_u32(&e->xform_stream, &e->n_xforms, &e->cap_xforms, xform_ix[k])) { e->status = -2; return e; }
                prev_xf = (int32_t)xform_ix[k];
            }
            if (enc_push_u32(&e->path_map, &e->n_paths, &e->cap_paths, k)) { e->status = -2; return e; }
        }
    }
    return e;
}

void ox_enc_free(ox_enc *e) {
    if (!e) return;
    free(e->tags); free(e->data); free(e->style_stream); free(e->xform_stream); free(e->path_map);
    free(e);
}
int ox_enc_status(const ox_enc *e) { return e->status; }
uint32_t ox_enc_ntags(const ox_enc *e) { return e->n_tags; }
uint32_t ox_enc_npts(const ox_enc *e) { return e->n_pts; }
uint32_t ox_enc_nstyles(const ox_enc *e) { return e->n_styles; }
uint32_t ox_enc_nxforms(const ox_enc *e) { return e->n_xforms; }
uint32_t ox_enc_npaths(const ox_enc *e) { return e->n_paths; }
const uint8_t *ox_enc_tags(const ox_enc *e) { return e->tags; }
const float *ox_enc_data(const ox_enc *e) { return e->data; }
const uint32_t *ox_enc_style_stream(const ox_enc *e) { return e->style_stream; }
const uint32_t *ox_enc_xform_stream(const ox_enc *e) { return e->xform_stream; }
const uint32_t *ox_enc_path_map(const ox_enc *e) { return e->path_map; }

/* ================================================== 2. tag monoid ======= */
/* Section 8.2: per-tag stream offsets are prefix sums of the tag's
 * increments.  Data offset (in points) and path index are exclusive sums;
 * style and transform indices are inclusive sums minus one (reading G15). */
void ox_monoids(const uint8_t *tags, uint32_t n, uint32_t *pathdata_off, uint32_t *path_ix,
                uint32_t *style_ix, uint32_t *xform_ix) {
    uint32_t off = 0, pth = 0, sty = 0, xf = 0;
    for (uint32_t i = 0; i < n; i++) {
        uint8_t t = tags[i];
        pathdata_off[i] = off;
        path_ix[i] = pth;
        sty += (t & OX_TAG_STYLE) ? 1u : 0u;
        xf += (t & OX_TAG_XFORM) ? 1u : 0u;
        style_ix[i] = sty - 1u;
        xform_ix[i] = xf - 1u;
        off += (t & OX_TAG_COUNT) + ((t & OX_TAG_SUBPATH_END) ? 1u : 0u);
        pth += (t & OX_TAG_PATH) ? 1u : 0u;
    }
}

/* ================================================ 3. curve math ========= */

/* Gauss-Legendre nodes on [-1,1] by Newton iteration on P_n (textbook). */
#define OX_GL_N 16
static double gl_x[OX_GL_N], gl_w[OX_GL_N];
static int gl_ready = 0;
static void gl_init(void) {
    if (gl_ready) return;
    int n = OX_GL_N;
    for (int i = 0; i < n; i++) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            double dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; k++) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        double dp = n * (x * p1 - p0) / (x * x - 1.0);
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}
void ox_gl_nodes(double *x, double *w) { gl_init(); for (int i = 0; i < OX_GL_N; i++) { x[i] = gl_x[i]; w[i] = gl_w[i]; } }

/* Normalised Euler spiral (Appendix A): unit arc length, tangent angle
 * phi(u) = k0 (u - 1/2) + k1/2 (u - 1/2)^2 for u in [0,1].
 * Z(u) = int_0^u exp(i phi(v)) dv by composite Gauss-Legendre with
 * sub-intervals of at most 0.25 rad turning bound. */
static double es_phi(double k0, double k1, double u) {
    double v = u - 0.5;
    return k0 * v + 0.5 * k1 * v * v;
}
static v2 es_integral(double k0, double k1, double u) {
    gl_init();
    double bound = (fabs(k0) + 0.5 * fabs(k1)) * fabs(u);
    int m = (int)ceil(bound / 0.25);
    if (m < 1) m = 1;
    double sx = 0.0, sy = 0.0;
    double h = u / m;
    for (int j = 0; j < m; j++) {
        double a = j * h;
        for (int i = 0; i < OX_GL_N; i++) {
            double v = a + 0.5 * h * (gl_x[i] + 1.0);
            double ph = es_phi(k0, k1, v);
            sx += gl_w[i] * 0.5 * h * cos(ph);
            sy += gl_w[i] * 0.5 * h * sin(ph);
        }
    }
    return v2m(sx, sy);
}
void ox_es_integral(double k0, double k1, double u, double *re, double *im) {
    v2 z = es_integral(k0, k1, u);
    *re = z.x; *im = z.y;
}

/* Appendix A: k1 and chord/arc-length ratio from k = th0 + th1 and
 * D = th1 - th0 (7th-order polynomials typed in from the appendix). */
double ox_es_k1(double th0, double th1) {
    double k = th0 + th1, d = th1 - th0;
    double k2 = k * k, k4 = k2 * k2, k6 = k4 * k2;
    double d2 = d * d, d3 = d2 * d, d5 = d3 * d2, d7 = d5 * d2;
    return 6.0 * d - d3 / 70.0 - d5 / 10780.0 + d7 * 2.769178184818219e-7
           - k2 * d / 10.0 + k2 * d3 / 4200.0 + k2 * d5 * 1.6959677820260655e-5
           - k4 * d / 1400.0 + k4 * d3 * 6.84915970574303e-5
           - k6 * d * 7.936475029053326e-6;
}
double ox_es_chord(double th0, double th1) {
    double k = th0 + th1, d = th1 - th0;
    double k2 = k * k, k4 = k2 * k2, k6 = k4 * k2;
    double d2 = d * d, d4 = d2 * d2, d6 = d4 * d2;
    return 1.0 - d2 / 40.0 + d4 * 0.00034226190482569864 - d6 * 1.9349474568904524e-6
           - k2 / 24.0 + k2 * d2 * 0.0024702380951963226 - k2 * d4 * 3.7297408997537985e-5
           + k4 / 1920.0 - k4 * d2 * 4.87350869747975e-5
           - k6 * 3.1001936068463107e-6;
}

/* Section 7.1: area between a chord-normalised cubic (end angles th0, th1
 * relative to the chord, arms d0, d1) and its chord, by Green's theorem. */
double ox_cubic_area(double th0, double th1, double d0, double d1) {
    return 3.0 / 20.0 * (2.0 * d0 * sin(th0) + 2.0 * d1 * sin(th1) - d0 * d1 * sin(th0 + th1));
}

/* Section 7.1: predicted (chord-normalised) distance between a cubic and
 * the Euler spiral with the same end tangents: ES-vs-its-cubic term,
 * 1.55 x area difference, and the arm-imbalance term. */
double ox_fit_estimate(double th0, double th1, double d0, double d1) {
    double s = fabs(th0 + th1), df = fabs(th0 - th1);
    double e0 = 4.6255e-6 * pow(s, 5) + 7.5e-3 * s * s * df;
    double db0 = 2.0 / (3.0 * (1.0 + cos(th0)));
    double db1 = 2.0 / (3.0 * (1.0 + cos(th1)));
    double ea = 1.55 * fabs(ox_cubic_area(th0, th1, d0, d1) - ox_cubic_area(th0, th1, db0, db1));
    double ei = (0.005 * s + 0.07 * df) * sqrt((db0 - d0) * (db0 - d0) + (db1 - d1) * (db1 - d1));
    return e0 + ea + ei;
}

/* Section 4.1: exact subdivision density integral of the ES parallel curve,
 * f(x) = int_0^x sqrt|u^2-1| du.  Reading G5: the |x|>=1 branch is
 * (x sqrt(x^2-1) - arcosh x)/2 + pi/4; odd symmetry for negative x. */
double ox_f_exact(double x) {
    double a = fabs(x), r;
    if (a <= 1.0) r = 0.5 * (a * sqrt(1.0 - a * a) + asin(a));
    else r = 0.5 * (a * sqrt(a * a - 1.0) - acosh(a)) + M_PI / 4.0;
    return x < 0 ? -r : r;
}

/* Section 4.2: piecewise approximation f_approx (given for x >= 0, odd).
 * c1, c2, c3 are the paper's printed constants.  Reading G6: the second
 * piece's (x-1)^1.5 means sign(x-1)|x-1|^1.5 on [0.8, 1). */
#define OX_C1 1.0976991822760038
#define OX_C2 0.9148117935952064
#define OX_C3 0.16145779359520596
double ox_f_approx(double x) {
    double a = fabs(x), r;
    if (a < 0.8) r = sin(OX_C1 * a) / OX_C1;
    else if (a < 1.25) {
        double e = a - 1.0;
        r = sqrt(8.0) / 3.0 * (e < 0 ? -pow(-e, 1.5) : pow(e, 1.5)) + M_PI / 4.0;
    } else if (a < 2.1) r = 0.6406 * a * a - 0.81 * a + OX_C2;
    else r = 0.5 * a * a - 0.156 * a + OX_C3;
    return x < 0 ? -r : r;
}
/* derivative of f_approx (the approximated density) */
double ox_f_approx_deriv(double x) {
    double a = fabs(x);
    if (a < 0.8) return cos(OX_C1 * a);
    if (a < 1.25) return sqrt(2.0) * sqrt(fabs(a - 1.0));
    if (a < 2.1) return 2.0 * 0.6406 * a - 0.81;
    return a - 0.156;
}
/* inverse of f_approx, branch by branch */
double ox_f_approx_inv(double y) {
    double a = fabs(y), r;
    double b1 = ox_f_approx(0.8), b2 = ox_f_approx(1.25), b3 = ox_f_approx(2.1);
    if (a < b1) r = asin(OX_C1 * a) / OX_C1;
    else if (a < b2) {
        double u = (a - M_PI / 4.0) * 3.0 / sqrt(8.0);
        r = 1.0 + (u < 0 ? -pow(-u, 2.0 / 3.0) : pow(u, 2.0 / 3.0));
    } else if (a < b3) r = (0.81 + sqrt(0.81 * 0.81 - 4.0 * 0.6406 * (OX_C2 - a))) / (2.0 * 0.6406);
    else r = 0.156 + sqrt(0.156 * 0.156 - 2.0 * (OX_C3 - a));
    return y < 0 ? -r : r;
}

/* Section 4.1: the exact subdivision density integral over [a, b] (signed),
 * D(a, b) = int_a^b sqrt|u^2 - 1| du, integrated directly (not as a
 * difference of f, which cancels on short ranges).  [a, b] is cut at -1, 0
 * and 1; by the density's symmetry each part is a part of [0, 1] or of
 * [1, inf), integrated after the substitution u = 1 - v^2 (integrand
 * 2 v^2 sqrt(2 - v^2)) or u = 1 + v^2 (integrand 2 v^2 sqrt(2 + v^2)), both
 * smooth in v, by 16-node Gauss-Legendre on panels of at most 1/4 in v. */
static double gl_panels(double va, double dv, double sgn) {
    gl_init();
    if (!(dv > 0.0)) return 0.0;
    int m = (int)ceil(dv / 0.25);
    if (m < 1) m = 1;
    double h = dv / m, sum = 0.0;
    for (int j = 0; j < m; j++) {
        double a = va + j * h;
        for (int i = 0; i < OX_GL_N; i++) {
            double v = a + 0.5 * h * (gl_x[i] + 1.0);
            sum += gl_w[i] * 0.5 * h * 2.0 * v * v * sqrt(2.0 + sgn * v * v);
        }
    }
    return sum;
}
/* int_p^q for 0 <= p <= q, with [p, q] inside [0, 1] or inside [1, inf); the
 * v interval's length is taken without cancellation,
 * |sqrt|q - 1| - sqrt|p - 1|| = (q - p) / (sqrt|q - 1| + sqrt|p - 1|) */
static double dens_part(double p, double q) {
    if (q <= 1.0) {
        double vq = sqrt(1.0 - q), vp = sqrt(1.0 - p);
        return gl_panels(vq, (q - p) / (vq + vp), -1.0);
    }
    double vp = sqrt(p - 1.0), vq = sqrt(q - 1.0);
    return gl_panels(vp, (q - p) / (vp + vq), 1.0);
}
double ox_dens_integral(double a, double b) {
    if (a == b) return 0.0;
    if (a > b) return -ox_dens_integral(b, a);
    const double cuts[3] = {-1.0, 0.0, 1.0};
    double pts[5];
    int n = 0;
    pts[n++] = a;
    for (int k = 0; k < 3; k++)
        if (cuts[k] > a && cuts[k] < b) pts[n++] = cuts[k];
    pts[n++] = b;
    double sum = 0.0;
    for (int k = 0; k + 1 < n; k++) {
        double p = pts[k], q = pts[k + 1];
        /* the density is even: a part at or below 0 is its mirror image */
        if (q <= 0.0) sum += dens_part(-q, -p);
        else sum += dens_part(p, q);
    }
    return sum;
}

/* Section 4.2's refinement: the point where f reaches y, from the f_approx
 * inverse as the initial guess, by two Newton steps x <- x - (f(x) - y) /
 * sqrt|x^2 - 1| on the exact f; each step kept inside [lo, hi] (the range
 * being flattened) and skipped where the density vanishes. */
double ox_f_newton_inv(double y, double lo, double hi) {
    double x = ox_f_approx_inv(y);
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    for (int it = 0; it < 2; it++) {
        double d = sqrt(fabs(x * x - 1.0));
        if (!(d > 0.0)) break;
        x -= (ox_f_exact(x) - y) / d;
        if (x < lo) x = lo;
        if (x > hi) x = hi;
    }
    return x;
}

/* ============================================ dashing (Sections 1, 9.3) == */
/* The dash pattern of a stroke (an SVG dash array and offset, in the path's
 * own units) cuts each subpath into dashes; every dash is then stroked as an
 * open subpath with the style's joins and caps.  The paper dashes on the CPU
 * and expands the dashes as individual strokes; this is that definition, as
 * an encoding of the dashed path.  Readings:
 *   G34  the pattern restarts at every subpath; a closed subpath is dashed
 *        along its closing line as well and no dash continues across its
 *        start point (every dash is open); zero-length dashes draw nothing;
 *        an odd-length array is repeated once; a pattern of total length 0
 *        leaves the stroke solid.
 *   G35  arc length of a segment: 16 equal parameter panels of 8-node
 *        Gauss-Legendre of |B'(t)|; lengths and pattern positions on a grid
 *        of 2^-24 units, so that sums along a subpath are exact; a dash
 *        boundary inside a segment lies at the parameter where the rule's
 *        partial integral reaches it; the dash's part of the segment is the
 *        segment restricted to that parameter range (its control points
 *        rounded to FP32).
 *   G36  the dashed encoding: every path opens with an empty closed subpath
 *        at its first point carrying its style and transform bits and ends
 *        with an empty closed subpath at its last subpath's start point
 *        carrying its path end bit (so that every path keeps its entries in
 *        the style, transform and path streams even when no dash falls on
 *        it); each dash is [start point][parts of segments][stroke cap
 *        marker (start, first control point that differs from it)].  A part
 *        whose rounded control points all equal its first point has no
 *        extent and is left out, as the encoding leaves out zero-length
 *        segments (G22); the dash starts at its first part with extent, and
 *        a dash without one draws nothing.
 * Fills are not dashed. */
#define OX_DASH_PANELS 16
#define OX_DASH_GRID 16777216.0 /* 2^24 */

static const double dash_gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
static const double dash_gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};

/* |B'(t)| of the degree-c Bezier P[0..c] */
static double bez_speed(const v2 *P, int c, double t) {
    double mt = 1.0 - t;
    v2 d;
    if (c == 1) d = vsub(P[1], P[0]);
    else if (c == 2) d = vscale(vadd(vscale(vsub(P[1], P[0]), mt), vscale(vsub(P[2], P[1]), t)), 2.0);
    else d = vscale(vadd(vadd(vscale(vsub(P[1], P[0]), mt * mt), vscale(vsub(P[2], P[1]), 2.0 * t * mt)),
                         vscale(vsub(P[3], P[2]), t * t)), 3.0);
    return vlen(d);
}
/* 8-node Gauss-Legendre of |B'| over [a, b] */
static double speed_gl8(const v2 *P, int c, double a, double b) {
    double m = 0.5 * (a + b), h = 0.5 * (b - a), sum = 0.0;
    for (int i = 0; i < 4; i++)
        sum += dash_gw[i] * (bez_speed(P, c, m - h * dash_gx[i]) + bez_speed(P, c, m + h * dash_gx[i]));
    return sum * h;
}
/* G35 arc length; panel[k] receives the integral over panel k */
double ox_dash_seg_len(const v2 *P, int c, double *panel) {
    double total = 0.0;
    for (int k = 0; k < OX_DASH_PANELS; k++) {
        panel[k] = speed_gl8(P, c, (double)k / OX_DASH_PANELS, (double)(k + 1) / OX_DASH_PANELS);
        total += panel[k];
    }
    return total;
}
/* parameter where the rule's partial integral reaches s (bisection) */
static double dash_t_at(const v2 *P, int c, const double *panel, double s) {
    double acc = 0.0;
    int k = 0;
    while (k < OX_DASH_PANELS - 1 && acc + panel[k] <= s) acc += panel[k++];
    double lo = (double)k / OX_DASH_PANELS, hi = (double)(k + 1) / OX_DASH_PANELS;
    const double t0 = lo, rest = s - acc;
    for (int it = 0; it < 200 && hi > lo; it++) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (speed_gl8(P, c, t0, mid) < rest) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}
/* blossom of the degree-c Bezier at (u[0..c-1]) */
static v2 bez_blossom(const v2 *P, int c, const double *u) {
    v2 q[4];
    for (int j = 0; j <= c; j++) q[j] = P[j];
    for (int l = 0; l < c; l++)
        for (int j = 0; j < c - l; j++) q[j] = vadd(vscale(q[j], 1.0 - u[l]), vscale(q[j + 1], u[l]));
    return q[0];
}
/* control points of the segment restricted to [ta, tb], rounded to FP32
 * (the segment's own end points where ta = 0 or tb = 1) */
static void bez_part(const v2 *P, int c, double ta, double tb, float *out) {
    for (int j = 0; j <= c; j++) {
        double u[3];
        for (int l = 0; l < c; l++) u[l] = (l < c - j) ? ta : tb;
        v2 q = bez_blossom(P, c, u);
        if (j == 0 && ta == 0.0) q = P[0];
        if (j == c && tb == 1.0) q = P[c];
        out[2 * j] = (float)q.x;
        out[2 * j + 1] = (float)q.y;
    }
}
static int64_t dash_fix(double v) { return (int64_t)llround(v * OX_DASH_GRID); }
static int64_t floor_div(int64_t a, int64_t b) { int64_t q = a / b; return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q; }

static void enc_marker(ox_enc *e, uint8_t extra, float sx, float sy, float dx, float dy) {
    e->tags[e->n_tags++] = (uint8_t)(2u | OX_TAG_SUBPATH_END | OX_TAG_F32 | extra);
    enc_pt(e, sx, sy);
    enc_pt(e, dx, dy);
}
/* an empty closed subpath at p (start point, then the marker's two points) */
static int enc_empty(ox_enc *e, uint8_t extra, float px, float py) {
    if (enc_reserve(e, 1, 3)) return -2;
    enc_pt(e, px, py);
    enc_marker(e, (uint8_t)(OX_TAG_CLOSED | extra), px, py, px + 1.0f, py);
    return 0;
}

/* The dashed encoding of an encoded scene (G34-G36).  Per user style:
 * dash values dash_arr[dash_off[k] .. dash_off[k+1]) and offset dash_phase[k];
 * style_fill[k] marks fills.  Paths whose style has no pattern (or a pattern
 * of total length 0) keep their tags and points unchanged. */
ox_enc *ox_encode_dashed(const ox_enc *src, const float *dash_arr, const uint32_t *dash_off,
                         const float *dash_phase, const uint8_t *style_fill, uint32_t n_user_styles) {
    ox_enc *e = (ox_enc *)calloc(1, sizeof(ox_enc));
    if (!e) return NULL;
    e->status = src->status;
    if (src->status) return e;
    for (uint32_t i = 0; i < src->n_styles; i++)
        if (enc_push_u32(&e->style_stream, &e->n_styles, &e->cap_styles, src->style_stream[i])) goto oom;
    for (uint32_t i = 0; i < src->n_xforms; i++)
        if (enc_push_u32(&e->xform_stream, &e->n_xforms, &e->cap_xforms, src->xform_stream[i])) goto oom;
    for (uint32_t i = 0; i < src->n_paths; i++)
        if (enc_push_u32(&e->path_map, &e->n_paths, &e->cap_paths, src->path_map[i])) goto oom;
    {
        uint32_t n = src->n_tags;
        uint32_t off = 0;
        int32_t sty = -1;
        uint32_t t = 0;
        while (t < n) {
            /* one path: tags t .. pe (the tag carrying the path end bit) */
            uint32_t pe = t;
            while (pe < n && !(src->tags[pe] & OX_TAG_PATH)) pe++;
            if (pe >= n) { e->status = -1; return e; }
            if (src->tags[t] & OX_TAG_STYLE) sty++;
            uint32_t us = src->style_stream[sty];
            if (us >= n_user_styles) { e->status = -1; return e; }
            const float *D0 = src->data + 2 * (size_t)off;
            float p0x = D0[0], p0y = D0[1];
            /* the pattern on the 2^-24 grid */
            int64_t pat[64];
            uint32_t np_ = dash_off[us + 1] - dash_off[us];
            int64_t period = 0;
            int solid = style_fill[us] != 0 || np_ == 0 || np_ > 32;
            if (!solid) {
                uint32_t m = (np_ & 1u) ? 2 * np_ : np_;
                for (uint32_t j = 0; j < m; j++) {
                    pat[j] = dash_fix((double)dash_arr[dash_off[us] + (j % np_)]);
                    period += pat[j];
                }
                np_ = m;
                solid = period <= 0;
            }
            if (enc_empty(e, (uint8_t)(src->tags[t] & (OX_TAG_STYLE | OX_TAG_XFORM)), p0x, p0y)) goto oom;
            if (solid) {
                /* copy the path's tags and points */
                for (uint32_t i = t; i <= pe; i++) {
                    uint32_t tg = src->tags[i];
                    uint32_t inc = (tg & OX_TAG_COUNT) + ((tg & OX_TAG_SUBPATH_END) ? 1u : 0u);
                    /* the first tag of each subpath brings its start point */
                    int first = (i == t) || (src->tags[i - 1] & OX_TAG_SUBPATH_END);
                    if (enc_reserve(e, 1, inc + 1)) goto oom;
                    const float *D = src->data + 2 * (size_t)off;
                    if (first) enc_pt(e, D[0], D[1]);
                    for (uint32_t j = 1; j <= (tg & OX_TAG_COUNT); j++) enc_pt(e, D[2 * j], D[2 * j + 1]);
                    e->tags[e->n_tags++] = (uint8_t)(tg & ~(OX_TAG_PATH | OX_TAG_STYLE | OX_TAG_XFORM));
                    off += inc;
                }
            } else {
                int64_t phase = dash_fix((double)dash_phase[us]) % period;
                if (phase < 0) phase += period;
                uint32_t i = t;
                while (i <= pe) {
                    /* one subpath: segments i .. me-1, marker me */
                    uint32_t me = i;
                    while (!(src->tags[me] & OX_TAG_SUBPATH_END)) me++;
                    int64_t S = 0; /* subpath position of the current segment's start */
                    /* total length first (for dashes running to the subpath end) */
                    int64_t Stot = 0;
                    {
                        uint32_t o2 = off;
                        for (uint32_t j = i; j < me; j++) {
                            uint32_t c = src->tags[j] & OX_TAG_COUNT;
                            v2 P[4];
                            double panel[OX_DASH_PANELS];
                            for (uint32_t q = 0; q <= c; q++) P[q] = v2m(src->data[2 * (o2 + q)], src->data[2 * (o2 + q) + 1]);
                            Stot += dash_fix(ox_dash_seg_len(P, (int)c, panel));
                            o2 += c;
                        }
                    }
                    float ds_x = 0, ds_y = 0, dd_x = 0, dd_y = 0;
                    int dash_written = 0; /* the current dash has a part with extent */
                    for (uint32_t j = i; j < me; j++) {
                        uint32_t c = src->tags[j] & OX_TAG_COUNT;
                        v2 P[4];
                        double panel[OX_DASH_PANELS];
                        for (uint32_t q = 0; q <= c; q++) P[q] = v2m(src->data[2 * (off + q)], src->data[2 * (off + q) + 1]);
                        int64_t len = dash_fix(ox_dash_seg_len(P, (int)c, panel));
                        int64_t S0 = S, S1 = S + len;
                        int last = (j + 1 == me);
                        /* dash intervals [a, b) meeting (S0, S1] */
                        int64_t mlo = floor_div(S0 + phase, period) - 1, mhi = floor_div(S1 + phase, period) + 1;
                        for (int64_t m = mlo; m <= mhi; m++) {
                            int64_t cpos = 0;
                            for (uint32_t k = 0; k < np_; k++) {
                                int64_t a = m * period + cpos - phase, b = a + pat[k];
                                cpos += pat[k];
                                if (k & 1u) continue; /* a gap */
                                if (a < 0) a = 0;
                                if (b > Stot) b = Stot;
                                int64_t lo = a > S0 ? a : S0, hi = b < S1 ? b : S1;
                                if (!(lo < hi)) continue;
                                double ta = lo == S0 ? 0.0 : dash_t_at(P, (int)c, panel, (double)(lo - S0) / OX_DASH_GRID);
                                double tb = hi == S1 ? 1.0 : dash_t_at(P, (int)c, panel, (double)(hi - S0) / OX_DASH_GRID);
                                if (tb < ta) tb = ta;
                                float part[8];
                                bez_part(P, (int)c, ta, tb, part);
                                if (enc_reserve(e, 2, c + 3)) goto oom;
                                if (a >= S0) dash_written = 0; /* a new dash */
                                /* the first control point that differs from the part's start */
                                int qd = 0;
                                for (uint32_t q = 1; q <= c && !qd; q++)
                                    if (!(part[2 * q] == part[0] && part[2 * q + 1] == part[1])) qd = (int)q;
                                if (qd) {
                                    if (!dash_written) {
                                        /* the dash's first part with extent: its start point, and its tangent point (G14) */
                                        dash_written = 1;
                                        ds_x = part[0]; ds_y = part[1];
                                        dd_x = part[2 * qd]; dd_y = part[2 * qd + 1];
                                        enc_pt(e, ds_x, ds_y);
                                    }
                                    for (uint32_t q = 1; q <= c; q++) enc_pt(e, part[2 * q], part[2 * q + 1]);
                                    e->tags[e->n_tags++] = (uint8_t)(c | OX_TAG_F32);
                                }
                                if (b <= S1 || last) {
                                    if (dash_written) enc_marker(e, 0, ds_x, ds_y, dd_x, dd_y);
                                    dash_written = 0;
                                }
                            }
                        }
                        S = S1;
                        off += c;
                    }
                    off += 3; /* the subpath's marker: its two points and the next start point */
                    i = me + 1;
                }
            }
            /* (off is now past the path's last marker: its start point is 2 back) */
            if (enc_empty(e, OX_TAG_PATH, src->data[2 * (size_t)(off - 2)], src->data[2 * (size_t)(off - 2) + 1]))
                goto oom;
            t = pe + 1;
        }
    }
    return e;
oom:
    e->status = -2;
    return e;
}

/* ===================================================== 4. expansion ===== */

typedef struct {
    double tau, tau_fit, tau_flat;
    int mode, fit_mode;
} ox_cfg;

typedef struct {
    v2 P[4];        /* elevated cubic, world space */
    v2 t_start, t_end; /* raw end tangent vectors (first nonzero difference) */
    double w;       /* world half-width (0 for a fill) */
    double lpoly;
    uint32_t path;
    uint32_t tag;
    int fill;       /* one side at offset 0, no joins or caps (reading G33) */
} ox_seg;

static void res_push(ox_res *r, v2 a, v2 b, double curv, uint32_t path, uint32_t kind, uint32_t tag) {
    if (r->n_out + 1 > r->cap_out) {
        uint64_t c = r->cap_out ? r->cap_out * 2 : 1024;
        ox_out *p = (ox_out *)realloc(r->out, c * sizeof(ox_out));
        if (!p) { r->status = -2; return; }
        r->out = p; r->cap_out = c;
    }
    ox_out *o = &r->out[r->n_out++];
    o->x0 = a.x; o->y0 = a.y; o->x1 = b.x; o->y1 = b.y; o->curv = curv;
    o->path = path; o->kind = kind; o->tag = tag;
}

static void piece_push(ox_res *r, const ox_piece *p) {
    if (r->n_pieces + 1 > r->cap_pieces) {
        uint64_t c = r->cap_pieces ? r->cap_pieces * 2 : 256;
        ox_piece *q = (ox_piece *)realloc(r->pieces, c * sizeof(ox_piece));
        if (!q) { r->status = -2; return; }
        r->pieces = q; r->cap_pieces = c;
    }
    r->pieces[r->n_pieces++] = *p;
}

static void margin_min(double *m, double v) { if (v < *m) *m = v; }

static void count_margin(ox_margin *m, double n_est) {
    if (n_est >= 0.5) {
        double d = fabs(n_est - floor(n_est + 0.5));
        margin_min(&m->count, d);
    }
}

/* n = max(1, ceil(n_est)) -- Section 2.1 "round up n" */
static uint32_t ceil_count(double n_est) {
    if (!(n_est > 1.0)) return 1;
    if (n_est > 1e7) return 10000000u;
    return (uint32_t)ceil(n_est);
}

/* Cubic point B(t) - P0 (evaluated relative to the start point so that
 * short chords far from the origin keep their precision) and q = B'/3 */
static v2 cubic_rel(const v2 *P, double t) {
    double mt = 1.0 - t;
    double b = 3.0 * mt * mt * t, c = 3.0 * mt * t * t, d = t * t * t;
    v2 d1 = vsub(P[1], P[0]), d2 = vsub(P[2], P[0]), d3 = vsub(P[3], P[0]);
    return v2m(b * d1.x + c * d2.x + d * d3.x, b * d1.y + c * d2.y + d * d3.y);
}
/* B(t0 + dt) - B(t0): a cubic's Taylor expansion terminates, so
 * B' dt + B'' dt^2 / 2 + B''' dt^3 / 6 is exact algebra; written with
 * q = B'/3 it keeps the chord's relative precision however short it is. */
static v2 cubic_chord(const v2 *P, double t0, double dt) {
    double mt = 1.0 - t0;
    v2 a = vsub(P[1], P[0]), b = vsub(P[2], P[1]), c = vsub(P[3], P[2]);
    v2 q0 = v2m(mt * mt * a.x + 2.0 * t0 * mt * b.x + t0 * t0 * c.x,
                mt * mt * a.y + 2.0 * t0 * mt * b.y + t0 * t0 * c.y);
    v2 s0 = vsub(b, a), s1 = vsub(c, b); /* B''/6 = (1-t) s0 + t s1 */
    v2 s2 = v2m(mt * s0.x + t0 * s1.x, mt * s0.y + t0 * s1.y);
    v2 s3 = vsub(s1, s0);                /* third derivative / 6 */
    return v2m(3.0 * dt * q0.x + 3.0 * dt * dt * s2.x + dt * dt * dt * s3.x,
               3.0 * dt * q0.y + 3.0 * dt * dt * s2.y + dt * dt * dt * s3.y);
}
/* test export: the chord B(t0 + dt) - B(t0) of the cubic P8 = (x0 y0 .. x3 y3) */
void ox_cubic_chord(const double *P8, double t0, double dt, double *out2) {
    v2 P[4];
    for (int j = 0; j < 4; j++) P[j] = v2m(P8[2 * j], P8[2 * j + 1]);
    v2 c = cubic_chord(P, t0, dt);
    out2[0] = c.x;
    out2[1] = c.y;
}
static v2 cubic_q(const v2 *P, double t) {
    double mt = 1.0 - t;
    v2 a = vsub(P[1], P[0]), b = vsub(P[2], P[1]), c = vsub(P[3], P[2]);
    return v2m(mt * mt * a.x + 2.0 * t * mt * b.x + t * t * c.x,
               mt * mt * a.y + 2.0 * t * mt * b.y + t * t * c.y);
}

/* Section 7.3: derivative sample at t; if it is (nearly) zero, sample at a
 * slightly perturbed parameter instead (reading G10). */
typedef struct { v2 dir; double mag; } ox_tan;
static ox_tan sample_q(const ox_seg *s, double t, ox_margin *m) {
    ox_tan r;
    if (t == 0.0) { r.dir = s->t_start; r.mag = vlen(vsub(s->P[1], s->P[0])); return r; }
    if (t == 1.0) { r.dir = s->t_end; r.mag = vlen(vsub(s->P[3], s->P[2])); return r; }
    v2 q = cubic_q(s->P, t);
    double ql = vlen(q);
    double thr = OX_EPS_Q * s->lpoly;
    if (thr > 0) margin_min(&m->q, fabs(ql / thr - 1.0));
    if (ql < thr) {
        q = cubic_q(s->P, t + OX_DELTA_T < 1.0 ? t + OX_DELTA_T : t - OX_DELTA_T);
        ql = vlen(q);
    }
    r.dir = q; r.mag = ql;
    return r;
}

/* ES piece placed in the world (Appendix A: scaled, rotated, translated). */
typedef struct {
    v2 p0, p1;      /* exact piece end points */
    v2 n0, n1;      /* end normals (from the cubic's tangents) */
    double k0, k1;  /* normalised curvature params */
    double L;       /* arc length, px (0 for a pivot of zero chord) */
    v2 rot;         /* chord / Z(1): complex factor mapping normalised -> world */
    double base;    /* world tangent angle = base + phi(u) */
    int pivot;      /* reading G28 */
} ox_es;

static v2 es_point(const ox_es *es, double u) {
    if (u == 0.0) return es->p0;
    if (u == 1.0) return es->p1;
    if (es->pivot) return vadd(es->p0, vscale(vsub(es->p1, es->p0), u));
    return vadd(es->p0, cmul(es->rot, es_integral(es->k0, es->k1, u)));
}
static double es_world_angle(const ox_es *es, double u) {
    return es->base + es_phi(es->k0, es->k1, u);
}
static v2 es_normal(const ox_es *es, double u) {
    if (u == 0.0) return es->n0;
    if (u == 1.0) return es->n1;
    double a = es_world_angle(es, u);
    return v2m(sin(a), -cos(a)); /* (T_y, -T_x) */
}
static double es_kappa(const ox_es *es, double u) { return (es->k0 + es->k1 * (u - 0.5)) / es->L; }
/* (1 + h kappa(u)) * L: same sign and zero as rho, finite for L = 0 */
static double es_rhoL(const ox_es *es, double h, double u) { return es->L + h * (es->k0 + es->k1 * (u - 0.5)); }

/* offset point at u on side h */
static v2 offset_point(const ox_es *es, double h, double u) {
    return vadd(es_point(es, u), vscale(es_normal(es, u), h));
}
/* evolute (centre of curvature) at u: E = p - N / kappa */
static v2 evolute_point(const ox_es *es, double u) {
    /* 1 / kappa = L / (k0 + k1 (u - 1/2)) */
    return vsub(es_point(es, u), vscale(es_normal(es, u), es->L / (es->k0 + es->k1 * (u - 0.5))));
}

/* ---- counts (Sections 4.1-4.2, 5, 6) ---------------------------------- */

/* Subdivision density integral of the parallel curve at offset h over
 * [ua, ub]:  I = int sqrt(|kappa| |1 + h kappa|) ds.  With x = -1 - 2 h kappa
 * (inflection at -1, parallel-curve cusp at +1):
 *     I = |F(x_b) - F(x_a)| / (4 |kappa'| |h|^1.5),  F = f_approx.
 * When the x range is tiny (kappa' ~ 0) the density is constant and
 * I = F'(x_mid) L_r / (2 sqrt|h|).  For h = 0 (zero-width stroke) the ES's own
 * density sqrt|kappa| is used (Section 2.2). */
static double line_integral(const ox_es *es, double h, double ua, double ub, int exact) {
    if (es->k1 == 0.0) {
        /* constant curvature k0 / L: I = sqrt(|kappa| |1 + h kappa|) L_r, written
         * so that it stays finite for a pivot of zero length */
        return (ub - ua) * sqrt(fabs(es->k0) * fabs(es->L + h * es->k0));
    }
    double ka = es_kappa(es, ua), kb = es_kappa(es, ub);
    double Lr = (ub - ua) * es->L;
    if (h == 0.0) {
        double dk = (kb - ka);
        if (fabs(dk) < 1e-12 * (fabs(ka) + fabs(kb)) || dk == 0.0) return sqrt(fabs(0.5 * (ka + kb))) * Lr;
        double kp = dk / Lr;
        if (ka * kb >= 0) return fabs(2.0 / (3.0 * kp) * (pow(fabs(kb), 1.5) - pow(fabs(ka), 1.5)));
        return 2.0 / (3.0 * fabs(kp)) * (pow(fabs(ka), 1.5) + pow(fabs(kb), 1.5));
    }
    double xa = -1.0 - 2.0 * h * ka, xb = -1.0 - 2.0 * h * kb;
    if (fabs(xb - xa) < 1e-9) {
        double xm = 0.5 * (xa + xb);
        return (exact ? sqrt(fabs(xm * xm - 1.0)) : ox_f_approx_deriv(xm)) * Lr / (2.0 * sqrt(fabs(h)));
    }
    double kp = es->k1 / (es->L * es->L);
    double dF = exact ? ox_dens_integral(xa, xb) : ox_f_approx(xb) - ox_f_approx(xa);
    return fabs(dF) / (4.0 * fabs(kp) * pow(fabs(h), 1.5));
}

/* ---- emission helpers ---------------------------------------------------- */

typedef struct {
    ox_res *r;
    uint32_t path, tag;
    int emit;        /* 0 = count only */
    uint64_t count;
    int mode;
} ox_sink;

static void sink_line(ox_sink *k, v2 a, v2 b, uint32_t kind) {
    k->count++;
    if (k->emit) res_push(k->r, a, b, 0.0, k->path, kind, k->tag);
}
static void sink_arc(ox_sink *k, v2 a, v2 b, double turn, uint32_t kind) {
    k->count++;
    if (k->emit) {
        double c = vlen(vsub(b, a));
        double curv = (c > 0.0 && turn != 0.0) ? 2.0 * sin(0.5 * turn) / c : 0.0;
        res_push(k->r, a, b, curv, k->path, kind, k->tag);
    }
}

/* One range [ua, ub] of a side of an ES piece.  Normal ranges are traversed
 * along the side's direction D (side A forward in u, side B backward);
 * reversed ranges (rho < 0) are handled per Section 6 / reading G17. */
static void emit_range(ox_sink *k, const ox_cfg *cfg, const ox_es *es, double h,
                       double ua, double ub, int reversed, int end_a_piece, int end_b_piece,
                       const v2 *Pa_shared, const v2 *Pb_shared, ox_margin *m) {
    int sideA = h > 0.0 || (h == 0.0);
    /* traversal direction of the offset in u: +1 forward, -1 backward */
    int D = sideA ? +1 : -1;
    int dir = reversed ? -D : D;
    double Lr = (ub - ua) * es->L;
    double kp = es->k1 == 0.0 ? 0.0 : es->k1 / (es->L * es->L);
    double ka = es->k1 == 0.0 ? 0.0 : es_kappa(es, ua), kb = es->k1 == 0.0 ? 0.0 : es_kappa(es, ub);
    uint32_t n;
    double *us = NULL;
    if (cfg->mode == OX_OUT_LINES) {
        double I = line_integral(es, h, ua, ub, (cfg->fit_mode & OX_DENSITY_NEWTON) != 0);
        double n_est = I * sqrt(1.0 / (8.0 * cfg->tau_flat));
        count_margin(m, n_est);
        n = ceil_count(n_est);
    } else {
        /* Section 5: n = s cbrt(|k'| (1 + 0.4 |h s k'|) / (120 d)), uniform in s;
         * reading G19: no arc sweeps more than pi/2. */
        double n_est = Lr * cbrt(fabs(kp) * (1.0 + 0.4 * fabs(h * Lr * kp)) / (120.0 * cfg->tau_flat));
        count_margin(m, n_est);
        n = ceil_count(n_est);
        double sweep = fmax(fabs(es->k0 + es->k1 * (ua - 0.5)), fabs(es->k0 + es->k1 * (ub - 0.5))) * (ub - ua) / (M_PI / 2.0);
        count_margin(m, sweep);
        uint32_t ns = ceil_count(sweep);
        if (ns > n) n = ns;
    }
    if (!k->emit) {
        k->count += n;
    } else {
        us = (double *)malloc((n + 1) * sizeof(double));
        us[0] = ua; us[n] = ub;
        if (cfg->mode == OX_OUT_LINES && h != 0.0 && es->k1 != 0.0 && (cfg->fit_mode & OX_DENSITY_NEWTON)) {
            /* exact density: points uniform in f between the range ends */
            double xa = -1.0 - 2.0 * h * ka, xb = -1.0 - 2.0 * h * kb;
            double Fa = ox_f_exact(xa), D = ox_dens_integral(xa, xb);
            double lo = fmin(xa, xb), hi = fmax(xa, xb);
            for (uint32_t i = 1; i < n; i++) {
                if (fabs(xb - xa) < 1e-9) { us[i] = ua + (ub - ua) * ((double)i / n); continue; }
                double x = ox_f_newton_inv(Fa + D * ((double)i / n), lo, hi);
                us[i] = ua + (ub - ua) * ((x - xa) / (xb - xa));
            }
        } else if (cfg->mode == OX_OUT_LINES && h != 0.0 && es->k1 != 0.0) {
            double xa = -1.0 - 2.0 * h * ka, xb = -1.0 - 2.0 * h * kb;
            double Fa = ox_f_approx(xa), Fb = ox_f_approx(xb);
            for (uint32_t i = 1; i < n; i++) {
                if (fabs(xb - xa) < 1e-9) { us[i] = ua + (ub - ua) * ((double)i / n); continue; }
                double y = Fa + (Fb - Fa) * ((double)i / n);
                double x = ox_f_approx_inv(y);
                us[i] = ua + (ub - ua) * ((x - xa) / (xb - xa));
            }
        } else if (cfg->mode == OX_OUT_LINES && es->k1 != 0.0) {
            /* h = 0: points uniform in the ES integral (2/3)|kappa|^1.5 / |kappa'|
             * (Section 2.2), split at an inflection inside the range */
            double Pa = pow(fabs(ka), 1.5), Pb = pow(fabs(kb), 1.5);
            int same = ka * kb >= 0.0;
            double total = same ? fabs(Pb - Pa) : Pa + Pb;
            for (uint32_t i = 1; i < n; i++) {
                double target = total * ((double)i / n), kap;
                if (same) {
                    double P = Pa + (Pb > Pa ? target : -target);
                    kap = (ka + kb >= 0.0 ? 1.0 : -1.0) * pow(P, 2.0 / 3.0);
                } else if (target <= Pa) {
                    kap = (ka >= 0.0 ? 1.0 : -1.0) * pow(Pa - target, 2.0 / 3.0);
                } else {
                    kap = (kb >= 0.0 ? 1.0 : -1.0) * pow(target - Pa, 2.0 / 3.0);
                }
                us[i] = 0.5 + (kap * es->L - es->k0) / es->k1;
            }
        } else {
            for (uint32_t i = 1; i < n; i++) us[i] = ua + (ub - ua) * ((double)i / n);
        }
        v2 *P = (v2 *)malloc((n + 1) * sizeof(v2));
        for (uint32_t i = 0; i <= n; i++) P[i] = offset_point(es, h, us[i]);
        if (Pa_shared) P[0] = *Pa_shared;
        if (Pb_shared) P[n] = *Pb_shared;
        for (uint32_t i = 0; i < n; i++) {
            v2 a = P[i], b = P[i + 1];
            if (cfg->mode == OX_OUT_LINES) {
                if (dir > 0) sink_line(k, a, b, OX_K_OFFSET); else sink_line(k, b, a, OX_K_OFFSET);
            } else {
                double turn = es_phi(es->k0, es->k1, us[i + 1]) - es_phi(es->k0, es->k1, us[i]);
                if (dir > 0) sink_arc(k, a, b, turn, OX_K_OFFSET); else sink_arc(k, b, a, -turn, OX_K_OFFSET);
            }
        }
        free(P);
    }
    if (!reversed) { free(us); return; }

    /* ---- evolute (Section 6): density |s - s0|^-1/2, points uniform in
     * sqrt|s - s0|; lines in both output modes (reading G20) ---- */
    double I_ev;
    /* 2 |sqrt|s_b - s0| - sqrt|s_a - s0||, s - s0 = kappa / kappa' */
    if (kp == 0.0) I_ev = 0.0;
    else I_ev = 2.0 * fabs(sqrt(fabs(kb / kp)) - sqrt(fabs(ka / kp)));
    double ne_est = I_ev * sqrt(1.0 / (8.0 * cfg->tau_flat));
    count_margin(m, ne_est);
    uint32_t ne = ceil_count(ne_est);
    uint32_t nconn = (end_a_piece ? 1u : 0u) + (end_b_piece ? 1u : 0u);
    if (!k->emit) {
        k->count += 2u * ne + 2u * nconn;
        free(us);
        return;
    }
    v2 *E = (v2 *)malloc((ne + 1) * sizeof(v2));
    for (uint32_t i = 0; i <= ne; i++) {
        double u;
        if (i == 0) u = ua;
        else if (i == ne) u = ub;
        else {
            double f = (double)i / ne;
            if (kp == 0.0 || fabs(es->k1) < 1e-7 * fabs(es->k0)) u = ua + (ub - ua) * f;
            else {
                /* uniform in r = sqrt|s - s0| between the range ends */
                double sa = ka / kp, sb = kb / kp; /* s - s0 at the ends (same sign) */
                double r = sqrt(fabs(sa)) + f * (sqrt(fabs(sb)) - sqrt(fabs(sa)));
                double s = (sa >= 0 ? 1.0 : -1.0) * r * r;
                u = ua + (ub - ua) * ((s - sa) / (sb - sa));
            }
        }
        E[i] = evolute_point(es, u);
    }
    /* at a rho = 0 end the evolute meets the offset: share the point */
    if (!end_a_piece && Pa_shared) E[0] = *Pa_shared;
    if (!end_b_piece && Pb_shared) E[ne] = *Pb_shared;
    for (int copy = 0; copy < 2; copy++)
        for (uint32_t i = 0; i < ne; i++) {
            /* evolute traversed along D */
            if (D > 0) sink_line(k, E[i], E[i + 1], OX_K_EVOLUTE);
            else sink_line(k, E[i + 1], E[i], OX_K_EVOLUTE);
        }
    /* connecting normal lines at piece-boundary ends, twice each:
     * P -> E at the end where D enters the range, E -> P where it leaves */
    v2 Pa = Pa_shared ? *Pa_shared : offset_point(es, h, ua);
    v2 Pb = Pb_shared ? *Pb_shared : offset_point(es, h, ub);
    if (end_a_piece)
        for (int copy = 0; copy < 2; copy++) {
            if (D > 0) sink_line(k, Pa, E[0], OX_K_CONNECT); else sink_line(k, E[0], Pa, OX_K_CONNECT);
        }
    if (end_b_piece)
        for (int copy = 0; copy < 2; copy++) {
            if (D > 0) sink_line(k, E[ne], Pb, OX_K_CONNECT); else sink_line(k, Pb, E[ne], OX_K_CONNECT);
        }
    free(E);
    free(us);
}

/* Parallel curve of one ES piece on side h (Algorithm 2's inner part):
 * split at the parallel-curve cusp (Section 7.3.1, linear in s), then each
 * range is normal or reversed. */
static void emit_side(ox_sink *k, const ox_cfg *cfg, const ox_es *es, double h, ox_margin *m) {
    double r0 = es_rhoL(es, h, 0.0), r1 = es_rhoL(es, h, 1.0);
    if (es->L > 0.0) {
        margin_min(&m->rho, fabs(r0 / es->L));
        margin_min(&m->rho, fabs(r1 / es->L));
    }
    v2 P0 = vadd(es->p0, vscale(es->n0, h));
    v2 P1 = vadd(es->p1, vscale(es->n1, h));
    if (r0 * r1 < 0.0) {
        /* reading G9: cusp where 1 + h kappa(u) = 0 */
        double tc = r0 / (r0 - r1);
        v2 Pc = offset_point(es, h, tc);
        emit_range(k, cfg, es, h, 0.0, tc, r0 < 0.0, 1, 0, &P0, &Pc, m);
        emit_range(k, cfg, es, h, tc, 1.0, r1 < 0.0, 0, 1, &Pc, &P1, m);
    } else {
        int rev = (r0 < 0.0 || r1 < 0.0);
        emit_range(k, cfg, es, h, 0.0, 1.0, rev, 1, 1, &P0, &P1, m);
    }
}

/* ---- test exports: one Euler spiral on its own ------------------------- */

/* An ES of arc length L with curvature parameters k0, k1 placed at the
 * origin with tangent angle phi(u) (base angle 0): p(u) = L Z(u). */
static ox_es es_at_origin(double k0, double k1, double L) {
    ox_es es;
    es.pivot = 0;
    es.k0 = k0; es.k1 = k1; es.L = L;
    es.rot = v2m(L, 0.0);
    es.base = 0.0;
    es.p0 = v2m(0.0, 0.0);
    es.p1 = cmul(es.rot, es_integral(k0, k1, 1.0));
    double a0 = es_phi(k0, k1, 0.0), a1 = es_phi(k0, k1, 1.0);
    es.n0 = v2m(sin(a0), -cos(a0));
    es.n1 = v2m(sin(a1), -cos(a1));
    return es;
}

/* Section 4.2 subdivision integral of side h over [ua, ub] of that ES, as the
 * line count uses it (before the sqrt(1 / (8 tau_flat)) factor). */
double ox_line_integral_es(double k0, double k1, double L, double h, double ua, double ub, int exact) {
    ox_es es = es_at_origin(k0, k1, L);
    return line_integral(&es, h, ua, ub, exact);
}

/* The records of side h of that ES (Sections 4-6: the range split at the
 * parallel-curve cusp, offsets, evolutes and connecting lines) at tolerance
 * tol in output mode `mode`; tag and path 0. */
ox_res *ox_es_side(double k0, double k1, double L, double h, double tol, int mode, int flags) {
    ox_res *r = (ox_res *)calloc(1, sizeof(ox_res));
    if (!r) return NULL;
    ox_cfg cfg;
    cfg.tau = tol;
    cfg.tau_fit = OX_FIT_FRAC * tol;
    cfg.tau_flat = OX_FLAT_FRAC * tol;
    cfg.mode = mode;
    cfg.fit_mode = flags;
    ox_es es = es_at_origin(k0, k1, L);
    ox_sink sk;
    sk.r = r; sk.path = 0; sk.tag = 0; sk.emit = 1; sk.count = 0; sk.mode = mode;
    ox_margin m;
    m.fit = m.count = m.rho = m.q = m.len = m.join = INFINITY;
    m.n_pieces = 0; m.max_depth_hits = 0;
    emit_side(&sk, &cfg, &es, h, &m);
    return r;
}

/* ---- joins and caps (Algorithm 1, SVG styles) --------------------------- */

static double round_step(double w, double tau_flat) {
    /* Section 2.1 exact arc flattening: each line spans 2 acos(1 - d/r) */
    double c = 1.0 - tau_flat / w;
    if (c < -1.0) c = -1.0;
    if (c > 1.0) c = 1.0;
    return 2.0 * acos(c);
}

/* round arc around centre c of radius w from angle a0 turning by sweep
 * (ccw positive); emits lines or arcs from point A to point B exactly. */
static void emit_round(ox_sink *k, const ox_cfg *cfg, v2 c, double w, double a0, double sweep,
                       v2 A, v2 B, uint32_t kind) {
    uint32_t n;
    if (cfg->mode == OX_OUT_LINES) {
        double st = round_step(w, cfg->tau_flat);
        n = ceil_count(fabs(sweep) / st);
    } else {
        n = ceil_count(fabs(sweep) / (M_PI / 2.0));
    }
    if (!k->emit) { k->count += n; return; }
    v2 prev = A;
    for (uint32_t i = 1; i <= n; i++) {
        v2 nx;
        if (i == n) nx = B;
        else {
            double a = a0 + sweep * ((double)i / n);
            nx = v2m(c.x + w * cos(a), c.y + w * sin(a));
        }
        if (cfg->mode == OX_OUT_LINES) sink_line(k, prev, nx, kind);
        else sink_arc(k, prev, nx, sweep / n, kind);
        prev = nx;
    }
}

static void emit_cap(ox_sink *k, const ox_cfg *cfg, int cap, v2 p, v2 u, double w, int start) {
    /* end cap: from P_A = p + wN to P_B = p - wN around the front (+u);
     * start cap: from P_B to P_A around the back (-u). */
    v2 N = vnormal(u);
    v2 PA = vadd(p, vscale(N, w)), PB = vsub(p, vscale(N, w));
    v2 from = start ? PB : PA, to = start ? PA : PB;
    v2 fwd = start ? vscale(u, -1.0) : u;
    if (cap == OX_CAP_BUTT) {
        sink_line(k, from, to, OX_K_CAP);
    } else if (cap == OX_CAP_SQUARE) {
        v2 a = vadd(from, vscale(fwd, w)), b = vadd(to, vscale(fwd, w));
        sink_line(k, from, a, OX_K_CAP);
        sink_line(k, a, b, OX_K_CAP);
        sink_line(k, b, to, OX_K_CAP);
    } else {
        double a0 = atan2(from.y - p.y, from.x - p.x);
        emit_round(k, cfg, p, w, a0, M_PI, from, to, OX_K_CAP);
    }
}

/* join at pivot p between unit tangents ua (end of this segment) and ub
 * (start of the next one).  Side A (h = +w) runs a -> b, side B runs b -> a. */
static void emit_join(ox_sink *k, const ox_cfg *cfg, const ox_style *st, v2 p, v2 ta, v2 tb,
                      double w, ox_margin *m) {
    v2 ua = vunit(ta), ub = vunit(tb);
    double cr = vcross(ua, ub), dp = vdot(ua, ub);
    v2 Na = vnormal(ua), Nb = vnormal(ub);
    /* reading G31: tangents within OX_SMOOTH_JOIN rad of each other close
     * each side with one straight line and no pivot lines; the wedge left out
     * is thinner than w * 1e-5.  Which side would be "outer" is then moot. */
    /* join margins are absolute distances of cr (unit vectors) to a threshold */
    if (dp > 0.0) margin_min(&m->join, fabs(fabs(cr) - OX_SMOOTH_JOIN));
    if (dp > 0.0 && fabs(cr) < OX_SMOOTH_JOIN) {
        sink_line(k, vadd(p, vscale(Na, w)), vadd(p, vscale(Nb, w)), OX_K_JOIN_OUTER);
        sink_line(k, vadd(p, vscale(Nb, -w)), vadd(p, vscale(Na, -w)), OX_K_JOIN_OUTER);
        return;
    }
    /* near-reversal: which side is outer hinges on the sign of cr */
    if (dp < 0.0) margin_min(&m->join, fabs(cr));
    /* reading G21: cr == 0 (reversal) counts as a left turn */
    int outerA = !(cr < 0.0);
    double h_out = outerA ? w : -w;
    double h_in = -h_out;
    v2 Oa = vadd(p, vscale(Na, h_out)), Ob = vadd(p, vscale(Nb, h_out));
    v2 Ia = vadd(p, vscale(Na, h_in)), Ib = vadd(p, vscale(Nb, h_in));
    /* outer contour in the outer side's traversal order */
    v2 from = outerA ? Oa : Ob, to = outerA ? Ob : Oa;
    /* emission order: side A's part first, then side B's */
    for (int side = 0; side < 2; side++) {
        int isA = side == 0;
        if (isA == outerA) {
            if (st->join == OX_JOIN_ROUND) {
                double dphi = atan2(cr, dp);
                /* around the pivot, body on the left: always ccw */
                double a0 = atan2(from.y - p.y, from.x - p.x);
                emit_round(k, cfg, p, w, a0, fabs(dphi), from, to, OX_K_JOIN_OUTER);
            } else if (st->join == OX_JOIN_MITER) {
                double lim = st->miter_limit;
                double crit = lim * lim * (1.0 + dp);
                margin_min(&m->join, fabs(crit / 2.0 - 1.0));
                if (crit >= 2.0) {
                    v2 Mp = vadd(p, vscale(vadd(Na, Nb), h_out / (1.0 + dp)));
                    sink_line(k, from, Mp, OX_K_JOIN_OUTER);
                    sink_line(k, Mp, to, OX_K_JOIN_OUTER);
                } else {
                    sink_line(k, from, to, OX_K_JOIN_OUTER);
                }
            } else {
                sink_line(k, from, to, OX_K_JOIN_OUTER);
            }
        } else {
            /* inner join through the pivot (strong correctness) */
            v2 f = outerA ? Ib : Ia, t = outerA ? Ia : Ib;
            sink_line(k, f, p, OX_K_JOIN_INNER);
            sink_line(k, p, t, OX_K_JOIN_INNER);
        }
    }
}

/* ---- cubic -> ES subdivision (Algorithm 2) ----------------------------- */

static void process_segment(ox_sink *k, const ox_cfg *cfg, const ox_seg *s, ox_margin *m) {
    uint32_t t0_u = 0;
    double dt = 1.0;
    v2 last_p = s->P[0];
    v2 last_rel = v2m(0.0, 0.0);
    ox_tan last_q = sample_q(s, 0.0, m);
    double hw = s->w;
    double tau_fit = cfg->tau_fit;
    while (1) {
        double t0 = (double)t0_u * dt;
        if (t0 == 1.0) break;
        double t1 = t0 + dt;
        v2 next_rel = (t1 == 1.0) ? vsub(s->P[3], s->P[0]) : cubic_rel(s->P, t1);
        v2 next_p = (t1 == 1.0) ? s->P[3] : vadd(s->P[0], next_rel);
        ox_tan next_q = sample_q(s, t1, m);
        v2 chord = cubic_chord(s->P, t0, dt);
        double cl = vlen(chord);
        double th0 = atan2(vcross(last_q.dir, chord), vdot(last_q.dir, chord));
        double th1 = atan2(vcross(chord, next_q.dir), vdot(chord, next_q.dir));
        double d0 = last_q.mag * dt / cl, d1 = next_q.mag * dt / cl;
        double est = ox_fit_estimate(th0, th1, d0, d1);
                double err = ((cfg->fit_mode & OX_FIT_PAPER) != 0) ? est * cl : est * (cl + OX_FIT_K * hw) * OX_FIT_S;
        /* reading G11: only a chord of exactly zero leaves the end angles
         * undefined; such a piece is subdivided */
        int len_ok = cl > 0.0;
        /* reading G29: the estimate only sees the end angles.  The sub-cubic's
         * hodograph control polygon a = q0 dt, b = chord - (q0 + q1) dt,
         * c = q1 dt bounds how far its tangent turns inside; when that polygon
         * turns by pi or more (angle(a,b) + angle(b,c) >= pi, i.e.
         * (a.b)|c| + (b.c)|a| <= 0) the piece may reverse (cusp) or loop
         * inside, invisible to the end angles, so it is subdivided. */
        int hodo_ok = 1;
        {
            double ma = last_q.mag * dt, mc = next_q.mag * dt;
            v2 a = vscale(vunit(last_q.dir), ma), c = vscale(vunit(next_q.dir), mc);
            v2 b = vsub(vsub(chord, a), c);
            /* a middle vector that is zero up to rounding leaves only the
             * turn from a to c, which is below pi: no test */
            if (!(cfg->fit_mode & OX_FIT_NO_HODO) && ma > 0.0 && mc > 0.0 && vlen(b) > 1e-9 * (ma + mc)) {
                double hv = vdot(a, b) * mc + vdot(b, c) * ma;
                double scale = vlen(b) * ma * mc;
                if (scale > 0.0) margin_min(&m->len, fabs(hv) / scale);
                hodo_ok = hv > 0.0;
            }
        }
        int forced = dt <= ldexp(1.0, -OX_MAX_DEPTH);
        int ok = len_ok && hodo_ok && err <= tau_fit;
        if (len_ok && hodo_ok && !forced && isfinite(err)) margin_min(&m->fit, fabs(err / tau_fit - 1.0));
        if (ok || forced) {
            int pivot = forced && !ok;
            if (pivot) m->max_depth_hits++;
            ox_es es;
            double c;
            es.pivot = pivot;
            es.p0 = last_p; es.p1 = next_p;
            es.n0 = vnormal(vunit(last_q.dir));
            es.n1 = vnormal(vunit(next_q.dir));
            if (pivot) {
                /* reading G28: a piece accepted only because of the depth cap
                 * holds a cusp the bisection cannot resolve; it is drawn as a
                 * pivot: constant curvature (k1 = 0), turning by the signed angle
                 * between its end tangents, oriented by its start tangent, so its
                 * parallel curves are circles about the point */
                es.k0 = atan2(vcross(last_q.dir, next_q.dir), vdot(last_q.dir, next_q.dir));
                es.k1 = 0.0;
                c = ox_es_chord(0.5 * es.k0, 0.5 * es.k0);
                es.base = atan2(last_q.dir.y, last_q.dir.x) + 0.5 * es.k0;
                es.rot = v2m(0.0, 0.0);
            } else {
                es.k0 = th0 + th1;
                es.k1 = ox_es_k1(th0, th1);
                c = ox_es_chord(th0, th1);
                v2 z1 = es_integral(es.k0, es.k1, 1.0);
                es.rot = cdiv(chord, z1);
                es.base = atan2(es.rot.y, es.rot.x);
            }
            if (!(c > OX_C_MIN)) c = OX_C_MIN;
            es.L = cl / c;
            m->n_pieces++;
            if (k->emit) {
                ox_piece pc = {t0, t1, es.k0, es.k1, cl, es.L, th0, th1, s->tag, (uint32_t)pivot};
                piece_push(k->r, &pc);
            }
            emit_side(k, cfg, &es, +hw, m);
            if (!s->fill) emit_side(k, cfg, &es, -hw, m);
            /* pop the two-word stack: count trailing zeros */
            t0_u += 1;
            uint32_t sh = 0;
            while (((t0_u >> sh) & 1u) == 0u) sh++;
            t0_u >>= sh;
            dt *= (double)(1u << sh);
            last_p = next_p;
            last_rel = next_rel;
            last_q = next_q;
        } else {
            t0_u *= 2;
            dt *= 0.5;
        }
    }
}

/* Reading G32: a line segment is exactly straight, so it is its own Euler
 * spiral piece: k0 = k1 = 0, arc length equal to the chord, tangent angle of
 * the chord.  The subdivision and fit test are skipped; on a line they would
 * only measure rounding noise (angles of order 1e-16 that leave the counts
 * unchanged but give arcs a curvature of that order). */
static void straight_segment(ox_sink *k, const ox_cfg *cfg, const ox_seg *s, ox_margin *m) {
    ox_es es;
    v2 chord = vsub(s->P[3], s->P[0]);
    es.pivot = 0;
    es.p0 = s->P[0];
    es.p1 = s->P[3];
    es.n0 = vnormal(vunit(s->t_start));
    es.n1 = es.n0;
    es.k0 = 0.0;
    es.k1 = 0.0;
    es.rot = chord;
    es.base = atan2(chord.y, chord.x);
    es.L = vlen(chord);
    m->n_pieces++;
    if (k->emit) {
        ox_piece pc = {0.0, 1.0, 0.0, 0.0, es.L, es.L, 0.0, 0.0, s->tag, 0u};
        piece_push(k->r, &pc);
    }
    emit_side(k, cfg, &es, +s->w, m);
    if (!s->fill) emit_side(k, cfg, &es, -s->w, m);
}

/* ---- segment fetch (Section 8.1: degree elevation) --------------------- */

static v2 xf_apply(const float *X, double x, double y) {
    /* x' = a x + c y + e, y' = b x + d y + f */
    return v2m((double)X[0] * x + (double)X[2] * y + (double)X[4],
               (double)X[1] * x + (double)X[3] * y + (double)X[5]);
}

static v2 first_nonzero(const v2 *cands, int n) {
    for (int i = 0; i < n; i++) if (!vzero(cands[i])) return cands[i];
    return v2m(1.0, 0.0);
}

int ox_affine_ok(const float *X) {
    for (int j = 0; j < 6; j++) if (!isfinite(X[j])) return 0;
    double det = (double)X[0] * X[3] - (double)X[1] * X[2];
    return det != 0.0 && isfinite(det);
}

int ox_xform_ok(const float *X) {
    /* reading G16: similarity transforms only (rotation / reflection with
     * uniform scale), exactly as encoded */
    int rot = (X[0] == X[3]) && (X[1] == -X[2]);
    int refl = (X[0] == -X[3]) && (X[1] == X[2]);
    double det = (double)X[0] * X[3] - (double)X[1] * X[2];
    return (rot || refl) && det != 0.0 && isfinite(det);
}

/* Full expansion of an encoded scene.  Output in canonical order (reading
 * G24): by tag; within a tag, ES pieces in t order, side A then side B,
 * ranges in u order; then the join or cap. */
ox_res *ox_expand(const ox_enc *e, const ox_style *styles, uint32_t n_styles,
                  const float *xforms, uint32_t n_xforms, double tolerance, int mode,
                  int fit_mode, int emit, uint32_t tag_begin, uint32_t tag_end) {
    ox_res *r = (ox_res *)calloc(1, sizeof(ox_res));
    if (!r) return NULL;
    uint32_t n = e->n_tags;
    if (tag_end > n) tag_end = n;
    if (tag_begin > tag_end) tag_begin = tag_end;
    r->n_tags = n;
    r->counts = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    r->margins = (ox_margin *)calloc(n ? n : 1, sizeof(ox_margin));
    if (!(tolerance > 0.0) || !isfinite(tolerance)) { r->status = -1; return r; }
    uint32_t *off = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *pth = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *sty = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *xfi = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    ox_monoids(e->tags, n, off, pth, sty, xfi);
    ox_cfg cfg;
    cfg.tau = tolerance;
    cfg.tau_fit = OX_FIT_FRAC * tolerance;
    cfg.tau_flat = OX_FLAT_FRAC * tolerance;
    cfg.mode = mode;
    cfg.fit_mode = fit_mode;
    for (uint32_t i = 0; i < e->n_xforms; i++) {
        if (e->xform_stream[i] >= n_xforms) { r->status = -1; goto done; }
    }
    for (uint32_t i = 0; i < e->n_styles; i++) {
        if (e->style_stream[i] >= n_styles) { r->status = -1; goto done; }
        const ox_style *st = &styles[e->style_stream[i]];
        if (st->flags & ~OX_STYLE_FILL) { r->status = -1; goto done; }
        /* a fill ignores width, miter limit, join and caps */
        if (!(st->flags & OX_STYLE_FILL) &&
            (!(st->half_width >= 0.0f) || !isfinite(st->half_width) || !(st->miter_limit >= 1.0f))) {
            r->status = -1;
            goto done;
        }
    }
    /* a transform drawn with a stroke must be a similarity (reading G16), one
     * drawn with a fill any invertible affine map (reading G33) */
    for (uint32_t i = 0; i < n; i++) {
        const ox_style *st = &styles[e->style_stream[sty[i]]];
        const float *X = xforms + 6 * (size_t)e->xform_stream[xfi[i]];
        int ok = (st->flags & OX_STYLE_FILL) ? ox_affine_ok(X) : ox_xform_ok(X);
        if (!ok) { r->status = -1; goto done; }
    }
    for (uint32_t i = tag_begin; i < tag_end; i++) {
        uint8_t tag = e->tags[i];
        ox_margin *m = &r->margins[i];
        m->fit = m->count = m->rho = m->q = m->len = m->join = INFINITY;
        const ox_style *st = &styles[e->style_stream[sty[i]]];
        const float *X = xforms + 6 * (size_t)e->xform_stream[xfi[i]];
        const int fill = (st->flags & OX_STYLE_FILL) != 0;
        double scale = sqrt(fabs((double)X[0] * X[3] - (double)X[1] * X[2]));
        double w = fill ? 0.0 : (double)st->half_width * scale;
        ox_sink sk;
        sk.r = r; sk.path = e->path_map[pth[i]]; sk.tag = i; sk.emit = emit; sk.count = 0; sk.mode = mode;
        const float *D = e->data + 2 * (size_t)off[i];
        if (tag & OX_TAG_SUBPATH_END) {
            /* stroke cap marker: start cap if the subpath is open */
            if (!fill && !(tag & OX_TAG_CLOSED)) {
                v2 ps = xf_apply(X, D[2], D[3]);
                v2 pd = xf_apply(X, D[4], D[5]);
                v2 dir = vsub(pd, ps);
                if (vzero(dir)) dir = v2m(1.0, 0.0);
                emit_cap(&sk, &cfg, st->start_cap, ps, vunit(dir), w, 1);
            }
        } else {
            uint32_t c = tag & OX_TAG_COUNT;
            v2 raw[4];
            for (uint32_t j = 0; j <= c; j++) raw[j] = xf_apply(X, D[2 * j], D[2 * j + 1]);
            ox_seg s;
            s.w = w; s.path = sk.path; s.tag = i; s.fill = fill;
            if (c == 1) {
                s.P[0] = raw[0]; s.P[3] = raw[1];
                v2 d = vsub(raw[1], raw[0]);
                s.P[1] = vadd(raw[0], vscale(d, 1.0 / 3.0));
                s.P[2] = vadd(raw[0], vscale(d, 2.0 / 3.0));
            } else if (c == 2) {
                s.P[0] = raw[0]; s.P[3] = raw[2];
                s.P[1] = vadd(raw[0], vscale(vsub(raw[1], raw[0]), 2.0 / 3.0));
                s.P[2] = vadd(raw[2], vscale(vsub(raw[1], raw[2]), 2.0 / 3.0));
            } else {
                for (int j = 0; j < 4; j++) s.P[j] = raw[j];
            }
            v2 cs[3], ce[3];
            for (uint32_t j = 0; j < c; j++) cs[j] = vsub(raw[j + 1], raw[0]);
            for (uint32_t j = 0; j < c; j++) ce[j] = vsub(raw[c], raw[c - 1 - j]);
            s.t_start = first_nonzero(cs, (int)c);
            s.t_end = first_nonzero(ce, (int)c);
            s.lpoly = vlen(vsub(s.P[1], s.P[0])) + vlen(vsub(s.P[2], s.P[1])) + vlen(vsub(s.P[3], s.P[2]));
            if (c == 1) straight_segment(&sk, &cfg, &s, m);
            else process_segment(&sk, &cfg, &s, m);
            /* join or end cap with the neighbour at i + 1 (Algorithm 1) */
            uint8_t nt = e->tags[i + 1];
            v2 pend = raw[c];
            if (fill) {
                /* a fill has no joins or caps */
            } else if ((nt & OX_TAG_SUBPATH_END) && !(nt & OX_TAG_CLOSED)) {
                emit_cap(&sk, &cfg, st->end_cap, pend, vunit(s.t_end), w, 0);
            } else {
                v2 tb;
                const float *Dn = e->data + 2 * (size_t)off[i + 1];
                if (nt & OX_TAG_SUBPATH_END) {
                    /* closed: join with the subpath's first segment, whose start
                     * tangent the marker carries as (start, dir) */
                    v2 ps = xf_apply(X, Dn[2], Dn[3]);
                    v2 pd = xf_apply(X, Dn[4], Dn[5]);
                    tb = vsub(pd, ps);
                    if (vzero(tb)) tb = v2m(1.0, 0.0);
                } else {
                    uint32_t cn = nt & OX_TAG_COUNT;
                    v2 rn[4];
                    for (uint32_t j = 0; j <= cn; j++) rn[j] = xf_apply(X, Dn[2 * j], Dn[2 * j + 1]);
                    v2 cn_s[3];
                    for (uint32_t j = 0; j < cn; j++) cn_s[j] = vsub(rn[j + 1], rn[0]);
                    tb = first_nonzero(cn_s, (int)cn);
                }
                emit_join(&sk, &cfg, st, pend, s.t_end, tb, w, m);
            }
        }
        if (sk.count > 0xffffffffull) { r->status = -4; goto done; }
        r->counts[i] = (uint32_t)sk.count;
        if (r->status) goto done;
    }
done:
    free(off); free(pth); free(sty); free(xfi);
    return r;
}

void ox_res_free(ox_res *r) {
    if (!r) return;
    free(r->out); free(r->counts); free(r->margins); free(r->pieces);
    free(r);
}
int ox_res_status(const ox_res *r) { return r->status; }
uint64_t ox_res_nout(const ox_res *r) { return r->n_out; }
const ox_out *ox_res_out(const ox_res *r) { return r->out; }
const uint32_t *ox_res_counts(const ox_res *r) { return r->counts; }
const ox_margin *ox_res_margins(const ox_res *r) { return r->margins; }
uint64_t ox_res_npieces(const ox_res *r) { return r->n_pieces; }
const ox_piece *ox_res_pieces(const ox_res *r) { return r->pieces; }
uint32_t ox_sizeof_out(void) { return (uint32_t)sizeof(ox_out); }
uint32_t ox_sizeof_margin(void) { return (uint32_t)sizeof(ox_margin); }
uint32_t ox_sizeof_piece(void) { return (uint32_t)sizeof(ox_piece); }
