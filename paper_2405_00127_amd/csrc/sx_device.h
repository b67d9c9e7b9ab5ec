// Device-side math of the stroke-expansion hot path (gfx950, wave64).
//
// Two stages share this header.  The piece stage, process_tag, runs the
// per-segment decisions of one tag (Algorithm 1 / Algorithm 2) and writes
// compact emission items: one per parallel-curve range, per evolute bundle
// and per join or cap, each split into chunks of at most K records, with the
// tag's record count.  The record stage, emit_item, expands one item chunk
// into output records at their final positions.
//
// Precision split.  CDNA4 issues FP64 vector FMA at the FP32 (unpacked)
// rate, so everything that *decides* -- the bisection and its fit estimate,
// the Euler spiral parameters, parallel-curve cusp splits, every count,
// join classification -- runs in FP64 from the exact FP32 inputs, once per
// piece.  The per-output-point work (spiral position, normal, offset and
// evolute points) runs in FP32 from the piece parameters; outputs are FP32
// records.  The library is built with -ffp-contract=off; every FMA here is
// explicit.
//
// Paper: Levien & Uguray, "GPU-friendly Stroke Expansion" (arXiv:2405.00127).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

// Every function is host+device so the same code can be unit-checked off the GPU.
#define SX_HD __host__ __device__
#define SX_FN __host__ __device__ __forceinline__

namespace sx {

// ------------------------------------------------------------ constants
// Table 1 (Section 8.2) tag bits; bit 7 marks a closed subpath on its
// stroke cap marker.
constexpr uint32_t kTagCount = 0x03u, kTagEnd = 0x04u, kTagF32 = 0x08u, kTagPath = 0x10u,
                   kTagXform = 0x20u, kTagStyle = 0x40u, kTagClosed = 0x80u;
enum { kJoinBevel = 0, kJoinMiter = 1, kJoinRound = 2 };
enum { kCapButt = 0, kCapSquare = 1, kCapRound = 2 };
enum { kOutLines = 0, kOutArcs = 1 };

// Tolerance split between the cubic->ES fit and parallel-curve flattening,
// and the offset-aware fit error err = est * (chord + K |h|) * S.
constexpr double kFitFrac = 0.15, kFlatFrac = 0.65, kFitK = 9.0, kFitS = 1.6;
// Section 7.3 cusp handling: near-zero derivative test and perturbation.
constexpr double kEpsQ = 1e-5, kDeltaT = 1.0 / 4096.0;
constexpr int kMaxDepth = 16;
constexpr double kCMin = 0.1;          // lower clamp of the chord / arc-length ratio
constexpr double kSmoothJoin = 1e-5;   // joins closer to tangent than this: one line per side
constexpr double kPi = 3.14159265358979323846;
constexpr double kHalfPi = 1.57079632679489661923;
// Section 4.2 constants of the piecewise approximation.
constexpr double kC1 = 1.0976991822760038, kC2 = 0.9148117935952064, kC3 = 0.16145779359520596;
constexpr double kA2 = 0.94280904158206336587;  // sqrt(8)/3
constexpr uint32_t kMaxCount = 10000000u;

struct StyleD {
    float half_width, miter_limit;
    uint32_t packed;  // join | start_cap << 8 | end_cap << 16 | flags << 24
};
// a fill: flattened at offset 0 (half_width 0), one side, no joins or caps
constexpr uint32_t kStyleFill = 1u << 24;

// ---------------------------------------------------------- small vectors
struct V2 {  // FP32 (per-point work, outputs)
    float x, y;
};
struct D2 {  // FP64 (decisions)
    double x, y;
};
SX_FN V2 v2(float x, float y) { return V2{x, y}; }
SX_FN V2 operator+(V2 a, V2 b) { return v2(a.x + b.x, a.y + b.y); }
SX_FN V2 operator-(V2 a, V2 b) { return v2(a.x - b.x, a.y - b.y); }
SX_FN V2 operator*(V2 a, float s) { return v2(a.x * s, a.y * s); }
SX_FN float len(V2 a) { return sqrtf(a.x * a.x + a.y * a.y); }

SX_FN D2 d2(double x, double y) { return D2{x, y}; }
SX_FN D2 operator+(D2 a, D2 b) { return d2(a.x + b.x, a.y + b.y); }
SX_FN D2 operator-(D2 a, D2 b) { return d2(a.x - b.x, a.y - b.y); }
SX_FN D2 operator*(D2 a, double s) { return d2(a.x * s, a.y * s); }
SX_FN double dot(D2 a, D2 b) { return a.x * b.x + a.y * b.y; }
SX_FN double cross(D2 a, D2 b) { return a.x * b.y - a.y * b.x; }
SX_FN double len(D2 a) { return sqrt(a.x * a.x + a.y * a.y); }
SX_FN bool is_zero(D2 a) { return a.x == 0.0 && a.y == 0.0; }
SX_FN D2 unit(D2 a) {
    const double r = 1.0 / len(a);
    return d2(a.x * r, a.y * r);
}
// right normal N = (T_y, -T_x); N' = kappa T
SX_FN D2 rnormal(D2 t) { return d2(t.y, -t.x); }
SX_FN V2 f32(D2 a) { return v2((float)a.x, (float)a.y); }
// offset point p + N h, rounded once
SX_FN V2 offs(D2 p, D2 n, double h) { return f32(p + n * h); }

// ------------------------------------------------------- Euler spirals
// Appendix A: k1 and chord / arc-length ratio as 7th-order polynomials in
// k = th0 + th1 and D = th1 - th0.
SX_FN double es_k1(double th0, double th1) {
    double k = th0 + th1, d = th1 - th0;
    double k2 = k * k, d2_ = d * d;
    double a = 6.0 + d2_ * (-1.0 / 70.0 + d2_ * (-1.0 / 10780.0 + d2_ * 2.769178184818219e-7));
    double b = -0.1 + d2_ * (1.0 / 4200.0 + d2_ * 1.6959677820260655e-5);
    double c = -1.0 / 1400.0 + d2_ * 6.84915970574303e-5;
    double e = -7.936475029053326e-6;
    return d * (a + k2 * (b + k2 * (c + k2 * e)));
}
SX_FN double es_chord(double th0, double th1) {
    double k = th0 + th1, d = th1 - th0;
    double k2 = k * k, d2_ = d * d;
    double a = 1.0 + d2_ * (-1.0 / 40.0 + d2_ * (0.00034226190482569864 - d2_ * 1.9349474568904524e-6));
    double b = -1.0 / 24.0 + d2_ * (0.0024702380951963226 - d2_ * 3.7297408997537985e-5);
    double c = 1.0 / 1920.0 - d2_ * 4.87350869747975e-5;
    double e = -3.1001936068463107e-6;
    return a + k2 * (b + k2 * (c + k2 * e));
}

// Section 7.1: chord-normalised distance estimate between a cubic with end
// angles th0, th1 and arms d0, d1 and the Euler spiral with those angles
// (sn0, c0, sn1, c1: the sines and cosines of th0 and th1).
SX_FN double fit_estimate_sc(double th0, double th1, double sn0, double c0, double sn1, double c1, double d0,
                             double d1) {
    double s = fabs(th0 + th1), df = fabs(th0 - th1);
    double s2 = s * s;
    double e0 = 4.6255e-6 * (s2 * s2 * s) + 7.5e-3 * s2 * df;
    const double sn01 = sn0 * c1 + c0 * sn1;
    double db0 = 2.0 / (3.0 * (1.0 + c0)), db1 = 2.0 / (3.0 * (1.0 + c1));
    // area(d0,d1) - area(db0,db1), area = 3/20 (2 d0 sin th0 + 2 d1 sin th1 - d0 d1 sin(th0+th1))
    double a_src = 2.0 * d0 * sn0 + 2.0 * d1 * sn1 - d0 * d1 * sn01;
    double a_es = 2.0 * db0 * sn0 + 2.0 * db1 * sn1 - db0 * db1 * sn01;
    double ea = 1.55 * 0.15 * fabs(a_src - a_es);
    double x0 = db0 - d0, x1 = db1 - d1;
    double ei = (0.005 * s + 0.07 * df) * sqrt(x0 * x0 + x1 * x1);
    return e0 + ea + ei;
}

// sin and cos in FP32 for the point placement, whose angles stay within a
// few turns: quadrant k = rint(2x / pi) and r = x - k pi/2 by Cody-Waite
// reduction (pi/2 as the float nearest to it plus the float nearest to the
// rest, each product taken inside an FMA), then the Taylor series of sin and
// cos on |r| <= pi/4 (truncation below 2e-9).  Within 2 ulp of the exact
// values for |x| < 1e4; the same operations on host and device.
SX_FN void sincos_r(float x, float* sn, float* cs) {
    const float k = rintf(x * 0.636619772367581343f);
    float r = fmaf(-k, 1.57079637050628662109375f, x);
    r = fmaf(-k, -4.37113900018624283e-8f, r);
    const float r2 = r * r;
    float ps = fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f);
    ps = fmaf(r2, ps, 1.0f / 120.0f);
    ps = fmaf(r2, ps, -1.0f / 6.0f);
    const float sr = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    pc = fmaf(r2, pc, -1.0f / 720.0f);
    pc = fmaf(r2, pc, 1.0f / 24.0f);
    pc = fmaf(r2, pc, -0.5f);
    const float cr = fmaf(r2, pc, 1.0f);
    const int q = (int)k & 3;
    const float a = (q & 1) ? cr : sr, b = (q & 1) ? sr : cr;
    *sn = (q & 2) ? -a : a;
    *cs = ((q + 1) & 2) ? -b : b;
}

// Normalised ES: unit arc length, phi(u) = k0 (u - 1/2) + k1/2 (u - 1/2)^2.
SX_FN float es_phi_f(float k0, float k1, float u) {
    float v = u - 0.5f;
    return v * (k0 + 0.5f * k1 * v);
}
SX_FN double es_phi(double k0, double k1, double u) {
    double v = u - 0.5;
    return v * (k0 + 0.5 * k1 * v);
}

// Z(u) = int_0^u exp(i phi(v)) dv by 4-point Gauss-Legendre on [0, u] (FP32).
SX_FN V2 es_integral_f(float k0, float k1, float u) {
    const float gx[4] = {-0.8611363115940526f, -0.3399810435848563f, 0.3399810435848563f, 0.8611363115940526f};
    const float gw[4] = {0.3478548451374538f, 0.6521451548625461f, 0.6521451548625461f, 0.3478548451374538f};
    float hu = 0.5f * u;
    float sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        float v = hu * (gx[i] + 1.0f);
        float ph = es_phi_f(k0, k1, v);
        float sn, cs;
        sincos_r(ph, &sn, &cs);
        sx = fmaf(gw[i], cs, sx);
        sy = fmaf(gw[i], sn, sy);
    }
    return v2(sx * hu, sy * hu);
}
// Z(1) (once per piece): 8-point Gauss-Legendre on v = u - 1/2.  The nodes
// come in pairs +-v, and exp(i phi(v)) + exp(i phi(-v)) = 2 cos(k0 v)
// exp(i k1 v^2 / 2), so each pair costs one sincos and one cos.  Z(1) only
// places the piece for the per-point work (p0 + chord / Z(1) * Z(u)), so the
// pipeline takes it in FP32; the FP64 form serves host checks.
SX_FN V2 es_integral1_f(float k0, float k1) {
    float sx = 0.0f, sy = 0.0f;
    if (fabsf(k0) + fabsf(k1) < 1.5f) {
        // 4 nodes (2 pairs) integrate the smooth phase to FP32 accuracy here
        const float gx[2] = {0.3399810435848563f, 0.8611363115940526f};
        const float gw[2] = {0.6521451548625461f, 0.3478548451374538f};
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const float v = 0.5f * gx[i];
            float sn, cs;
            sincos_r(0.5f * k1 * v * v, &sn, &cs);
            float s0, c0;
            sincos_r(k0 * v, &s0, &c0);
            const float c = gw[i] * c0;
            sx += c * cs;
            sy += c * sn;
        }
    } else {
        const float gx[4] = {0.1834346424956498f, 0.5255324099163290f, 0.7966664774136267f, 0.9602898564975363f};
        const float gw[4] = {0.3626837833783620f, 0.3137066458778873f, 0.2223810344533745f, 0.1012285362903763f};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const float v = 0.5f * gx[i];
            float sn, cs;
            sincos_r(0.5f * k1 * v * v, &sn, &cs);
            float s0, c0;
            sincos_r(k0 * v, &s0, &c0);
            const float c = gw[i] * c0;
            sx += c * cs;
            sy += c * sn;
        }
    }
    return v2(sx, sy);
}
SX_FN D2 es_integral1(double k0, double k1) {
    const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < 4; i++) {
        const double v = 0.5 * gx[i];
        double sn, cs;
        sincos(0.5 * k1 * v * v, &sn, &cs);
        const double c = gw[i] * cos(k0 * v);
        sx += c * cs;
        sy += c * sn;
    }
    return d2(sx, sy);
}

struct ES {
    D2 p0, p1, n0, n1;  // exact end points and end normals
    double k0, k1, L;   // curvature params and arc length (px)
    bool pivot;
    // from the exact ends, rounded once: offset end points of sides A / B
    // and the evolute's end points (p - N / kappa at u = 0 and 1)
    V2 P0A, P1A, P0B, P1B, E0, E1;
    // FP32 copies for the per-point work
    V2 fp0, frot, fd;   // world p0, chord / Z(1), p1 - p0 (pivot)
    float fk0, fk1, fL, fbase;
};

SX_FN V2 es_point_f(const ES& es, float u) {
    if (es.pivot) return es.fp0 + es.fd * u;
    V2 z = es_integral_f(es.fk0, es.fk1, u);
    return es.fp0 + v2(es.frot.x * z.x - es.frot.y * z.y, es.frot.x * z.y + es.frot.y * z.x);
}
SX_FN V2 es_normal_f(const ES& es, float u) {
    float a = es.fbase + es_phi_f(es.fk0, es.fk1, u);
    float sn, cs;
    sincos_r(a, &sn, &cs);
    return v2(sn, -cs);
}
SX_FN double es_kn(const ES& es, double u) { return es.k0 + es.k1 * (u - 0.5); }
// (1 + h kappa(u)) L: sign and zero of rho, finite for a zero-length pivot
SX_FN double es_rhoL(const ES& es, double h, double u) { return es.L + h * es_kn(es, u); }
// interior offset point (FP32)
SX_FN V2 offset_point_f(const ES& es, float h, float u) { return es_point_f(es, u) + es_normal_f(es, u) * h; }
// evolute point E = p - N / kappa, 1/kappa = L / (k0 + k1 (u - 1/2))
SX_FN V2 evolute_point_f(const ES& es, float u) {
    float kn = es.fk0 + es.fk1 * (u - 0.5f);
    return es_point_f(es, u) - es_normal_f(es, u) * (es.fL / kn);
}
SX_FN V2 evolute_end(const ES& es, bool at_end) {
    // exact end points and normals, FP64 (infinite where kappa = 0: only
    // read on reversed ranges, where kappa is not 0)
    D2 p = at_end ? es.p1 : es.p0, n = at_end ? es.n1 : es.n0;
    double kn = es_kn(es, at_end ? 1.0 : 0.0);
    return f32(p - n * (es.L / kn));
}
// the rounded end points of the spiral's sides and evolute (see ES)
SX_FN void es_ends(ES& es, double w) {
    es.P0A = offs(es.p0, es.n0, w);
    es.P1A = offs(es.p1, es.n1, w);
    es.P0B = offs(es.p0, es.n0, -w);
    es.P1B = offs(es.p1, es.n1, -w);
    es.E0 = evolute_end(es, false);
    es.E1 = evolute_end(es, true);
}

// FP32 copies of an ES for the record pass: p0, chord / Z(1) (or p1 - p0 for
// a pivot), k0, k1, L, base angle
SX_FN void set_es_f(const ES& es, float* d) {
    V2 r = es.pivot ? es.fd : es.frot;
    d[0] = es.fp0.x; d[1] = es.fp0.y; d[2] = r.x; d[3] = r.y;
    d[4] = es.fk0; d[5] = es.fk1; d[6] = es.fL; d[7] = es.fbase;
}

// ------------------------------------------- subdivision density integral
// x = -1 - 2 h kappa maps the ES inflection to -1 and the parallel-curve
// cusp to +1 (Section 4.1).  A point on this axis keeps x and, precisely,
// e = |x| - 1 (2 h kappa when x <= 0, -2 rho when x > 0).
// The helpers are templates: FP64 where they decide counts (piece stage),
// FP32 where they only place points (record stage).
template <class T>
SX_FN T absT(T v) { return v < T(0) ? -v : v; }
template <class T>
struct XPT {
    T x, e;
};
using XP = XPT<double>;
template <class T>
SX_FN XPT<T> make_xp(T hk) {
    const T x = T(-1) - T(2) * hk;
    const T e = (x <= T(0)) ? T(2) * hk : T(-2) * (T(1) + hk);
    return XPT<T>{x, e};
}
template <class T>
SX_FN XPT<T> bp_xp(T x) { return XPT<T>{x, absT(x) - T(1)}; }

// branch of f_approx by |x|: 0 [0,0.8) sin, 1 [0.8,1.25) 1.5-power, 2 [1.25,2.1) and 3 quadratics
template <class T>
SX_FN int branch_of(T ax) { return ax < T(0.8) ? 0 : (ax < T(1.25) ? 1 : (ax < T(2.1) ? 2 : 3)); }
SX_FN double pow15(double a) { return a * sqrt(a); }
SX_FN float pow15f(float a) { return a * sqrtf(a); }

// Divided difference (F(b) - F(a)) / (b - a) of f_approx over one branch,
// in a cancellation-free form; dx = b - a given precisely.
template <class T>
SX_HD inline T branch_dd(int br, XPT<T> a, XPT<T> b, T dx) {
    if (br == 0) {
        // cos(c1 m) sin(hz) / hz.  A piece of this branch lies in
        // [-0.8, 0.8], so |c1 m| < 0.88 and |hz| <= 0.8 c1 < 0.88: both by
        // their Taylor series (truncation below 1e-18 relative for |hz| < 1).
        const T m = T(0.5) * (a.x + b.x);
        const T hz = T(0.5) * T(kC1) * dx;
        const T z = T(kC1) * m;
        const T h2 = hz * hz;
        const T sc = T(1) + h2 * (T(-1.0 / 6) + h2 * (T(1.0 / 120) + h2 * (T(-1.0 / 5040) + h2 * (T(1.0 / 362880) +
                     h2 * (T(-1.0 / 39916800) + h2 * (T(1.0 / 6227020800.0) + h2 * (T(-1.0 / 1307674368000.0) +
                     h2 * (T(1.0 / 355687428096000.0) + h2 * (T(-1.0 / 121645100408832000.0) +
                     h2 * T(1.0 / 51090942171709440000.0))))))))));
        const T z2 = z * z;
        const T cz = T(1) + z2 * (T(-1.0 / 2) + z2 * (T(1.0 / 24) + z2 * (T(-1.0 / 720) + z2 * (T(1.0 / 40320) +
                     z2 * (T(-1.0 / 3628800) + z2 * (T(1.0 / 479001600.0) + z2 * (T(-1.0 / 87178291200.0) +
                     z2 * (T(1.0 / 20922789888000.0) + z2 * (T(-1.0 / 6402373705728000.0) +
                     z2 * T(1.0 / 2432902008176640000.0))))))))));
        return cz * sc;
    }
    if (br == 1) {
        const T ea = absT(a.e), eb = absT(b.e);
        if (a.e * b.e >= T(0)) {
            const T ra = sqrt(ea), rb = sqrt(eb);
            const T den = ra + rb;
            if (den == T(0)) return T(0);
            return T(kA2) * (ea + ra * rb + eb) / den;
        }
        return T(kA2) * (ea * sqrt(ea) + eb * sqrt(eb)) / (ea + eb);
    }
    const T aa = absT(a.x), ab = absT(b.x);
    if (br == 2) return T(0.6406) * (aa + ab) - T(0.81);
    return T(0.5) * (aa + ab) - T(0.156);
}

// Range of the x axis split at the branch breaks of f_approx.
template <class T>
struct XSegT {
    XPT<T> a;
    T len;  // signed x length
    T dF;   // F increment over the piece
    T G;    // dF / len (the piece's divided difference)
    int br;
};
using XSeg = XSegT<double>;
// Total F increment over [xa, xb], split at the branch breaks of f_approx
// (each piece within one branch, by its divided difference).  Pieces
// between two breaks have fixed increments (xinc, see set_break_increments),
// so at most the two end pieces are evaluated.  *dF0 and *len0 receive the
// first piece's increment and x length, *xbits the split: breaks crossed
// (bits 0-2), index of the first one crossed (bits 3-5), walking up the x
// axis (bit 6).
constexpr double kXBreak[6] = {-2.1, -1.25, -0.8, 0.8, 1.25, 2.1};
SX_HD inline double split_x_sum(XP xa, XP xb, double dx_total, const double* xinc, double* dF0, double* len0,
                                uint32_t* xbits) {
    const bool up = xb.x > xa.x;
    // the breaks strictly between xa and xb are consecutive ones: walk them
    // from xa, summing the fixed increments between them
    int n = 0, kf = 0;
    double bf = 0.0, bl = 0.0, mid = 0.0;
#pragma unroll
    for (int kk = 0; kk < 6; kk++) {
        const double b = up ? kXBreak[kk] : kXBreak[5 - kk];
        const bool in = up ? (b > xa.x && b < xb.x) : (b < xa.x && b > xb.x);
        if (in) {
            if (n == 0) {
                bf = b;
                kf = up ? kk : 5 - kk;
            } else if (kk > 0) {
                mid += up ? xinc[kk - 1] : -xinc[5 - kk];
            }
            bl = b;
            n++;
        }
    }
    const bool cross = n > 0;
    const double l1 = cross ? bf - xa.x : dx_total;
    const int br1 = cross ? branch_of(fabs(xa.x + 0.5 * l1)) : branch_of(fabs(0.5 * (xa.x + xb.x)));
    double dF = branch_dd(br1, xa, cross ? bp_xp(bf) : xb, l1) * l1;
    *dF0 = dF;
    *len0 = l1;
    if (cross) {
        const double l2 = xb.x - bl;
        dF += mid;
        dF += branch_dd(branch_of(fabs(bl + 0.5 * l2)), bp_xp(bl), xb, l2) * l2;
    }
    *xbits = (uint32_t)n | ((uint32_t)kf << 3) | (up ? 64u : 0u);
    return dF;
}
// F increments of the pieces between consecutive branch breaks (break k to
// break k + 1), by the same divided differences.
SX_HD inline void set_break_increments(double* xinc) {
    for (int k = 0; k < 5; k++) {
        const double a = kXBreak[k], b = kXBreak[k + 1], l = b - a;
        xinc[k] = branch_dd(branch_of(fabs(a + 0.5 * l)), bp_xp(a), bp_xp(b), l) * l;
    }
}

// Fraction of a branch segment at which F has risen by f * seg.dF
// (local, cancellation-free inverse of f_approx; FP32 per output point).
SX_HD inline float branch_inv_frac(const XSegT<float>& s, float f) {
    const float G = s.G;  // divided difference (len != 0 here)
    const float ax = s.a.x, ae = s.a.e, dF = s.dF, ln = s.len;
    if (s.br == 0) {
        const float c1 = (float)kC1;
        float th = c1 * ax;
        float S, C;
        sincos_r(th, &S, &C);
        float dy = c1 * f * dF;
        float Sp = S + dy;
        if (S * Sp < 0.0f || fabsf(dy) > 0.25f) {
            float d = asinf(fminf(fmaxf(Sp, -1.0f), 1.0f)) / c1 - ax;
            return d / ln;
        }
        float rp = sqrtf(fmaxf(1.0f - Sp * Sp, 0.0f));
        float coef = C + S * (S + Sp) / (C + rp);
        float arg = dy * coef;
        float as = (fabsf(arg) < 1e-4f) ? 1.0f + arg * arg * (1.0f / 6.0f) : asinf(fminf(fmaxf(arg, -1.0f), 1.0f)) / arg;
        return f * G * coef * as;
    }
    float sgn = (ax + 0.5f * ln) >= 0.0f ? 1.0f : -1.0f;  // side of the axis
    float dFa = sgn * f * dF;                              // F increment on |x|
    if (s.br == 1) {
        const float A2 = (float)kA2;
        float vs = (ae < 0.0f ? -1.0f : 1.0f) * pow15f(fabsf(ae));
        float dg = dFa / A2;
        float vp = vs + dg;
        float lena = sgn * ln;
        if (vs * vp >= 0.0f) {
            float avp = fabsf(vp), avs = fabsf(vs);
            float p = cbrtf(avp), q = cbrtf(avs);
            float D = p * p * p * p + p * p * q * q + q * q * q * q;
            if (D == 0.0f) return f;
            return f * G * (avp + avs) / (A2 * D);
        }
        float ep = (vp < 0.0f ? -1.0f : 1.0f) * cbrtf(vp * vp);
        return (ep - ae) / lena;
    }
    float a = fabsf(ax);
    if (s.br == 2) {
        float B = 1.2812f * a - 0.81f;
        return 2.0f * f * G / (B + sqrtf(fmaxf(B * B + 4.0f * 0.6406f * dFa, 0.0f)));
    }
    float B = a - 0.156f;
    return 2.0f * f * G / (B + sqrtf(fmaxf(B * B + 2.0f * dFa, 0.0f)));
}

// ------------------------------- exact density integral, refined inverse
// The higher-quality option of Section 4.2: counts from the exact integral
// f(x) = int_0^x sqrt|u^2 - 1| du, points where f reaches each target, found
// from the f_approx inverse by two Newton steps on f.  FP64 throughout.

// f in closed form (reading G5 for |x| > 1), odd
SX_FN double f_exact_d(double x) {
    const double a = fabs(x);
    const double r = a <= 1.0 ? 0.5 * (a * sqrt(1.0 - a * a) + asin(a))
                              : 0.5 * (a * sqrt(a * a - 1.0) - acosh(a)) + 0.25 * kPi;
    return x < 0.0 ? -r : r;
}
// int of 2 v^2 sqrt(2 + s v^2) over [v0, v0 + dv] by 8-node Gauss-Legendre
// (the density after the substitution u = 1 + s v^2, smooth in v)
SX_HD inline double sub_gl8(double v0, double dv, double s) {
    const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const double c = v0 + 0.5 * dv, hw = 0.5 * dv;
    double sum = 0.0;
    for (int i = 0; i < 4; i++) {
        const double va = c - hw * gx[i], vb = c + hw * gx[i];
        sum += gw[i] * (va * va * sqrt(2.0 + s * va * va) + vb * vb * sqrt(2.0 + s * vb * vb));
    }
    return sum * dv;  // (dv / 2) x weights x 2 v^2 sqrt(...)
}
// int_p^q sqrt|u^2 - 1| du, 0 <= p <= q on one side of 1, by the substitution
// u = 1 -+ v^2 (v's interval length without cancellation)
SX_HD inline double dens_side(double p, double q) {
    if (q <= 1.0) {
        const double vq = sqrt(1.0 - q), vp = sqrt(1.0 - p);
        return (vp + vq > 0.0) ? sub_gl8(vq, (q - p) / (vp + vq), -1.0) : 0.0;
    }
    const double vp = sqrt(p - 1.0), vq = sqrt(q - 1.0);
    return (vp + vq > 0.0) ? sub_gl8(vp, (q - p) / (vp + vq), 1.0) : 0.0;
}
// int_a^b sqrt|u^2 - 1| du (signed), relative-accurate: the closed-form
// difference when it keeps at least 1e-4 of the larger |f| (rounding then
// costs at most ~1e-12 of the result), else -- a short range -- the
// substituted quadrature on each part between -1, 0 and 1
SX_HD inline double dens_int_d(double a, double b) {
    if (a == b) return 0.0;
    const double fa = f_exact_d(a), fb = f_exact_d(b);
    const double d = fb - fa;
    if (fabs(d) >= 1e-4 * fmax(fabs(fa), fabs(fb))) return d;
    const double lo = fmin(a, b), hi = fmax(a, b);
    const double cut[3] = {-1.0, 0.0, 1.0};
    double sum = 0.0, p = lo;
    for (int k = 0; k <= 3; k++) {
        const double q = (k < 3 && cut[k] > p && cut[k] < hi) ? cut[k] : (k == 3 ? hi : p);
        if (q > p) {
            sum += (q <= 0.0) ? dens_side(-q, -p) : dens_side(p, q);
            p = q;
        }
    }
    return b > a ? sum : -sum;
}
// inverse of f_approx, branch by branch (Section 4.2)
SX_HD inline double f_approx_inv_d(double y) {
    const double a = fabs(y);
    const double b1 = 0.7010707591262915;  // sin(0.8 c1) / c1: f_approx at 0.8
    const double b2 = kA2 * 0.125 + 0.25 * kPi;  // sqrt(8)/3 (1/4)^1.5 + pi/4
    const double b3 = 0.6406 * 2.1 * 2.1 - 0.81 * 2.1 + kC2;
    double r;
    if (a < b1) {
        r = asin(kC1 * a) / kC1;
    } else if (a < b2) {
        const double u = (a - 0.25 * kPi) / kA2;
        r = 1.0 + (u < 0.0 ? -cbrt(u * u) : cbrt(u * u));
    } else if (a < b3) {
        r = (0.81 + sqrt(0.81 * 0.81 - 4.0 * 0.6406 * (kC2 - a))) / (2.0 * 0.6406);
    } else {
        r = 0.156 + sqrt(0.156 * 0.156 - 2.0 * (kC3 - a));
    }
    return y < 0.0 ? -r : r;
}
// x in [lo, hi] where f(x) = y: the f_approx inverse, then two Newton steps
// x <- x - (f(x) - y) / sqrt|x^2 - 1| (each kept in [lo, hi], skipped where
// the density vanishes)
SX_HD inline double f_newton_inv_d(double y, double lo, double hi) {
    double x = fmin(fmax(f_approx_inv_d(y), lo), hi);
    for (int it = 0; it < 2; it++) {
        const double d = sqrt(fabs(x * x - 1.0));
        if (!(d > 0.0)) break;
        x = fmin(fmax(x - (f_exact_d(x) - y) / d, lo), hi);
    }
    return x;
}
SX_FN float bits_f(uint32_t v) {
    float f;
    memcpy(&f, &v, 4);
    return f;
}
SX_FN uint32_t f_bits(float f) {
    uint32_t v;
    memcpy(&v, &f, 4);
    return v;
}

SX_FN uint32_t ceil_count(double n_est) {
    if (!(n_est > 1.0)) return 1u;
    if (n_est > 1e7) return kMaxCount;
    return (uint32_t)ceil(n_est);
}

// ------------------------------------------------------------- items
// The piece pass turns each tag into emission items in canonical order:
// one per parallel-curve range (offset lines / arcs), one per reversed
// range's evolute bundle (evolute twice + connecting lines), one per join or
// cap.  Items longer than K records are split into chunks of K.  The record
// pass then runs one thread per item: FP32 per-point work only, at most K
// records each, so the load is balanced and the register footprint small.
enum { kItemOffset = 1, kItemEvolute = 2, kItemJoin = 3 };
// item header flags (bits 4..)
constexpr uint32_t kIfDirNeg = 1u << 4;     // offset: records run backwards in u
constexpr uint32_t kIfArcs = 1u << 5;       // arc records
constexpr uint32_t kIfPivot = 1u << 6;      // ES is a pivot (straight position)
constexpr uint32_t kIfPlaceF = 1u << 7;     // offset: place points by the density inverse (h != 0)
constexpr uint32_t kIfPlaceES = 1u << 8;    // offset: place points uniform in |kappa|^1.5 (h == 0)
constexpr uint32_t kIfEndA = 1u << 9;       // evolute: connecting lines at ua
constexpr uint32_t kIfEndB = 1u << 10;      // evolute: connecting lines at ub
constexpr uint32_t kIfDneg = 1u << 11;      // evolute: side traversed backwards
constexpr uint32_t kIfInnerFirst = 1u << 12;  // join: inner part before the outer part
constexpr uint32_t kIfKSame = 1u << 13;       // offset, h == 0: curvature keeps its sign over the range
constexpr uint32_t kIfNewton = 1u << 14;      // offset: place points by the Newton-refined exact inverse
constexpr uint32_t kXBitsShift = 16;          // offset: the split at the branch breaks (bits 16-22)
// join outer part kind (bits 16..19), inner part kind (bits 20..21)
enum { kOutLine1 = 0, kOutLine2 = 1, kOutLine3 = 2, kOutRound = 3 };
enum { kInNone = 0, kInPivot = 1, kInSmooth = 2 };

// Items live in 64-byte units.  Offset items take one unit; evolute, join
// and cap items two (their payload keeps word 16 at zero, so a scan over
// units reads the second unit as an empty slot).  The Euler spiral of a
// piece is stored once per slot (the slot's ES record), not per item.
constexpr uint32_t kUnitWords = 16;
struct __align__(16) Unit {
    uint32_t w[kUnitWords];
};
struct ItemHdr {
    uint32_t hdr;    // kind | flags | outer kind << 16 | inner kind << 20 | records in this chunk << 24
    uint32_t path;   // output path id of the records
    uint32_t slot;   // slot index (canonical position of the piece or tail)
    uint32_t local;  // record offset of this chunk within the slot
    uint32_t k0;     // first record of the chunk within the whole item
    uint32_t ntot;   // records of the whole item
};
constexpr uint32_t kHdrWords = 6;
SX_FN uint32_t item_n(uint32_t hdr) { return hdr >> 24; }

// offset-item payload: the range [ua, ub] of side h, its exact end points,
// and for density placement the F increment over the range and the FP32 sum
// of its branch pieces' x lengths (from the FP64 count)
struct OffsetP {
    float ua, du, len0, fh;  // u range, x length of its first branch piece, side h
    float Pax, Pay, Pbx, Pby;
    float dF, dF0;  // F increment of the range and of its first branch piece
    // (with kIfNewton: len0 and dF0 hold the low and high words of the FP64
    // density coordinate x at ua, dF the x length of the range)
};
// evolute-item payload: the range, its density split alpha and evolute
// count, the exact offset and evolute end points
struct EvoluteP {
    float ua, du, alpha;
    uint32_t ne;
    float Pax, Pay, Pbx, Pby;
    float E0x, E0y;
    uint32_t zero;  // word 16 of the item
    float E1x, E1y;
};
// join- and cap-item payload: the outer part's end points (exact offsets,
// shared with the adjacent sides), the inner part, the join point and the
// round or miter / square geometry
struct JoinP {
    float fromx, fromy, tox, toy;
    float fx, fy, tx, ty;  // inner part (pivot: f -> p -> t; smooth: f -> t)
    float px, py;          // join / cap point (round centre)
    uint32_t zero;         // word 16 of the item
    float a0, sweep, w;    // round part
    float ax, ay, bx, by;  // miter point / square corners
    uint32_t n_outer;
};
template <class P>
struct Units {
    static constexpr uint32_t n = (kHdrWords + (uint32_t)(sizeof(P) / 4) + kUnitWords - 1) / kUnitWords;
};
static_assert(Units<OffsetP>::n == 1 && Units<EvoluteP>::n == 2 && Units<JoinP>::n == 2, "item units");
static_assert(offsetof(EvoluteP, zero) == (kUnitWords - kHdrWords) * 4 && offsetof(JoinP, zero) == (kUnitWords - kHdrWords) * 4,
              "second unit starts with a zero word");

SX_FN uint32_t chunks(uint32_t n, uint32_t K) { return (n + K - 1) / K; }

struct Cfg {
    double tau_fit, tau_flat, inv_sqrt8tf;  // sqrt(1 / (8 tau_flat))
    double cbrt_inv120tf;                   // cbrt(1 / (120 tau_flat))
    int arcs;
    int paper_fit;                          // fit error: Section 7.1 estimate x chord (else offset-aware)
    int newton;                             // exact density integral, Newton-refined inverse (Section 4.2)
    uint32_t K;                             // records per item chunk
    double xinc[5];                         // F increments between the branch breaks
};

// Item sink: writes a tag's items into slots handed out by the allocator and
// counts the tag's records.  Alloc::alloc(nc) returns the first of nc
// consecutive slots owned by the caller, or ~0 when the workspace is full
// (the items are then dropped; the caller sees the overflow count).
// With Stats, the sink also counts the work done (fit trials, accepted
// pieces, items by kind) for the algorithmic-work figures of the roofline.
enum { kStTrials = 0, kStPieces = 1, kStRanges = 2, kStEvolutes = 3, kStJoins = 4, kStLines = 5, kStN = 6 };

// An item of nrec records as chunks of at most K records, each chunk a copy
// of the header (with its own count and position) and the payload, at unit
// `base` of the workspace; n0 = the item's first record within its slot.
template <class P>
SX_HD void write_item(Unit* units, uint64_t base, uint32_t hdr, uint32_t path, uint32_t slot, uint32_t n0,
                      uint32_t nrec, uint32_t K, const P& p) {
    constexpr uint32_t U = Units<P>::n;
    const uint32_t nc = chunks(nrec, K);
    for (uint32_t c = 0; c < nc; c++) {
        uint32_t* dst = units[base + (uint64_t)c * U].w;
        const uint32_t nchunk = (c + 1 < nc) ? K : nrec - c * K;
        *reinterpret_cast<uint4*>(dst) = make_uint4(hdr | (nchunk << 24), path, slot, n0 + c * K);
        *reinterpret_cast<uint2*>(dst + 4) = make_uint2(c * K, nrec);
        *reinterpret_cast<P*>(dst + kHdrWords) = p;
    }
}

template <class Alloc, bool Stats = false>
struct ItemSink {
    Unit* units;
    float* es_tab;  // 8 floats per slot
    Alloc al;
    uint32_t path, slot;  // output path id, slot index
    uint32_t n;           // records of the slot so far
    uint32_t st[Stats ? kStN : 1];
    static constexpr bool kStats = Stats;
    template <class P>
    SX_HD void put(uint32_t hdr, uint32_t nrec, uint32_t K, const P& p) {
        if constexpr (Stats) {
            const uint32_t kind = hdr & 15u;
            st[kind == kItemOffset ? kStRanges : (kind == kItemEvolute ? kStEvolutes : kStJoins)]++;
        }
        const uint64_t base = al.alloc(chunks(nrec, K) * Units<P>::n);
        if (base != ~0ull) write_item(units, base, hdr, path, slot, n, nrec, K, p);
        n += nrec;
    }
};

// ----------------------------------------------- one range of one side
// Section 4 (lines), Section 5 (arcs) and Section 6 (evolute for rho < 0).
// The decisions of a range (its counts and the density increment that places
// its points) depend only on the spiral's k0, k1, L, the side h and the u
// range; writing its items needs the rest.
struct RangeRes {
    float dF;           // F increment over the range (density placement)
    float dF0, len0, alpha;  // increment and x length of its first branch piece; evolute point split
    uint32_t n, ne, place, xbits;  // xbits: the split at the branch breaks (split_x_sum)
};
// Newton: the build that can count with the exact integral (cfg.newton);
// the default build leaves that code out.
template <bool Newton = true>
SX_FN RangeRes range_count(const Cfg& cfg, double k0, double k1, double L, double h, double ua, double ub,
                           bool reversed) {
    RangeRes r;
    const double du = ub - ua;
    const double kna = k0 + k1 * (ua - 0.5), knb = k0 + k1 * (ub - 0.5);
    r.dF = 0.0f;
    r.dF0 = 0.0f;
    r.len0 = 0.0f;
    r.place = 0;
    r.xbits = 0;
    if (!cfg.arcs) {
        double I;
        if (k1 == 0.0) {
            I = du * sqrt(fabs(k0) * fabs(L + h * k0));
        } else if (h == 0.0) {
            r.place = kIfPlaceES;
            double aa = fabs(kna), ab = fabs(knb);
            if (kna * knb >= 0.0) {
                r.place |= kIfKSame;
                double den = pow15(aa) + pow15(ab);
                I = den > 0.0 ? (2.0 / 3.0) * du * sqrt(L) * (aa * aa + aa * ab + ab * ab) / den : 0.0;
            } else {
                I = (2.0 / 3.0) * du * sqrt(L) * (pow15(aa) + pow15(ab)) / (aa + ab);
            }
        } else if (Newton && cfg.newton) {
            // the exact integral (counts) and the range's x in FP64 (placement)
            r.place = kIfNewton;
            const double hL = h / L;
            const double xa = -1.0 - 2.0 * (hL * kna), xb = -1.0 - 2.0 * (hL * knb);
            const double dx = -2.0 * hL * k1 * du;
            const double D = dens_int_d(xa, xb);
            uint64_t xw;
            memcpy(&xw, &xa, 8);
            r.len0 = bits_f((uint32_t)xw);
            r.dF0 = bits_f((uint32_t)(xw >> 32));
            r.dF = (float)dx;
            I = (dx != 0.0) ? fabs(D) * L * L / (4.0 * fabs(h * k1) * sqrt(fabs(h))) : 0.0;
        } else {
            r.place = kIfPlaceF;
            const double hL = h / L;
            const double hka = hL * kna, hkb = hL * knb;
            const double dx = -2.0 * hL * k1 * du;
            double d0, l0;
            const double dF = split_x_sum(make_xp(hka), make_xp(hkb), dx, cfg.xinc, &d0, &l0, &r.xbits);
            r.dF = (float)dF;
            r.dF0 = (float)d0;
            r.len0 = (float)l0;
            // I = |dF| / (4 |kappa'| |h|^1.5) = |dF/dx| L_r / (2 sqrt|h|)
            // (dx = -2 h k1 du / L, so |dF/dx| du L = |dF| L^2 / (2 |h k1|))
            I = (dx != 0.0) ? fabs(dF) * L * L / (4.0 * fabs(h * k1) * sqrt(fabs(h))) : 0.0;
        }
        r.n = ceil_count(I * cfg.inv_sqrt8tf);
    } else {
        double n_est = 0.0;
        if (k1 != 0.0) {
            double Lr = du * L;
            double kp = k1 / (L * L);
            n_est = Lr * cbrt(fabs(kp) * (1.0 + 0.4 * fabs(h * Lr * kp))) * cfg.cbrt_inv120tf;
        }
        r.n = ceil_count(n_est);
        double sweep = fmax(fabs(kna), fabs(knb)) * du * (1.0 / kHalfPi);
        uint32_t ns = ceil_count(sweep);
        r.n = ns > r.n ? ns : r.n;
    }
    r.ne = 0;
    r.alpha = 0.5f;
    if (reversed) {
        // evolute: density |s - s0|^-1/2 (Section 6); lines in both modes
        const double ra = sqrt(fabs(kna)), rb = sqrt(fabs(knb));
        double Iev = (k1 != 0.0 && ra + rb > 0.0) ? 2.0 * du * sqrt(fabs(k1) * L) / (ra + rb) : 0.0;
        r.ne = ceil_count(Iev * cfg.inv_sqrt8tf);
        if (ra + rb > 0.0) r.alpha = (float)(ra / (ra + rb));
    }
    return r;
}

// The range's items: the offset (or reversed offset) range, then for a
// reversed range its evolute bundle (the evolute twice and the connecting
// lines at ends that are piece ends).  Pa, Pb: the range's end points (exact
// piece ends or the shared cusp point).
template <class Sink>
SX_FN void range_put(Sink& k, const Cfg& cfg, const ES& es, double h, double ua, double ub, bool reversed,
                     bool end_a_piece, bool end_b_piece, V2 Pa, V2 Pb, const RangeRes& r) {
    const int D = h >= 0.0 ? 1 : -1;
    const int dir = reversed ? -D : D;
    const double du = ub - ua;
    {
        OffsetP p;
        p.ua = (float)ua; p.du = (float)du; p.len0 = r.len0; p.fh = (float)h;
        p.dF = r.dF; p.dF0 = r.dF0;
        p.Pax = Pa.x; p.Pay = Pa.y; p.Pbx = Pb.x; p.Pby = Pb.y;
        uint32_t hdr = kItemOffset | (dir < 0 ? kIfDirNeg : 0u) | (cfg.arcs ? kIfArcs : 0u) |
                       (es.pivot ? kIfPivot : 0u) | r.place | (r.xbits << kXBitsShift);
        k.put(hdr, r.n, cfg.K, p);
    }
    if (reversed) {
        const uint32_t nconn = (end_a_piece ? 1u : 0u) + (end_b_piece ? 1u : 0u);
        EvoluteP p;
        p.ua = (float)ua; p.du = (float)du;
        p.alpha = r.alpha;
        p.ne = r.ne;
        const V2 E0 = end_a_piece ? es.E0 : Pa;  // a range ending at a piece end: ua = 0, ub = 1
        const V2 E1 = end_b_piece ? es.E1 : Pb;
        p.E0x = E0.x; p.E0y = E0.y; p.E1x = E1.x; p.E1y = E1.y;
        p.Pax = Pa.x; p.Pay = Pa.y; p.Pbx = Pb.x; p.Pby = Pb.y;
        p.zero = 0u;
        uint32_t hdr = kItemEvolute | (D < 0 ? kIfDneg : 0u) | (es.pivot ? kIfPivot : 0u) |
                       (end_a_piece ? kIfEndA : 0u) | (end_b_piece ? kIfEndB : 0u);
        k.put(hdr, 2u * r.ne + 2u * nconn, cfg.K, p);
    }
}

template <class Sink>
SX_FN void emit_range(Sink& k, const Cfg& cfg, const ES& es, double h, double ua, double ub, bool reversed,
                      bool end_a_piece, bool end_b_piece, V2 Pa, V2 Pb) {
    range_put(k, cfg, es, h, ua, ub, reversed, end_a_piece, end_b_piece, Pa, Pb,
              range_count(cfg, es.k0, es.k1, es.L, h, ua, ub, reversed));
}

// One side (h = +w for side 0, -w for side 1) of a piece: rho = 1 + h kappa
// changes sign at most once along it (kappa is linear in u), splitting the
// side at the parallel-curve cusp tc into two ranges (reading G9).
struct SideGeo {
    double h, tc;
    bool split, rev1, rev2;  // two ranges; first / second range reversed (rho < 0)
    V2 P0, P1, Pc;           // side end points and the cusp point
};
SX_FN SideGeo side_geo(const ES& es, double w, int side) {
    SideGeo g;
    g.h = side == 0 ? w : -w;
    const double r0 = es_rhoL(es, g.h, 0.0), r1 = es_rhoL(es, g.h, 1.0);
    g.P0 = side == 0 ? es.P0A : es.P0B;
    g.P1 = side == 0 ? es.P1A : es.P1B;
    g.split = r0 * r1 < 0.0;
    g.tc = g.split ? r0 / (r0 - r1) : 1.0;
    g.Pc = g.split ? offset_point_f(es, (float)g.h, (float)g.tc) : g.P1;
    g.rev1 = g.split ? r0 < 0.0 : (r0 < 0.0 || r1 < 0.0);
    g.rev2 = r1 < 0.0;
    return g;
}

template <class Sink>
SX_FN void emit_sides(Sink& k, const Cfg& cfg, const ES& es, double w, bool fill) {
    for (int side = 0; side < (fill ? 1 : 2); side++) {
        const SideGeo g = side_geo(es, w, side);
        emit_range(k, cfg, es, g.h, 0.0, g.tc, g.rev1, true, !g.split, g.P0, g.Pc);
        if (g.split) emit_range(k, cfg, es, g.h, g.tc, 1.0, g.rev2, false, true, g.Pc, g.P1);
    }
}

// ----------------------------------------------------- joins and caps
SX_FN double round_step(double w, double tau_flat) {
    double c = 1.0 - tau_flat / w;
    c = fmin(fmax(c, -1.0), 1.0);
    return 2.0 * acos(c);
}
SX_FN uint32_t round_count(const Cfg& cfg, double w, double sweep) {
    return cfg.arcs ? ceil_count(fabs(sweep) * (1.0 / kHalfPi)) : ceil_count(fabs(sweep) / round_step(w, cfg.tau_flat));
}
SX_FN uint32_t inner_count(uint32_t inner) { return inner == kInPivot ? 2u : (inner == kInSmooth ? 1u : 0u); }
SX_FN uint32_t outer_count(uint32_t outer, uint32_t n_round) {
    return outer == kOutLine1 ? 1u : (outer == kOutLine2 ? 2u : (outer == kOutLine3 ? 3u : n_round));
}

template <class Sink>
SX_FN void put_join(Sink& k, const Cfg& cfg, uint32_t outer, uint32_t inner, bool inner_first, const JoinP& p) {
    uint32_t nrec = outer_count(outer, p.n_outer) + inner_count(inner);
    uint32_t hdr = kItemJoin | (cfg.arcs ? kIfArcs : 0u) | (inner_first ? kIfInnerFirst : 0u) | (outer << 16) |
                   (inner << 20);
    k.put(hdr, nrec, cfg.K, p);
}

template <class Sink>
SX_HD void emit_cap(Sink& k, const Cfg& cfg, int cap, D2 p, D2 u, double w, bool start) {
    D2 N = rnormal(u);
    D2 PA = p + N * w, PB = p + N * (-w);
    D2 from = start ? PB : PA, to = start ? PA : PB;
    D2 fwd = start ? d2(-u.x, -u.y) : u;
    JoinP jp = {};
    V2 f = f32(from), t = f32(to);
    jp.fromx = f.x; jp.fromy = f.y; jp.tox = t.x; jp.toy = t.y;
    const V2 fpc = f32(p);
    jp.px = fpc.x; jp.py = fpc.y;
    if (cap == kCapButt) {
        put_join(k, cfg, kOutLine1, kInNone, false, jp);
    } else if (cap == kCapSquare) {
        V2 a = f32(from + fwd * w), b = f32(to + fwd * w);
        jp.ax = a.x; jp.ay = a.y; jp.bx = b.x; jp.by = b.y;
        put_join(k, cfg, kOutLine3, kInNone, false, jp);
    } else {
        // the start angle only places FP32 points: FP32 is enough
        jp.a0 = atan2f((float)(from.y - p.y), (float)(from.x - p.x));
        jp.sweep = (float)kPi; jp.w = (float)w;
        jp.n_outer = round_count(cfg, w, kPi);
        put_join(k, cfg, kOutRound, kInNone, false, jp);
    }
}

template <class Sink>
SX_HD void emit_join(Sink& k, const Cfg& cfg, int join, double miter_limit, D2 p, D2 ta, D2 tb, double w) {
    D2 ua = unit(ta), ub = unit(tb);
    double cr = cross(ua, ub), dp = dot(ua, ub);
    D2 Na = rnormal(ua), Nb = rnormal(ub);
    JoinP jp = {};
    // nearly tangent-continuous: one straight line per side, no pivot lines
    if (dp > 0.0 && fabs(cr) < kSmoothJoin) {
        V2 a0 = offs(p, Na, w), a1 = offs(p, Nb, w), b0 = offs(p, Nb, -w), b1 = offs(p, Na, -w);
        jp.fromx = a0.x; jp.fromy = a0.y; jp.tox = a1.x; jp.toy = a1.y;
        jp.fx = b0.x; jp.fy = b0.y; jp.tx = b1.x; jp.ty = b1.y;
        put_join(k, cfg, kOutLine1, kInSmooth, false, jp);
        return;
    }
    bool outerA = !(cr < 0.0);
    double h_out = outerA ? w : -w, h_in = -h_out;
    D2 Oa = p + Na * h_out, Ob = p + Nb * h_out;
    V2 Ia = offs(p, Na, h_in), Ib = offs(p, Nb, h_in);
    D2 from = outerA ? Oa : Ob, to = outerA ? Ob : Oa;
    V2 ff = f32(from), ft = f32(to), fp = f32(p);
    jp.fromx = ff.x; jp.fromy = ff.y; jp.tox = ft.x; jp.toy = ft.y;
    V2 fi = outerA ? Ib : Ia, ti = outerA ? Ia : Ib;
    jp.fx = fi.x; jp.fy = fi.y; jp.px = fp.x; jp.py = fp.y; jp.tx = ti.x; jp.ty = ti.y;
    uint32_t outer = kOutLine1;
    if (join == kJoinRound) {
        double dphi = atan2(cr, dp);  // FP64: it decides the count
        jp.a0 = atan2f((float)(from.y - p.y), (float)(from.x - p.x));
        jp.sweep = (float)fabs(dphi); jp.w = (float)w;
        jp.n_outer = round_count(cfg, w, fabs(dphi));
        outer = kOutRound;
    } else if (join == kJoinMiter) {
        double crit = miter_limit * miter_limit * (1.0 + dp);
        if (crit >= 2.0) {
            V2 M = offs(p, Na + Nb, h_out / (1.0 + dp));
            jp.ax = M.x; jp.ay = M.y;
            outer = kOutLine2;
        }
    }
    // canonical order: side A's part first, then side B's
    put_join(k, cfg, outer, kInPivot, !outerA, jp);
}

// ------------------------------------------------------ record emission
// FP32 per-point work of one item chunk; records go to out at `dst`.
struct RecOut {
    float* out;
    uint64_t idx, end;
    uint32_t path;
    int arcs;
    float* stage;        // staging copy of records [lo, hi) (LDS), or null
    uint64_t lo, hi;
    SX_FN void put(V2 a, V2 b, float curv) {
        if (idx >= lo && idx < hi) {
            float* r = stage + (idx - lo) * (arcs ? 6 : 5);
            r[0] = a.x; r[1] = a.y; r[2] = b.x; r[3] = b.y;
            if (arcs) {
                r[4] = curv;
                reinterpret_cast<uint32_t*>(r)[5] = path;
            } else {
                reinterpret_cast<uint32_t*>(r)[4] = path;
            }
        } else if (idx < end) {
            if (arcs) {
                float* r = out + idx * 6;
                r[0] = a.x; r[1] = a.y; r[2] = b.x; r[3] = b.y; r[4] = curv;
                reinterpret_cast<uint32_t*>(r)[5] = path;
            } else {
                float* r = out + idx * 5;
                r[0] = a.x; r[1] = a.y; r[2] = b.x; r[3] = b.y;
                reinterpret_cast<uint32_t*>(r)[4] = path;
            }
        }
        idx++;
    }
    SX_FN void line(V2 a, V2 b) { put(a, b, 0.0f); }
    SX_FN void arc(V2 a, V2 b, float turn) {
        float c = len(b - a);
        float sh, ch;
        sincos_r(0.5f * turn, &sh, &ch);
        float curv = (c > 0.0f && turn != 0.0f) ? 2.0f * sh / c : 0.0f;
        put(a, b, curv);
    }
};

SX_FN ES es_from_f(const float* d, bool pivot) {
    ES es;
    es.fp0 = v2(d[0], d[1]);
    es.frot = v2(d[2], d[3]);
    es.fd = es.frot;
    es.fk0 = d[4]; es.fk1 = d[5]; es.fL = d[6]; es.fbase = d[7];
    es.pivot = pivot;
    return es;
}

// Walk state over the branch pieces of an offset range's density axis.
// Points are placed in increasing order, so the piece holding each point's
// share of F only moves forward; the pieces are produced one at a time.
struct XWalk {
    XPT<float> xa, xb;
    float dx;  // xb.x - xa.x, cancellation-free
    float cum, dF, dF0, len0;
    XSegT<float> seg;
    int j, nseg, kf;
    bool up;
    float acc_len;
};

// the branch breaks of f_approx and the increments between them, as floats
SX_FN float xbreak_f(int k) {
    return k == 0 ? -2.1f : (k == 1 ? -1.25f : (k == 2 ? -0.8f : (k == 3 ? 0.8f : (k == 4 ? 1.25f : 2.1f))));
}
struct XIncF {
    float v[5];
};
SX_FN float xinc_f(const XIncF& t, int k) {
    return k == 0 ? t.v[0] : (k == 1 ? t.v[1] : (k == 2 ? t.v[2] : (k == 3 ? t.v[3] : t.v[4])));
}

// Branch piece j of an offset range's density axis (the split the piece
// stage decided): from xa or the (j-1)-th break crossed to the j-th break
// or xb.  Increments: the first piece's and the total come from the FP64
// decisions, the pieces between breaks from the fixed increments, the last
// one is the rest.
SX_FN void walk_piece(XWalk& w, const XIncF& xi, int j) {
    const int nc = w.nseg - 1;
    const int kprev = w.up ? w.kf + j - 1 : w.kf - j + 1;
    const int knext = w.up ? w.kf + j : w.kf - j;
    const float a = (j == 0) ? w.xa.x : xbreak_f(kprev);
    const float e = (j < nc) ? xbreak_f(knext) : w.xb.x;
    w.seg.a = (j == 0) ? w.xa : bp_xp(a);
    // lengths from the decided first piece and the exact breaks; the last
    // piece is the rest of the cancellation-free total
    w.seg.len = (j == 0) ? w.len0 : ((j < nc) ? e - a : w.dx - w.acc_len);
    w.seg.dF = (j == 0) ? (nc ? w.dF0 : w.dF)
                        : ((j < nc) ? (w.up ? xinc_f(xi, kprev) : -xinc_f(xi, knext)) : w.dF - w.cum);
    w.seg.G = (w.seg.len != 0.0f) ? w.seg.dF / w.seg.len : 0.0f;
    w.seg.br = branch_of(absT(a + 0.5f * w.seg.len));
}

// Point placement data of an offset range, from the piece's FP32 spiral:
// the density axis of side h (the counts were decided in FP64; here the
// points only have to follow the same density), or the h = 0 curvatures.
struct Place {
    XWalk w;
    float kna, knb;
    float inv_n;  // 1 / (records of the range)
};
// Exact-density placement of a range (kIfNewton): its x interval and the
// exact integral over it, FP64.
struct PlaceN {
    double xa, dx, lo, hi, Fa, D;
};
SX_HD inline void place_newton_init(PlaceN& pn, const OffsetP& p) {
    const uint64_t xw = (uint64_t)f_bits(p.len0) | ((uint64_t)f_bits(p.dF0) << 32);
    memcpy(&pn.xa, &xw, 8);
    pn.dx = (double)p.dF;
    const double xb = pn.xa + pn.dx;
    pn.lo = fmin(pn.xa, xb);
    pn.hi = fmax(pn.xa, xb);
    pn.Fa = f_exact_d(pn.xa);
    pn.D = dens_int_d(pn.xa, xb);
}
// u of point i (0 < i < n): uniform in the exact integral, x from the
// Newton-refined inverse (a range of x length below 1e-9 has constant
// density: uniform in u)
SX_HD inline float offset_u_newton(const OffsetP& p, const PlaceN& pn, uint32_t i, uint32_t n) {
    const double f = (double)i / (double)n;
    double tau = f;
    if (fabs(pn.dx) >= 1e-9) {
        const double x = f_newton_inv_d(pn.Fa + pn.D * f, pn.lo, pn.hi);
        tau = fmin(fmax((x - pn.xa) / pn.dx, 0.0), 1.0);
    }
    return (float)((double)p.ua + (double)p.du * tau);
}
SX_HD inline void place_init(Place& pl, const ES& es, const OffsetP& p, uint32_t hdr, const XIncF& xi) {
    pl.kna = es.fk0 + es.fk1 * (p.ua - 0.5f);
    pl.knb = es.fk0 + es.fk1 * (p.ua + p.du - 0.5f);
    XWalk& w = pl.w;
    w.j = 0;
    w.nseg = 1;
    w.cum = 0.0f;
    w.acc_len = 0.0f;
    w.dF = 0.0f;
    if (hdr & kIfPlaceF) {
        w.xa = make_xp(p.fh * pl.kna / es.fL);
        w.xb = make_xp(p.fh * pl.knb / es.fL);
        w.dx = -2.0f * p.fh * es.fk1 * p.du / es.fL;
        w.dF = p.dF;
        w.dF0 = p.dF0;
        w.len0 = p.len0;
        const uint32_t xbits = (hdr >> kXBitsShift) & 127u;
        w.nseg = 1 + (int)(xbits & 7u);
        w.kf = (int)((xbits >> 3) & 7u);
        w.up = (xbits & 64u) != 0u;
        walk_piece(w, xi, 0);
    }
}

// u of point i (0 < i < n) of an offset range
SX_HD inline float offset_u(const OffsetP& p, uint32_t hdr, uint32_t i, uint32_t n, Place& pl, const XIncF& xi) {
    const float f = (float)i * pl.inv_n;
    float tau = f;
    if (hdr & kIfPlaceF) {
        // advance to the branch piece holding f * dF
        XWalk& w = pl.w;
        const float target = f * w.dF;
        while (w.j < w.nseg - 1 && !(fabsf(w.cum + w.seg.dF) >= fabsf(target))) {
            w.cum += w.seg.dF;
            w.acc_len += w.seg.len;
            w.j++;
            walk_piece(w, xi, w.j);
        }
        float fl = (w.nseg == 1) ? f : ((w.seg.dF != 0.0f) ? (target - w.cum) / w.seg.dF : 0.0f);
        fl = fminf(fmaxf(fl, 0.0f), 1.0f);
        const float phi = (w.seg.len != 0.0f) ? branch_inv_frac(w.seg, fl) : fl;
        tau = (w.nseg == 1 || w.dx == 0.0f) ? phi : (w.acc_len + phi * w.seg.len) / w.dx;
    } else if (hdr & kIfPlaceES) {
        // h = 0: uniform in |kappa|^1.5 (Section 2.2)
        const float aa = fabsf(pl.kna), ab = fabsf(pl.knb);
        const float a = sqrtf(aa), b = sqrtf(ab);
        const float Pa15 = aa * a, Pb15 = ab * b;  // |kappa|^1.5
        float kap;
        if (hdr & kIfKSame) {
            // with a = sqrt|kappa_a|, b = sqrt|kappa_b| and p^3 = a^3 +
            // f (b^3 - a^3), tau = (p^2 - a^2) / (b^2 - a^2); dividing
            // p^3 - a^3 by b^3 - a^3 gives it without cancellation (nearly
            // constant curvature): tau = f (a^2 + ab + b^2)(p + a) /
            // ((a^2 + ap + p^2)(a + b))
            const float p = cbrtf(Pa15 + f * (Pb15 - Pa15));
            const float den = (aa + a * p + p * p) * (a + b);
            tau = (den > 0.0f) ? f * (aa + a * b + ab) * (p + a) / den : f;
        } else {
            const float target = f * (Pa15 + Pb15);
            if (target <= Pa15) {
                const float t15 = Pa15 - target;
                kap = cbrtf(t15 * t15);
                tau = (aa - kap) / (aa + ab);
            } else {
                const float t15 = target - Pa15;
                kap = cbrtf(t15 * t15);
                tau = (aa + kap) / (aa + ab);
            }
        }
    }
    tau = fminf(fmaxf(tau, 0.0f), 1.0f);
    return p.ua + p.du * tau;
}

// One item chunk (header + payload words) into records; es: the slot's
// spiral (8 floats) for offset and evolute items.  Newton: the build that
// handles exact-density offset items (kIfNewton).
template <bool Newton = false>
SX_HD inline void emit_item(const uint32_t* it, const float* es_rec, const XIncF& xi, RecOut& o) {
    const ItemHdr h = *reinterpret_cast<const ItemHdr*>(it);
    const uint32_t* pw = it + kHdrWords;
    const uint32_t hdr = h.hdr;
    const uint32_t kind = hdr & 15u;
    const uint32_t nrec = item_n(hdr);
    const bool arcs = (hdr & kIfArcs) != 0;
    if (kind == kItemOffset) {
        const OffsetP p = *reinterpret_cast<const OffsetP*>(pw);
        const ES es = es_from_f(es_rec, (hdr & kIfPivot) != 0);
        Place pl;
        PlaceN pn;
        const bool newton = Newton && (hdr & kIfNewton) != 0;
        if (newton) place_newton_init(pn, p);
        else place_init(pl, es, p, hdr, xi);
        const uint32_t n = h.ntot;
        pl.inv_n = 1.0f / (float)n;
        const bool neg = (hdr & kIfDirNeg) != 0;
        // point k0 of the chunk
        float uprev;
        V2 prev;
        if (h.k0 == 0) {
            uprev = p.ua;
            prev = v2(p.Pax, p.Pay);
        } else {
            uprev = newton ? offset_u_newton(p, pn, h.k0, n) : offset_u(p, hdr, h.k0, n, pl, xi);
            prev = offset_point_f(es, p.fh, uprev);
        }
        for (uint32_t r = 0; r < nrec; r++) {
            const uint32_t i = h.k0 + r + 1;
            float u;
            V2 P;
            if (i == n) {
                u = p.ua + p.du;
                P = v2(p.Pbx, p.Pby);
            } else {
                u = newton ? offset_u_newton(p, pn, i, n) : offset_u(p, hdr, i, n, pl, xi);
                P = offset_point_f(es, p.fh, u);
            }
            if (!arcs) {
                if (!neg) o.line(prev, P); else o.line(P, prev);
            } else {
                const float turn = es_phi_f(es.fk0, es.fk1, u) - es_phi_f(es.fk0, es.fk1, uprev);
                if (!neg) o.arc(prev, P, turn); else o.arc(P, prev, -turn);
            }
            prev = P;
            uprev = u;
        }
    } else if (kind == kItemEvolute) {
        const EvoluteP p = *reinterpret_cast<const EvoluteP*>(pw);
        const ES es = es_from_f(es_rec, (hdr & kIfPivot) != 0);
        const uint32_t ne = p.ne;
        const bool Dneg = (hdr & kIfDneg) != 0;
        const V2 E0 = v2(p.E0x, p.E0y), E1 = v2(p.E1x, p.E1y), Pa = v2(p.Pax, p.Pay), Pb = v2(p.Pbx, p.Pby);
        const float inv_ne = 1.0f / (float)ne;
        auto ev = [&](uint32_t i) -> V2 {
            if (i == 0) return E0;
            if (i == ne) return E1;
            const float f = (float)i * inv_ne;
            const float tau = f * (2.0f * p.alpha + f * (1.0f - 2.0f * p.alpha));
            return evolute_point_f(es, p.ua + p.du * tau);
        };
        const bool ca = (hdr & kIfEndA) != 0;
        V2 cache_a = v2(0.0f, 0.0f);
        uint32_t cache_i = 0xffffffffu;
        for (uint32_t r = 0; r < nrec; r++) {
            const uint32_t k = h.k0 + r;
            if (k < 2u * ne) {
                const uint32_t s = k % ne;  // segment s of copy k / ne
                const V2 A = (cache_i == s) ? cache_a : ev(s);
                const V2 B = ev(s + 1);
                cache_a = B;
                cache_i = s + 1;
                if (!Dneg) o.line(A, B); else o.line(B, A);
            } else {
                const uint32_t c = k - 2u * ne;  // connecting lines: 2 at ua (if any), then 2 at ub
                if (ca && c < 2u) {
                    if (!Dneg) o.line(Pa, E0); else o.line(E0, Pa);
                } else {
                    if (!Dneg) o.line(E1, Pb); else o.line(Pb, E1);
                }
            }
        }
    } else {
        const JoinP p = *reinterpret_cast<const JoinP*>(pw);
        const uint32_t outer = (hdr >> 16) & 15u, inner = (hdr >> 20) & 3u;
        const bool inner_first = (hdr & kIfInnerFirst) != 0;
        const uint32_t no = outer_count(outer, p.n_outer), ni = inner_count(inner);
        const V2 from = v2(p.fromx, p.fromy), to = v2(p.tox, p.toy), A = v2(p.ax, p.ay), B = v2(p.bx, p.by);
        const V2 F = v2(p.fx, p.fy), Pp = v2(p.px, p.py), T = v2(p.tx, p.ty);
        for (uint32_t r = 0; r < nrec; r++) {
            const uint32_t k = h.k0 + r;
            const bool is_inner = inner_first ? (k < ni) : (k >= no);
            if (is_inner) {
                const uint32_t j = inner_first ? k : k - no;
                if (inner == kInSmooth) o.line(F, T);
                else if (j == 0) o.line(F, Pp);
                else o.line(Pp, T);
                continue;
            }
            const uint32_t j = inner_first ? k - ni : k;
            if (outer == kOutLine1) {
                o.line(from, to);
            } else if (outer == kOutLine2) {
                if (j == 0) o.line(from, A); else o.line(A, to);
            } else if (outer == kOutLine3) {
                if (j == 0) o.line(from, A); else if (j == 1) o.line(A, B); else o.line(B, to);
            } else {
                const uint32_t nr = p.n_outer;
                const float inv_nr = 1.0f / (float)nr;
                auto rp = [&](uint32_t q) -> V2 {
                    if (q == 0) return from;
                    if (q == nr) return to;
                    const float a = p.a0 + p.sweep * ((float)q * inv_nr);
                    float sn, cs;
                    sincos_r(a, &sn, &cs);
                    return v2(p.px + p.w * cs, p.py + p.w * sn);
                };
                const V2 a = rp(j), b = rp(j + 1);
                if (arcs) o.arc(a, b, p.sweep / (float)nr); else o.line(a, b);
            }
        }
    }
}

// --------------------------------------------------------- segments
// A segment in coordinates relative to its world start point P0w: the
// control points' offsets D1..D3 are transformed differences of the input
// points, so sub-piece chords keep full relative precision wherever the
// segment sits on the canvas.
struct Seg {
    D2 P0w, P3w;      // world end points (bit-identical with the neighbours')
    D2 D1, D2_, D3;   // world offsets of the elevated control points from P0w
    D2 A2, B2, C3;    // D2 - 2 D1, D3 - 2 D2 + D1, D3 - 3 D2 + 3 D1
    D2 ts, te;        // end tangents (transformed raw differences)
    double w, lpoly;
    bool fill;        // one side at offset 0 (the path itself)
};

struct Tan {
    D2 dir;
    double mag;
};

// B(t) - P0
SX_FN D2 cubic_rel(const Seg& s, double t) {
    double mt = 1.0 - t;
    double b = 3.0 * mt * mt * t, c = 3.0 * mt * t * t, d = t * t * t;
    return d2(b * s.D1.x + c * s.D2_.x + d * s.D3.x, b * s.D1.y + c * s.D2_.y + d * s.D3.y);
}
SX_FN D2 cubic_world(const Seg& s, double t) {
    if (t == 0.0) return s.P0w;
    if (t == 1.0) return s.P3w;
    return s.P0w + cubic_rel(s, t);
}
// q = B'/3
SX_FN D2 cubic_q(const Seg& s, double t) {
    double mt = 1.0 - t;
    D2 a = s.D1, b = s.D2_ - s.D1, c = s.D3 - s.D2_;
    double wa = mt * mt, wb = 2.0 * t * mt, wc = t * t;
    return d2(wa * a.x + wb * b.x + wc * c.x, wa * a.y + wb * b.y + wc * c.y);
}
// B(t0 + dt) - B(t0) by the (terminating) Taylor expansion of the cubic
SX_FN D2 cubic_chord(const Seg& s, double t0, double dt, D2 q0) {
    double mt = 1.0 - t0;
    D2 b2 = d2(mt * s.A2.x + t0 * s.B2.x, mt * s.A2.y + t0 * s.B2.y);
    double e1 = 3.0 * dt, e2 = 3.0 * dt * dt, e3 = dt * dt * dt;
    return d2(e1 * q0.x + e2 * b2.x + e3 * s.C3.x, e1 * q0.y + e2 * b2.y + e3 * s.C3.y);
}
SX_FN Tan sample_q(const Seg& s, double t) {
    if (t == 0.0) return Tan{s.ts, len(s.D1)};
    if (t == 1.0) return Tan{s.te, len(s.D3 - s.D2_)};
    D2 q = cubic_q(s, t);
    double ql = len(q);
    if (ql < kEpsQ * s.lpoly) {
        q = cubic_q(s, (t + kDeltaT < 1.0) ? t + kDeltaT : t - kDeltaT);
        ql = len(q);
    }
    return Tan{q, ql};
}

// ------------------------------------------------------ segment fetch
// linear part of the transform applied to a difference vector (FP64 from FP32)
SX_FN D2 xf_vec(const float* X, double dx, double dy) {
    return d2((double)X[0] * dx + (double)X[2] * dy, (double)X[1] * dx + (double)X[3] * dy);
}
SX_FN D2 xf_apply(const float* X, float x, float y) {
    // x' = a x + c y + e, y' = b x + d y + f
    return d2((double)X[0] * x + (double)X[2] * y + (double)X[4], (double)X[1] * x + (double)X[3] * y + (double)X[5]);
}


struct SceneView {
    const uint8_t* tags;
    const float2* pts;
    const StyleD* styles;
    const float* xforms;  // 6 floats each
    const uint32_t* path_map;
    const uint32_t* mon;  // 4 x mon_stride SoA (point offset, path, style, transform)
    uint32_t n_tags, n_pts, n_styles, n_xforms, n_paths;
    uint32_t mon_stride;  // n_tags rounded up to a multiple of 4 (16-byte aligned rows)
};
// row stride of the monoid SoA for n tags
SX_FN uint32_t mon_stride_of(uint32_t n) { return (n + 3u) & ~3u; }

enum { kTagInvalid = 0, kTagSegment = 1, kTagMarker = 2 };

// What one tag's work needs besides the segment geometry.
struct TagInfo {
    uint32_t kind, tag, off;
    const float* X;  // transform
    double w;        // half-width in output units
    float miter;
    int join, scap, ecap;
    bool line;
    bool fill;       // one side at offset 0, no join or cap
};

// Input path id of tag i (all ones for a tag outside every path).
SX_FN uint32_t path_of(const SceneView& sv, uint32_t i) {
    const uint32_t pi = sv.mon[(size_t)sv.mon_stride + i];
    return pi < sv.n_paths ? sv.path_map[pi] : 0xffffffffu;
}

// Segment fetch and degree elevation (Section 8.1) of tag i; bounds derived
// from the monoids are checked (a consistent scan never trips them).
// The kind of tag i (kTagInvalid when its indices or its points, or for a
// segment the next tag's points, fall outside the scene), and whether a
// segment is a line: what fetch_tag decides, without loading the segment.
SX_HD inline int tag_kind(const SceneView& sv, uint32_t i, bool& line) {
    line = false;
    const uint32_t tag = sv.tags[i];
    const uint32_t off = sv.mon[i];
    const uint32_t sty = sv.mon[2 * (size_t)sv.mon_stride + i];
    const uint32_t xfi = sv.mon[3 * (size_t)sv.mon_stride + i];
    const uint32_t need = (tag & kTagEnd) ? 3u : (tag & kTagCount) + 1u;
    if (sty >= sv.n_styles || xfi >= sv.n_xforms || (size_t)off + need > sv.n_pts) return kTagInvalid;
    if (tag & kTagEnd) return kTagMarker;
    if (i + 1 >= sv.n_tags) return kTagInvalid;
    const uint32_t t1 = sv.tags[i + 1];
    const uint32_t need1 = (t1 & kTagEnd) ? 3u : (t1 & kTagCount) + 1u;
    if ((size_t)sv.mon[i + 1] + need1 > sv.n_pts) return kTagInvalid;
    line = (tag & kTagCount) == 1u;
    return kTagSegment;
}

SX_HD inline void fetch_tag(const SceneView& sv, uint32_t i, TagInfo& ti, Seg& s) {
    ti.fill = false;
    ti.kind = tag_kind(sv, i, ti.line);
    if (ti.kind == kTagInvalid) return;
    const uint32_t tag = sv.tags[i];
    const uint32_t off = sv.mon[i];
    const uint32_t sty = sv.mon[2 * (size_t)sv.mon_stride + i];
    const uint32_t xfi = sv.mon[3 * (size_t)sv.mon_stride + i];
    const StyleD st = sv.styles[sty];
    const float* X = sv.xforms + 6 * (size_t)xfi;
    const double scale = sqrt(fabs((double)X[0] * X[3] - (double)X[1] * X[2]));
    ti.tag = tag;
    ti.off = off;
    ti.X = X;
    ti.w = (double)st.half_width * scale;
    ti.miter = st.miter_limit;
    ti.join = st.packed & 0xff;
    ti.scap = (st.packed >> 8) & 0xff;
    ti.ecap = (st.packed >> 16) & 0xff;
    ti.fill = (st.packed & kStyleFill) != 0u;
    if (ti.kind == kTagMarker) return;
    const float2* D = sv.pts + off;
    const int c = tag & kTagCount;
    // the segment's c + 1 points, loaded without a runtime-indexed array
    // (indices clamped to the segment, so every load stays in it)
    const float2 r0 = D[0], r1 = D[1], r2 = D[c >= 2 ? 2 : 1], r3 = D[c >= 3 ? 3 : c];
    const float2 rc = (c == 1) ? r1 : ((c == 2) ? r2 : r3);
    s.w = ti.w;
    s.fill = ti.fill;
    s.P0w = xf_apply(X, r0.x, r0.y);
    s.P3w = xf_apply(X, rc.x, rc.y);
    // transformed differences r_j - r_0
    const D2 e0 = xf_vec(X, (double)r1.x - r0.x, (double)r1.y - r0.y);
    const D2 e1 = xf_vec(X, (double)r2.x - r0.x, (double)r2.y - r0.y);
    const D2 e2 = xf_vec(X, (double)r3.x - r0.x, (double)r3.y - r0.y);
    if (c == 1) {
        s.D1 = e0 * (1.0 / 3.0);
        s.D2_ = e0 * (2.0 / 3.0);
        s.D3 = e0;
    } else if (c == 2) {
        s.D1 = e0 * (2.0 / 3.0);
        s.D2_ = e1 + (e0 - e1) * (2.0 / 3.0);
        s.D3 = e1;
    } else {
        s.D1 = e0;
        s.D2_ = e1;
        s.D3 = e2;
    }
    s.A2 = s.D2_ - s.D1 * 2.0;
    s.B2 = s.D3 - s.D2_ * 2.0 + s.D1;
    s.C3 = s.D3 - s.D2_ * 3.0 + s.D1 * 3.0;
    // end tangents: the first nonzero difference from each end (r_c - r_{c-1-j})
    const float2 q0 = (c == 1) ? r0 : ((c == 2) ? r1 : r2);  // r_{c-1}
    const float2 q1 = (c == 2) ? r0 : r1;                    // r_{c-2}
    const D2 ce0 = xf_vec(X, (double)rc.x - q0.x, (double)rc.y - q0.y);
    const D2 ce1 = xf_vec(X, (double)rc.x - q1.x, (double)rc.y - q1.y);
    const D2 ce2 = xf_vec(X, (double)rc.x - r0.x, (double)rc.y - r0.y);
    const D2 one = d2(1.0, 0.0);
    s.ts = !is_zero(e0) ? e0 : (c >= 2 && !is_zero(e1)) ? e1 : (c >= 3 && !is_zero(e2)) ? e2 : one;
    s.te = !is_zero(ce0) ? ce0 : (c >= 2 && !is_zero(ce1)) ? ce1 : (c >= 3 && !is_zero(ce2)) ? ce2 : one;
    s.lpoly = len(s.D1) + len(s.D2_ - s.D1) + len(s.D3 - s.D2_);
}

// ------------------------------------------- Algorithm 2: the bisection
// One candidate piece [t0, t0 + dt] of the segment: its chord, end angles and
// the accept test (Section 7.1 estimate with reading G2, the hodograph test
// of reading G29; a line is its own piece and skips the test).
struct Trial {
    D2 chord;
    double cl, th0, th1;
    bool ok;
};
SX_HD inline Trial trial(const Seg& s, const Cfg& cfg, bool line, double dt, const Tan& last_q, const Tan& next_q,
                         D2 chord) {
    Trial r;
    r.chord = chord;
    r.cl = len(chord);
    r.th0 = 0.0;
    r.th1 = 0.0;
    r.ok = true;
    if (line) return r;
    // the end angles, and their sines and cosines from the same cross and
    // dot products (a zero vector gives angle 0)
    const double x0 = cross(last_q.dir, chord), y0 = dot(last_q.dir, chord);
    const double x1 = cross(chord, next_q.dir), y1 = dot(chord, next_q.dir);
    r.th0 = atan2(x0, y0);
    r.th1 = atan2(x1, y1);
    const double h0 = sqrt(x0 * x0 + y0 * y0), h1 = sqrt(x1 * x1 + y1 * y1);
    const double r0 = 1.0 / h0, r1 = 1.0 / h1, rcl = dt / r.cl;
    const double sn0 = h0 > 0.0 ? x0 * r0 : 0.0, c0 = h0 > 0.0 ? y0 * r0 : 1.0;
    const double sn1 = h1 > 0.0 ? x1 * r1 : 0.0, c1 = h1 > 0.0 ? y1 * r1 : 1.0;
    const double d0 = last_q.mag * rcl, d1 = next_q.mag * rcl;
    const double est = fit_estimate_sc(r.th0, r.th1, sn0, c0, sn1, c1, d0, d1);
    const double err = cfg.paper_fit ? est * r.cl : est * (r.cl + kFitK * s.w) * kFitS;
    const bool len_ok = r.cl > 0.0;
    bool hodo_ok = true;
    {
        const double ma = last_q.mag * dt, mc = next_q.mag * dt;
        const D2 a = unit(last_q.dir) * ma, c = unit(next_q.dir) * mc;
        const D2 b = chord - a - c;
        // a middle vector that is zero up to rounding leaves only the turn from a to c (< pi)
        if (ma > 0.0 && mc > 0.0 && len(b) > 1e-9 * (ma + mc)) hodo_ok = (dot(a, b) * mc + dot(b, c) * ma) > 0.0;
    }
    r.ok = len_ok && hodo_ok && (err <= cfg.tau_fit);
    return r;
}

// The bisection state of one segment: the two-word stack (t0_u, depth with
// dt = 2^-depth) and the samples at t0.
struct Bisect {
    uint32_t t0_u, depth;
    Tan last_q;
    D2 last_qtrue;
};
SX_FN void bisect_init(Bisect& b, const Seg& s) {
    b.t0_u = 0;
    b.depth = 0;
    b.last_q = sample_q(s, 0.0);
    b.last_qtrue = s.D1;
}
SX_FN double depth_dt(uint32_t depth) { return ldexp(1.0, -(int)depth); }  // 2^-depth, exact

// One trial of the bisection.  Returns true when [t0, t0 + dt] is accepted
// (its t0_u and depth are reported before the stack pops); *done is set when
// the segment is fully covered.
SX_HD inline bool bisect_step(Bisect& b, const Seg& s, const Cfg& cfg, bool line, uint32_t& acc_t0u,
                              uint32_t& acc_depth, bool& acc_pivot, bool& done) {
    const double dt = depth_dt(b.depth);
    const double t0 = (double)b.t0_u * dt;
    const double t1 = t0 + dt;
    const Tan next_q = line ? b.last_q : sample_q(s, t1);
    const D2 chord = line ? s.D3 : cubic_chord(s, t0, dt, b.last_qtrue);
    const Trial tr = trial(s, cfg, line, dt, b.last_q, next_q, chord);
    const bool forced = b.depth >= (uint32_t)kMaxDepth;
    done = false;
    if (tr.ok || forced) {
        acc_t0u = b.t0_u;
        acc_depth = b.depth;
        acc_pivot = !tr.ok;
        // pop: count trailing zeros
        b.t0_u += 1;
        const uint32_t sh = __builtin_ctz(b.t0_u);
        b.t0_u >>= sh;
        b.depth -= sh;
        b.last_q = next_q;
        b.last_qtrue = (t1 == 1.0) ? s.D3 - s.D2_ : cubic_q(s, t1);
        done = (double)b.t0_u * depth_dt(b.depth) == 1.0;
        return true;
    }
    b.t0_u *= 2;
    b.depth += 1;
    return false;
}

// The accepted piece [t0, t0 + 2^-depth] of the segment (accepted by the
// fit, or only at the depth cap: a pivot): the same chord and end angles as
// in the bisection and its Euler spiral (Appendix A; a pivot for reading
// G28), whose FP32 record goes to the slot's row of the spiral table;
// emit_piece adds both parallel-curve sides.
template <class Sink>
SX_HD void piece_es(Sink& k, const Cfg& cfg, const Seg& s, bool line, uint32_t t0_u, uint32_t depth, bool pivot,
                    ES& es) {
    const double dt = depth_dt(depth);
    const double t0 = (double)t0_u * dt;
    const double t1 = t0 + dt;
    const Tan last_q = sample_q(s, t0);
    const D2 last_qtrue = (t0 == 0.0) ? s.D1 : cubic_q(s, t0);
    const Tan next_q = line ? last_q : sample_q(s, t1);
    const D2 chord = line ? s.D3 : cubic_chord(s, t0, dt, last_qtrue);
    Trial tr;
    tr.chord = chord;
    tr.cl = len(chord);
    tr.th0 = 0.0;
    tr.th1 = 0.0;
    if (!line && !pivot) {
        tr.th0 = atan2(cross(last_q.dir, chord), dot(last_q.dir, chord));
        tr.th1 = atan2(cross(chord, next_q.dir), dot(chord, next_q.dir));
    }
    if constexpr (Sink::kStats) k.st[kStPieces]++;
    es.pivot = pivot;
    es.p0 = cubic_world(s, t0);
    es.p1 = cubic_world(s, t1);
    es.n0 = rnormal(unit(last_q.dir));
    es.n1 = rnormal(unit(next_q.dir));
    double c, base;
    D2 rot = d2(0.0, 0.0);
    if (line) {
        es.k0 = 0.0;
        es.k1 = 0.0;
        c = 1.0;
        rot = chord;
        base = atan2(rot.y, rot.x);
    } else if (pivot) {
        es.k0 = atan2(cross(last_q.dir, next_q.dir), dot(last_q.dir, next_q.dir));
        es.k1 = 0.0;
        c = es_chord(0.5 * es.k0, 0.5 * es.k0);
        base = atan2(last_q.dir.y, last_q.dir.x) + 0.5 * es.k0;
    } else {
        es.k0 = tr.th0 + tr.th1;
        es.k1 = es_k1(tr.th0, tr.th1);
        c = es_chord(tr.th0, tr.th1);
        // rotation chord / Z(1) in FP32: it only places the per-point work
        const V2 z1 = es_integral1_f((float)es.k0, (float)es.k1);
        const V2 ch = f32(chord);
        const float rzz = 1.0f / (z1.x * z1.x + z1.y * z1.y);
        const V2 fr = v2((ch.x * z1.x + ch.y * z1.y) * rzz, (ch.y * z1.x - ch.x * z1.y) * rzz);
        rot = d2(fr.x, fr.y);
        base = (double)atan2f(fr.y, fr.x);
    }
    if (!(c > kCMin)) c = kCMin;
    es.L = tr.cl / c;
    es.fp0 = f32(es.p0);
    es.fd = f32(es.p1 - es.p0);
    es.frot = f32(rot);
    es.fk0 = (float)es.k0;
    es.fk1 = (float)es.k1;
    es.fL = (float)es.L;
    es.fbase = (float)base;
    es_ends(es, s.w);
    set_es_f(es, k.es_tab + 8 * (size_t)k.slot);
}
template <class Sink>
SX_HD void emit_piece(Sink& k, const Cfg& cfg, const Seg& s, bool line, uint32_t t0_u, uint32_t depth, bool pivot) {
    ES es;
    piece_es(k, cfg, s, line, t0_u, depth, pivot, es);
    emit_sides(k, cfg, es, s.w, s.fill);
}

// The tail of tag i: the start cap of an open subpath (stroke cap marker),
// or the join with tag i + 1 / the end cap of a segment (Algorithm 1);
// nothing for a fill.
template <class Sink>
SX_HD void emit_tail(Sink& k, const Cfg& cfg, const SceneView& sv, uint32_t i, const TagInfo& ti, const Seg& s) {
    if (ti.fill) return;  // a fill has no joins or caps
    if (ti.kind == kTagMarker) {
        if (!(ti.tag & kTagClosed)) {
            const float2* D = sv.pts + ti.off;
            const float2 a = D[1], bb = D[2];
            const D2 ps = xf_apply(ti.X, a.x, a.y);
            D2 dir = xf_vec(ti.X, (double)bb.x - a.x, (double)bb.y - a.y);
            if (is_zero(dir)) dir = d2(1.0, 0.0);
            emit_cap(k, cfg, ti.scap, ps, unit(dir), ti.w, true);
        }
        return;
    }
    if (ti.kind != kTagSegment) return;
    const uint32_t nt = sv.tags[i + 1];
    const D2 pend = s.P3w;
    if ((nt & kTagEnd) && !(nt & kTagClosed)) {
        emit_cap(k, cfg, ti.ecap, pend, unit(s.te), ti.w, false);
        return;
    }
    const float* X = ti.X;
    const float2* Dn = sv.pts + sv.mon[i + 1];
    D2 tb;
    if (nt & kTagEnd) {
        const float2 a = Dn[1], bb = Dn[2];
        tb = xf_vec(X, (double)bb.x - a.x, (double)bb.y - a.y);
        if (is_zero(tb)) tb = d2(1.0, 0.0);
    } else {
        // the next segment's start tangent: its first nonzero difference
        const int cn = nt & kTagCount;
        const float2 r0 = Dn[0], r1 = Dn[1], r2 = Dn[cn >= 2 ? 2 : 1], r3 = Dn[cn >= 3 ? 3 : cn];
        const D2 c0 = xf_vec(X, (double)r1.x - r0.x, (double)r1.y - r0.y);
        const D2 c1 = xf_vec(X, (double)r2.x - r0.x, (double)r2.y - r0.y);
        const D2 c2 = xf_vec(X, (double)r3.x - r0.x, (double)r3.y - r0.y);
        tb = !is_zero(c0) ? c0 : (cn >= 2 && !is_zero(c1)) ? c1 : (cn >= 3 && !is_zero(c2)) ? c2 : d2(1.0, 0.0);
    }
    emit_join(k, cfg, ti.join, (double)ti.miter, pend, s.te, tb, ti.w);
}

// The single pass of one tag (Section 8.1's organisation): its bisection,
// each accepted piece's parallel curves as soon as it is accepted, then its
// join or cap, all into one sink.  Shared by the single-pass kernel and its
// host build.
template <class Sink>
SX_HD void soup_tag(Sink& k, const Cfg& cfg, const SceneView& sv, uint32_t i) {
    TagInfo ti;
    Seg sg;
    fetch_tag(sv, i, ti, sg);
    if (ti.kind == kTagSegment) {
        Bisect bs;
        bisect_init(bs, sg);
        for (;;) {
            uint32_t t0u = 0, depth = 0;
            bool done = false, pivot = false;
            if (bisect_step(bs, sg, cfg, ti.line, t0u, depth, pivot, done)) {
                emit_piece(k, cfg, sg, ti.line, t0u, depth, pivot);
                if (done) break;
            }
        }
    }
    emit_tail(k, cfg, sv, i, ti, sg);
}

// ------------------------------------------------------------ slots
// Every tag owns (pieces + 1) consecutive *slots* in canonical order: one
// per accepted piece in t order, then its tail (join / cap).  A slot code is
// (t0_u << 6) | pivot << 5 | depth for a piece (bit 31 marks the single
// piece of a line segment, reading G32), kSlotTail for the tail.
constexpr uint32_t kSlotTail = 0xffffffffu;
constexpr uint32_t kCodeLine = 0x80000000u;
struct Slot {
    uint32_t tag, code;
};
SX_FN uint32_t slot_code(uint32_t t0_u, uint32_t depth, bool pivot) {
    return (t0_u << 6) | (pivot ? 32u : 0u) | depth;
}
SX_FN uint32_t code_t0u(uint32_t code) { return (code & ~kCodeLine) >> 6; }
SX_FN bool code_line(uint32_t code) { return code != kSlotTail && (code & kCodeLine) != 0u; }
SX_FN uint32_t code_depth(uint32_t code) { return code & 31u; }
SX_FN bool code_pivot(uint32_t code) { return (code & 32u) != 0u; }


// ------------------------------------------------------------- dashing
// Dash patterns (Sections 1 and 9.3) cut a stroke's subpaths into dashes,
// each then stroked as an open subpath.  Lengths are measured in the path's
// own units by 16 panels of 8-node Gauss-Legendre of |B'(t)| and kept on a
// grid of 2^-24 units (64-bit integers), so prefix sums over a subpath are
// exact and order-free; a dash boundary inside a segment sits at the
// parameter where the panels' partial integral reaches it (Newton steps kept
// inside the panel), and the dash's part of the segment is the segment
// restricted to that parameter range (blossom), rounded to FP32.
constexpr int kDashPanels = 16;
constexpr double kDashGrid = 16777216.0;  // 2^24
// per style entry: pattern values pat[off .. off + n) (n even; 0 = solid),
// their sum and the offset, on the grid
struct DashDesc {
    uint32_t off, n;
    int64_t period, phase;
};

// |B'(t)| of the degree-C Bezier P[0..C] (the degree a template parameter,
// so that every array of the dashing code is indexed statically)
template <int C>
SX_FN double bez_speed_c(const D2* P, double t) {
    const double mt = 1.0 - t;
    double dx, dy;
    if (C == 1) {
        dx = P[1].x - P[0].x;
        dy = P[1].y - P[0].y;
    } else if (C == 2) {
        dx = 2.0 * (mt * (P[1].x - P[0].x) + t * (P[2].x - P[1].x));
        dy = 2.0 * (mt * (P[1].y - P[0].y) + t * (P[2].y - P[1].y));
    } else {
        const double a = mt * mt, b = 2.0 * t * mt, e = t * t;
        dx = 3.0 * (a * (P[1].x - P[0].x) + b * (P[2].x - P[1].x) + e * (P[3].x - P[2].x));
        dy = 3.0 * (a * (P[1].y - P[0].y) + b * (P[2].y - P[1].y) + e * (P[3].y - P[2].y));
    }
    return hypot(dx, dy);
}
// 8-node Gauss-Legendre of |B'| over [a, b]
template <int C>
SX_FN double speed_gl8_c(const D2* P, double a, double b) {
    const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const double m = 0.5 * (a + b), h = 0.5 * (b - a);
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++) sum += gw[i] * (bez_speed_c<C>(P, m - h * gx[i]) + bez_speed_c<C>(P, m + h * gx[i]));
    return sum * h;
}
// arc length (sum of the panels' integrals, panel[k] each)
template <int C>
SX_FN double dash_len_c(const D2* P, double* panel) {
    double total = 0.0;
#pragma unroll
    for (int k = 0; k < kDashPanels; k++) {
        panel[k] = speed_gl8_c<C>(P, (double)k / kDashPanels, (double)(k + 1) / kDashPanels);
        total += panel[k];
    }
    return total;
}
// the same for the degree c of a tag (1, 2 or 3; P[0..c])
SX_HD inline double dash_len_d(const D2* P, int c, double* panel) {
    if (c == 1) return dash_len_c<1>(P, panel);
    if (c == 2) return dash_len_c<2>(P, panel);
    return dash_len_c<3>(P, panel);
}
SX_FN int64_t dash_fix(double v) { return (int64_t)llround(v * kDashGrid); }
SX_FN int64_t floor_div64(int64_t a, int64_t b) {
    const int64_t q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
// parameter where the panels' partial integral reaches s
template <int C>
SX_FN double dash_t_c(const D2* P, const double* panel, double s) {
    // the panel holding s: the first k (< 15) with acc + panel[k] > s, where
    // acc sums the panels before it (unrolled: the panels stay in registers)
    double acc = 0.0, pk = panel[kDashPanels - 1];
    int k = kDashPanels - 1;
    bool found = false;
#pragma unroll
    for (int q = 0; q < kDashPanels - 1; q++) {
        if (!found) {
            if (acc + panel[q] <= s) {
                acc += panel[q];
            } else {
                found = true;
                k = q;
                pk = panel[q];
            }
        }
    }
    double lo = (double)k / kDashPanels, hi = (double)(k + 1) / kDashPanels;
    const double t0 = lo, rest = s - acc;
    double t = lo + (hi - lo) * fmin(fmax(pk > 0.0 ? rest / pk : 0.5, 0.0), 1.0);
    for (int it = 0; it < 60; it++) {
        const double g = speed_gl8_c<C>(P, t0, t) - rest;
        if (g == 0.0) break;
        if (g < 0.0) lo = t;
        else hi = t;
        const double d = bez_speed_c<C>(P, t);
        double tn = d > 0.0 ? t - g / d : 0.5 * (lo + hi);
        if (!(tn >= lo && tn <= hi)) tn = 0.5 * (lo + hi);
        // converged: the step is down to a few ulps of t <= 1
        if (fabs(tn - t) <= 4.0e-16 || !(hi > lo)) {
            t = tn;
            break;
        }
        t = tn;
    }
    return t;
}
// A dash's part of one segment: its control points (the segment restricted
// to [ta, tb] by blossoming, rounded to FP32; the segment's own end points
// where ta = 0 or tb = 1), whether it has extent (a control point differs
// from its start; a part without extent is left out, as the encoding
// leaves out zero-length segments) and the first such point.
struct DashPart {
    float2 p[4];
    bool extent;
    float2 dv;
};
template <int C>
SX_FN DashPart dash_part_c(const float2* Dq, const double* pan, int64_t Q0, int64_t Q1, int64_t lo, int64_t hi) {
    D2 P[C + 1];
#pragma unroll
    for (int j = 0; j <= C; j++) P[j] = d2((double)Dq[j].x, (double)Dq[j].y);
    const double ta = lo == Q0 ? 0.0 : dash_t_c<C>(P, pan, (double)(lo - Q0) / kDashGrid);
    double tb = hi == Q1 ? 1.0 : dash_t_c<C>(P, pan, (double)(hi - Q0) / kDashGrid);
    if (tb < ta) tb = ta;
    DashPart r;
#pragma unroll
    for (int j = 0; j <= C; j++) {
        D2 q[C + 1];
#pragma unroll
        for (int l = 0; l <= C; l++) q[l] = P[l];
#pragma unroll
        for (int l = 0; l < C; l++) {
            const double u = (l < C - j) ? ta : tb;
#pragma unroll
            for (int m = 0; m < C - l; m++) q[m] = q[m] * (1.0 - u) + q[m + 1] * u;
        }
        D2 v = q[0];
        if (j == 0 && ta == 0.0) v = P[0];
        if (j == C && tb == 1.0) v = P[C];
        r.p[j] = make_float2((float)v.x, (float)v.y);
    }
    r.extent = false;
    r.dv = make_float2(r.p[0].x + 1.0f, r.p[0].y);
#pragma unroll
    for (int j = 1; j <= C; j++)
        if (!r.extent && !(r.p[j].x == r.p[0].x && r.p[j].y == r.p[0].y)) {
            r.extent = true;
            r.dv = r.p[j];
        }
    return r;
}
// A part of grid length lp of a segment of grid length ls whose control
// points lie within +-M cannot have rounded control points that all
// coincide when lp is longer than their control polygon could then be
// (3 legs of at most a diagonal of the 2^-23 M rounding box: under 8 x
// 2^-22 M), plus the arc-length rule's own error (below 2e-3 ls even
// beside a cusp) and 2^-20: such a part has extent without computing it.
// Both dashing passes take the same decision, so their counts agree.
SX_FN bool dash_surely_extent(int64_t lp, int64_t ls, double M) {
    return (double)lp / kDashGrid > 8.0 * M * 0x1p-22 + 2e-3 * ((double)ls / kDashGrid) + 0x1p-20;
}
template <int C>
SX_FN double dash_max_coord(const float2* D) {
    double m = 0.0;
#pragma unroll
    for (int j = 0; j <= C; j++) m = fmax(m, fmax(fabs((double)D[j].x), fabs((double)D[j].y)));
    return m;
}
SX_HD inline double dash_max_coord_d(int c, const float2* D) {
    if (c == 1) return dash_max_coord<1>(D);
    if (c == 2) return dash_max_coord<2>(D);
    return dash_max_coord<3>(D);
}
// the same for the degree c of a tag
SX_HD inline DashPart dash_part_d(int c, const float2* Dq, const double* pan, int64_t Q0, int64_t Q1, int64_t lo,
                                  int64_t hi) {
    if (c == 1) return dash_part_c<1>(Dq, pan, Q0, Q1, lo, hi);
    if (c == 2) return dash_part_c<2>(Dq, pan, Q0, Q1, lo, hi);
    return dash_part_c<3>(Dq, pan, Q0, Q1, lo, hi);
}
// The dash intervals [a, b) (clipped to the subpath [0, Stot]) meeting the
// segment (S0, S1], in order: f(lo, hi, a, b) for each, lo < hi.
// Only the pattern periods m in [m_begin, m_end] are visited (a chunk of the
// segment's work; the whole span is [dash_m_lo, dash_m_hi]).
SX_FN int64_t dash_m_lo(int64_t S0, int64_t period, int64_t phase) { return floor_div64(S0 + phase, period) - 1; }
SX_FN int64_t dash_m_hi(int64_t S1, int64_t period, int64_t phase) { return floor_div64(S1 + phase, period) + 1; }
template <class F>
SX_HD void dash_parts(int64_t S0, int64_t S1, int64_t Stot, const int64_t* pat, uint32_t n, int64_t period,
                      int64_t phase, int64_t m_begin, int64_t m_end, F f) {
    const int64_t mlo = dash_m_lo(S0, period, phase), mhi = dash_m_hi(S1, period, phase);
    const int64_t ma = mlo > m_begin ? mlo : m_begin, mb = mhi < m_end ? mhi : m_end;
    for (int64_t m = ma; m <= mb; m++) {
        int64_t cpos = 0;
        for (uint32_t k = 0; k < n; k++) {
            int64_t a = m * period + cpos - phase, b = a + pat[k];
            cpos += pat[k];
            if (k & 1u) continue;  // a gap
            if (a < 0) a = 0;
            if (b > Stot) b = Stot;
            const int64_t lo = a > S0 ? a : S0, hi = b < S1 ? b : S1;
            if (lo < hi) f(lo, hi, a, b);
        }
    }
}


struct DashIn {
    SceneView sv;
    const DashDesc* desc;       // per style entry
    const int64_t* pat;         // pattern values on the grid
    const double* panels;       // per dashed segment tag i: panel k's integral at [k * n_tags + i]
    const uint64_t* len;        // per tag: grid length of a dashed segment, else 0
    const uint64_t* cum;        // per tag: exclusive prefix of len
    const uint32_t* subix;      // per tag: subpaths ended before it
    const uint64_t* sub_start;  // per subpath: cum at its first tag
};

// Work split of the count and write passes: a dashed segment's dash
// intervals are taken a few pattern periods at a time (about kDashChunk
// dashes), one chunk per thread, so a long segment with hundreds of dashes
// does not hold up its wave; every other tag is one chunk.  A chunk's
// output is the part of its tag's output that its periods produce (the
// first chunk also opens the path, the last one ends it), so the chunks'
// outputs in order are the tag's.
constexpr int64_t kDashChunk = 16;
constexpr uint32_t kDashMaxChunks = 1u << 20;  // per segment; more is refused
struct DashSpan {
    int64_t S0, S1, Stot, base;  // the segment on its subpath (grid units)
    int64_t mlo, per;            // first pattern period, periods per chunk
    uint32_t nq;                 // chunks
};
SX_HD inline DashSpan dash_span(const DashIn& in, uint32_t i, const DashDesc& dd) {
    DashSpan sp{0, 0, 0, 0, 0, 1, 1u};
    const uint32_t tag = in.sv.tags[i];
    if (dd.n == 0 || (tag & kTagEnd)) return sp;
    const uint32_t k = in.subix[i];
    sp.base = (int64_t)in.sub_start[k];
    sp.S0 = (int64_t)in.cum[i] - sp.base;
    sp.S1 = sp.S0 + (int64_t)in.len[i];
    sp.Stot = (int64_t)in.sub_start[k + 1] - sp.base;
    sp.mlo = dash_m_lo(sp.S0, dd.period, dd.phase);
    const int64_t span = dash_m_hi(sp.S1, dd.period, dd.phase) - sp.mlo + 1;
    const int64_t dashes = (int64_t)(dd.n / 2u);
    sp.per = dashes >= kDashChunk ? 1 : kDashChunk / dashes;
    const int64_t nq = (span + sp.per - 1) / sp.per;
    sp.nq = nq > (int64_t)kDashMaxChunks ? kDashMaxChunks + 1u : (uint32_t)nq;
    return sp;
}
SX_HD inline DashDesc dash_desc_of(const DashIn& in, uint32_t i) {
    const uint32_t sty = in.sv.mon[2 * (size_t)in.sv.mon_stride + i];
    return sty < in.sv.n_styles ? in.desc[sty] : DashDesc{0, 0, 0, 0};
}
SX_HD inline uint32_t dash_chunks(const DashIn& in, uint32_t i) { return dash_span(in, i, dash_desc_of(in, i)).nq; }

// Chunk q of dashed segment i (degree C): its dashes' parts and markers.
template <bool Write, int C, class PutPt, class PutTag>
SX_HD void dash_segment(const DashIn& in, uint32_t i, uint32_t q, const DashDesc& dd, const DashSpan& spn,
                        PutPt& put_pt, PutTag& put_tag) {
    const SceneView& sv = in.sv;
    const float2* D = sv.pts + sv.mon[i];
    double panel[kDashPanels];
#pragma unroll
    for (int k = 0; k < kDashPanels; k++) panel[k] = in.panels[(size_t)k * sv.n_tags + i];
    const int64_t base = spn.base, S0 = spn.S0, S1 = spn.S1, Stot = spn.Stot;
    const int64_t m_begin = spn.mlo + (int64_t)q * spn.per, m_end = m_begin + spn.per - 1;
    const bool last = (sv.tags[i + 1] & kTagEnd) != 0;
    const int64_t* pat = in.pat + dd.off;
    // A dash that started in an earlier segment (at subpath position a <
    // S0): whether one of its parts before this tag has extent and, when
    // want_pt, the start and tangent points of the first such part.  Its
    // start tag j is the last tag at or before position a; the tags between
    // j and this one hold full parts (with extent) exactly when they have
    // length.
    auto earlier_extent = [&](int64_t a, int64_t b, bool want_pt, float2& ds, float2& dv) {
        const uint64_t pos = (uint64_t)(base + a);
        // the last j < i with cum[j] <= pos (cum[i] > pos; the subpath's
        // first tag qualifies): usually i - 1, so gallop back from there,
        // then bisect the last step
        uint32_t h = i - 1, l = h, step = 1;
        while (in.cum[l] > pos) {
            h = l - 1;
            l = l >= step ? l - step : 0u;
            step *= 2u;
        }
        while (l < h) {
            const uint32_t mid = l + (h - l + 1) / 2;
            if (in.cum[mid] <= pos) l = mid;
            else h = mid - 1;
        }
        const uint32_t j = l;
        const uint64_t xj = in.cum[j] + in.len[j];  // where j's part ends
        const bool between = xj < in.cum[i];
        if (between && !want_pt) return true;
        const int cj = (int)(sv.tags[j] & kTagCount);
        const float2* Dj = sv.pts + sv.mon[j];
        const int64_t Q0 = (int64_t)in.cum[j] - base, Q1 = Q0 + (int64_t)in.len[j];
        const int64_t hj = b < Q1 ? b : Q1;
        const bool sure = dash_surely_extent(hj - a, Q1 - Q0, dash_max_coord_d(cj, Dj));
        if (sure && !want_pt) return true;
        double pj[kDashPanels];
#pragma unroll
        for (int k = 0; k < kDashPanels; k++) pj[k] = in.panels[(size_t)k * sv.n_tags + j];
        const DashPart pt2 = dash_part_d(cj, Dj, pj, Q0, Q1, a, hj);
        if (sure || pt2.extent) {
            ds = pt2.p[0];
            dv = pt2.dv;
            return true;
        }
        if (!between) return false;
        // the first tag after j with length: the last k < i with cum[k] <=
        // xj (cum[j + 1] = xj), usually j + 1: gallop forward, then bisect
        uint32_t lk = j + 1, hk = lk, stp = 1;
        while (hk < i - 1 && in.cum[hk + 1] <= xj) {
            lk = hk + 1;
            hk = (i - 1 - hk > stp) ? hk + stp : i - 1;
            stp *= 2u;
        }
        while (lk < hk) {
            const uint32_t mid = lk + (hk - lk + 1) / 2;
            if (in.cum[mid] <= xj) lk = mid;
            else hk = mid - 1;
        }
        const float2* Dk = sv.pts + sv.mon[lk];
        const int ck = (int)(sv.tags[lk] & kTagCount);
        ds = Dk[0];
        dv = make_float2(Dk[0].x + 1.0f, Dk[0].y);  // (a full part always has extent)
        for (int m = ck; m >= 1; m--)
            if (!(Dk[m].x == Dk[0].x && Dk[m].y == Dk[0].y)) dv = Dk[m];
        return true;
    };
    const double M = dash_max_coord<C>(D);
    dash_parts(S0, S1, Stot, pat, dd.n, dd.period, dd.phase, m_begin, m_end,
               [&](int64_t lo, int64_t hi, int64_t a, int64_t b) {
        // (the count pass needs the part's points only when its extent is in doubt)
        const bool sure = dash_surely_extent(hi - lo, S1 - S0, M);
        DashPart pa{};
        if (Write || !sure) pa = dash_part_c<C>(D, panel, S0, S1, lo, hi);
        const bool extent = sure || pa.extent;
        const bool ends = b <= S1 || last;
        float2 ds = make_float2(0.0f, 0.0f), dv = ds;
        // an earlier part of this dash (in an earlier tag) had extent; its
        // start and tangent points are needed only to write the marker here
        const bool written = a < S0 && earlier_extent(a, b, Write && ends, ds, dv);
        if (extent) {
            if (!written) {
                put_pt(pa.p[0].x, pa.p[0].y);
                ds = pa.p[0];
                dv = pa.dv;
            }
#pragma unroll
            for (int m = 1; m <= C; m++) put_pt(pa.p[m].x, pa.p[m].y);
            put_tag((uint32_t)C | kTagF32);
        }
        if (ends && (written || extent)) {
            put_pt(ds.x, ds.y);
            put_pt(dv.x, dv.y);
            put_tag(2u | kTagEnd | kTagF32);
        }
    });
}

// The dashed encoding's tags and points of chunk q of source tag i: counted
// (Write false) or written at tags_out[t0 ..], pts_out[p0 ..] (Write true).
template <bool Write>
SX_HD void dash_tag(const DashIn& in, uint32_t i, uint32_t q, uint8_t* tags_out, float2* pts_out,
                         uint64_t t0, uint64_t p0, uint32_t& nt, uint32_t& np) {
    const SceneView& sv = in.sv;
    auto put_pt = [&](float x, float y) {
        if (Write) pts_out[p0 + np] = make_float2(x, y);
        np++;
    };
    auto put_tag = [&](uint32_t t) {
        if (Write) tags_out[t0 + nt] = (uint8_t)t;
        nt++;
    };
    auto put_empty = [&](uint32_t extra, float2 p) {
        put_pt(p.x, p.y);
        put_pt(p.x, p.y);
        put_pt(p.x + 1.0f, p.y);
        put_tag(2u | kTagEnd | kTagF32 | kTagClosed | extra);
    };
    const uint32_t tag = sv.tags[i];
    const uint32_t off = sv.mon[i];
    const float2* D = sv.pts + off;
    const bool first_of_path = i == 0 || (sv.tags[i - 1] & kTagPath);
    const bool first_of_sub = i == 0 || (sv.tags[i - 1] & kTagEnd);
    const DashDesc dd = dash_desc_of(in, i);
    const DashSpan spn = dash_span(in, i, dd);
    if (first_of_path && q == 0) put_empty(tag & (kTagStyle | kTagXform), D[0]);
    if (dd.n == 0) {
        // a solid stroke or a fill: the tag and its points as they are
        if (first_of_sub) put_pt(D[0].x, D[0].y);
        const uint32_t cnt = tag & kTagCount;
        for (uint32_t j = 1; j <= cnt; j++) put_pt(D[j].x, D[j].y);
        put_tag(tag & ~(kTagPath | kTagStyle | kTagXform));
    } else if (!(tag & kTagEnd)) {
        const int c = (int)(tag & kTagCount);
        if (c == 1) dash_segment<Write, 1>(in, i, q, dd, spn, put_pt, put_tag);
        else if (c == 2) dash_segment<Write, 2>(in, i, q, dd, spn, put_pt, put_tag);
        else dash_segment<Write, 3>(in, i, q, dd, spn, put_pt, put_tag);
    }
    // (a dashed stroke's own markers give way to its dashes' markers)
    if ((tag & kTagPath) && q + 1 == spn.nq) put_empty(kTagPath, D[1]);
}

}  // namespace sx
