// Device-side FP32 math of the stroke-expansion hot path (gfx950, wave64).
//
// One function template, process_tag<Sink>, runs the whole per-segment
// computation; the count kernel instantiates it with a counting sink and
// the emit kernel with a writing sink, so both passes take bit-identical
// decisions (the library is built with -ffp-contract=off; every FMA here
// is explicit).
//
// Paper: Levien & Uguray, "GPU-friendly Stroke Expansion" (arXiv:2405.00127).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
constexpr float kFitFrac = 0.15f, kFlatFrac = 0.65f, kFitK = 9.0f, kFitS = 1.6f;
// Section 7.3 cusp handling: near-zero derivative test and perturbation.
constexpr float kEpsQ = 1e-5f, kDeltaT = 1.0f / 4096.0f;
constexpr int kMaxDepth = 16;
constexpr float kCMin = 0.1f;  // lower clamp of the chord / arc-length ratio
constexpr float kPi = 3.14159265358979323846f;
constexpr float kHalfPi = 1.57079632679489661923f;
// Section 4.2 constants of the piecewise approximation.
constexpr float kC1 = 1.0976991822760038f, kC2 = 0.9148117935952064f, kC3 = 0.16145779359520596f;
constexpr float kA2 = 0.94280904158206336587f;  // sqrt(8)/3
constexpr float kQ4 = 0.78539816339744830962f;  // pi/4
constexpr uint32_t kMaxCount = 10000000u;

struct StyleD {
    float half_width, miter_limit;
    uint32_t packed;  // join | start_cap << 8 | end_cap << 16 | flags << 24
};

// ---------------------------------------------------------- small vectors
struct V2 {
    float x, y;
};
__device__ __forceinline__ V2 v2(float x, float y) { return V2{x, y}; }
__device__ __forceinline__ V2 operator+(V2 a, V2 b) { return v2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ V2 operator-(V2 a, V2 b) { return v2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ V2 operator*(V2 a, float s) { return v2(a.x * s, a.y * s); }
__device__ __forceinline__ float dot(V2 a, V2 b) { return a.x * b.x + a.y * b.y; }
__device__ __forceinline__ float cross(V2 a, V2 b) { return a.x * b.y - a.y * b.x; }
__device__ __forceinline__ float len(V2 a) { return sqrtf(a.x * a.x + a.y * a.y); }
__device__ __forceinline__ bool is_zero(V2 a) { return a.x == 0.0f && a.y == 0.0f; }
__device__ __forceinline__ V2 unit(V2 a) {
    float l = len(a);
    return v2(a.x / l, a.y / l);
}
// right normal N = (T_y, -T_x); N' = kappa T
__device__ __forceinline__ V2 rnormal(V2 t) { return v2(t.y, -t.x); }
// offset point: p + N * h
__device__ __forceinline__ V2 offs(V2 p, V2 n, float h) { return p + n * h; }

// ------------------------------------------------------- Euler spirals
// Appendix A: k1 and chord / arc-length ratio as 7th-order polynomials in
// k = th0 + th1 and D = th1 - th0.
__device__ __forceinline__ float es_k1(float th0, float th1) {
    float k = th0 + th1, d = th1 - th0;
    float k2 = k * k, d2 = d * d;
    float a = 6.0f + d2 * (-1.0f / 70.0f + d2 * (-1.0f / 10780.0f + d2 * 2.769178184818219e-7f));
    float b = -0.1f + d2 * (1.0f / 4200.0f + d2 * 1.6959677820260655e-5f);
    float c = -1.0f / 1400.0f + d2 * 6.84915970574303e-5f;
    float e = -7.936475029053326e-6f;
    return d * (a + k2 * (b + k2 * (c + k2 * e)));
}
__device__ __forceinline__ float es_chord(float th0, float th1) {
    float k = th0 + th1, d = th1 - th0;
    float k2 = k * k, d2 = d * d;
    float a = 1.0f + d2 * (-1.0f / 40.0f + d2 * (0.00034226190482569864f - d2 * 1.9349474568904524e-6f));
    float b = -1.0f / 24.0f + d2 * (0.0024702380951963226f - d2 * 3.7297408997537985e-5f);
    float c = 1.0f / 1920.0f - d2 * 4.87350869747975e-5f;
    float e = -3.1001936068463107e-6f;
    return a + k2 * (b + k2 * (c + k2 * e));
}

// Section 7.1: chord-normalised distance estimate between a cubic with end
// angles th0, th1 and arms d0, d1 and the Euler spiral with those angles.
__device__ __forceinline__ float fit_estimate(float th0, float th1, float d0, float d1) {
    float s = fabsf(th0 + th1), df = fabsf(th0 - th1);
    float s2 = s * s;
    float e0 = 4.6255e-6f * (s2 * s2 * s) + 7.5e-3f * s2 * df;
    float c0 = cosf(th0), c1 = cosf(th1);
    float sn0 = sinf(th0), sn1 = sinf(th1), sn01 = sinf(th0 + th1);
    float db0 = 2.0f / (3.0f * (1.0f + c0)), db1 = 2.0f / (3.0f * (1.0f + c1));
    // area(d0,d1) - area(db0,db1), area = 3/20 (2 d0 sin th0 + 2 d1 sin th1 - d0 d1 sin(th0+th1))
    float a_src = 2.0f * d0 * sn0 + 2.0f * d1 * sn1 - d0 * d1 * sn01;
    float a_es = 2.0f * db0 * sn0 + 2.0f * db1 * sn1 - db0 * db1 * sn01;
    float ea = 1.55f * 0.15f * fabsf(a_src - a_es);
    float x0 = db0 - d0, x1 = db1 - d1;
    float ei = (0.005f * s + 0.07f * df) * sqrtf(x0 * x0 + x1 * x1);
    return e0 + ea + ei;
}

// Normalised ES: unit arc length, phi(u) = k0 (u - 1/2) + k1/2 (u - 1/2)^2.
__device__ __forceinline__ float es_phi(float k0, float k1, float u) {
    float v = u - 0.5f;
    return v * (k0 + 0.5f * k1 * v);
}

// Z(u) = int_0^u exp(i phi(v)) dv by 4-point Gauss-Legendre on [0, u].
__device__ __forceinline__ V2 es_integral(float k0, float k1, float u) {
    const float gx[4] = {-0.8611363115940526f, -0.3399810435848563f, 0.3399810435848563f, 0.8611363115940526f};
    const float gw[4] = {0.3478548451374538f, 0.6521451548625461f, 0.6521451548625461f, 0.3478548451374538f};
    float hu = 0.5f * u;
    float sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        float v = hu * (gx[i] + 1.0f);
        float ph = es_phi(k0, k1, v);
        float sn, cs;
        sincosf(ph, &sn, &cs);
        sx = fmaf(gw[i], cs, sx);
        sy = fmaf(gw[i], sn, sy);
    }
    return v2(sx * hu, sy * hu);
}

struct ES {
    V2 p0, p1, n0, n1;
    V2 rot;  // chord / Z(1)
    float k0, k1, L, base;
    bool pivot;
};

__device__ __forceinline__ V2 es_point(const ES& es, float u) {
    if (u == 0.0f) return es.p0;
    if (u == 1.0f) return es.p1;
    if (es.pivot) return es.p0 + (es.p1 - es.p0) * u;
    V2 z = es_integral(es.k0, es.k1, u);
    return es.p0 + v2(es.rot.x * z.x - es.rot.y * z.y, es.rot.x * z.y + es.rot.y * z.x);
}
__device__ __forceinline__ V2 es_normal(const ES& es, float u) {
    if (u == 0.0f) return es.n0;
    if (u == 1.0f) return es.n1;
    float a = es.base + es_phi(es.k0, es.k1, u);
    float sn, cs;
    sincosf(a, &sn, &cs);
    return v2(sn, -cs);
}
__device__ __forceinline__ float es_kn(const ES& es, float u) { return es.k0 + es.k1 * (u - 0.5f); }
// (1 + h kappa(u)) L: sign and zero of rho, finite for a zero-length pivot
__device__ __forceinline__ float es_rhoL(const ES& es, float h, float u) { return es.L + h * es_kn(es, u); }
__device__ __forceinline__ V2 offset_point(const ES& es, float h, float u) {
    return offs(es_point(es, u), es_normal(es, u), h);
}
__device__ __forceinline__ V2 evolute_point(const ES& es, float u) {
    // E = p - N / kappa, 1/kappa = L / (k0 + k1 (u - 1/2))
    return es_point(es, u) - es_normal(es, u) * (es.L / es_kn(es, u));
}

// ------------------------------------------- subdivision density integral
// x = -1 - 2 h kappa maps the ES inflection to -1 and the parallel-curve
// cusp to +1 (Section 4.1).  A point on this axis keeps x and, precisely,
// e = |x| - 1 (2 h kappa when x <= 0, -2 rho when x > 0).
struct XP {
    float x, e;
};
__device__ __forceinline__ XP make_xp(float hk) {
    float x = -1.0f - 2.0f * hk;
    float e = (x <= 0.0f) ? 2.0f * hk : -2.0f * (1.0f + hk);
    return XP{x, e};
}
__device__ __forceinline__ XP bp_xp(float x) { return XP{x, fabsf(x) - 1.0f}; }

// branch of f_approx by |x|: 0 [0,0.8) sin, 1 [0.8,1.25) 1.5-power, 2 [1.25,2.1) and 3 quadratics
__device__ __forceinline__ int branch_of(float ax) {
    return ax < 0.8f ? 0 : (ax < 1.25f ? 1 : (ax < 2.1f ? 2 : 3));
}
__device__ __forceinline__ float pow15(float a) { return a * sqrtf(a); }

// Divided difference (F(b) - F(a)) / (b - a) of f_approx over one branch,
// in a cancellation-free form; dx = b - a given precisely.
__device__ float branch_dd(int br, XP a, XP b, float dx) {
    if (br == 0) {
        float m = 0.5f * (a.x + b.x);
        float hz = 0.5f * kC1 * dx;
        float sc = (fabsf(hz) < 1e-4f) ? 1.0f - hz * hz * (1.0f / 6.0f) : sinf(hz) / hz;
        return cosf(kC1 * m) * sc;
    }
    if (br == 1) {
        float ea = fabsf(a.e), eb = fabsf(b.e);
        if (a.e * b.e >= 0.0f) {
            float ra = sqrtf(ea), rb = sqrtf(eb);
            float den = ra + rb;
            if (den == 0.0f) return 0.0f;
            return kA2 * (ea + ra * rb + eb) / den;
        }
        return kA2 * (pow15(ea) + pow15(eb)) / (ea + eb);
    }
    float aa = fabsf(a.x), ab = fabsf(b.x);
    if (br == 2) return 0.6406f * (aa + ab) - 0.81f;
    return 0.5f * (aa + ab) - 0.156f;
}

// Range of the x axis split at the branch breaks of f_approx.
struct XSeg {
    XP a;
    float len;  // signed x length
    float dF;   // F increment over the piece
    int br;
};
constexpr int kMaxXSeg = 7;
__device__ int split_x(XP xa, XP xb, float dx_total, XSeg* segs) {
    const float bps[6] = {-2.1f, -1.25f, -0.8f, 0.8f, 1.25f, 2.1f};
    int n = 0;
    XP cur = xa;
    bool up = xb.x > xa.x;
    float covered = 0.0f;
    if (up) {
        for (int k = 0; k < 6; k++) {
            if (bps[k] > xa.x && bps[k] < xb.x) {
                XP nb = bp_xp(bps[k]);
                float l = bps[k] - cur.x;
                segs[n].a = cur; segs[n].len = l;
                segs[n].br = branch_of(fabsf(cur.x + 0.5f * l));
                segs[n].dF = branch_dd(segs[n].br, cur, nb, l) * l;
                covered += l; cur = nb; n++;
            }
        }
    } else {
        for (int k = 5; k >= 0; k--) {
            if (bps[k] < xa.x && bps[k] > xb.x) {
                XP nb = bp_xp(bps[k]);
                float l = bps[k] - cur.x;
                segs[n].a = cur; segs[n].len = l;
                segs[n].br = branch_of(fabsf(cur.x + 0.5f * l));
                segs[n].dF = branch_dd(segs[n].br, cur, nb, l) * l;
                covered += l; cur = nb; n++;
            }
        }
    }
    float l = (n == 0) ? dx_total : xb.x - cur.x;
    segs[n].a = cur; segs[n].len = l;
    segs[n].br = (n == 0) ? branch_of(fabsf(0.5f * (xa.x + xb.x))) : branch_of(fabsf(cur.x + 0.5f * l));
    segs[n].dF = branch_dd(segs[n].br, cur, xb, l) * l;
    return n + 1;
}

// Fraction phi of a branch segment at which F has risen by f * seg.dF
// (local, cancellation-free inverse of f_approx).
__device__ float branch_inv_frac(const XSeg& s, float f) {
    float G = s.dF / s.len;  // divided difference (len != 0 here)
    if (s.br == 0) {
        float th = kC1 * s.a.x;
        float S = sinf(th), C = cosf(th);
        float dy = kC1 * f * s.dF;
        float Sp = S + dy;
        float rp = sqrtf(fmaxf(1.0f - Sp * Sp, 0.0f));
        float coef = C + S * (S + Sp) / (C + rp);
        float arg = dy * coef;
        float as = (fabsf(arg) < 1e-4f) ? 1.0f + arg * arg * (1.0f / 6.0f) : asinf(fminf(fmaxf(arg, -1.0f), 1.0f)) / arg;
        return f * G * coef * as;
    }
    float sgn = (s.a.x + 0.5f * s.len) >= 0.0f ? 1.0f : -1.0f;  // side of the axis
    float dFa = sgn * f * s.dF;                                 // F increment on |x|
    if (s.br == 1) {
        float es = s.a.e;
        float vs = (es < 0.0f ? -1.0f : 1.0f) * pow15(fabsf(es));
        float dg = dFa / kA2;
        float vp = vs + dg;
        float lena = sgn * s.len;
        if (vs * vp >= 0.0f) {
            float avp = fabsf(vp), avs = fabsf(vs);
            float p = cbrtf(avp), q = cbrtf(avs);
            float D = p * p * p * p + p * p * q * q + q * q * q * q;
            if (D == 0.0f) return f;
            return (f * G * sgn * sgn) * (avp + avs) / (kA2 * D);
        }
        float ep = (vp < 0.0f ? -1.0f : 1.0f) * cbrtf(vp * vp);
        return (ep - es) / lena;
    }
    float a = fabsf(s.a.x);
    float dFa_pos = dFa;
    if (s.br == 2) {
        float B = 1.2812f * a - 0.81f;
        return 2.0f * f * G / (B + sqrtf(fmaxf(B * B + 4.0f * 0.6406f * dFa_pos, 0.0f)));
    }
    float B = a - 0.156f;
    return 2.0f * f * G / (B + sqrtf(fmaxf(B * B + 2.0f * dFa_pos, 0.0f)));
}

__device__ __forceinline__ uint32_t ceil_count(float n_est) {
    if (!(n_est > 1.0f)) return 1u;
    if (n_est > 1e7f) return kMaxCount;
    return (uint32_t)ceilf(n_est);
}

// ------------------------------------------------------------- the sink
// Counting sink: only counts.  Writing sink: writes records at base + n.
struct CountSink {
    uint32_t n;
    __device__ __forceinline__ void line(V2, V2) { n++; }
    __device__ __forceinline__ void arc(V2, V2, float) { n++; }
    __device__ __forceinline__ void skip(uint32_t k) { n += k; }
    static constexpr bool kEmit = false;
};

struct WriteSink {
    float* out;      // records base (float words)
    uint64_t idx;    // next record index
    uint64_t end;    // one past this tag's last record (never written beyond)
    uint32_t path;
    int arcs;        // 0: 5-word lines, 1: 6-word arcs
    uint32_t n;
    __device__ __forceinline__ void put(V2 a, V2 b, float curv) {
        if (idx >= end) { n++; return; }
        if (arcs) {
            float* r = out + idx * 6;
            r[0] = a.x; r[1] = a.y; r[2] = b.x; r[3] = b.y; r[4] = curv;
            reinterpret_cast<uint32_t*>(r)[5] = path;
        } else {
            float* r = out + idx * 5;
            r[0] = a.x; r[1] = a.y; r[2] = b.x; r[3] = b.y;
            reinterpret_cast<uint32_t*>(r)[4] = path;
        }
        idx++;
        n++;
    }
    __device__ __forceinline__ void line(V2 a, V2 b) { put(a, b, 0.0f); }
    __device__ __forceinline__ void arc(V2 a, V2 b, float turn) {
        float c = len(b - a);
        float curv = (c > 0.0f && turn != 0.0f) ? 2.0f * sinf(0.5f * turn) / c : 0.0f;
        put(a, b, curv);
    }
    __device__ __forceinline__ void skip(uint32_t) {}
    static constexpr bool kEmit = true;
};

struct Cfg {
    float tau_fit, tau_flat, inv_sqrt8tf;  // sqrt(1 / (8 tau_flat))
    float cbrt_inv120tf;                   // cbrt(1 / (120 tau_flat))
    float round_step;                      // unused placeholder (per-width)
    int arcs;
    int paper_fit;
};

// ----------------------------------------------- one range of one side
// Section 4 (lines), Section 5 (arcs) and Section 6 (evolute for rho < 0).
template <class Sink>
__device__ void emit_range(Sink& k, const Cfg& cfg, const ES& es, float h, float ua, float ub, bool reversed,
                           bool end_a_piece, bool end_b_piece, V2 Pa, V2 Pb) {
    const bool sideA = h >= 0.0f;
    const int D = sideA ? 1 : -1;
    const int dir = reversed ? -D : D;
    const float du = ub - ua;
    const float kna = es_kn(es, ua), knb = es_kn(es, ub);
    uint32_t n;
    XSeg segs[kMaxXSeg];
    int nseg = 0;
    float dF = 0.0f;
    // arc-length dependent quantities
    if (!cfg.arcs) {
        float I;
        if (es.k1 == 0.0f) {
            I = du * sqrtf(fabsf(es.k0) * fabsf(es.L + h * es.k0));
        } else if (h == 0.0f) {
            float aa = fabsf(kna), ab = fabsf(knb);
            if (kna * knb >= 0.0f) {
                float den = pow15(aa) + pow15(ab);
                I = den > 0.0f ? (2.0f / 3.0f) * du * sqrtf(es.L) * (aa * aa + aa * ab + ab * ab) / den : 0.0f;
            } else {
                I = (2.0f / 3.0f) * du * sqrtf(es.L) * (pow15(aa) + pow15(ab)) / (aa + ab);
            }
        } else {
            XP xa = make_xp(h * kna / es.L), xb = make_xp(h * knb / es.L);
            float dx = -2.0f * h * es.k1 * du / es.L;
            nseg = split_x(xa, xb, dx, segs);
            for (int j = 0; j < nseg; j++) dF += segs[j].dF;
            // I = |dF| / (4 |kappa'| |h|^1.5) = |dF/dx| L_r / (2 sqrt|h|)
            float G = (dx != 0.0f) ? dF / dx : 0.0f;
            I = fabsf(G) * du * es.L / (2.0f * sqrtf(fabsf(h)));
        }
        n = ceil_count(I * cfg.inv_sqrt8tf);
    } else {
        float n_est = 0.0f;
        if (es.k1 != 0.0f) {
            float Lr = du * es.L;
            float kp = es.k1 / (es.L * es.L);
            n_est = Lr * cbrtf(fabsf(kp) * (1.0f + 0.4f * fabsf(h * Lr * kp))) * cfg.cbrt_inv120tf;
        }
        n = ceil_count(n_est);
        float sweep = fmaxf(fabsf(kna), fabsf(knb)) * du * (1.0f / kHalfPi);
        uint32_t ns = ceil_count(sweep);
        n = ns > n ? ns : n;
    }

    if (!Sink::kEmit) {
        k.skip(n);
    } else {
        V2 prev = Pa;
        float uprev = ua;
        for (uint32_t i = 1; i <= n; i++) {
            float u;
            V2 P;
            if (i == n) {
                u = ub;
                P = Pb;
            } else {
                float f = (float)i / (float)n;
                float tau = f;
                if (!cfg.arcs && es.k1 != 0.0f) {
                    if (h != 0.0f) {
                        if (nseg > 0) {
                            // walk the branch pieces to the one holding f * dF
                            float target = f * dF, cum = 0.0f, acc_len = 0.0f, dx_total = 0.0f;
                            for (int j = 0; j < nseg; j++) dx_total += segs[j].len;
                            int j = 0;
                            for (; j < nseg - 1; j++) {
                                if (fabsf(cum + segs[j].dF) >= fabsf(target)) break;
                                cum += segs[j].dF;
                                acc_len += segs[j].len;
                            }
                            float fl = (segs[j].dF != 0.0f) ? (target - cum) / segs[j].dF : 0.0f;
                            fl = fminf(fmaxf(fl, 0.0f), 1.0f);
                            float phi = (segs[j].len != 0.0f) ? branch_inv_frac(segs[j], fl) : fl;
                            tau = (nseg == 1) ? phi : (acc_len + phi * segs[j].len) / dx_total;
                        }
                    } else {
                        // h = 0: uniform in |kappa|^1.5 (Section 2.2)
                        float aa = fabsf(kna), ab = fabsf(knb);
                        float Pa15 = pow15(aa), Pb15 = pow15(ab);
                        float kap;
                        if (kna * knb >= 0.0f) {
                            float P15 = Pa15 + f * (Pb15 - Pa15);
                            kap = cbrtf(P15 * P15);
                            tau = (ab != aa) ? (kap - aa) / (ab - aa) : f;
                        } else {
                            float target = f * (Pa15 + Pb15);
                            if (target <= Pa15) {
                                float t15 = Pa15 - target;
                                kap = cbrtf(t15 * t15);
                                tau = (aa - kap) / (aa + ab);
                            } else {
                                float t15 = target - Pa15;
                                kap = cbrtf(t15 * t15);
                                tau = (aa + kap) / (aa + ab);
                            }
                        }
                    }
                }
                tau = fminf(fmaxf(tau, 0.0f), 1.0f);
                u = ua + du * tau;
                P = offset_point(es, h, u);
            }
            if (!cfg.arcs) {
                if (dir > 0) k.line(prev, P); else k.line(P, prev);
            } else {
                float turn = es_phi(es.k0, es.k1, u) - es_phi(es.k0, es.k1, uprev);
                if (dir > 0) k.arc(prev, P, turn); else k.arc(P, prev, -turn);
            }
            prev = P;
            uprev = u;
        }
    }
    if (!reversed) return;

    // ---- evolute: density |s - s0|^-1/2 (Section 6); lines in both modes
    float aa = fabsf(kna), ab = fabsf(knb);
    float ra = sqrtf(aa), rb = sqrtf(ab);
    float Iev = (es.k1 != 0.0f && ra + rb > 0.0f) ? 2.0f * du * sqrtf(fabsf(es.k1) * es.L) / (ra + rb) : 0.0f;
    uint32_t ne = ceil_count(Iev * cfg.inv_sqrt8tf);
    uint32_t nconn = (end_a_piece ? 1u : 0u) + (end_b_piece ? 1u : 0u);
    if (!Sink::kEmit) {
        k.skip(2u * ne + 2u * nconn);
        return;
    }
    float alpha = (ra + rb > 0.0f) ? ra / (ra + rb) : 0.5f;
    auto ev_at = [&](uint32_t i) -> V2 {
        if (i == 0) return end_a_piece ? evolute_point(es, ua) : Pa;
        if (i == ne) return end_b_piece ? evolute_point(es, ub) : Pb;
        float f = (float)i / (float)ne;
        float tau = f * (2.0f * alpha + f * (1.0f - 2.0f * alpha));
        return evolute_point(es, ua + du * tau);
    };
    for (int copy = 0; copy < 2; copy++) {
        V2 prev = ev_at(0);
        for (uint32_t i = 1; i <= ne; i++) {
            V2 E = ev_at(i);
            if (D > 0) k.line(prev, E); else k.line(E, prev);
            prev = E;
        }
    }
    if (end_a_piece) {
        V2 E0 = evolute_point(es, ua);
        for (int c = 0; c < 2; c++) { if (D > 0) k.line(Pa, E0); else k.line(E0, Pa); }
    }
    if (end_b_piece) {
        V2 E1 = evolute_point(es, ub);
        for (int c = 0; c < 2; c++) { if (D > 0) k.line(E1, Pb); else k.line(Pb, E1); }
    }
}

template <class Sink>
__device__ void emit_side(Sink& k, const Cfg& cfg, const ES& es, float h) {
    float r0 = es_rhoL(es, h, 0.0f), r1 = es_rhoL(es, h, 1.0f);
    V2 P0 = offs(es.p0, es.n0, h), P1 = offs(es.p1, es.n1, h);
    if (r0 * r1 < 0.0f) {
        float tc = r0 / (r0 - r1);
        V2 Pc = offset_point(es, h, tc);
        emit_range(k, cfg, es, h, 0.0f, tc, r0 < 0.0f, true, false, P0, Pc);
        emit_range(k, cfg, es, h, tc, 1.0f, r1 < 0.0f, false, true, Pc, P1);
    } else {
        emit_range(k, cfg, es, h, 0.0f, 1.0f, (r0 < 0.0f || r1 < 0.0f), true, true, P0, P1);
    }
}

// ----------------------------------------------------- joins and caps
__device__ __forceinline__ float round_step(float w, float tau_flat) {
    float c = 1.0f - tau_flat / w;
    c = fminf(fmaxf(c, -1.0f), 1.0f);
    return 2.0f * acosf(c);
}

template <class Sink>
__device__ void emit_round(Sink& k, const Cfg& cfg, V2 c, float w, float a0, float sweep, V2 A, V2 B) {
    uint32_t n = cfg.arcs ? ceil_count(fabsf(sweep) * (1.0f / kHalfPi))
                          : ceil_count(fabsf(sweep) / round_step(w, cfg.tau_flat));
    if (!Sink::kEmit) { k.skip(n); return; }
    V2 prev = A;
    for (uint32_t i = 1; i <= n; i++) {
        V2 nx;
        if (i == n) nx = B;
        else {
            float a = a0 + sweep * ((float)i / (float)n);
            float sn, cs;
            sincosf(a, &sn, &cs);
            nx = v2(c.x + w * cs, c.y + w * sn);
        }
        if (cfg.arcs) k.arc(prev, nx, sweep / (float)n); else k.line(prev, nx);
        prev = nx;
    }
}

template <class Sink>
__device__ void emit_cap(Sink& k, const Cfg& cfg, int cap, V2 p, V2 u, float w, bool start) {
    V2 N = rnormal(u);
    V2 PA = offs(p, N, w), PB = offs(p, N, -w);
    V2 from = start ? PB : PA, to = start ? PA : PB;
    V2 fwd = start ? v2(-u.x, -u.y) : u;
    if (cap == kCapButt) {
        k.line(from, to);
    } else if (cap == kCapSquare) {
        V2 a = from + fwd * w, b = to + fwd * w;
        k.line(from, a);
        k.line(a, b);
        k.line(b, to);
    } else {
        float a0 = atan2f(from.y - p.y, from.x - p.x);
        emit_round(k, cfg, p, w, a0, kPi, from, to);
    }
}

template <class Sink>
__device__ void emit_join(Sink& k, const Cfg& cfg, int join, float miter_limit, V2 p, V2 ta, V2 tb, float w) {
    V2 ua = unit(ta), ub = unit(tb);
    if (ua.x == ub.x && ua.y == ub.y) return;
    float cr = cross(ua, ub), dp = dot(ua, ub);
    V2 Na = rnormal(ua), Nb = rnormal(ub);
    bool outerA = !(cr < 0.0f);
    float h_out = outerA ? w : -w, h_in = -h_out;
    V2 Oa = offs(p, Na, h_out), Ob = offs(p, Nb, h_out);
    V2 Ia = offs(p, Na, h_in), Ib = offs(p, Nb, h_in);
    V2 from = outerA ? Oa : Ob, to = outerA ? Ob : Oa;
    for (int side = 0; side < 2; side++) {
        bool isA = side == 0;
        if (isA == outerA) {
            if (join == kJoinRound) {
                float dphi = atan2f(cr, dp);
                float a0 = atan2f(from.y - p.y, from.x - p.x);
                emit_round(k, cfg, p, w, a0, fabsf(dphi), from, to);
            } else if (join == kJoinMiter) {
                float crit = miter_limit * miter_limit * (1.0f + dp);
                if (crit >= 2.0f) {
                    V2 M = offs(p, Na + Nb, h_out / (1.0f + dp));
                    k.line(from, M);
                    k.line(M, to);
                } else {
                    k.line(from, to);
                }
            } else {
                k.line(from, to);
            }
        } else {
            V2 f = outerA ? Ib : Ia, t = outerA ? Ia : Ib;
            k.line(f, p);
            k.line(p, t);
        }
    }
}

// --------------------------------------------------------- segments
struct Seg {
    V2 P[4];
    V2 ts, te;
    float w, lpoly;
};

struct Tan {
    V2 dir;
    float mag;
};

__device__ __forceinline__ V2 cubic_point(const Seg& s, float t) {
    float mt = 1.0f - t;
    float a = mt * mt * mt, b = 3.0f * mt * mt * t, c = 3.0f * mt * t * t, d = t * t * t;
    return v2(a * s.P[0].x + b * s.P[1].x + c * s.P[2].x + d * s.P[3].x,
              a * s.P[0].y + b * s.P[1].y + c * s.P[2].y + d * s.P[3].y);
}
__device__ __forceinline__ V2 cubic_q(const Seg& s, float t) {
    float mt = 1.0f - t;
    V2 a = s.P[1] - s.P[0], b = s.P[2] - s.P[1], c = s.P[3] - s.P[2];
    float wa = mt * mt, wb = 2.0f * t * mt, wc = t * t;
    return v2(wa * a.x + wb * b.x + wc * c.x, wa * a.y + wb * b.y + wc * c.y);
}
__device__ __forceinline__ Tan sample_q(const Seg& s, float t) {
    if (t == 0.0f) return Tan{s.ts, len(s.P[1] - s.P[0])};
    if (t == 1.0f) return Tan{s.te, len(s.P[3] - s.P[2])};
    V2 q = cubic_q(s, t);
    float ql = len(q);
    if (ql < kEpsQ * s.lpoly) {
        q = cubic_q(s, (t + kDeltaT < 1.0f) ? t + kDeltaT : t - kDeltaT);
        ql = len(q);
    }
    return Tan{q, ql};
}

// Algorithm 2: adaptive bisection of the cubic into Euler spiral pieces with
// the two-word stack (t0_u, dt), then the parallel curves of each piece.
template <class Sink>
__device__ void process_segment(Sink& k, const Cfg& cfg, const Seg& s) {
    uint32_t t0_u = 0;
    float dt = 1.0f;
    V2 last_p = s.P[0];
    Tan last_q = sample_q(s, 0.0f);
    const float hw = s.w;
    const float min_dt = 1.0f / (float)(1u << kMaxDepth);
    for (;;) {
        float t0 = (float)t0_u * dt;
        if (t0 == 1.0f) break;
        float t1 = t0 + dt;
        V2 next_p = (t1 == 1.0f) ? s.P[3] : cubic_point(s, t1);
        Tan next_q = sample_q(s, t1);
        V2 chord = next_p - last_p;
        float cl = len(chord);
        float th0 = atan2f(cross(last_q.dir, chord), dot(last_q.dir, chord));
        float th1 = atan2f(cross(chord, next_q.dir), dot(chord, next_q.dir));
        float d0 = last_q.mag * dt / cl, d1 = next_q.mag * dt / cl;
        float est = fit_estimate(th0, th1, d0, d1);
        float err = cfg.paper_fit ? est * cl : est * (cl + kFitK * hw) * kFitS;
        bool len_ok = cl > 0.0f;
        bool hodo_ok = true;
        {
            float ma = last_q.mag * dt, mc = next_q.mag * dt;
            V2 a = unit(last_q.dir) * ma, c = unit(next_q.dir) * mc;
            V2 b = chord - a - c;
            if (ma > 0.0f && mc > 0.0f && !is_zero(b)) hodo_ok = (dot(a, b) * mc + dot(b, c) * ma) > 0.0f;
        }
        bool forced = dt <= min_dt;
        bool ok = len_ok && hodo_ok && (err <= cfg.tau_fit);
        if (ok || forced) {
            bool pivot = !ok;
            ES es;
            es.pivot = pivot;
            es.p0 = last_p;
            es.p1 = next_p;
            es.n0 = rnormal(unit(last_q.dir));
            es.n1 = rnormal(unit(next_q.dir));
            float c;
            if (pivot) {
                es.k0 = atan2f(cross(last_q.dir, next_q.dir), dot(last_q.dir, next_q.dir));
                es.k1 = 0.0f;
                c = es_chord(0.5f * es.k0, 0.5f * es.k0);
                es.base = atan2f(last_q.dir.y, last_q.dir.x) + 0.5f * es.k0;
                es.rot = v2(0.0f, 0.0f);
            } else {
                es.k0 = th0 + th1;
                es.k1 = es_k1(th0, th1);
                c = es_chord(th0, th1);
                V2 z1 = es_integral(es.k0, es.k1, 1.0f);
                float zz = z1.x * z1.x + z1.y * z1.y;
                es.rot = v2((chord.x * z1.x + chord.y * z1.y) / zz, (chord.y * z1.x - chord.x * z1.y) / zz);
                es.base = atan2f(es.rot.y, es.rot.x);
            }
            if (!(c > kCMin)) c = kCMin;
            es.L = cl / c;
            emit_side(k, cfg, es, hw);
            emit_side(k, cfg, es, -hw);
            // pop: count trailing zeros
            t0_u += 1;
            uint32_t sh = __builtin_ctz(t0_u);
            t0_u >>= sh;
            dt *= (float)(1u << sh);
            last_p = next_p;
            last_q = next_q;
        } else {
            t0_u *= 2;
            dt *= 0.5f;
        }
    }
}

__device__ __forceinline__ V2 xf_apply(const float* X, float x, float y) {
    // x' = a x + c y + e, y' = b x + d y + f (explicit order, no contraction)
    return v2(X[0] * x + X[2] * y + X[4], X[1] * x + X[3] * y + X[5]);
}

__device__ __forceinline__ V2 first_nonzero(const V2* c, int n) {
    for (int i = 0; i < n; i++)
        if (!is_zero(c[i])) return c[i];
    return v2(1.0f, 0.0f);
}

struct SceneView {
    const uint8_t* tags;
    const float2* pts;
    const StyleD* styles;
    const float* xforms;  // 6 floats each
    const uint32_t* path_map;
    const uint32_t* mon;  // 4 x n SoA
    uint32_t n_tags;
};

// Algorithm 1: the work of thread `i` (one tag).
template <class Sink>
__device__ void process_tag(Sink& k, const Cfg& cfg, const SceneView& sv, uint32_t i) {
    const uint32_t n = sv.n_tags;
    uint32_t tag = sv.tags[i];
    uint32_t off = sv.mon[i];
    uint32_t sty = sv.mon[2 * (size_t)n + i];
    uint32_t xfi = sv.mon[3 * (size_t)n + i];
    StyleD st = sv.styles[sty];
    const float* X = sv.xforms + 6 * (size_t)xfi;
    float scale = sqrtf(fabsf(X[0] * X[3] - X[1] * X[2]));
    float w = st.half_width * scale;
    int join = st.packed & 0xff, scap = (st.packed >> 8) & 0xff, ecap = (st.packed >> 16) & 0xff;
    const float2* D = sv.pts + off;
    if (tag & kTagEnd) {
        if (!(tag & kTagClosed)) {
            float2 a = D[1], b = D[2];
            V2 ps = xf_apply(X, a.x, a.y), pd = xf_apply(X, b.x, b.y);
            V2 dir = pd - ps;
            if (is_zero(dir)) dir = v2(1.0f, 0.0f);
            emit_cap(k, cfg, scap, ps, unit(dir), w, true);
        }
        return;
    }
    int c = tag & kTagCount;
    V2 raw[4];
    for (int j = 0; j <= c; j++) {
        float2 q = D[j];
        raw[j] = xf_apply(X, q.x, q.y);
    }
    Seg s;
    s.w = w;
    if (c == 1) {
        V2 d = raw[1] - raw[0];
        s.P[0] = raw[0]; s.P[3] = raw[1];
        s.P[1] = raw[0] + d * (1.0f / 3.0f);
        s.P[2] = raw[0] + d * (2.0f / 3.0f);
    } else if (c == 2) {
        s.P[0] = raw[0]; s.P[3] = raw[2];
        s.P[1] = raw[0] + (raw[1] - raw[0]) * (2.0f / 3.0f);
        s.P[2] = raw[2] + (raw[1] - raw[2]) * (2.0f / 3.0f);
    } else {
        for (int j = 0; j < 4; j++) s.P[j] = raw[j];
    }
    V2 cs[3], ce[3];
    for (int j = 0; j < c; j++) cs[j] = raw[j + 1] - raw[0];
    for (int j = 0; j < c; j++) ce[j] = raw[c] - raw[c - 1 - j];
    s.ts = first_nonzero(cs, c);
    s.te = first_nonzero(ce, c);
    s.lpoly = len(s.P[1] - s.P[0]) + len(s.P[2] - s.P[1]) + len(s.P[3] - s.P[2]);
    process_segment(k, cfg, s);

    // join with tag i + 1 or end cap (Algorithm 1)
    uint32_t nt = sv.tags[i + 1];
    V2 pend = raw[c];
    if ((nt & kTagEnd) && !(nt & kTagClosed)) {
        emit_cap(k, cfg, ecap, pend, unit(s.te), w, false);
        return;
    }
    const float2* Dn = sv.pts + sv.mon[i + 1];
    V2 tb;
    if (nt & kTagEnd) {
        float2 a = Dn[1], b = Dn[2];
        V2 ps = xf_apply(X, a.x, a.y), pd = xf_apply(X, b.x, b.y);
        tb = pd - ps;
        if (is_zero(tb)) tb = v2(1.0f, 0.0f);
    } else {
        int cn = nt & kTagCount;
        V2 r0;
        {
            float2 q = Dn[0];
            r0 = xf_apply(X, q.x, q.y);
        }
        V2 cands[3];
        for (int j = 0; j < cn; j++) {
            float2 q = Dn[j + 1];
            cands[j] = xf_apply(X, q.x, q.y) - r0;
        }
        tb = first_nonzero(cands, cn);
    }
    emit_join(k, cfg, join, st.miter_limit, pend, s.te, tb, w);
}

}  // namespace sx
