// prox.h -- FP32 device minimisers of the three-weight planner for gfx950.
//
// Every minimiser returns the argmin of  f_b(x) + sum_k (w_k/2)|x_k - n_k|^2
// (eq. general_minimizer_definition).  The collision and wall minimisers use
// the separating-line form of the non-convex constraint: a segment avoids
// the open capsule R (all points within r of [x_L, x_R]) iff some unit
// normal u has both segment ends in {y : <y, u> >= h(u)}, h the support
// function of R.  For a fixed u the best ends are the projections of n onto
// that half-plane, so the minimiser is
//     min_u F(u),  F(u) = sum_k (w_k/2) max(0, h(u) - <n_k, u>)^2 .
// F is C^1 on the circle away from the two kinks of h, so its minimum is at
// (a) a stationary point of a smooth piece where both ends are pushed (the
// paper's tangent-slab family, App. I), (b) the outward normal of the point
// of R nearest to one end while the other end is already clear (the
// paper's configuration with one spring at rest), or (c) a kink of h (slab
// resting on a flat side of the wall).  Candidates of each kind are
// enumerated in closed form or by a bracketed 1-D root solve, and the one
// of least F wins.  The stationary points of a piece are Lagrange points of
// a quadratic on the unit circle; the global one is the root below the
// smallest eigenvalue of the secular equation (trust-region theory), found
// by safeguarded Newton.
#pragma once
#include <hip/hip_runtime.h>

namespace twa {

// host and device: the minimisers are plain arithmetic
#define TWA_HD __host__ __device__ __forceinline__

TWA_HD float inv_sqrt(float x) { return 1.0f / sqrtf(x); }

enum : int { W_ZERO = 0, W_STD = 1, W_INF = 2 };

struct f2 {
    float x, y;
};
TWA_HD f2 mk(float x, float y) { return f2{x, y}; }
TWA_HD f2 add(f2 a, f2 b) { return f2{a.x + b.x, a.y + b.y}; }
TWA_HD f2 sub(f2 a, f2 b) { return f2{a.x - b.x, a.y - b.y}; }
TWA_HD f2 scl(f2 a, float s) { return f2{a.x * s, a.y * s}; }
TWA_HD float dot(f2 a, f2 b) { return a.x * b.x + a.y * b.y; }
TWA_HD f2 perp(f2 a) { return f2{-a.y, a.x}; }
TWA_HD float pos(float v) { return v > 0.f ? v : 0.f; }

struct f3 {
    float x, y, z;
};
TWA_HD f3 sub3(f3 a, f3 b) { return f3{a.x - b.x, a.y - b.y, a.z - b.z}; }
TWA_HD float dot3(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Squared closest approach of (1-a) d0 + a d1 over a in [0, 1]
// (the constraint of eq. basic_opt_prob on the relative positions).
TWA_HD float cpa_sq(f3 d0, f3 d1) {
    f3 e = sub3(d1, d0);
    float ee = dot3(e, e);
    float a = 0.f;
    if (ee > 0.f) a = fminf(fmaxf(-dot3(d0, e) / ee, 0.f), 1.f);
    f3 v{d0.x + a * e.x, d0.y + a * e.y, d0.z + a * e.z};
    return dot3(v, v);
}

// Whether (1-a) d0 + a d1 comes closer to the origin than sqrt(R2) for some
// a in [0, 1], without a division: the closest point is an end unless the
// projection of the origin falls inside, and then its squared distance is
// |d0 x e|^2 / |e|^2 with e = d1 - d0.
TWA_HD bool cpa_below(f3 d0, f3 d1, float R2) {
    // all three cases evaluated and selected (no divergent branches)
    f3 e = sub3(d1, d0);
    f3 c{d0.y * e.z - d0.z * e.y, d0.z * e.x - d0.x * e.z, d0.x * e.y - d0.y * e.x};
    const bool at0 = dot3(d0, e) >= 0.f, at1 = dot3(d1, e) <= 0.f;
    const bool in0 = dot3(d0, d0) < R2, in1 = dot3(d1, d1) < R2, inm = dot3(c, c) < R2 * dot3(e, e);
    return at0 ? in0 : (at1 ? in1 : inm);
}

TWA_HD float point_seg_sq(f2 q, f2 a, f2 b) {
    f2 d = sub(b, a);
    float L2 = dot(d, d);
    float t = 0.f;
    if (L2 > 0.f) t = fminf(fmaxf(dot(sub(q, a), d) / L2, 0.f), 1.f);
    f2 v = sub(add(a, scl(d, t)), q);
    return dot(v, v);
}

TWA_HD float orient(f2 a, f2 b, f2 c) {
    return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

// Squared distance between planar segments [p0,p1] and [q0,q1]
// (the constraint of eq. wall_minimizer over all alpha, beta).
TWA_HD float segseg_sq(f2 p0, f2 p1, f2 q0, f2 q1) {
    float o1 = orient(p0, p1, q0), o2 = orient(p0, p1, q1);
    float o3 = orient(q0, q1, p0), o4 = orient(q0, q1, p1);
    if (((o1 > 0.f && o2 < 0.f) || (o1 < 0.f && o2 > 0.f)) && ((o3 > 0.f && o4 < 0.f) || (o3 < 0.f && o4 > 0.f)))
        return 0.f;
    float m = point_seg_sq(p0, q0, q1);
    m = fminf(m, point_seg_sq(p1, q0, q1));
    m = fminf(m, point_seg_sq(q0, p0, p1));
    m = fminf(m, point_seg_sq(q1, p0, p1));
    return m;
}

// ---------------------------------------------------------------------------
// Energy minimiser, App. E (eq. energy_minimizer_output) with the limits of
// infinite weights and of two equal weights tending to zero.
// ---------------------------------------------------------------------------
TWA_HD void energy_prox(float nl, float nh, float wl, float wh, int kl, int kh, float C,
                                            float &xl, float &xh) {
    if (C <= 0.f || (kl == W_INF && kh == W_INF)) {
        xl = nl;
        xh = nh;
    } else if (kl == W_INF) {
        xl = nl;
        xh = (wh * nh + 2.f * C * nl) / (2.f * C + wh);
    } else if (kh == W_INF) {
        xh = nh;
        xl = (wl * nl + 2.f * C * nh) / (2.f * C + wl);
    } else if (kl == W_ZERO && kh == W_ZERO) {
        xl = xh = 0.5f * (nl + nh);
    } else {
        float den = 2.f * C * (wl + wh) + wl * wh;
        float cm = 2.f * C * (wl * nl + wh * nh);
        xl = (wl * wh * nl + cm) / den;
        xh = (wl * wh * nh + cm) / den;
    }
}

// ---------------------------------------------------------------------------
// Velocity-limit minimiser, App. F (maximum) and App. G (minimum): the
// closest pair (xl, xh) to (nl, nh) in the weighted norm with |xl - xh| <= C
// (>= C).  When the limit binds, the KKT conditions keep the weighted mean
// (wl nl + wh nh)/(wl + wh) and put the ends at distance C along nl - nh; a
// certain end stays and the other moves to distance C of it.  Returns whether
// the limit binds (the factor then sends weight rho0).  Coinciding ends under
// a minimum: direction +e1.
// ---------------------------------------------------------------------------
template <int D>
TWA_HD bool vel_prox(const float *nl, const float *nh, float wl, float wh, int kl, int kh, float C, bool minimum,
                     float *xl, float *xh) {
    float d[3] = {0.f, 0.f, 0.f}, dd = 0.f;
    for (int c = 0; c < D; ++c) {
        d[c] = nl[c] - nh[c];
        dd += d[c] * d[c];
    }
    const bool bind = minimum ? (dd < C * C) : (dd > C * C);
    for (int c = 0; c < D; ++c) xl[c] = nl[c], xh[c] = nh[c];
    if (!bind || (kl == W_INF && kh == W_INF)) return bind;
    float e[3] = {1.f, 0.f, 0.f};
    if (dd > 0.f) {
        const float inv = 1.f / sqrtf(dd);
        for (int c = 0; c < D; ++c) e[c] = d[c] * inv;
    }
    // share of the correction taken by the lower end
    float sl;
    if (kl == W_INF) sl = 0.f;
    else if (kh == W_INF) sl = 1.f;
    else if (kl == W_ZERO && kh == W_ZERO) sl = 0.5f;
    else sl = wh / (wl + wh);
    for (int c = 0; c < D; ++c) {
        const float corr = C * e[c] - d[c]; // change of xl - xh
        xl[c] = nl[c] + sl * corr;
        xh[c] = nh[c] - (1.f - sl) * corr;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Quadratic on the unit circle: E(u) = 1/2 u^T Q u - <b, u>,
// Q = [[a, c], [c, e]] positive semi-definite.
// ---------------------------------------------------------------------------
struct Eig2 {
    f2 v1, v2;       // eigenvectors of q1 <= q2
    float gap;       // q2 - q1
    float b1, b2;    // coordinates of b
};

TWA_HD Eig2 eig2(float a, float c, float e, f2 b) {
    Eig2 r;
    float d = 0.5f * (a - e);
    float rad = sqrtf(d * d + c * c);
    f2 v;
    if (rad <= 1e-30f) v = mk(1.f, 0.f);
    else if (d >= 0.f) v = mk(-c, d + rad);
    else v = mk(rad - d, -c);
    float inv = inv_sqrt(dot(v, v));
    r.v1 = scl(v, inv);
    r.v2 = perp(r.v1);
    r.gap = 2.f * rad;
    r.b1 = dot(b, r.v1);
    r.b2 = dot(b, r.v2);
    return r;
}

// Global minimiser of E on the circle.  Writes a second candidate (the
// mirror point of the degenerate "hard case", where two minimisers tie)
// into *alt and returns 2, else returns 1.
TWA_HD int trs_global(const Eig2 &g, f2 *out, f2 *alt) {
    float b1 = g.b1, b2 = g.b2, gap = g.gap;
    float bn = sqrtf(b1 * b1 + b2 * b2);
    if (!(bn > 0.f)) {
        // E = 1/2 u^T Q u: minimised along v1 (both signs)
        out[0] = g.v1;
        *alt = scl(g.v1, -1.f);
        return 2;
    }
    // t = q1 - lambda > 0 solves b1^2/t^2 + b2^2/(t+gap)^2 = 1.  The root
    // lies in [lo, hi]; when |b2| < gap and t << gap it is close to
    // |b1| / sqrt(1 - (b2/gap)^2), a good first guess.  Newton on
    // 1/sqrt(S) - 1 (nearly linear in t at both ends), with geometric
    // bisection whenever a step leaves the bracket.
    float lo = fmaxf(fabsf(b1), bn - gap), hi = bn;
    float t = hi;
    float q = b2 / fmaxf(gap, 1e-30f);
    if (q * q < 1.f) {
        float ta = fabsf(b1) * inv_sqrt(1.f - q * q);
        if (ta > lo && ta < hi) t = ta;
    }
    for (int it = 0; it < 60; ++it) {
        float y1 = b1 / t, y2 = b2 / (t + gap);
        float S = y1 * y1 + y2 * y2;
        float rs = inv_sqrt(S);
        float h = rs - 1.f; // increasing in t; root where h == 0
        if (h > 0.f) hi = t;
        else lo = t;
        if (fabsf(h) <= 2.4e-7f) break;
        float dS = y1 * y1 / t + y2 * y2 / (t + gap); // = -S'/2
        float hp = rs * rs * rs * dS;
        float tn = t - h / hp;
        if (!(tn > lo && tn < hi)) tn = lo > 0.f ? sqrtf(lo * hi) : 0.5f * hi;
        if (tn == t) break;
        t = tn;
    }
    float y1, y2;
    bool hard = t <= 1e-6f * (bn + gap);
    if (hard) {
        y2 = fminf(fmaxf(b2 / (t + gap), -1.f), 1.f);
        y1 = sqrtf(fmaxf(0.f, 1.f - y2 * y2));
        if (b1 < 0.f) y1 = -y1;
    } else {
        y1 = b1 / t;
        y2 = b2 / (t + gap);
    }
    float inv = inv_sqrt(y1 * y1 + y2 * y2);
    y1 *= inv;
    y2 *= inv;
    out[0] = add(scl(g.v1, y1), scl(g.v2, y2));
    if (hard) {
        *alt = add(scl(g.v1, -y1), scl(g.v2, y2));
        return 2;
    }
    return 1;
}

// Root in (0, xm] of  bn^2/x^2 + bf^2/(gap - x)^2 = 1, where the left side
// is convex in x with its minimum (< 1) at xm: Newton's method from x = |bn|
// (where the left side is > 1) increases monotonically onto the root.
TWA_HD float secular_side(float bn, float bf, float gap, float xm) {
    float x = fabsf(bn);
    for (int it = 0; it < 32; ++it) {
        float y = gap - x;
        float r1 = bn / x, r2 = bf / y;
        float f = r1 * r1 + r2 * r2 - 1.f;
        float fp = 2.f * (r2 * r2 / y - r1 * r1 / x);
        float xn = x - f / fp;
        if (!(xn > x)) break; // converged: rounding turns the step back
        x = fminf(xn, xm);
    }
    return x;
}

// The two stationary points between the eigenvalues (a local minimum and a
// local maximum), when they exist.  Returns how many were written.
// With t = lambda - q1 they are the roots in (0, gap) of
//     b1^2/t^2 + b2^2/(gap - t)^2 = 1,
// whose left side is convex with its minimum at tm (closed form): when that
// minimum is below 1 there is one root on each side of tm.  Each side is
// solved in the distance from its own end (t, and gap - t), which keeps
// full precision when the root lies close to that end.
TWA_HD int trs_middle(const Eig2 &g, f2 *out) {
    float b1 = g.b1, b2 = g.b2, gap = g.gap;
    if (!(gap > 0.f) || b1 == 0.f || b2 == 0.f) return 0;
    float c1 = cbrtf(b1 * b1), c2 = cbrtf(b2 * b2);
    float tm = gap * c1 / (c1 + c2);
    float y1 = b1 / tm, y2 = b2 / (gap - tm);
    if (y1 * y1 + y2 * y2 >= 1.f) return 0;
    float t = secular_side(b1, b2, gap, tm);
    float sr = secular_side(b2, b1, gap, gap - tm);
    // (q1 - lambda) = -t, (q2 - lambda) = gap - t
    float z[2][2] = {{-b1 / t, b2 / (gap - t)}, {-b1 / (gap - sr), b2 / sr}};
    for (int k = 0; k < 2; ++k) {
        float inv = inv_sqrt(z[k][0] * z[k][0] + z[k][1] * z[k][1]);
        out[k] = add(scl(g.v1, z[k][0] * inv), scl(g.v2, z[k][1] * inv));
    }
    return 2;
}

// Q and b of E_c(u) = sum_k (w_k/2)(r - <m_k, u>)^2 up to a constant
TWA_HD Eig2 piece_quadratic(f2 m0, f2 m1, float w0, float w1, float r) {
    float a = w0 * m0.x * m0.x + w1 * m1.x * m1.x;
    float c = w0 * m0.x * m0.y + w1 * m1.x * m1.y;
    float e = w0 * m0.y * m0.y + w1 * m1.y * m1.y;
    f2 b = scl(add(scl(m0, w0), scl(m1, w1)), r);
    return eig2(a, c, e, b);
}

// Which candidate a minimiser chose (for its derivative).
enum : int { CH_NONE = 0, CH_T = 1, CH_R0 = 2, CH_R1 = 3, CH_TAN = 4, CH_RADF = 5, CH_FLAT = 6 };
struct Choice {
    int kind; // CH_*
    f2 u;     // unit normal of the separating line
    f2 c;     // centre of the arc the configuration rests on (disk: origin)
};

// ---------------------------------------------------------------------------
// Disk (collision) minimiser on the difference variables (App. C, I):
// min (w0/2)|v0 - m0|^2 + (w1/2)|v1 - m1|^2  s.t.  dist(0, [v0, v1]) >= R.
// k0/k1: W_INF marks a certain end that must stay.
// ---------------------------------------------------------------------------
TWA_HD float disk_F(f2 u, f2 m0, f2 m1, float w0, float w1, float R) {
    float g0 = pos(R - dot(m0, u)), g1 = pos(R - dot(m1, u));
    return 0.5f * (w0 * g0 * g0 + w1 * g1 * g1);
}

// tangent normals from point q (|q| >= r) to the circle of radius r at c
TWA_HD int tangent_normals(f2 q, f2 c, float r, f2 *out) {
    f2 w = sub(q, c);
    float L2 = dot(w, w);
    float s2 = L2 - r * r;
    if (!(L2 > 0.f) || s2 < 0.f) return 0;
    float s = sqrtf(s2);
    f2 wp = perp(w);
    float inv = 1.f / L2;
    out[0] = scl(add(scl(w, r), scl(wp, s)), inv);
    out[1] = scl(sub(scl(w, r), scl(wp, s)), inv);
    return 2;
}

TWA_HD void disk_prox(f2 m0, f2 m1, float w0, float w1, int k0, int k1, float R, f2 &v0, f2 &v1,
                      Choice *ch = nullptr) {
    bool i0 = k0 == W_INF, i1 = k1 == W_INF;
    if (ch) {
        ch->kind = CH_NONE;
        ch->u = mk(1.f, 0.f);
        ch->c = mk(0.f, 0.f);
    }
    if (i0 && i1) {
        v0 = m0;
        v1 = m1;
        return;
    }
    if (i0 || i1) {
        f2 q = i0 ? m0 : m1, m = i0 ? m1 : m0;
        f2 best = mk(1.f, 0.f);
        int bk = CH_NONE;
        float bg = INFINITY;
        auto consider = [&](f2 u, int kind) {
            float g = pos(R - dot(m, u));
            if (g < bg) {
                bg = g;
                best = u;
                bk = kind;
            }
        };
        f2 tn[2];
        int nt = tangent_normals(q, mk(0.f, 0.f), R, tn);
        for (int k = 0; k < nt; ++k) consider(tn[k], CH_TAN);
        float mm = dot(m, m);
        if (mm > 0.f) {
            f2 u = scl(m, inv_sqrt(mm));
            if (dot(q, u) >= R) consider(u, CH_RADF);
        }
        f2 vm = (bg < INFINITY) ? add(m, scl(best, bg)) : m;
        v0 = i0 ? m0 : vm;
        v1 = i0 ? vm : m1;
        if (ch) {
            ch->kind = bk;
            ch->u = best;
        }
        return;
    }
    Eig2 g = piece_quadratic(m0, m1, w0, w1, R);
    f2 best = mk(1.f, 0.f);
    int bk = CH_NONE;
    float bF = INFINITY;
    auto consider = [&](f2 u, int kind) {
        float Fk = disk_F(u, m0, m1, w0, w1, R);
        if (Fk < bF || bk == CH_NONE) {
            bF = Fk;
            best = u;
            bk = kind;
        }
    };
    // one end pushed straight out while the other is clear: when valid it
    // is the minimiser outright (that end moves the least any feasible
    // configuration can move it, the other not at all), taken without
    // comparing F, which rounding decides wrongly when the tangent family's
    // root lies within ~1e-4 rad of it (F is stationary there).  Otherwise
    // both ends are pushed and the tangent family holds the minimum.
    float q0 = dot(m0, m0), q1 = dot(m1, m1);
    if (q0 > 0.f && q0 < R * R) {
        f2 u = scl(m0, inv_sqrt(q0));
        if (dot(m1, u) >= R) consider(u, CH_R0);
    }
    if (bk == CH_NONE && q1 > 0.f && q1 < R * R) {
        f2 u = scl(m1, inv_sqrt(q1));
        if (dot(m0, u) >= R) consider(u, CH_R1);
    }
    if (bk == CH_NONE) {
        f2 t0, alt;
        int nt = trs_global(g, &t0, &alt);
        consider(t0, CH_T);
        if (nt == 2) consider(alt, CH_T);
    }
    v0 = add(m0, scl(best, pos(R - dot(m0, best))));
    v1 = add(m1, scl(best, pos(R - dot(m1, best))));
    if (ch) {
        ch->kind = bk;
        ch->u = best;
    }
}

// ---------------------------------------------------------------------------
// Capsule (wall) minimiser, App. D and I.
// ---------------------------------------------------------------------------
struct Capsule {
    f2 a, b;
    float r;
};
TWA_HD float cap_h(const Capsule &C, f2 u) { return fmaxf(dot(C.a, u), dot(C.b, u)) + C.r; }
TWA_HD float cap_F(const Capsule &C, f2 u, f2 n0, f2 n1, float w0, float w1) {
    float h = cap_h(C, u);
    float g0 = pos(h - dot(n0, u)), g1 = pos(h - dot(n1, u));
    return 0.5f * (w0 * g0 * g0 + w1 * g1 * g1);
}
TWA_HD f2 closest_on_seg(f2 q, f2 a, f2 b) {
    f2 d = sub(b, a);
    float L2 = dot(d, d);
    float t = 0.f;
    if (L2 > 0.f) t = fminf(fmaxf(dot(sub(q, a), d) / L2, 0.f), 1.f);
    return add(a, scl(d, t));
}

// Best candidate so far of the capsule minimiser: least F, the earliest
// candidate on ties.
struct CapBest {
    f2 u = f2{1.f, 0.f};
    float F = INFINITY;
    int kind = CH_NONE, ctr = 0;
};

// Candidates of smooth piece pc (the arc around C.a, or C.b) in their fixed
// order: the global stationary point of the piece's quadratic (and its
// mirror in the hard case), and the two middle ones when the global point
// lies on the wrong half-circle.
TWA_HD void capsule_piece(const Capsule &C, f2 n0, f2 n1, float w0, float w1, int pc, f2 d, bool seg, CapBest &bb) {
    auto consider = [&](f2 u) {
        float Fk = cap_F(C, u, n0, n1, w0, w1);
        if (Fk < bb.F || bb.kind == CH_NONE) {
            bb.F = Fk;
            bb.u = u;
            bb.kind = CH_T;
            bb.ctr = pc;
        }
    };
    f2 c = pc ? C.b : C.a;
    Eig2 g = piece_quadratic(sub(n0, c), sub(n1, c), w0, w1, C.r);
    f2 t0, alt, mid[2];
    int k = trs_global(g, &t0, &alt);
    consider(t0);
    if (k == 2) consider(alt);
    // the piece's other local minimum can only matter when its global one
    // lies on the half-circle where the other end cap is the support
    float side = dot(d, t0);
    bool valid = !seg || (pc ? side >= 0.f : side <= 0.f);
    if (!valid) {
        int nm = trs_middle(g, mid);
        for (int q = 0; q < nm; ++q) consider(mid[q]);
    }
}

TWA_HD void capsule_finish(const Capsule C, f2 n0, f2 n1, float w0, float w1, f2 d, float L2, bool seg, f2 sw,
                           CapBest &bb, f2 &x0, f2 &x1, Choice *ch);

TWA_HD void capsule_prox(const Capsule C, f2 n0, f2 n1, float w0, float w1, int k0, int k1, f2 &x0, f2 &x1,
                         Choice *ch = nullptr) {
    bool i0 = k0 == W_INF, i1 = k1 == W_INF;
    if (ch) {
        ch->kind = CH_NONE;
        ch->u = mk(1.f, 0.f);
        ch->c = C.a;
    }
    if (i0 && i1) {
        x0 = n0;
        x1 = n1;
        return;
    }
    f2 d = sub(C.b, C.a);
    float L2 = dot(d, d);
    bool seg = L2 > 0.f;
    f2 sw = seg ? scl(perp(d), inv_sqrt(L2)) : mk(0.f, 1.f);
    if (i0 || i1) {
        // one end certain: the other moves along normals u visible from it
        // (<q, u> >= h(u)).  A tangent normal from q to the circle at one
        // end of the segment has q on its line, so it is visible exactly
        // when that end is the support in direction u: the sign of <d, u>,
        // tested with a slack of a few roundings of |d| only.  The other
        // candidates are tested as they stand.
        f2 q = i0 ? n0 : n1, m = i0 ? n1 : n0;
        const float dtol = 1e-6f * (fabsf(d.x) + fabsf(d.y));
        f2 best = mk(1.f, 0.f);
        int bk = CH_NONE, bc = 0;
        float bg = INFINITY;
        auto consider = [&](f2 u, int kind, int ctr) {
            float h = cap_h(C, u);
            if (kind == CH_TAN) {
                float side = dot(d, u); // > 0: the end b supports direction u
                if (ctr ? side < -dtol : side > dtol) return;
            } else if (dot(q, u) < h) {
                return; // not visible from the certain end
            }
            float g = pos(h - dot(m, u));
            if (g < bg) {
                bg = g;
                best = u;
                bk = kind;
                bc = ctr;
            }
        };
        // m's nearest boundary point, when visible from q, is the minimiser
        // outright (m must move at least that far, and q stays), so rounding
        // gets no say between it and a candidate of nearly the same direction
        {
            float tpar = seg ? fminf(fmaxf(dot(sub(m, C.a), d) / L2, 0.f), 1.f) : 0.f;
            f2 t = sub(m, closest_on_seg(m, C.a, C.b));
            float tt = dot(t, t);
            if (tt > 0.f) {
                const bool flat = seg && tpar > 0.f && tpar < 1.f;
                f2 u = flat ? (dot(t, sw) >= 0.f ? sw : scl(sw, -1.f)) : scl(t, inv_sqrt(tt));
                float h = cap_h(C, u);
                if (dot(q, u) >= h) {
                    bg = pos(h - dot(m, u));
                    best = u;
                    bk = flat ? CH_FLAT : CH_RADF;
                    bc = (seg && tpar >= 1.f) ? 1 : 0;
                }
            }
        }
        if (bk == CH_NONE) {
            f2 tn[2];
            int nt = tangent_normals(q, C.a, C.r, tn);
            for (int k = 0; k < nt; ++k) consider(tn[k], CH_TAN, 0);
            if (seg) {
                nt = tangent_normals(q, C.b, C.r, tn);
                for (int k = 0; k < nt; ++k) consider(tn[k], CH_TAN, 1);
            }
            f2 t0 = sub(m, C.a);
            if (dot(t0, t0) > 0.f) consider(scl(t0, inv_sqrt(dot(t0, t0))), CH_RADF, 0);
            if (seg) {
                f2 t1 = sub(m, C.b);
                if (dot(t1, t1) > 0.f) consider(scl(t1, inv_sqrt(dot(t1, t1))), CH_RADF, 1);
                consider(sw, CH_FLAT, 0);
                consider(scl(sw, -1.f), CH_FLAT, 0);
            }
        }
        f2 xm = (bg < INFINITY) ? add(m, scl(best, bg)) : m;
        x0 = i0 ? n0 : xm;
        x1 = i0 ? xm : n1;
        if (ch && bk != CH_NONE) {
            ch->kind = bk;
            ch->u = best;
            ch->c = bc ? C.b : C.a;
        }
        return;
    }
    CapBest bb;
    // (a) stationary points of each smooth piece
    for (int pc = 0; pc < (seg ? 2 : 1); ++pc) capsule_piece(C, n0, n1, w0, w1, pc, d, seg, bb);
    capsule_finish(C, n0, n1, w0, w1, d, L2, seg, sw, bb, x0, x1, ch);
}

TWA_HD void capsule_finish(const Capsule C, f2 n0, f2 n1, float w0, float w1, f2 d, float L2, bool seg, f2 sw,
                           CapBest &bb, f2 &x0, f2 &x1, Choice *ch) {
    f2 &best = bb.u;
    int &bk = bb.kind, &bc = bb.ctr;
    float &bF = bb.F;
    auto consider = [&](f2 u, int kind, int ctr) {
        float Fk = cap_F(C, u, n0, n1, w0, w1);
        if (Fk < bF || bk == CH_NONE) {
            bF = Fk;
            best = u;
            bk = kind;
            bc = ctr;
        }
    };
    // (c) kinks: slab against a flat side
    if (seg) {
        consider(sw, CH_FLAT, 0);
        consider(scl(sw, -1.f), CH_FLAT, 0);
    }
    // (b) nearest boundary point of one end while the other end is clear.
    // When it exists it is the minimiser outright: every feasible
    // configuration moves that end at least to the capsule's boundary, and
    // this one moves nothing else.  It is taken without comparing F, which
    // rounding decides wrongly when another candidate's direction lies
    // within a few 1e-4 of it (F is stationary there) while its x differs.
    for (int e = 0; e < 2; ++e) {
        f2 n = e ? n1 : n0, other = e ? n0 : n1;
        float tpar = seg ? fminf(fmaxf(dot(sub(n, C.a), d) / L2, 0.f), 1.f) : 0.f;
        f2 c = closest_on_seg(n, C.a, C.b);
        f2 t = sub(n, c);
        float tt = dot(t, t);
        if (tt > 0.f && tt < C.r * C.r) {
            // against the flat side the normal is +-sw exactly (n - c is
            // short and carries the rounding of c when n is near the segment)
            const bool flat = seg && tpar > 0.f && tpar < 1.f;
            f2 u = flat ? (dot(t, sw) >= 0.f ? sw : scl(sw, -1.f)) : scl(t, inv_sqrt(tt));
            if (dot(other, u) >= cap_h(C, u)) {
                best = u;
                bk = flat ? CH_FLAT : (e ? CH_R1 : CH_R0);
                bc = (seg && tpar >= 1.f) ? 1 : 0;
                break;
            }
        }
    }
    float h = cap_h(C, best);
    x0 = add(n0, scl(best, pos(h - dot(n0, best))));
    x1 = add(n1, scl(best, pos(h - dot(n1, best))));
    if (ch) {
        ch->kind = bk;
        ch->u = best;
        ch->c = bc ? C.b : C.a;
    }
}

// ---------------------------------------------------------------------------
// Derivatives (vector-Jacobian products) of the minimisers, holding the
// chosen candidate fixed.  The tangent family's optimal direction theta*
// depends on the inputs through E_theta(theta*, m, R) = 0 (implicit function
// theorem: dtheta = -E_theta,q dq / E_theta,theta).
// ---------------------------------------------------------------------------

// v_k = m_k + g_k u, g_k = max(0, R - <m_k, u>), around the origin.
// Given vb_k = dL/dv_k returns mb_k = dL/dm_k (added) and dL/dR (added).
TWA_HD void disk_vjp(f2 m0, f2 m1, float w0, float w1, int k0, int k1, float R, const Choice &ch, f2 vb0, f2 vb1,
                     f2 &mb0, f2 &mb1, float &Rb) {
    f2 u = ch.u, up = perp(u);
    bool i0 = k0 == W_INF, i1 = k1 == W_INF;
    if (ch.kind == CH_NONE) {
        mb0 = add(mb0, vb0);
        mb1 = add(mb1, vb1);
        return;
    }
    if (ch.kind == CH_TAN || ch.kind == CH_RADF) {
        // one certain end q stays; the free end m moves
        f2 q = i0 ? m0 : m1, m = i0 ? m1 : m0;
        f2 vq = i0 ? vb0 : vb1, vm = i0 ? vb1 : vb0;
        f2 qb = vq, mb;
        float g = R - dot(m, u);
        float a = g > 0.f ? 1.f : 0.f;
        if (ch.kind == CH_TAN) {
            // u on a tangent through q: <q, u(theta)> = R
            f2 du_b = scl(sub(scl(vm, g), scl(m, dot(u, vm))), a);
            float thb = dot(up, du_b);
            float qu = dot(q, up);
            float inv = fabsf(qu) > 1e-30f ? 1.f / qu : 0.f;
            mb = sub(vm, scl(u, a * dot(u, vm)));
            Rb += a * dot(u, vm) + thb * inv;
            qb = sub(qb, scl(u, thb * inv));
        } else {
            float L = sqrtf(dot(m, m));
            if (a > 0.f && L > 0.f) {
                // v = R m/|m|
                mb = scl(sub(vm, scl(u, dot(u, vm))), R / L);
                Rb += dot(u, vm);
            } else {
                mb = vm;
            }
        }
        if (i0) {
            mb0 = add(mb0, qb);
            mb1 = add(mb1, mb);
        } else {
            mb1 = add(mb1, qb);
            mb0 = add(mb0, mb);
        }
        return;
    }
    float g0 = R - dot(m0, u), g1 = R - dot(m1, u);
    float a0 = g0 > 0.f ? 1.f : 0.f, a1 = g1 > 0.f ? 1.f : 0.f;
    if (ch.kind == CH_T) {
        f2 r0 = sub(vb0, scl(u, a0 * dot(u, vb0)));
        f2 r1 = sub(vb1, scl(u, a1 * dot(u, vb1)));
        Rb += a0 * dot(u, vb0) + a1 * dot(u, vb1);
        float p0 = dot(m0, up), p1 = dot(m1, up);
        float thb = a0 * dot(sub(scl(up, g0), scl(u, p0)), vb0) + a1 * dot(sub(scl(up, g1), scl(u, p1)), vb1);
        float Ett = w0 * a0 * (p0 * p0 + g0 * dot(m0, u)) + w1 * a1 * (p1 * p1 + g1 * dot(m1, u));
        float c = fabsf(Ett) > 1e-30f ? -thb / Ett : 0.f;
        // dE_theta/dm_k = w_k a_k (<m_k,up> u - g_k up);  dE_theta/dR = -sum w_k a_k <m_k,up>
        r0 = add(r0, scl(sub(scl(u, p0), scl(up, g0)), c * w0 * a0));
        r1 = add(r1, scl(sub(scl(u, p1), scl(up, g1)), c * w1 * a1));
        Rb += c * (-(w0 * a0 * p0 + w1 * a1 * p1));
        mb0 = add(mb0, r0);
        mb1 = add(mb1, r1);
        return;
    }
    // radial: u = m_e/|m_e| for end e, the other end pushed along u if needed
    bool e1 = ch.kind == CH_R1;
    f2 me = e1 ? m1 : m0, mo = e1 ? m0 : m1;
    f2 ve = e1 ? vb1 : vb0, vo = e1 ? vb0 : vb1;
    float go = e1 ? g0 : g1, ao = e1 ? a0 : a1;
    float L = sqrtf(dot(me, me));
    f2 ub = add(scl(ve, R), scl(sub(scl(vo, go), scl(mo, dot(u, vo))), ao));
    Rb += dot(u, ve) + ao * dot(u, vo);
    f2 mbo = sub(vo, scl(u, ao * dot(u, vo)));
    f2 mbe = L > 0.f ? scl(sub(ub, scl(u, dot(u, ub))), 1.f / L) : mk(0.f, 0.f);
    if (e1) {
        mb1 = add(mb1, mbe);
        mb0 = add(mb0, mbo);
    } else {
        mb0 = add(mb0, mbe);
        mb1 = add(mb1, mbo);
    }
}

// x_k = n_k + g_k u around the capsule: arc kinds reduce to the disk at the
// chosen centre; a flat side keeps u fixed.
TWA_HD void capsule_vjp(const Capsule C, f2 n0, f2 n1, float w0, float w1, int k0, int k1, const Choice &ch, f2 xb0,
                        f2 xb1, f2 &nb0, f2 &nb1, float &rb) {
    if (ch.kind == CH_FLAT) {
        f2 u = ch.u;
        float h = cap_h(C, u);
        for (int e = 0; e < 2; ++e) {
            f2 n = e ? n1 : n0, xb = e ? xb1 : xb0;
            bool fixed = (e ? k1 : k0) == W_INF;
            float a = (!fixed && h - dot(n, u) > 0.f) ? 1.f : 0.f;
            f2 r = sub(xb, scl(u, a * dot(u, xb)));
            rb += a * dot(u, xb);
            if (e) nb1 = add(nb1, r);
            else nb0 = add(nb0, r);
        }
        return;
    }
    disk_vjp(sub(n0, ch.c), sub(n1, ch.c), w0, w1, k0, k1, C.r, ch, xb0, xb1, nb0, nb1, rb);
}

// ---------------------------------------------------------------------------
// Agent-agent minimiser through the difference variables v = x' - x of each
// break-point (App. C).  At fixed v the best x is
//   x = (rho n + rho' (n' - v)) / (rho + rho'),
// leaving (omega/2)|v - (n' - n)|^2 with omega = rho rho'/(rho + rho').
// ---------------------------------------------------------------------------
TWA_HD void pair_weight(float r, float rp, int k, int kp, float &om, int &kom) {
    if (k == W_INF && kp == W_INF) {
        om = 0.f;
        kom = W_INF;
    } else if (k == W_INF) {
        om = rp;
        kom = W_STD;
    } else if (kp == W_INF) {
        om = r;
        kom = W_STD;
    } else {
        om = r * rp / (r + rp);
        kom = W_STD;
    }
}

// rebuild one break-point pair from v (component-wise)
TWA_HD void pair_rebuild(float r, float rp, int k, int kp, float n, float np, float v, float &x,
                                             float &xp) {
    if (k == W_INF && kp == W_INF) {
        x = n;
        xp = np;
    } else if (k == W_INF) {
        x = n;
        xp = n + v;
    } else if (kp == W_INF) {
        xp = np;
        x = np - v;
    } else {
        x = (r * n + rp * (np - v)) / (r + rp);
        xp = x + v;
    }
}

// Full collision minimiser (App. C): n, weights -> x.  D == 3 solves in the
// plane spanned by the two difference vectors (the optimum lies there).
template <int D>
TWA_HD void coll_prox(const float *n, const float *w, const int *k, float R, float *x, Choice *ch = nullptr) {
    float om_l, om_h;
    int ko_l, ko_h;
    pair_weight(w[0], w[2], k[0], k[2], om_l, ko_l);
    pair_weight(w[1], w[3], k[1], k[3], om_h, ko_h);
    float vl[3], vh[3];
    if constexpr (D == 2) {
        f2 ml = mk(n[4] - n[0], n[5] - n[1]);
        f2 mh = mk(n[6] - n[2], n[7] - n[3]);
        f2 a, b;
        disk_prox(ml, mh, om_l, om_h, ko_l, ko_h, R, a, b, ch);
        vl[0] = a.x, vl[1] = a.y, vh[0] = b.x, vh[1] = b.y;
    } else {
        float ml[3] = {n[6] - n[0], n[7] - n[1], n[8] - n[2]};
        float mh[3] = {n[9] - n[3], n[10] - n[4], n[11] - n[5]};
        float nl = sqrtf(ml[0] * ml[0] + ml[1] * ml[1] + ml[2] * ml[2]);
        float nh = sqrtf(mh[0] * mh[0] + mh[1] * mh[1] + mh[2] * mh[2]);
        const float *f = nl > 0.f ? ml : mh;
        float nf = nl > 0.f ? nl : nh;
        float e1[3] = {1.f, 0.f, 0.f}, e2[3];
        if (nf > 0.f) e1[0] = f[0] / nf, e1[1] = f[1] / nf, e1[2] = f[2] / nf;
        const float *g = nl > 0.f ? mh : ml;
        float pr = g[0] * e1[0] + g[1] * e1[1] + g[2] * e1[2];
        float w3[3] = {g[0] - pr * e1[0], g[1] - pr * e1[1], g[2] - pr * e1[2]};
        float nw = sqrtf(w3[0] * w3[0] + w3[1] * w3[1] + w3[2] * w3[2]);
        if (!(nw > 1e-6f * (nf + nh))) {
            int ax = 0;
            if (fabsf(e1[1]) < fabsf(e1[ax])) ax = 1;
            if (fabsf(e1[2]) < fabsf(e1[ax])) ax = 2;
            float t[3] = {0.f, 0.f, 0.f};
            t[ax] = 1.f;
            float p2 = e1[ax];
            w3[0] = t[0] - p2 * e1[0], w3[1] = t[1] - p2 * e1[1], w3[2] = t[2] - p2 * e1[2];
            nw = sqrtf(w3[0] * w3[0] + w3[1] * w3[1] + w3[2] * w3[2]);
        }
        for (int q = 0; q < 3; ++q) e2[q] = w3[q] / nw;
        f2 a2 = mk(ml[0] * e1[0] + ml[1] * e1[1] + ml[2] * e1[2], ml[0] * e2[0] + ml[1] * e2[1] + ml[2] * e2[2]);
        f2 b2 = mk(mh[0] * e1[0] + mh[1] * e1[1] + mh[2] * e1[2], mh[0] * e2[0] + mh[1] * e2[1] + mh[2] * e2[2]);
        f2 a, b;
        disk_prox(a2, b2, om_l, om_h, ko_l, ko_h, R, a, b);
        for (int q = 0; q < 3; ++q) {
            vl[q] = a.x * e1[q] + a.y * e2[q];
            vh[q] = b.x * e1[q] + b.y * e2[q];
        }
    }
    for (int c = 0; c < D; ++c) {
        pair_rebuild(w[0], w[2], k[0], k[2], n[c], n[2 * D + c], vl[c], x[c], x[2 * D + c]);
        pair_rebuild(w[1], w[3], k[1], k[3], n[D + c], n[3 * D + c], vh[c], x[D + c], x[3 * D + c]);
    }
}


// VJP of pair_rebuild for one coordinate: x = a n + b np - b v, xp = x + v.
TWA_HD void pair_rebuild_vjp(float r, float rp, int k, int kp, float xb, float xpb, float &nb, float &npb, float &vb) {
    if (k == W_INF && kp == W_INF) {
        nb += xb;
        npb += xpb;
        vb = 0.f;
    } else if (k == W_INF) {
        nb += xb + xpb;
        vb = xpb;
    } else if (kp == W_INF) {
        npb += xb + xpb;
        vb = -xb;
    } else {
        float a = r / (r + rp), b = rp / (r + rp);
        nb += a * (xb + xpb);
        npb += b * (xb + xpb);
        vb = -b * xb + (1.f - b) * xpb;
    }
}

// VJP of the planar collision minimiser: xb [8] -> nb [8] (added), Rb (added).
TWA_HD void coll_vjp2(const float *n, const float *w, const int *k, float R, const float *xb, float *nb, float &Rb) {
    float x[8];
    Choice ch;
    coll_prox<2>(n, w, k, R, x, &ch);
    float om_l, om_h;
    int ko_l, ko_h;
    pair_weight(w[0], w[2], k[0], k[2], om_l, ko_l);
    pair_weight(w[1], w[3], k[1], k[3], om_h, ko_h);
    float vl[2], vh[2];
    for (int c = 0; c < 2; ++c) {
        pair_rebuild_vjp(w[0], w[2], k[0], k[2], xb[c], xb[4 + c], nb[c], nb[4 + c], vl[c]);
        pair_rebuild_vjp(w[1], w[3], k[1], k[3], xb[2 + c], xb[6 + c], nb[2 + c], nb[6 + c], vh[c]);
    }
    f2 ml = mk(n[4] - n[0], n[5] - n[1]);
    f2 mh = mk(n[6] - n[2], n[7] - n[3]);
    f2 mbl = mk(0.f, 0.f), mbh = mk(0.f, 0.f);
    disk_vjp(ml, mh, om_l, om_h, ko_l, ko_h, R, ch, mk(vl[0], vl[1]), mk(vh[0], vh[1]), mbl, mbh, Rb);
    nb[4] += mbl.x, nb[5] += mbl.y, nb[0] -= mbl.x, nb[1] -= mbl.y;
    nb[6] += mbh.x, nb[7] += mbh.y, nb[2] -= mbh.x, nb[3] -= mbh.y;
}

// VJP of the energy minimiser (linear in n) for one coordinate.
TWA_HD void energy_vjp(float wl, float wh, int kl, int kh, float C, float xlb, float xhb, float &nlb, float &nhb) {
    if (C <= 0.f || (kl == W_INF && kh == W_INF)) {
        nlb += xlb;
        nhb += xhb;
    } else if (kl == W_INF) {
        float a = 2.f * C / (2.f * C + wh), b = wh / (2.f * C + wh);
        nlb += xlb + a * xhb;
        nhb += b * xhb;
    } else if (kh == W_INF) {
        float a = 2.f * C / (2.f * C + wl), b = wl / (2.f * C + wl);
        nhb += xhb + a * xlb;
        nlb += b * xlb;
    } else if (kl == W_ZERO && kh == W_ZERO) {
        nlb += 0.5f * (xlb + xhb);
        nhb += 0.5f * (xlb + xhb);
    } else {
        float den = 2.f * C * (wl + wh) + wl * wh;
        nlb += (wl * (wh + 2.f * C) * xlb + 2.f * C * wl * xhb) / den;
        nhb += (2.f * C * wh * xlb + wh * (wl + 2.f * C) * xhb) / den;
    }
}

} // namespace twa
