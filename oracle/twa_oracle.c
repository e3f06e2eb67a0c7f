/*
 * twa_oracle.c -- plain FP64 CPU reference of the three-weight message-passing
 * trajectory planner (Bento, Derbinsky, Alonso-Mora, Yedidia, NIPS 2013).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file: only the tests, the smoke check and the benchmark's CPU-baseline leg.
 * It shares no code, header, table or helper with the GPU library.
 *
 * What it computes, step by step in the paper's order (App. B, steps 1-7):
 *   1. n = z - u per edge
 *   2. x = g_b(n, <-rho) per factor, each minimiser solved exactly
 *   3. ->rho per factor (0, rho0 or infinity)
 *   4. m = x + u per edge
 *   5. z = weighted mean of m per equality node
 *   6. <-rho per node
 *   7. u update per edge
 * Minimisers:
 *   fixed start/goal   : a unary factor emitting the constant with weight inf
 *   energy             : closed form of App. E (eq. energy_minimizer_output)
 *   agent-agent        : reduction to the wall minimiser of App. C (with the
 *                        weight/target of the difference variable re-derived,
 *                        see twa_coll_prox) and the spring-slab analogue
 *   agent-wall         : spring-slab analogue of App. D and App. I:
 *                        scenario 1 (no crossing -> x = n), otherwise the
 *                        cheaper of (a) the slab tangent to the capsule
 *                        region, argmin over theta of E_tangent, and (b) one
 *                        spring relaxed, the other end at the nearest visible
 *                        boundary point of the region.
 * The tangent family is minimised exactly: every stationary point of each
 * smooth piece of E_tangent is a Lagrange point of a quadratic on the unit
 * circle, found by bracketing the roots of its secular equation, plus the
 * two kink directions of the capsule (App. I notes at most two kinks).
 *
 * Readings where the paper is silent or garbled (all listed in the design
 * notes of the repository):
 *   - the <-rho rule and the special u rule live in a lost figure (App. B):
 *     <-rho_j = INF if any incoming ->rho is INF, ZERO if all are ZERO, else
 *     STD; u <- 0 unless both ->rho^k and <-rho^{k+1} are STD.
 *   - start and goal are constants (Sec. 3) yet equality nodes (Sec. 3.3):
 *     each gets a unary factor x = const with weight infinity.
 *   - weight infinity is taken as the exact limit; weight zero is replaced by
 *     a small value shared by both weights (App. C, D, E).
 *   - the capsule support point P(theta) uses <x_R - x_L, n(theta)> >= 0.
 *   - exact ties of the argmin are broken deterministically: lowest energy,
 *     then tangent before boundary candidates, then smallest theta in
 *     [0, 2 pi).  The paper draws uniformly at random (App. B, step 2).
 *   - non-collision means distance >= r_i + r_j (Sec. 3.1 footnote), so a
 *     collision factor is active iff the closest approach is < r_i + r_j.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TOR_PI 3.14159265358979323846264338327950288
#define TOR_2PI (2.0 * TOR_PI)

enum { TOR_ZERO = 0, TOR_STD = 1, TOR_INF = 2 };
enum { TOR_F_FIXED = 0, TOR_F_ENERGY = 1, TOR_F_COLL = 2, TOR_F_WALL = 3 };
enum { TOR_MODE_TWA = 0, TOR_MODE_ADMM = 1 };
/* the per-segment factor of each agent (eq. velo_cost_pair_wise, eq. max_vel_min) */
enum { TOR_COST_ENERGY = 0, TOR_COST_NONE = 1, TOR_COST_MAXVEL = 2, TOR_COST_MINVEL = 3, TOR_COST_VO = 4 };
/* TOR_COST_VO: one planning epoch of the velocity-obstacle local planner
 * (Sec. 5, App. H), eta = 1: x(0) are the current positions, xT the
 * reference end positions x^ref, C[i] the cost c_i of deviating from them.
 * The energy factors are absent and each goal factor becomes the VO cost
 * minimiser g^cost(x^ref, n, inf, rho, c) (eq. minimizer_rvo_cost), weight
 * rho0; the agent-agent and agent-wall factors with their start ends fixed
 * are eq. minimizer_rvo_coll and eq. minimizer_rvo_wall as they stand. */

/* Relative size of the small value shared by both weights when a zero weight is replaced (App. C-E). */
#define TOR_ZERO_WEIGHT 1e-9

/* ------------------------------------------------------------------------ */
/* small 2D helpers                                                           */
/* ------------------------------------------------------------------------ */

static double dot2(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1]; }
static double wrap2pi(double t) {
    t = fmod(t, TOR_2PI);
    if (t < 0) t += TOR_2PI;
    if (t >= TOR_2PI) t -= TOR_2PI;
    return t;
}
/* is angle t inside the arc [lo, lo+len] (len in [0, 2pi]) ? */
static int ang_in(double t, double lo, double len) {
    double d = wrap2pi(t - lo);
    return d <= len + 1e-13 || d >= TOR_2PI - 1e-13;
}

/* Closest approach of two agents moving at constant velocity between two
 * break-points, given the relative positions d0 (at alpha=0) and d1 (at
 * alpha=1): min over alpha in [0,1] of |(1-alpha) d0 + alpha d1|
 * (constraint of eq. basic_opt_prob). */
double tor_cpa(const double *d0, const double *d1, int dim) {
    double e[3], ee = 0, de = 0;
    for (int k = 0; k < dim; k++) {
        e[k] = d1[k] - d0[k];
        ee += e[k] * e[k];
        de += d0[k] * e[k];
    }
    double a = 0.0;
    if (ee > 0) {
        a = -de / ee;
        if (a < 0) a = 0;
        if (a > 1) a = 1;
    }
    double s = 0;
    for (int k = 0; k < dim; k++) {
        double v = d0[k] + a * e[k];
        s += v * v;
    }
    return sqrt(s);
}

static double point_seg_dist2d(const double *q, const double *a, const double *b) {
    double d[2] = {b[0] - a[0], b[1] - a[1]};
    double L2 = dot2(d, d);
    double t = 0;
    if (L2 > 0) {
        t = ((q[0] - a[0]) * d[0] + (q[1] - a[1]) * d[1]) / L2;
        if (t < 0) t = 0;
        if (t > 1) t = 1;
    }
    double x = a[0] + t * d[0] - q[0], y = a[1] + t * d[1] - q[1];
    return sqrt(x * x + y * y);
}

static double orient(const double *a, const double *b, const double *c) {
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

/* Minimum distance between planar segments [p0,p1] and [q0,q1] (the
 * constraint of eq. wall_minimizer over all alpha, beta in [0,1]). */
double tor_segseg(const double *p0, const double *p1, const double *q0, const double *q1) {
    double o1 = orient(p0, p1, q0), o2 = orient(p0, p1, q1);
    double o3 = orient(q0, q1, p0), o4 = orient(q0, q1, p1);
    if (((o1 > 0 && o2 < 0) || (o1 < 0 && o2 > 0)) && ((o3 > 0 && o4 < 0) || (o3 < 0 && o4 > 0)))
        return 0.0;
    double m = point_seg_dist2d(p0, q0, q1);
    double t = point_seg_dist2d(p1, q0, q1);
    if (t < m) m = t;
    t = point_seg_dist2d(q0, p0, p1);
    if (t < m) m = t;
    t = point_seg_dist2d(q1, p0, p1);
    if (t < m) m = t;
    return m;
}

/* ------------------------------------------------------------------------ */
/* Energy minimiser (App. E)                                                  */
/* ------------------------------------------------------------------------ */

/* weights: value >= 0, or isinf for the certain weight.  A zero weight is a
 * small positive value by the time it reaches here, except both-zero which
 * is handled as the equal-weights limit. */
void tor_prox_energy(const double *nl, const double *nh, double wl, double wh, double C, int dim,
                     double *xl, double *xh) {
    int il = isinf(wl), ih = isinf(wh);
    for (int k = 0; k < dim; k++) {
        double a = nl[k], b = nh[k];
        if (C <= 0) {
            xl[k] = a;
            xh[k] = b;
        } else if (il && ih) {
            xl[k] = a;
            xh[k] = b;
        } else if (il) {
            /* limit wl -> inf: x_lo = n_lo, x_hi = (wh n_hi + 2C n_lo) / (2C + wh) */
            xl[k] = a;
            xh[k] = (wh * b + 2 * C * a) / (2 * C + wh);
        } else if (ih) {
            xh[k] = b;
            xl[k] = (wl * a + 2 * C * b) / (2 * C + wl);
        } else if (wl == 0 && wh == 0) {
            xl[k] = xh[k] = 0.5 * (a + b);
        } else {
            double den = 2 * C * (wl + wh) + wl * wh;
            xl[k] = (wl * wh * a + 2 * C * (wl * a + wh * b)) / den;
            xh[k] = (wl * wh * b + 2 * C * (wl * a + wh * b)) / den;
        }
    }
}

/*
 * Maximum / minimum velocity minimiser (App. F and App. G): minimise
 *   (wl/2)|xl - nl|^2 + (wh/2)|xh - nh|^2  subject to  |xl - xh| <= C
 * (maximum) or |xl - xh| >= C (minimum).  Returns 1 when the constraint
 * binds (the factor then sends weight rho0, Sec. 3.3.3), 0 when x = n (weight
 * zero).  With the constraint active the KKT conditions give x as a function
 * of the multiplier lambda (eq. sol_paramterized_max_vel), and lambda follows
 * from |xl - xh| = C (eq. unique_lambda_val_max_vel, the same expression for
 * both: positive for the maximum, negative for the minimum).  Infinite
 * weights are taken as exact limits: the certain end stays, the other end
 * moves to distance C of it.  Both weights zero: equal small weights (the
 * result does not depend on their common value).  A minimum-velocity factor
 * whose two ends coincide has no direction to push along: +e1 is used.
 */
int tor_prox_vel(const double *nl, const double *nh, double wl, double wh, double C, int dim, int minimum,
                 double *xl, double *xh) {
    double d[3] = {0, 0, 0}, dn = 0;
    for (int k = 0; k < dim; k++) {
        d[k] = nl[k] - nh[k];
        dn += d[k] * d[k];
    }
    dn = sqrt(dn);
    int bind = minimum ? (dn < C) : (dn > C);
    if (!bind) {
        for (int k = 0; k < dim; k++) xl[k] = nl[k], xh[k] = nh[k];
        return 0;
    }
    int il = isinf(wl), ih = isinf(wh);
    if (il && ih) {
        for (int k = 0; k < dim; k++) xl[k] = nl[k], xh[k] = nh[k];
        return 1;
    }
    if (wl == 0 && wh == 0) wl = wh = 1.0;
    if (dn == 0) {
        /* coinciding ends (minimum velocity only; lambda is then singular):
         * the KKT conditions keep the weighted mean and put the ends C apart
         * along the chosen direction +e1 */
        double sl = il ? 0.0 : (ih ? 1.0 : wh / (wl + wh));
        for (int k = 0; k < dim; k++) {
            double e = (k == 0) ? C : 0.0;
            xl[k] = nl[k] + sl * e;
            xh[k] = nh[k] - (1.0 - sl) * e;
        }
        return 1;
    }
    double ratio = dn / C; /* |n_lo - n_hi| / C */
    if (il || ih) {
        /* lambda / w_free -> ratio - 1 as w_certain -> infinity */
        const double *nf = il ? nl : nh, *nv = il ? nh : nl;
        double *xf = il ? xl : xh, *xv = il ? xh : xl;
        for (int k = 0; k < dim; k++) {
            xf[k] = nf[k];
            xv[k] = (nv[k] + (ratio - 1.0) * nf[k]) / ratio;
        }
        return 1;
    }
    double lambda = (ratio - 1.0) / (1.0 / wl + 1.0 / wh);
    double den = wl * wh + lambda * (wl + wh);
    for (int k = 0; k < dim; k++) {
        double a = nl[k], b = nh[k];
        xl[k] = (wl * (wh + lambda) * a + lambda * wh * b) / den;
        xh[k] = (wh * (wl + lambda) * b + lambda * wl * a) / den;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Lagrange points of a quadratic on the unit circle                          */
/* ------------------------------------------------------------------------ */
/*
 * E(n) = sum_k (w_k/2) (r - <m_k, n>)^2 on |n| = 1 equals
 *   1/2 n^T Q n - <b, n> + const,  Q = sum w_k m_k m_k^T,  b = r sum w_k m_k.
 * Stationary points satisfy (Q - lambda I) n = b.  In the eigenbasis of Q
 * (q1 <= q2, coordinates beta of b) n has coordinates beta_k/(q_k - lambda)
 * and lambda solves f(lambda) = sum beta_k^2/(q_k-lambda)^2 - 1 = 0, which has
 * one root below q1, one above q2 and 0 or 2 between (f is convex there).
 * Zero beta_k add the points lambda = q_k.  Every case is enumerated, so all
 * (at most four) stationary points are returned as unit vectors.
 */
static double secf(double b1, double b2, double q1, double q2, double l) {
    double t1 = b1 / (q1 - l), t2 = b2 / (q2 - l);
    return t1 * t1 + t2 * t2 - 1.0;
}
static double bisect_sec(double b1, double b2, double q1, double q2, double lo, double hi) {
    double flo = secf(b1, b2, q1, q2, lo);
    for (int it = 0; it < 400; it++) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm = secf(b1, b2, q1, q2, mid);
        if (isnan(fm)) fm = INFINITY;
        if ((fm < 0) == (flo < 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

static void energy_derivs(const double *w, const double m[][2], double r, double th, double *e1,
                          double *e2) {
    double c = cos(th), s = sin(th);
    double d1 = 0, d2 = 0;
    for (int k = 0; k < 2; k++) {
        double a = m[k][0] * c + m[k][1] * s;   /* <m, n>  */
        double ap = -m[k][0] * s + m[k][1] * c; /* <m, n'> */
        d1 += w[k] * (r - a) * (-ap);
        d2 += w[k] * (ap * ap + (r - a) * a);
    }
    *e1 = d1;
    *e2 = d2;
}

/* Fills th[] with the angles of all stationary points; returns their count. */
static int circle_stationary(const double *w, const double m[][2], double r, double *th) {
    double a = 0, c = 0, e = 0, bx = 0, by = 0, scale = 0;
    for (int k = 0; k < 2; k++) {
        a += w[k] * m[k][0] * m[k][0];
        c += w[k] * m[k][0] * m[k][1];
        e += w[k] * m[k][1] * m[k][1];
        bx += r * w[k] * m[k][0];
        by += r * w[k] * m[k][1];
        scale += r * w[k] * sqrt(m[k][0] * m[k][0] + m[k][1] * m[k][1]);
    }
    double mean = 0.5 * (a + e), rad = hypot(0.5 * (a - e), c);
    double q1 = mean - rad, q2 = mean + rad;
    double psi = 0.5 * atan2(2 * c, a - e);
    double v2[2] = {cos(psi), sin(psi)}, v1[2] = {-v2[1], v2[0]};
    double b1 = bx * v1[0] + by * v1[1], b2 = bx * v2[0] + by * v2[1];
    double tol = 1e-13 * (scale + fabs(q2) + 1e-300);
    if (fabs(b1) <= tol) b1 = 0;
    if (fabs(b2) <= tol) b2 = 0;
    double y[8][2];
    int n = 0;
    double gap = q2 - q1;
    if (gap <= 1e-13 * (fabs(q1) + fabs(q2) + 1e-300)) {
        /* Q is a multiple of the identity: E = const - <b, n> */
        double bn = hypot(b1, b2);
        if (bn > 0) {
            y[n][0] = b1 / bn, y[n][1] = b2 / bn, n++;
            y[n][0] = -b1 / bn, y[n][1] = -b2 / bn, n++;
        } else {
            /* E is constant: every direction is stationary */
            y[n][0] = 1, y[n][1] = 0, n++;
        }
    } else if (b1 != 0 && b2 != 0) {
        double bn = hypot(b1, b2);
        double l = bisect_sec(b1, b2, q1, q2, q1 - bn, q1 - fabs(b1));
        y[n][0] = b1 / (q1 - l), y[n][1] = b2 / (q2 - l), n++;
        l = bisect_sec(b1, b2, q1, q2, q2 + fabs(b2), q2 + bn);
        y[n][0] = b1 / (q1 - l), y[n][1] = b2 / (q2 - l), n++;
        double t = cbrt((b1 * b1) / (b2 * b2));
        double lm = (q1 + t * q2) / (1 + t);
        double fm = secf(b1, b2, q1, q2, lm);
        if (fm < 0) {
            l = bisect_sec(b1, b2, q1, q2, q1, lm);
            y[n][0] = b1 / (q1 - l), y[n][1] = b2 / (q2 - l), n++;
            l = bisect_sec(b1, b2, q1, q2, lm, q2);
            y[n][0] = b1 / (q1 - l), y[n][1] = b2 / (q2 - l), n++;
        } else if (fm == 0) {
            y[n][0] = b1 / (q1 - lm), y[n][1] = b2 / (q2 - lm), n++;
        }
    } else if (b1 == 0 && b2 != 0) {
        y[n][0] = 0, y[n][1] = 1, n++;
        y[n][0] = 0, y[n][1] = -1, n++;
        double t = b2 / gap; /* lambda = q1 */
        if (t * t <= 1) {
            double s = sqrt(1 - t * t);
            y[n][0] = s, y[n][1] = t, n++;
            y[n][0] = -s, y[n][1] = t, n++;
        }
    } else if (b2 == 0 && b1 != 0) {
        y[n][0] = 1, y[n][1] = 0, n++;
        y[n][0] = -1, y[n][1] = 0, n++;
        double t = -b1 / gap; /* lambda = q2 */
        if (t * t <= 1) {
            double s = sqrt(1 - t * t);
            y[n][0] = t, y[n][1] = s, n++;
            y[n][0] = t, y[n][1] = -s, n++;
        }
    } else {
        y[n][0] = 1, y[n][1] = 0, n++;
        y[n][0] = -1, y[n][1] = 0, n++;
        y[n][0] = 0, y[n][1] = 1, n++;
        y[n][0] = 0, y[n][1] = -1, n++;
    }
    for (int i = 0; i < n; i++) {
        double nx = y[i][0] * v1[0] + y[i][1] * v2[0];
        double ny = y[i][0] * v1[1] + y[i][1] * v2[1];
        double t = atan2(ny, nx);
        /* polish on E'(theta) = 0; keep a step only if it reduces |E'| */
        for (int it = 0; it < 4; it++) {
            double d1, d2;
            energy_derivs(w, m, r, t, &d1, &d2);
            if (d2 == 0) break;
            double tn = t - d1 / d2, e1n, e2n;
            energy_derivs(w, m, r, tn, &e1n, &e2n);
            if (fabs(e1n) < fabs(d1) && fabs(tn - t) < 0.1) t = tn;
            else break;
        }
        th[i] = wrap2pi(t);
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Spring-slab analogue for a capsule region (App. D and App. I)              */
/* ------------------------------------------------------------------------ */
/*
 * Region R: all points within distance r of the segment [xa, xb] (xa == xb
 * gives a disk).  Problem: min (w0/2)|x0 - n0|^2 + (w1/2)|x1 - n1|^2 subject
 * to segment [x0, x1] not entering the interior of R.
 */
typedef struct {
    double a[2], b[2], r;
} capsule;

/* support value h(theta) = <P(theta), n(theta)> with P the capsule point of
 * outward normal n(theta): x_R + r n if <x_R - x_L, n> >= 0, else x_L + r n */
static void support_point(const capsule *R, double th, double P[2]) {
    double n[2] = {cos(th), sin(th)};
    double d[2] = {R->b[0] - R->a[0], R->b[1] - R->a[1]};
    const double *c = (dot2(d, n) >= 0) ? R->b : R->a;
    P[0] = c[0] + R->r * n[0];
    P[1] = c[1] + R->r * n[1];
}

static int in_region(const capsule *R, const double *q) {
    return point_seg_dist2d(q, R->a, R->b) < R->r;
}

typedef struct {
    double E;   /* energy */
    int kind;   /* 0 = tangent, 1 = boundary with x1 fixed, 2 = boundary with x0 fixed */
    double th;  /* tangent direction, or the contact normal angle for boundary */
    double x0[2], x1[2];
} cand;

static int better(const cand *c, const cand *best) {
    double tol = 1e-11 * fmax(fabs(best->E), 1e-300);
    if (c->E < best->E - tol) return 1;
    if (c->E > best->E + tol) return 0;
    if (c->kind != best->kind) return c->kind < best->kind;
    return c->th < best->th;
}

/* E_tangent(theta) (eq. one_dime_prob_mech_analog_function) and the
 * configuration it stands for. */
static void tangent_config(const capsule *R, const double *n0, const double *n1, double w0, double w1,
                           double th, cand *out) {
    double P[2], n[2] = {cos(th), sin(th)};
    support_point(R, th, P);
    double g0 = (P[0] - n0[0]) * n[0] + (P[1] - n0[1]) * n[1];
    double g1 = (P[0] - n1[0]) * n[0] + (P[1] - n1[1]) * n[1];
    out->kind = 0;
    out->th = wrap2pi(th);
    out->x0[0] = n0[0] + g0 * n[0], out->x0[1] = n0[1] + g0 * n[1];
    out->x1[0] = n1[0] + g1 * n[0], out->x1[1] = n1[1] + g1 * n[1];
    double e0 = isinf(w0) ? 0.0 : 0.5 * w0 * g0 * g0;
    double e1 = isinf(w1) ? 0.0 : 0.5 * w1 * g1 * g1;
    out->E = e0 + e1;
}

/* Visible normal-angle arc of the disk piece centred at c, seen from q:
 * <q - c, n> >= r, i.e. [phi - beta, phi + beta].  Returns 0 if q is inside. */
static int disk_visible(const double *c, double r, const double *q, double *lo, double *len) {
    double v[2] = {q[0] - c[0], q[1] - c[1]};
    double L = sqrt(dot2(v, v));
    if (L < r) return 0;
    double beta = acos(fmin(1.0, r / L));
    *lo = wrap2pi(atan2(v[1], v[0]) - beta);
    *len = 2 * beta;
    return 1;
}

/* Nearest point of the boundary of R to t among points visible from q (the
 * segment from the point to q does not cross the interior of R).  Boundary
 * points are parametrised by their outward normal angle; a point of normal
 * n is visible iff <q, n> >= h(n).  Returns 0 if none. */
static int nearest_visible(const capsule *R, const double *q, const double *t, double out[2],
                           double *out_th) {
    double d[2] = {R->b[0] - R->a[0], R->b[1] - R->a[1]};
    double L = sqrt(dot2(d, d));
    double best = INFINITY;
    int found = 0;
    const double *ctr[2] = {R->b, R->a};
    double phid = atan2(d[1], d[0]);
    for (int piece = 0; piece < (L > 0 ? 2 : 1); piece++) {
        const double *c = ctr[piece];
        double plo, plen;
        if (L > 0) {
            plo = wrap2pi(phid + (piece == 0 ? -0.5 * TOR_PI : 0.5 * TOR_PI));
            plen = TOR_PI;
        } else {
            plo = 0;
            plen = TOR_2PI;
        }
        double vlo, vlen;
        if (!disk_visible(c, R->r, q, &vlo, &vlen)) continue;
        double cands[5];
        int nc = 0;
        double tv[2] = {t[0] - c[0], t[1] - c[1]};
        if (dot2(tv, tv) > 0) cands[nc++] = atan2(tv[1], tv[0]);
        cands[nc++] = vlo;
        cands[nc++] = vlo + vlen;
        if (L > 0) {
            cands[nc++] = plo;
            cands[nc++] = plo + plen;
        }
        for (int k = 0; k < nc; k++) {
            double th = wrap2pi(cands[k]);
            if (!ang_in(th, plo, plen) || !ang_in(th, vlo, vlen)) continue;
            double p[2] = {c[0] + R->r * cos(th), c[1] + R->r * sin(th)};
            double dd = (p[0] - t[0]) * (p[0] - t[0]) + (p[1] - t[1]) * (p[1] - t[1]);
            if (dd < best - 1e-15 * fmax(best, 1e-300) || (!found)) {
                best = dd;
                out[0] = p[0], out[1] = p[1];
                *out_th = th;
                found = 1;
            }
        }
    }
    if (L > 0) {
        /* the two flat sides, normals +-d_perp */
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            double nn[2] = {-sgn * d[1] / L, sgn * d[0] / L};
            double h = dot2(R->a, nn) + R->r;
            if (dot2(q, nn) < h) continue; /* side not visible */
            double s = ((t[0] - R->a[0]) * d[0] + (t[1] - R->a[1]) * d[1]) / (L * L);
            if (s < 0) s = 0;
            if (s > 1) s = 1;
            double p[2] = {R->a[0] + s * d[0] + R->r * nn[0], R->a[1] + s * d[1] + R->r * nn[1]};
            double dd = (p[0] - t[0]) * (p[0] - t[0]) + (p[1] - t[1]) * (p[1] - t[1]);
            if (dd < best - 1e-15 * fmax(best, 1e-300) || (!found)) {
                best = dd;
                out[0] = p[0], out[1] = p[1];
                *out_th = wrap2pi(atan2(nn[1], nn[0]));
                found = 1;
            }
        }
    }
    return found;
}

/* Tangent directions through a point q outside R: the two ends of the
 * normal-angle arc visible from q (intersection of the two disks' arcs). */
static int tangents_through(const capsule *R, const double *q, double th[2]) {
    double lo1, len1;
    if (!disk_visible(R->a, R->r, q, &lo1, &len1)) return 0;
    double lo2, len2;
    if (!disk_visible(R->b, R->r, q, &lo2, &len2)) return 0;
    /* intersection of two arcs each shorter than pi is one arc */
    double lo, hi;
    if (ang_in(lo2, lo1, len1)) lo = lo2;
    else lo = lo1;
    double e1 = lo1 + len1, e2 = lo2 + len2;
    if (ang_in(e2, lo1, len1)) hi = e2;
    else hi = e1;
    th[0] = wrap2pi(lo);
    th[1] = wrap2pi(hi);
    return 2;
}

/*
 * Capsule minimiser: returns 1 if the constraint was active (x moved or was
 * solved), 0 if scenario 1 (x = n).  w = INFINITY marks a certain weight.
 */
/* relative energy gap between the chosen configuration and the best other
 * (distinct) candidate; a diagnostic for near-ties, not part of the method */
static double tie_gap(const cand *all, int na, const cand *best) {
    double second = INFINITY;
    double scale = fabs(best->x0[0]) + fabs(best->x0[1]) + fabs(best->x1[0]) + fabs(best->x1[1]) + 1e-300;
    for (int k = 0; k < na; k++) {
        double d = fabs(all[k].x0[0] - best->x0[0]) + fabs(all[k].x0[1] - best->x0[1]) +
                   fabs(all[k].x1[0] - best->x1[0]) + fabs(all[k].x1[1] - best->x1[1]);
        if (d <= 1e-9 * scale) continue;
        if (all[k].E < second) second = all[k].E;
    }
    if (!(second < INFINITY)) return INFINITY;
    return (second - best->E) / fmax(fabs(best->E), 1e-300);
}

int tor_prox_capsule_gap(const double *xa, const double *xb, double r, const double *n0, const double *n1,
                         double w0, double w1, double *x0, double *x1, int *kind_out, double *theta_out,
                         double *gap_out);

int tor_prox_capsule(const double *xa, const double *xb, double r, const double *n0, const double *n1,
                     double w0, double w1, double *x0, double *x1, int *kind_out, double *theta_out) {
    return tor_prox_capsule_gap(xa, xb, r, n0, n1, w0, w1, x0, x1, kind_out, theta_out, NULL);
}

int tor_prox_capsule_gap(const double *xa, const double *xb, double r, const double *n0, const double *n1,
                         double w0, double w1, double *x0, double *x1, int *kind_out, double *theta_out,
                         double *gap_out) {
    cand all[40];
    int na = 0;
    if (gap_out) *gap_out = INFINITY;
    capsule R = {{xa[0], xa[1]}, {xb[0], xb[1]}, r};
    if (tor_segseg(n0, n1, xa, xb) >= r) {
        x0[0] = n0[0], x0[1] = n0[1], x1[0] = n1[0], x1[1] = n1[1];
        if (kind_out) *kind_out = -1;
        if (theta_out) *theta_out = 0;
        return 0;
    }
    int i0 = isinf(w0), i1 = isinf(w1);
    cand best, c;
    best.E = INFINITY;
    best.kind = 99;
    best.th = 0;
    if (i0 && i1) {
        /* nothing can move */
        x0[0] = n0[0], x0[1] = n0[1], x1[0] = n1[0], x1[1] = n1[1];
        if (kind_out) *kind_out = -2;
        if (theta_out) *theta_out = 0;
        return 1;
    }
    if (!i0 && !i1) {
        /* (a) tangent family: all stationary points of each smooth piece,
         * plus the two kink directions */
        double d[2] = {R.b[0] - R.a[0], R.b[1] - R.a[1]};
        double ths[16];
        int nt = 0;
        const double *ctr[2] = {R.a, R.b};
        int npc = (d[0] != 0 || d[1] != 0) ? 2 : 1;
        for (int pc = 0; pc < npc; pc++) {
            const double *cc = ctr[pc];
            double w[2] = {w0, w1};
            double m[2][2] = {{n0[0] - cc[0], n0[1] - cc[1]}, {n1[0] - cc[0], n1[1] - cc[1]}};
            nt += circle_stationary(w, m, r, ths + nt);
        }
        if (npc == 2) {
            double pd = atan2(d[1], d[0]);
            ths[nt++] = wrap2pi(pd + 0.5 * TOR_PI);
            ths[nt++] = wrap2pi(pd - 0.5 * TOR_PI);
        }
        for (int k = 0; k < nt; k++) {
            tangent_config(&R, n0, n1, w0, w1, ths[k], &c);
            all[na++] = c;
            if (better(&c, &best)) best = c;
        }
        /* (b) one spring relaxed, the other end on the visible boundary */
        int in0 = in_region(&R, n0), in1 = in_region(&R, n1);
        if (in0 && !in1) {
            double p[2], th;
            if (nearest_visible(&R, n1, n0, p, &th)) {
                c.kind = 1, c.th = th;
                c.x0[0] = p[0], c.x0[1] = p[1], c.x1[0] = n1[0], c.x1[1] = n1[1];
                c.E = 0.5 * w0 * ((p[0] - n0[0]) * (p[0] - n0[0]) + (p[1] - n0[1]) * (p[1] - n0[1]));
                all[na++] = c;
            if (better(&c, &best)) best = c;
            }
        } else if (in1 && !in0) {
            double p[2], th;
            if (nearest_visible(&R, n0, n1, p, &th)) {
                c.kind = 2, c.th = th;
                c.x0[0] = n0[0], c.x0[1] = n0[1], c.x1[0] = p[0], c.x1[1] = p[1];
                c.E = 0.5 * w1 * ((p[0] - n1[0]) * (p[0] - n1[0]) + (p[1] - n1[1]) * (p[1] - n1[1]));
                all[na++] = c;
            if (better(&c, &best)) best = c;
            }
        } else if (!in0 && !in1) {
            double p[2], th;
            if (nearest_visible(&R, n1, n0, p, &th)) {
                c.kind = 1, c.th = th;
                c.x0[0] = p[0], c.x0[1] = p[1], c.x1[0] = n1[0], c.x1[1] = n1[1];
                c.E = 0.5 * w0 * ((p[0] - n0[0]) * (p[0] - n0[0]) + (p[1] - n0[1]) * (p[1] - n0[1]));
                all[na++] = c;
            if (better(&c, &best)) best = c;
            }
            if (nearest_visible(&R, n0, n1, p, &th)) {
                c.kind = 2, c.th = th;
                c.x0[0] = n0[0], c.x0[1] = n0[1], c.x1[0] = p[0], c.x1[1] = p[1];
                c.E = 0.5 * w1 * ((p[0] - n1[0]) * (p[0] - n1[0]) + (p[1] - n1[1]) * (p[1] - n1[1]));
                all[na++] = c;
            if (better(&c, &best)) best = c;
            }
        }
    } else {
        /* one end certain (weight infinity): it stays at its n.  Tangent
         * configurations must then pass through it (two tangent lines); the
         * boundary configuration keeps it and moves the other end. */
        const double *nf = i0 ? n0 : n1, *nv = i0 ? n1 : n0;
        double wv = i0 ? w1 : w0;
        double ths[2];
        int nt = tangents_through(&R, nf, ths);
        for (int k = 0; k < nt; k++) {
            double P[2], n[2] = {cos(ths[k]), sin(ths[k])};
            support_point(&R, ths[k], P);
            double g = (P[0] - nv[0]) * n[0] + (P[1] - nv[1]) * n[1];
            double xv[2] = {nv[0] + g * n[0], nv[1] + g * n[1]};
            c.kind = 0, c.th = ths[k];
            c.E = 0.5 * wv * g * g;
            if (i0) {
                c.x0[0] = nf[0], c.x0[1] = nf[1], c.x1[0] = xv[0], c.x1[1] = xv[1];
            } else {
                c.x1[0] = nf[0], c.x1[1] = nf[1], c.x0[0] = xv[0], c.x0[1] = xv[1];
            }
            all[na++] = c;
            if (better(&c, &best)) best = c;
        }
        double p[2], th;
        if (nearest_visible(&R, nf, nv, p, &th)) {
            c.kind = i0 ? 2 : 1, c.th = th;
            c.E = 0.5 * wv * ((p[0] - nv[0]) * (p[0] - nv[0]) + (p[1] - nv[1]) * (p[1] - nv[1]));
            if (i0) {
                c.x0[0] = nf[0], c.x0[1] = nf[1], c.x1[0] = p[0], c.x1[1] = p[1];
            } else {
                c.x1[0] = nf[0], c.x1[1] = nf[1], c.x0[0] = p[0], c.x0[1] = p[1];
            }
            all[na++] = c;
            if (better(&c, &best)) best = c;
        }
    }
    if (!(best.E < INFINITY)) {
        /* no feasible configuration (fixed end inside the region) */
        x0[0] = n0[0], x0[1] = n0[1], x1[0] = n1[0], x1[1] = n1[1];
        if (kind_out) *kind_out = -3;
        if (theta_out) *theta_out = 0;
        return 1;
    }
    x0[0] = best.x0[0], x0[1] = best.x0[1], x1[0] = best.x1[0], x1[1] = best.x1[1];
    if (gap_out) *gap_out = tie_gap(all, na, &best);
    if (kind_out) *kind_out = best.kind;
    if (theta_out) *theta_out = best.th;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Agent-agent minimiser through the wall minimiser (App. C)                  */
/* ------------------------------------------------------------------------ */
/*
 * Combined weight of the difference variable v = x' - x for one break-point.
 * Minimising (rho/2)|x - n|^2 + (rho'/2)|x + v - n'|^2 over x at fixed v
 * leaves (omega/2)|v - (n' - n)|^2 with omega = rho rho' / (rho + rho') and
 * x = (rho n + rho' (n' - v)) / (rho + rho').  (App. C writes the weight as
 * (rho + rho')/4 and the target as 2(rho' n' - rho n)/(rho + rho'); the two
 * agree when rho == rho', which is the only case the planner produces.)
 */
static double pair_weight(double r, double rp) {
    if (isinf(r) && isinf(rp)) return INFINITY;
    if (isinf(r)) return rp;
    if (isinf(rp)) return r;
    return r * rp / (r + rp);
}
static void pair_rebuild(double r, double rp, const double *n, const double *np, const double *v, int dim,
                         double *x, double *xp) {
    for (int k = 0; k < dim; k++) {
        double xv;
        if (isinf(r) && isinf(rp)) {
            /* both ends certain: v equals n' - n, nothing moves */
            x[k] = n[k];
            xp[k] = np[k];
            continue;
        } else if (isinf(r)) xv = n[k];
        else if (isinf(rp)) xv = np[k] - v[k];
        else xv = (r * n[k] + rp * (np[k] - v[k])) / (r + rp);
        x[k] = xv;
        xp[k] = xv + v[k];
    }
}

/* in 3D the optimum lies in the plane spanned by m_lo and m_hi (through the
 * origin): an orthonormal basis e1, e2 of that plane */
static void plane_basis(const double *a, const double *b, double *e1, double *e2) {
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double *f = na > 0 ? a : b;
    double nf = na > 0 ? na : nb;
    if (nf > 0) {
        for (int k = 0; k < 3; k++) e1[k] = f[k] / nf;
    } else {
        e1[0] = 1, e1[1] = 0, e1[2] = 0;
    }
    const double *g = na > 0 ? b : a;
    double pr = g[0] * e1[0] + g[1] * e1[1] + g[2] * e1[2];
    double w[3] = {g[0] - pr * e1[0], g[1] - pr * e1[1], g[2] - pr * e1[2]};
    double nw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (nw <= 1e-12 * (nf + nb + 1e-300)) {
        /* collinear: a fixed plane through the axis least aligned with e1 */
        int ax = 0;
        for (int k = 1; k < 3; k++)
            if (fabs(e1[k]) < fabs(e1[ax])) ax = k;
        double t[3] = {0, 0, 0};
        t[ax] = 1;
        double p2 = e1[ax];
        w[0] = t[0] - p2 * e1[0], w[1] = t[1] - p2 * e1[1], w[2] = t[2] - p2 * e1[2];
        nw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    }
    for (int k = 0; k < 3; k++) e2[k] = w[k] / nw;
}

/*
 * Agent-agent minimiser g_coll (eq. coll_minimizer_problem).  Inputs are
 * the four n-messages (agent 1 at break-points s, s+1: nl, nh; agent 2: nlp,
 * nhp), their weights (INFINITY = certain) and the radius sum R.  Returns 1
 * if the pair collides (weights rho0 out), 0 otherwise (x = n, weights 0).
 */
int tor_prox_coll_gap(const double *nl, const double *nh, const double *nlp, const double *nhp, double wl,
                      double wh, double wlp, double whp, double R, int dim, double *xl, double *xh, double *xlp,
                      double *xhp, int *kind_out, double *theta_out, double *gap_out);

int tor_prox_coll(const double *nl, const double *nh, const double *nlp, const double *nhp, double wl,
                  double wh, double wlp, double whp, double R, int dim, double *xl, double *xh, double *xlp,
                  double *xhp, int *kind_out, double *theta_out) {
    return tor_prox_coll_gap(nl, nh, nlp, nhp, wl, wh, wlp, whp, R, dim, xl, xh, xlp, xhp, kind_out, theta_out,
                             NULL);
}

int tor_prox_coll_gap(const double *nl, const double *nh, const double *nlp, const double *nhp, double wl,
                      double wh, double wlp, double whp, double R, int dim, double *xl, double *xh, double *xlp,
                      double *xhp, int *kind_out, double *theta_out, double *gap_out) {
    if (gap_out) *gap_out = INFINITY;
    double ml[3], mh[3];
    for (int k = 0; k < dim; k++) {
        ml[k] = nlp[k] - nl[k];
        mh[k] = nhp[k] - nh[k];
    }
    if (tor_cpa(ml, mh, dim) >= R) {
        memcpy(xl, nl, sizeof(double) * dim);
        memcpy(xh, nh, sizeof(double) * dim);
        memcpy(xlp, nlp, sizeof(double) * dim);
        memcpy(xhp, nhp, sizeof(double) * dim);
        if (kind_out) *kind_out = -1;
        if (theta_out) *theta_out = 0;
        return 0;
    }
    double om_l = pair_weight(wl, wlp), om_h = pair_weight(wh, whp);
    double zero[2] = {0, 0};
    double vl[3], vh[3];
    if (dim == 2) {
        tor_prox_capsule_gap(zero, zero, R, ml, mh, om_l, om_h, vl, vh, kind_out, theta_out, gap_out);
    } else {
        double e1[3], e2[3];
        plane_basis(ml, mh, e1, e2);
        double a[2] = {ml[0] * e1[0] + ml[1] * e1[1] + ml[2] * e1[2], ml[0] * e2[0] + ml[1] * e2[1] + ml[2] * e2[2]};
        double b[2] = {mh[0] * e1[0] + mh[1] * e1[1] + mh[2] * e1[2], mh[0] * e2[0] + mh[1] * e2[1] + mh[2] * e2[2]};
        double va[2], vb[2];
        tor_prox_capsule_gap(zero, zero, R, a, b, om_l, om_h, va, vb, kind_out, theta_out, gap_out);
        /* the component of m orthogonal to the plane is zero by construction */
        for (int k = 0; k < 3; k++) {
            vl[k] = va[0] * e1[k] + va[1] * e2[k];
            vh[k] = vb[0] * e1[k] + vb[1] * e2[k];
        }
    }
    pair_rebuild(wl, wlp, nl, nlp, vl, dim, xl, xlp);
    pair_rebuild(wh, whp, nh, nhp, vh, dim, xh, xhp);
    return 1;
}

/* ------------------------------------------------------------------------ */
/* The planner: factor graph and iteration (App. B)                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int p, eta, dim, W, mode;
    double rho0, alpha, rho0_init;
    int n_warm;
    long iter;
    double *radii, *x0, *xT, *walls, *C;
    long F, E, N;
    unsigned char *ftype;
    long *fe0;      /* first edge of each factor */
    int *fa, *fb;   /* agent(s) of the factor */
    int *fs, *fw;   /* segment / wall index */
    long *enode;
    long *adj_off, *adj; /* node -> incident edges (CSR) */
    double *z, *u, *x, *n, *m; /* z: [N][dim]; others [E][dim] */
    unsigned char *rout;  /* ->rho per edge */
    unsigned char *rin;   /* <-rho per edge */
    /* reverse-mode tape: every iteration's state (small instances only) */
    int taping;
    long tape_len, tape_cap;
    double *tape_z, *tape_u;          /* [t][N*dim], [t][E*dim] state before iteration t */
    unsigned char *tape_rin, *tape_rout; /* [t][E] <-rho used by iteration t, ->rho it produced */
    unsigned char *tape_rin_next;     /* [E] <-rho after the last taped iteration */
    double tape_rho[4096];            /* rho0 of each taped iteration (schedule) */
    double *act_margin;   /* |closest approach - R| / R of the last activity test, per factor */
    double *tie_margin;   /* relative energy gap to the runner-up candidate, per factor */
    int cost;             /* TOR_COST_*: what the per-segment factors are */
    /* test support: minimiser outputs given for the next iteration */
    long *ovr;            /* [F] offset of the factor's x in ovr_x, or -1 (NULL: none) */
    double *ovr_x;        /* per listed factor: its edges' x, canonical order */
    unsigned char *ovr_rho; /* [F] ->rho of a listed factor */
} tor_t;

static long node_id(const tor_t *T, int i, int s) { return (long)i * (T->eta + 1) + s; }

void *tor_create(int p, int eta, int dim, const double *radii, const double *x0, const double *xT, int W,
                 const double *walls, const double *C, double rho0, double alpha, int mode, int cost) {
    if (p < 1 || eta < 1 || (dim != 2 && dim != 3) || W < 0 || (W > 0 && dim != 2)) return NULL;
    if (cost < TOR_COST_ENERGY || cost > TOR_COST_VO || (cost == TOR_COST_VO && eta != 1)) return NULL;
    tor_t *T = (tor_t *)calloc(1, sizeof(tor_t));
    T->p = p, T->eta = eta, T->dim = dim, T->W = W, T->mode = mode, T->cost = cost;
    T->rho0 = rho0, T->alpha = alpha, T->rho0_init = rho0, T->n_warm = 0;
    T->radii = (double *)malloc(sizeof(double) * p);
    memcpy(T->radii, radii, sizeof(double) * p);
    T->x0 = (double *)malloc(sizeof(double) * p * dim);
    memcpy(T->x0, x0, sizeof(double) * p * dim);
    T->xT = (double *)malloc(sizeof(double) * p * dim);
    memcpy(T->xT, xT, sizeof(double) * p * dim);
    T->walls = (double *)malloc(sizeof(double) * (W > 0 ? W : 1) * 4);
    if (W) memcpy(T->walls, walls, sizeof(double) * W * 4);
    T->C = (double *)malloc(sizeof(double) * p * eta);
    memcpy(T->C, C, sizeof(double) * p * eta);
    long fc = (long)eta * p * (p - 1) / 2, fe = (long)eta * p, fw = (long)eta * p * W, ff = 2L * p;
    T->F = fc + fe + fw + ff;
    T->E = 4 * fc + 2 * fe + 2 * fw + ff;
    T->N = (long)(eta + 1) * p;
    T->ftype = (unsigned char *)malloc(T->F);
    T->fe0 = (long *)malloc(sizeof(long) * (T->F + 1));
    T->fa = (int *)malloc(sizeof(int) * T->F);
    T->fb = (int *)malloc(sizeof(int) * T->F);
    T->fs = (int *)malloc(sizeof(int) * T->F);
    T->fw = (int *)malloc(sizeof(int) * T->F);
    T->enode = (long *)malloc(sizeof(long) * T->E);
    long f = 0, e = 0;
    for (int i = 0; i < p; i++) {
        for (int g = 0; g < 2; g++) {
            T->ftype[f] = TOR_F_FIXED, T->fe0[f] = e, T->fa[f] = i, T->fb[f] = -1;
            T->fs[f] = g ? eta : 0, T->fw[f] = -1;
            T->enode[e++] = node_id(T, i, g ? eta : 0);
            f++;
        }
    }
    for (int i = 0; i < p; i++)
        for (int s = 0; s < eta; s++) {
            T->ftype[f] = TOR_F_ENERGY, T->fe0[f] = e, T->fa[f] = i, T->fb[f] = -1, T->fs[f] = s, T->fw[f] = -1;
            T->enode[e++] = node_id(T, i, s);
            T->enode[e++] = node_id(T, i, s + 1);
            f++;
        }
    for (int s = 0; s < eta; s++)
        for (int i = 0; i < p; i++)
            for (int j = i + 1; j < p; j++) {
                T->ftype[f] = TOR_F_COLL, T->fe0[f] = e, T->fa[f] = i, T->fb[f] = j, T->fs[f] = s, T->fw[f] = -1;
                T->enode[e++] = node_id(T, i, s);
                T->enode[e++] = node_id(T, i, s + 1);
                T->enode[e++] = node_id(T, j, s);
                T->enode[e++] = node_id(T, j, s + 1);
                f++;
            }
    for (int s = 0; s < eta; s++)
        for (int i = 0; i < p; i++)
            for (int w = 0; w < W; w++) {
                T->ftype[f] = TOR_F_WALL, T->fe0[f] = e, T->fa[f] = i, T->fb[f] = -1, T->fs[f] = s, T->fw[f] = w;
                T->enode[e++] = node_id(T, i, s);
                T->enode[e++] = node_id(T, i, s + 1);
                f++;
            }
    T->fe0[f] = e;
    /* node adjacency */
    T->adj_off = (long *)calloc(T->N + 1, sizeof(long));
    for (long k = 0; k < T->E; k++) T->adj_off[T->enode[k] + 1]++;
    for (long j = 0; j < T->N; j++) T->adj_off[j + 1] += T->adj_off[j];
    T->adj = (long *)malloc(sizeof(long) * T->E);
    long *fill = (long *)calloc((size_t)(T->N > 0 ? T->N : 1), sizeof(long));
    for (long k = 0; k < T->E; k++) {
        long j = T->enode[k];
        T->adj[T->adj_off[j] + fill[j]++] = k;
    }
    free(fill);
    T->z = (double *)calloc(T->N * dim, sizeof(double));
    T->u = (double *)calloc(T->E * dim, sizeof(double));
    T->x = (double *)calloc(T->E * dim, sizeof(double));
    T->n = (double *)calloc(T->E * dim, sizeof(double));
    T->m = (double *)calloc(T->E * dim, sizeof(double));
    T->rout = (unsigned char *)calloc(T->E, 1);
    T->rin = (unsigned char *)calloc(T->E, 1);
    T->act_margin = (double *)malloc(sizeof(double) * T->F);
    T->tie_margin = (double *)malloc(sizeof(double) * T->F);
    for (long q = 0; q < T->F; q++) T->act_margin[q] = T->tie_margin[q] = INFINITY;
    /* default state: straight lines, u = 0, <-rho INF at end points, STD inside */
    for (int i = 0; i < p; i++)
        for (int s = 0; s <= eta; s++)
            for (int k = 0; k < dim; k++)
                T->z[node_id(T, i, s) * dim + k] =
                    x0[i * dim + k] + ((double)s / eta) * (xT[i * dim + k] - x0[i * dim + k]);
    for (long k = 0; k < T->E; k++) {
        int s = (int)(T->enode[k] % (eta + 1));
        T->rin[k] = (mode == TOR_MODE_TWA && (s == 0 || (s == eta && cost != TOR_COST_VO))) ? TOR_INF : TOR_STD;
    }
    return T;
}

void tor_destroy(void *h) {
    tor_t *T = (tor_t *)h;
    if (!T) return;
    free(T->radii), free(T->x0), free(T->xT), free(T->walls), free(T->C);
    free(T->ftype), free(T->fe0), free(T->fa), free(T->fb), free(T->fs), free(T->fw);
    free(T->enode), free(T->adj_off), free(T->adj);
    free(T->z), free(T->u), free(T->x), free(T->n), free(T->m), free(T->rout), free(T->rin);
    free(T->act_margin), free(T->tie_margin);
    free(T->tape_z), free(T->tape_u), free(T->tape_rin), free(T->tape_rout), free(T->tape_rin_next);
    free(T->ovr), free(T->ovr_x), free(T->ovr_rho);
    free(T);
}

long tor_num_factors(void *h) { return ((tor_t *)h)->F; }
long tor_num_edges(void *h) { return ((tor_t *)h)->E; }
long tor_iteration(void *h) { return ((tor_t *)h)->iter; }

/* Sec. 4's warm-up: rho0 = rho0_init in the minimisers' weights for the
 * first n_warm iterations (counted from 0), then the configuration's rho0.
 * The u step stays alpha / rho0 of the configuration throughout (step 7). */
void tor_set_schedule(void *h, double rho0_init, int n_warm) {
    tor_t *T = (tor_t *)h;
    T->rho0_init = rho0_init;
    T->n_warm = n_warm;
}

/* state: z [p][eta+1][dim], u [E][dim] canonical order, <-rho per node
 * [p][eta+1] (the rule makes it uniform over a node's edges), iteration k */
void tor_set_state(void *h, const double *z, const double *u, const unsigned char *lrho, long k) {
    tor_t *T = (tor_t *)h;
    memcpy(T->z, z, sizeof(double) * T->N * T->dim);
    memcpy(T->u, u, sizeof(double) * T->E * T->dim);
    for (long e = 0; e < T->E; e++) T->rin[e] = lrho[T->enode[e]];
    T->iter = k;
}

void tor_get_state(void *h, double *z, double *u, unsigned char *lrho) {
    tor_t *T = (tor_t *)h;
    if (z) memcpy(z, T->z, sizeof(double) * T->N * T->dim);
    if (u) memcpy(u, T->u, sizeof(double) * T->E * T->dim);
    if (lrho)
        for (long j = 0; j < T->N; j++) lrho[j] = T->adj_off[j + 1] > T->adj_off[j] ? T->rin[T->adj[T->adj_off[j]]] : TOR_STD;
}

/* x of the last iteration per edge and ->rho per factor */
void tor_get_last(void *h, double *x, unsigned char *rho_f) {
    tor_t *T = (tor_t *)h;
    if (x) memcpy(x, T->x, sizeof(double) * T->E * T->dim);
    if (rho_f)
        for (long f = 0; f < T->F; f++) rho_f[f] = T->rout[T->fe0[f]];
}

/* near-tie diagnostics of the last iteration, per factor (test use) */
void tor_get_margins(void *h, double *act_margin, double *tie_margin) {
    tor_t *T = (tor_t *)h;
    if (act_margin) memcpy(act_margin, T->act_margin, sizeof(double) * T->F);
    if (tie_margin) memcpy(tie_margin, T->tie_margin, sizeof(double) * T->F);
}

/* Test support, not a step of the method: for the next iteration only, the
 * listed factors skip their minimiser and emit the given x (each factor's
 * edges in canonical order, dim values per edge, factors one after another in
 * the order listed) and ->rho; m, z, <-rho and u then follow App. B as usual.
 * Lets a test follow the iteration after a factor whose argmin is a near-tie
 * took the other (equally good) candidate. */
void tor_override_next(void *h, long nf, const long *factors, const double *x, const unsigned char *rho) {
    tor_t *T = (tor_t *)h;
    free(T->ovr), free(T->ovr_x), free(T->ovr_rho);
    T->ovr = NULL, T->ovr_x = NULL, T->ovr_rho = NULL;
    if (nf <= 0) return;
    long nx = 0;
    for (long q = 0; q < nf; q++) nx += (T->fe0[factors[q] + 1] - T->fe0[factors[q]]) * T->dim;
    T->ovr = (long *)malloc(sizeof(long) * T->F);
    T->ovr_x = (double *)malloc(sizeof(double) * (size_t)nx);
    T->ovr_rho = (unsigned char *)malloc((size_t)T->F);
    for (long f = 0; f < T->F; f++) T->ovr[f] = -1;
    long off = 0;
    for (long q = 0; q < nf; q++) {
        long f = factors[q];
        long n = (T->fe0[f + 1] - T->fe0[f]) * T->dim;
        T->ovr[f] = off; /* where factor f's x starts in ovr_x */
        T->ovr_rho[f] = rho[q];
        memcpy(T->ovr_x + off, x + off, sizeof(double) * (size_t)n);
        off += n;
    }
}

static double weight_value(const tor_t *T, unsigned char w, double rho) {
    (void)T;
    if (w == TOR_INF) return INFINITY;
    if (w == TOR_ZERO) return TOR_ZERO_WEIGHT * rho;
    return rho;
}

/* step 2 and 3 for one factor */
static void run_factor(tor_t *T, long f, double rho) {
    int dim = T->dim;
    long e = T->fe0[f];
    int t = T->ftype[f];
    double *n = T->n, *x = T->x;
    unsigned char out = TOR_STD;
    if (T->ovr && T->ovr[f] >= 0) {
        /* outputs given for this iteration (tor_override_next) */
        long ne = T->fe0[f + 1] - e;
        memcpy(x + e * dim, T->ovr_x + T->ovr[f], sizeof(double) * (size_t)(ne * dim));
        for (long q = 0; q < ne; q++) T->rout[e + q] = T->ovr_rho[f];
        return;
    }
    if (t == TOR_F_FIXED && T->cost == TOR_COST_VO && T->fs[f] != 0) {
        /* VO cost: the energy minimiser with its first end certain at x^ref */
        int i = T->fa[f];
        double tmp[3];
        tor_prox_energy(T->xT + i * dim, n + e * dim, INFINITY, weight_value(T, T->rin[e], rho), T->C[i], dim, tmp,
                        x + e * dim);
        out = TOR_STD;
    } else if (t == TOR_F_FIXED) {
        int i = T->fa[f];
        const double *c = (T->fs[f] == 0) ? T->x0 + i * dim : T->xT + i * dim;
        for (int k = 0; k < dim; k++) x[e * dim + k] = c[k];
        out = TOR_INF;
    } else if (t == TOR_F_ENERGY) {
        double wl = weight_value(T, T->rin[e], rho), wh = weight_value(T, T->rin[e + 1], rho);
        if (T->rin[e] == TOR_ZERO && T->rin[e + 1] == TOR_ZERO) wl = wh = 0; /* equal-weight limit */
        double Cf = T->C[T->fa[f] * T->eta + T->fs[f]];
        if (T->cost == TOR_COST_ENERGY) {
            tor_prox_energy(n + e * dim, n + (e + 1) * dim, wl, wh, Cf, dim, x + e * dim, x + (e + 1) * dim);
            out = TOR_STD;
        } else if (T->cost == TOR_COST_NONE || T->cost == TOR_COST_VO) {
            /* no cost: the factor is absent (x = n, weight zero) */
            for (int k = 0; k < 2 * dim; k++) x[e * dim + k] = n[e * dim + k];
            out = TOR_ZERO;
        } else {
            double dd = 0;
            for (int k = 0; k < dim; k++) {
                double q = n[e * dim + k] - n[(e + 1) * dim + k];
                dd += q * q;
            }
            T->act_margin[f] = fabs(sqrt(dd) - Cf) / Cf;
            int b = tor_prox_vel(n + e * dim, n + (e + 1) * dim, wl, wh, Cf, dim, T->cost == TOR_COST_MINVEL,
                                 x + e * dim, x + (e + 1) * dim);
            out = b ? TOR_STD : TOR_ZERO;
        }
    } else if (t == TOR_F_COLL) {
        double R = T->radii[T->fa[f]] + T->radii[T->fb[f]];
        double w[4];
        for (int q = 0; q < 4; q++) w[q] = weight_value(T, T->rin[e + q], rho);
        double d0[3], d1[3];
        for (int k = 0; k < dim; k++) {
            d0[k] = n[(e + 2) * dim + k] - n[e * dim + k];
            d1[k] = n[(e + 3) * dim + k] - n[(e + 1) * dim + k];
        }
        T->act_margin[f] = fabs(tor_cpa(d0, d1, dim) - R) / R;
        int act = tor_prox_coll_gap(n + e * dim, n + (e + 1) * dim, n + (e + 2) * dim, n + (e + 3) * dim, w[0],
                                    w[1], w[2], w[3], R, dim, x + e * dim, x + (e + 1) * dim, x + (e + 2) * dim,
                                    x + (e + 3) * dim, NULL, NULL, &T->tie_margin[f]);
        out = act ? TOR_STD : TOR_ZERO;
    } else {
        const double *wa = T->walls + T->fw[f] * 4, *wb = wa + 2;
        double r = T->radii[T->fa[f]];
        double wl = weight_value(T, T->rin[e], rho), wh = weight_value(T, T->rin[e + 1], rho);
        T->act_margin[f] = fabs(tor_segseg(n + e * dim, n + (e + 1) * dim, wa, wb) - r) / r;
        int act = tor_prox_capsule_gap(wa, wb, r, n + e * dim, n + (e + 1) * dim, wl, wh, x + e * dim,
                                       x + (e + 1) * dim, NULL, NULL, &T->tie_margin[f]);
        out = act ? TOR_STD : TOR_ZERO;
    }
    if (T->mode == TOR_MODE_ADMM) out = TOR_STD;
    long ne = T->fe0[f + 1] - e;
    for (long q = 0; q < ne; q++) T->rout[e + q] = out;
}

static void one_iteration(tor_t *T) {
    int dim = T->dim;
    double rho = (T->iter < T->n_warm) ? T->rho0_init : T->rho0;
    long E = T->E, N = T->N, F = T->F;
    if (T->taping && T->tape_len < T->tape_cap) {
        long t = T->tape_len;
        memcpy(T->tape_z + t * N * dim, T->z, sizeof(double) * N * dim);
        memcpy(T->tape_u + t * E * dim, T->u, sizeof(double) * E * dim);
        memcpy(T->tape_rin + t * E, T->rin, E);
        T->tape_rho[t] = rho;
    }
    /* 1. n = z - u */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; e++)
        for (int k = 0; k < dim; k++) T->n[e * dim + k] = T->z[T->enode[e] * dim + k] - T->u[e * dim + k];
    /* 2-3. minimisers and outgoing weights */
#pragma omp parallel for schedule(dynamic, 4096)
    for (long f = 0; f < F; f++) run_factor(T, f, rho);
    /* 4. m = x + u */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E * dim; e++) T->m[e] = T->x[e] + T->u[e];
    /* 5-6. z and <-rho per node */
#pragma omp parallel for schedule(dynamic, 64)
    for (long j = 0; j < N; j++) {
        long a = T->adj_off[j], b = T->adj_off[j + 1];
        int ninf = 0, nstd = 0;
        for (long q = a; q < b; q++) {
            unsigned char w = T->rout[T->adj[q]];
            ninf += (w == TOR_INF);
            nstd += (w == TOR_STD);
        }
        double acc[3] = {0, 0, 0}, wsum = 0;
        for (long q = a; q < b; q++) {
            long e = T->adj[q];
            unsigned char w = T->rout[e];
            double wv;
            if (ninf) wv = (w == TOR_INF) ? 1.0 : 0.0; /* limit: mean over the certain edges */
            else if (nstd) wv = (w == TOR_STD) ? rho : 0.0;
            else wv = 1.0; /* all weights zero: treat them as 1 */
            if (wv == 0) continue;
            for (int k = 0; k < dim; k++) acc[k] += wv * T->m[e * dim + k];
            wsum += wv;
        }
        if (b > a)
            for (int k = 0; k < dim; k++) T->z[j * dim + k] = acc[k] / wsum;
        unsigned char back = ninf ? TOR_INF : (nstd ? TOR_STD : TOR_ZERO);
        if (T->mode == TOR_MODE_ADMM) back = TOR_STD;
        for (long q = a; q < b; q++) T->rin[T->adj[q]] = back;
    }
    /* 7. u update.  The step is alpha / rho0 with the configuration's rho0
     * even while the warm-up's small rho0 is in force (Sec. 4): that small
     * value enters the minimisers' weights only.  Over the warm-up value the
     * step would be alpha / (eta p 1e-5), in the hundreds, and the iterates
     * diverge (see the design notes). */
    double step = T->alpha / T->rho0;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; e++) {
        if (T->rout[e] == TOR_STD && T->rin[e] == TOR_STD) {
            for (int k = 0; k < dim; k++)
                T->u[e * dim + k] += step * (T->x[e * dim + k] - T->z[T->enode[e] * dim + k]);
        } else {
            for (int k = 0; k < dim; k++) T->u[e * dim + k] = 0;
        }
    }
    if (T->ovr) tor_override_next(T, 0, NULL, NULL, NULL); /* one iteration only */
    if (T->taping && T->tape_len < T->tape_cap) {
        memcpy(T->tape_rout + T->tape_len * E, T->rout, E);
        memcpy(T->tape_rin_next, T->rin, E);
        T->tape_len++;
    }
    T->iter++;
}

void tor_iterate(void *h, long k) {
    tor_t *T = (tor_t *)h;
    for (long it = 0; it < k; it++) one_iteration(T);
}

/* objective sum_{i,s} C_{i,s} |z_i(s+1) - z_i(s)|^2 of the current z */
double tor_objective(void *h) {
    tor_t *T = (tor_t *)h;
    double acc = 0;
    for (int i = 0; i < T->p; i++)
        for (int s = 0; s < T->eta; s++) {
            double d2 = 0;
            for (int k = 0; k < T->dim; k++) {
                double d = T->z[node_id(T, i, s + 1) * T->dim + k] - T->z[node_id(T, i, s) * T->dim + k];
                d2 += d * d;
            }
            acc += T->C[i * T->eta + s] * d2;
        }
    return acc;
}

/* smallest clearance of trajectories z (layout [p][eta+1][dim]):
 * closest approach - (r_i + r_j) over all segment pairs, and
 * segment-wall distance - r_i over all walls (planar only) */
double tor_min_clearance(int p, int eta, int dim, const double *radii, const double *z, int W,
                         const double *walls) {
    double best = INFINITY;
    for (int s = 0; s < eta; s++) {
        for (int i = 0; i < p; i++) {
            const double *ai = z + ((long)i * (eta + 1) + s) * dim, *bi = ai + dim;
            for (int j = i + 1; j < p; j++) {
                const double *aj = z + ((long)j * (eta + 1) + s) * dim, *bj = aj + dim;
                double d0[3], d1[3];
                for (int k = 0; k < dim; k++) d0[k] = aj[k] - ai[k], d1[k] = bj[k] - bi[k];
                double c = tor_cpa(d0, d1, dim) - (radii[i] + radii[j]);
                if (c < best) best = c;
            }
            for (int w = 0; w < W && dim == 2; w++) {
                double c = tor_segseg(ai, bi, walls + w * 4, walls + w * 4 + 2) - radii[i];
                if (c < best) best = c;
            }
        }
    }
    return best;
}

/* ======================================================================== */
/* Reverse mode of K unrolled iterations (test reference of the adjoint)     */
/* ======================================================================== */
/*
 * tor_tape(h, K) runs K iterations from the current state and keeps every
 * iteration's state.  tor_backward(h, dz, ...) then returns the gradient of
 * L(z^K) given dL/dz^K, with respect to the start and goal positions, the
 * radii and the initial break-points, holding every discrete decision of
 * the forward run fixed (weights, minimiser configuration).
 *
 * The reverse sweep follows App. B backwards, per iteration:
 *   step 7  u' = u + s (x - z') on edges whose ->rho and new <-rho are rho0,
 *           else 0   (s = alpha/rho0)
 *   step 5  z' = weighted mean of m over the edges that carried weight
 *   step 4  m = x + u
 *   step 2  x = g(n): each minimiser's local Jacobian (with respect to its
 *           n-messages and its radius) by FP64 central differences with a
 *           step of 1e-9, small enough to stay inside the smooth piece the
 *           input lies on (the minimisers are piecewise smooth: a segment
 *           end that is pushed or just clear of the separating line, the
 *           candidate that wins); the energy minimiser is linear in n; a
 *           fixed factor's x is the start or goal itself
 *   step 1  n = z - u
 */
static void coll_eval(tor_t *T, long f, const double *nin, double R, const double *w, double *xout) {
    int dim = T->dim;
    tor_prox_coll(nin, nin + dim, nin + 2 * dim, nin + 3 * dim, w[0], w[1], w[2], w[3], R, dim, xout, xout + dim,
                  xout + 2 * dim, xout + 3 * dim, NULL, NULL);
    (void)f;
}

static void wall_eval(tor_t *T, long f, const double *nin, double r, const double *w, double *xout) {
    const double *wa = T->walls + T->fw[f] * 4, *wb = wa + 2;
    tor_prox_capsule(wa, wb, r, nin, nin + 2, w[0], w[1], xout, xout + 2, NULL, NULL);
}

long tor_tape(void *h, long K) {
    tor_t *T = (tor_t *)h;
    if (T->cost != TOR_COST_ENERGY) return -2; /* the reverse sweep covers the energy cost only */
    long N = T->N, E = T->E;
    int dim = T->dim;
    if (K > 4096) K = 4096;
    free(T->tape_z), free(T->tape_u), free(T->tape_rin), free(T->tape_rout), free(T->tape_rin_next);
    T->tape_z = (double *)malloc(sizeof(double) * (K + 1) * N * dim);
    T->tape_u = (double *)malloc(sizeof(double) * (K + 1) * E * dim);
    T->tape_rin = (unsigned char *)malloc((size_t)(K + 1) * E);
    T->tape_rout = (unsigned char *)malloc((size_t)(K + 1) * E);
    T->tape_rin_next = (unsigned char *)malloc((size_t)E);
    if (!T->tape_z || !T->tape_u || !T->tape_rin || !T->tape_rout || !T->tape_rin_next) return -1;
    T->tape_len = 0;
    T->tape_cap = K;
    T->taping = 1;
    tor_iterate(h, K);
    T->taping = 0;
    return T->tape_len;
}

/* dz [N][dim] = dL/dz^K (node order i*(eta+1)+s).  Outputs (accumulated,
 * caller zeroes them): dx0, dxT [p][dim], dr [p], dz0 [N][dim]. */
void tor_backward(void *h, const double *dz, double *dx0, double *dxT, double *dr, double *dz0) {
    tor_t *T = (tor_t *)h;
    long N = T->N, E = T->E, F = T->F;
    int dim = T->dim;
    double *zb = (double *)calloc(N * dim, sizeof(double));   /* adjoint of z^{k+1} */
    double *ub = (double *)calloc(E * dim, sizeof(double));   /* adjoint of u^{k+1} */
    double *xb = (double *)calloc(E * dim, sizeof(double));
    double *ubn = (double *)calloc(E * dim, sizeof(double));
    double *zbn = (double *)calloc(N * dim, sizeof(double));
    double *zhat = (double *)calloc(N * dim, sizeof(double));
    double *n = (double *)calloc(E * dim, sizeof(double));
    memcpy(zb, dz, sizeof(double) * N * dim);
    for (long t = T->tape_len - 1; t >= 0; t--) {
        const double *z = T->tape_z + t * N * dim, *u = T->tape_u + t * E * dim;
        const unsigned char *rin = T->tape_rin + t * E, *rout = T->tape_rout + t * E;
        const unsigned char *rin1 = (t + 1 < T->tape_len) ? T->tape_rin + (t + 1) * E : T->tape_rin_next;
        double rho = T->tape_rho[t], s = T->alpha / T->rho0;
        for (long e = 0; e < E; e++)
            for (int k = 0; k < dim; k++) n[e * dim + k] = z[T->enode[e] * dim + k] - u[e * dim + k];
        /* step 7 */
        memcpy(zhat, zb, sizeof(double) * N * dim);
        for (long e = 0; e < E; e++) {
            int a = rout[e] == TOR_STD && rin1[e] == TOR_STD;
            for (int k = 0; k < dim; k++) {
                double g = a ? ub[e * dim + k] : 0.0;
                xb[e * dim + k] = s * g;
                ubn[e * dim + k] = g;
                zhat[T->enode[e] * dim + k] -= s * g;
            }
        }
        /* step 5 and 4 */
        for (long j = 0; j < N; j++) {
            long a0 = T->adj_off[j], a1 = T->adj_off[j + 1];
            int ninf = 0, nstd = 0;
            for (long q = a0; q < a1; q++) {
                unsigned char w = rout[T->adj[q]];
                ninf += (w == TOR_INF);
                nstd += (w == TOR_STD);
            }
            double wsum = 0;
            for (long q = a0; q < a1; q++) {
                unsigned char w = rout[T->adj[q]];
                wsum += ninf ? (w == TOR_INF) : (nstd ? (w == TOR_STD) * rho : 1.0);
            }
            for (long q = a0; q < a1; q++) {
                long e = T->adj[q];
                unsigned char w = rout[e];
                double wv = ninf ? (w == TOR_INF) : (nstd ? (w == TOR_STD) * rho : 1.0);
                if (wv == 0) continue;
                for (int k = 0; k < dim; k++) {
                    double mb = zhat[j * dim + k] * wv / wsum;
                    xb[e * dim + k] += mb;
                    ubn[e * dim + k] += mb;
                }
            }
        }
        /* step 2 and 1 */
        memset(zbn, 0, sizeof(double) * N * dim);
        for (long f = 0; f < F; f++) {
            long e0 = T->fe0[f], ne = T->fe0[f + 1] - e0;
            int tp = T->ftype[f];
            double nb[12];
            for (int q = 0; q < ne * dim; q++) nb[q] = 0;
            if (tp == TOR_F_FIXED) {
                double *dst = (T->fs[f] == 0) ? dx0 : dxT;
                for (int k = 0; k < dim; k++) dst[T->fa[f] * dim + k] += xb[e0 * dim + k];
            } else if (tp == TOR_F_ENERGY) {
                double C = T->C[T->fa[f] * T->eta + T->fs[f]];
                double wl = weight_value(T, rin[e0], rho), wh = weight_value(T, rin[e0 + 1], rho);
                int both0 = rin[e0] == TOR_ZERO && rin[e0 + 1] == TOR_ZERO;
                /* the minimiser is linear in n: its Jacobian from unit inputs */
                for (int c = 0; c < 2; c++) {
                    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0}, xl[3], xh[3];
                    if (c == 0) a[0] = 1; else b[0] = 1;
                    tor_prox_energy(a, b, both0 ? 0.0 : wl, both0 ? 0.0 : wh, C, 1, xl, xh);
                    for (int k = 0; k < dim; k++)
                        nb[c * dim + k] = xl[0] * xb[e0 * dim + k] + xh[0] * xb[(e0 + 1) * dim + k];
                }
            } else {
                int act = rout[e0] == TOR_STD;
                if (!act) {
                    for (int q = 0; q < ne * dim; q++) nb[q] = xb[e0 * dim + q];
                } else {
                    int nin = (int)(ne * dim);
                    double w[4], R;
                    for (int q = 0; q < ne; q++) w[q] = weight_value(T, rin[e0 + q], rho);
                    if (tp == TOR_F_COLL) R = T->radii[T->fa[f]] + T->radii[T->fb[f]];
                    else R = T->radii[T->fa[f]];
                    double base[12], xp[12], xm[12];
                    for (int q = 0; q < nin; q++) base[q] = n[e0 * dim + q];
                    double sc = 1e-9; /* inside one smooth piece of the minimiser */
                    for (int q = 0; q <= nin; q++) {
                        double in_p[12], in_m[12], Rp = R, Rm = R;
                        memcpy(in_p, base, sizeof(double) * nin);
                        memcpy(in_m, base, sizeof(double) * nin);
                        if (q < nin) in_p[q] += sc, in_m[q] -= sc;
                        else Rp += sc, Rm -= sc;
                        if (tp == TOR_F_COLL) {
                            coll_eval(T, f, in_p, Rp, w, xp);
                            coll_eval(T, f, in_m, Rm, w, xm);
                        } else {
                            wall_eval(T, f, in_p, Rp, w, xp);
                            wall_eval(T, f, in_m, Rm, w, xm);
                        }
                        double g = 0;
                        for (int o = 0; o < nin; o++) g += (xp[o] - xm[o]) / (2 * sc) * xb[e0 * dim + o];
                        if (q < nin) nb[q] = g;
                        else if (tp == TOR_F_COLL) dr[T->fa[f]] += g, dr[T->fb[f]] += g;
                        else dr[T->fa[f]] += g;
                    }
                }
            }
            for (long q = 0; q < ne; q++) {
                long e = e0 + q;
                for (int k = 0; k < dim; k++) {
                    zbn[T->enode[e] * dim + k] += nb[q * dim + k];
                    ubn[e * dim + k] -= nb[q * dim + k];
                }
            }
        }
        memcpy(zb, zbn, sizeof(double) * N * dim);
        memcpy(ub, ubn, sizeof(double) * E * dim);
    }
    /* z^0: its end points are x(0) and x(T) */
    for (int i = 0; i < T->p; i++)
        for (int k = 0; k < dim; k++) {
            dx0[i * dim + k] += zb[node_id(T, i, 0) * dim + k];
            dxT[i * dim + k] += zb[node_id(T, i, T->eta) * dim + k];
        }
    for (long j = 0; j < N; j++) {
        int sj = (int)(j % (T->eta + 1));
        if (sj == 0 || sj == T->eta) continue;
        for (int k = 0; k < dim; k++) dz0[j * dim + k] += zb[j * dim + k];
    }
    free(zb), free(ub), free(xb), free(ubn), free(zbn), free(zhat), free(n);
}
