/*
 * yarn_oracle.c -- plain FP64 CPU oracle of ray / yarn-tube intersection
 * (explicit yarn curves, Sec. 3.3 of arXiv 2401.12724).
 *
 * TEST INFRASTRUCTURE ONLY (see yarn_oracle.h for the definitions).  The
 * search is brute force: every yarn and span whose box the ray crosses is
 * scanned with dense samples of the curve parameter and the best sample is
 * polished by golden-section search.  The rotation-minimising frame and the
 * arc length are integrated with many small steps (double reflection,
 * composite Simpson).
 */
#include "yarn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SUB 64          /* RMF / arc-length sub-steps per span */
#define SCAN 256        /* curve samples per span in the hit scan */
#define DIST_SCAN 64    /* curve samples per span in the distance scan */
#define EXCLUDE_FRAC 1e-3

typedef struct { double x, y, z; } d3;

static d3 mk(double x, double y, double z) { d3 r = {x, y, z}; return r; }
static d3 add(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static d3 sub(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static d3 scl(d3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static d3 cross(d3 a, d3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static d3 unit(d3 a) { return scl(a, 1.0 / sqrt(dot(a, a))); }

typedef struct {
    int32_t n_yarns;
    int64_t* off;      /* control-point CSR */
    int64_t* span_off; /* span CSR: yarn Y owns spans span_off[Y] .. span_off[Y+1]-1 */
    d3* P;             /* control points */
    double* R;         /* per yarn */
    double* ybox;      /* per yarn lo(3) hi(3), grown by R */
    double* sbox;      /* per span lo(3) hi(3), grown by R */
    d3* N0;            /* RMF normal at each span start */
    double* v0;        /* arc length at each span start */
} scene_t;

/* uniform cubic B-spline span on p[0..3] */
static d3 bs_pos(const d3* p, double s)
{
    double u = 1.0 - s;
    double b0 = u * u * u / 6.0;
    double b1 = (3.0 * s * s * s - 6.0 * s * s + 4.0) / 6.0;
    double b2 = (-3.0 * s * s * s + 3.0 * s * s + 3.0 * s + 1.0) / 6.0;
    double b3 = s * s * s / 6.0;
    return add(add(scl(p[0], b0), scl(p[1], b1)), add(scl(p[2], b2), scl(p[3], b3)));
}
static d3 bs_der(const d3* p, double s)
{
    double u = 1.0 - s;
    double b0 = -u * u / 2.0;
    double b1 = (3.0 * s * s - 4.0 * s) / 2.0;
    double b2 = (-3.0 * s * s + 2.0 * s + 1.0) / 2.0;
    double b3 = s * s / 2.0;
    return add(add(scl(p[0], b0), scl(p[1], b1)), add(scl(p[2], b2), scl(p[3], b3)));
}

/* one double-reflection step of the rotation-minimising frame (Wang,
 * Juettler, Zheng, Liu 2008) from (x0, t0, n0) to the point x1 with
 * tangent t1 */
static d3 rmf_step(d3 x0, d3 t0, d3 n0, d3 x1, d3 t1)
{
    d3 v1 = sub(x1, x0);
    double c1 = dot(v1, v1);
    /* a chord at rounding level has a random direction; its limit for a
     * vanishing step is the tangent */
    if (!(c1 > 1e-16 * (dot(x0, x0) + dot(x1, x1)))) {
        v1 = t0;
        c1 = 1.0;
    }
    d3 nl = sub(n0, scl(v1, 2.0 * dot(v1, n0) / c1));
    d3 tl = sub(t0, scl(v1, 2.0 * dot(v1, t0) / c1));
    d3 v2 = sub(t1, tl);
    double c2 = dot(v2, v2);
    if (c2 > 0.0) nl = sub(nl, scl(v2, 2.0 * dot(v2, nl) / c2));
    return nl;
}

static d3 initial_normal(d3 t)
{
    d3 up = fabs(t.z) > cos(25.0 * 3.14159265358979323846 / 180.0) ? mk(1, 0, 0) : mk(0, 0, 1);
    return unit(sub(up, scl(t, dot(up, t))));
}

/* arc length of a span over [0, s] by composite Simpson with SUB intervals */
static double span_len(const d3* p, double s)
{
    double h = s / SUB, acc = 0.0;
    for (int i = 0; i <= SUB; ++i) {
        double w = (i == 0 || i == SUB) ? 1.0 : (i % 2 ? 4.0 : 2.0);
        d3 dd = bs_der(p, i * h);
        acc += w * sqrt(dot(dd, dd));
    }
    return acc * h / 3.0;
}

/* transport the frame from the span start to parameter s in SUB-sized steps */
static d3 span_normal(const d3* p, d3 n0, double s)
{
    d3 n = n0;
    d3 x = bs_pos(p, 0.0), t = unit(bs_der(p, 0.0));
    int steps = (int)ceil(s * SUB - 1e-12);
    for (int i = 1; i <= steps; ++i) {
        double si = i == steps ? s : (double)i / SUB;
        d3 x1 = bs_pos(p, si), t1 = unit(bs_der(p, si));
        n = rmf_step(x, t, n, x1, t1);
        x = x1;
        t = t1;
    }
    return n;
}

void* orc_scene_create(const float* ctrl, const int64_t* yarn_off, int32_t n_yarns)
{
    scene_t* S = (scene_t*)calloc(1, sizeof(scene_t));
    S->n_yarns = n_yarns;
    int64_t ncp = yarn_off[n_yarns];
    S->off = (int64_t*)malloc(sizeof(int64_t) * (n_yarns + 1));
    memcpy(S->off, yarn_off, sizeof(int64_t) * (n_yarns + 1));
    S->span_off = (int64_t*)malloc(sizeof(int64_t) * (n_yarns + 1));
    S->span_off[0] = 0;
    for (int y = 0; y < n_yarns; ++y) S->span_off[y + 1] = S->span_off[y] + (yarn_off[y + 1] - yarn_off[y] - 3);
    int64_t nsp = S->span_off[n_yarns];
    S->P = (d3*)malloc(sizeof(d3) * ncp);
    for (int64_t i = 0; i < ncp; ++i) S->P[i] = mk(ctrl[4 * i], ctrl[4 * i + 1], ctrl[4 * i + 2]);
    S->R = (double*)malloc(sizeof(double) * n_yarns);
    S->ybox = (double*)malloc(sizeof(double) * 6 * n_yarns);
    S->sbox = (double*)malloc(sizeof(double) * 6 * nsp);
    S->N0 = (d3*)malloc(sizeof(d3) * nsp);
    S->v0 = (double*)malloc(sizeof(double) * nsp);
    for (int y = 0; y < n_yarns; ++y) {
        double R = ctrl[4 * yarn_off[y] + 3];
        S->R[y] = R;
        double* yb = S->ybox + 6 * y;
        for (int k = 0; k < 3; ++k) { yb[k] = INFINITY; yb[3 + k] = -INFINITY; }
        d3 n = mk(0, 0, 0);
        double v = 0.0;
        for (int64_t g = S->span_off[y]; g < S->span_off[y + 1]; ++g) {
            const d3* p = S->P + yarn_off[y] + (g - S->span_off[y]);
            double* b = S->sbox + 6 * g;
            for (int k = 0; k < 3; ++k) { b[k] = INFINITY; b[3 + k] = -INFINITY; }
            for (int c = 0; c < 4; ++c) {
                double q[3] = {p[c].x, p[c].y, p[c].z};
                for (int k = 0; k < 3; ++k) {
                    if (q[k] - R < b[k]) b[k] = q[k] - R;
                    if (q[k] + R > b[3 + k]) b[3 + k] = q[k] + R;
                }
            }
            for (int k = 0; k < 3; ++k) {
                if (b[k] < yb[k]) yb[k] = b[k];
                if (b[3 + k] > yb[3 + k]) yb[3 + k] = b[3 + k];
            }
            if (g == S->span_off[y]) n = initial_normal(unit(bs_der(p, 0.0)));
            S->N0[g] = n;
            S->v0[g] = v;
            n = span_normal(p, n, 1.0);
            /* the next span starts where this one ends: same point and
             * tangent, so the frame carries over unchanged */
            v += span_len(p, 1.0);
        }
    }
    return S;
}

void orc_scene_free(void* scene)
{
    scene_t* S = (scene_t*)scene;
    if (!S) return;
    free(S->off); free(S->span_off); free(S->P); free(S->R); free(S->ybox);
    free(S->sbox); free(S->N0); free(S->v0); free(S);
}

static const d3* span_cp(const scene_t* S, int y, int64_t g) { return S->P + S->off[y] + (g - S->span_off[y]); }

void orc_scene_frame(const void* scene, int32_t yarn, int32_t seg, double s, double* out)
{
    const scene_t* S = (const scene_t*)scene;
    int64_t g = S->span_off[yarn] + seg;
    const d3* p = span_cp(S, yarn, g);
    d3 t = unit(bs_der(p, s));
    d3 n = span_normal(p, S->N0[g], s);
    n = unit(sub(n, scl(t, dot(n, t))));
    d3 x = bs_pos(p, s);
    out[0] = t.x; out[1] = t.y; out[2] = t.z;
    out[3] = n.x; out[4] = n.y; out[5] = n.z;
    out[6] = S->v0[g] + span_len(p, s);
    out[7] = x.x; out[8] = x.y; out[9] = x.z;
}

/* slab test of the ray against a box over [t0, t1] */
static int box_hit(const double* b, d3 o, d3 d, double t0, double t1)
{
    double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    for (int k = 0; k < 3; ++k) {
        if (dd[k] == 0.0) {
            if (oo[k] < b[k] || oo[k] > b[3 + k]) return 0;
            continue;
        }
        double ta = (b[k] - oo[k]) / dd[k], tb = (b[3 + k] - oo[k]) / dd[k];
        if (ta > tb) { double tt = ta; ta = tb; tb = tt; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

static const double GOLD = 0.61803398874989484820;

/* squared distance from point q to the span at s */
static double dist2_at(const d3* p, d3 q, double s)
{
    d3 c = sub(bs_pos(p, s), q);
    return dot(c, c);
}

/* minimum distance from q to a span: dense scan, golden-section polish */
static double span_dist(const d3* p, d3 q)
{
    int best = 0;
    double bv = INFINITY;
    for (int i = 0; i <= DIST_SCAN; ++i) {
        double v = dist2_at(p, q, (double)i / DIST_SCAN);
        if (v < bv) { bv = v; best = i; }
    }
    double a = best > 0 ? (double)(best - 1) / DIST_SCAN : 0.0;
    double b = best < DIST_SCAN ? (double)(best + 1) / DIST_SCAN : 1.0;
    for (int it = 0; it < 100; ++it) {
        double x1 = b - GOLD * (b - a), x2 = a + GOLD * (b - a);
        if (dist2_at(p, q, x1) < dist2_at(p, q, x2)) b = x2; else a = x1;
    }
    double v = dist2_at(p, q, 0.5 * (a + b));
    if (v < bv) bv = v;
    return sqrt(bv);
}

/* entry parameter of the ray into the ball of radius R at C(s), or +inf
 * when the ball misses the ray or does not lie ahead of t_min; *depth
 * receives 1 - (distance of the ray from C(s)) / R */
static double entry_at(const d3* p, d3 o, d3 d, double R, double t_min, double s, double* depth)
{
    d3 c = sub(bs_pos(p, s), o);
    double z = dot(c, d);
    double r2 = dot(c, c) - z * z;
    if (r2 < 0.0) r2 = 0.0;
    if (depth) *depth = 1.0 - sqrt(r2) / R;
    if (r2 >= R * R) return INFINITY;
    double t = z - sqrt(R * R - r2);
    return t > t_min ? t : INFINITY;
}

/* derivative dT/ds of the entry parameter (ball at C(s) ahead and hit),
 * or NAN where the ball misses the ray */
static double entry_slope(const d3* p, d3 o, d3 d, double R, double s)
{
    d3 c = sub(bs_pos(p, s), o), c1 = bs_der(p, s);
    double z = dot(c, d), z1 = dot(c1, d);
    double r2 = dot(c, c) - z * z;
    if (r2 >= R * R) return NAN;
    double q = sqrt(R * R - r2);
    return z1 + (dot(c, c1) - z * z1) / q;
}

typedef struct { double t, s, depth; int64_t g; int y; } cand_t;

static void scan_span(const scene_t* S, int y, int64_t g, d3 o, d3 d, double t_min, cand_t* best)
{
    const d3* p = span_cp(S, y, g);
    double R = S->R[y];
    int bi = -1;
    double bt = INFINITY, bdep = -INFINITY;
    for (int i = 0; i <= SCAN; ++i) {
        double dep;
        double t = entry_at(p, o, d, R, t_min, (double)i / SCAN, &dep);
        if (t < bt) { bt = t; bi = i; }
        if (t < INFINITY && dep > bdep) bdep = dep;
    }
    if (bi < 0) return;
    double a = bi > 0 ? (double)(bi - 1) / SCAN : 0.0;
    double b = bi < SCAN ? (double)(bi + 1) / SCAN : 1.0;
    double bs = (double)bi / SCAN;
    /* the minimum in [a, b] is where dT/ds changes sign (a ball that misses
     * the ray counts as a steep wall: -inf on the left, +inf on the right);
     * bisection on that sign is exact to rounding even where T is flat */
    double sm = bs;
    double ga = entry_slope(p, o, d, R, a), gb = entry_slope(p, o, d, R, b);
    if (!(ga == ga)) ga = -INFINITY;
    if (!(gb == gb)) gb = INFINITY;
    if (ga < 0.0 && gb > 0.0) {
        double lo = a, hi = b;
        for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
            double m = 0.5 * (lo + hi);
            if (m <= lo || m >= hi) break;
            double gm = entry_slope(p, o, d, R, m);
            if (!(gm == gm)) {
                /* a gap inside the bracket: fall back to golden section */
                lo = hi = -1.0;
                break;
            }
            if (gm < 0.0) lo = m; else hi = m;
        }
        if (lo >= 0.0) {
            sm = 0.5 * (lo + hi);
        } else {
            double aa = a, bb = b;
            for (int it = 0; it < 100; ++it) {
                double x1 = bb - GOLD * (bb - aa), x2 = aa + GOLD * (bb - aa);
                double f1 = entry_at(p, o, d, R, t_min, x1, NULL), f2 = entry_at(p, o, d, R, t_min, x2, NULL);
                if (f1 < f2) bb = x2; else aa = x1;
            }
            sm = 0.5 * (aa + bb);
        }
    }
    double tm = entry_at(p, o, d, R, t_min, sm, NULL);
    /* where T is flat the refined value ties the best sample to rounding:
     * keep the refined parameter */
    if (tm <= bt + 1e-12 * (fabs(bt) > 1.0 ? fabs(bt) : 1.0)) { if (tm < bt) bt = tm; bs = sm; }
    /* the end points themselves (a minimum on the boundary) */
    for (int e = 0; e < 2; ++e) {
        double te = entry_at(p, o, d, R, t_min, (double)e, NULL);
        if (te < bt) { bt = te; bs = (double)e; }
    }
    if (bt < best->t) {
        best->t = bt;
        best->s = bs;
        best->g = g;
        best->y = y;
        best->depth = bdep;
    }
}

static void intersect_one(const scene_t* S, d3 o, d3 d, double t_max, double t_min, int skip, double* out)
{
    unsigned flags = 0;
    cand_t best = {INFINITY, 0.0, -INFINITY, -1, -1};
    double second = INFINITY; /* best entry of any other yarn */
    for (int y = 0; y < S->n_yarns; ++y) {
        if (y == skip) continue;
        const double* yb = S->ybox + 6 * y;
        double R = S->R[y];
        /* exclusion: the origin lies inside this yarn's tube */
        if (o.x >= yb[0] && o.x <= yb[3] && o.y >= yb[1] && o.y <= yb[4] && o.z >= yb[2] &&
            o.z <= yb[5]) {
            double dm = INFINITY;
            for (int64_t g = S->span_off[y]; g < S->span_off[y + 1]; ++g) {
                const double* b = S->sbox + 6 * g;
                if (o.x < b[0] || o.x > b[3] || o.y < b[1] || o.y > b[4] || o.z < b[2] || o.z > b[5])
                    continue;
                double dd = span_dist(span_cp(S, y, g), o);
                if (dd < dm) dm = dd;
            }
            double lim = R * (1.0 - EXCLUDE_FRAC);
            if (fabs(dm - lim) < 1e-6 * R) flags |= ORC_HIT_ORIGIN_EDGE;
            if (dm < lim) {
                flags |= ORC_HIT_EXCLUDED;
                continue;
            }
        }
        if (!box_hit(yb, o, d, t_min, t_max)) continue;
        cand_t yc = {INFINITY, 0.0, -INFINITY, -1, -1};
        for (int64_t g = S->span_off[y]; g < S->span_off[y + 1]; ++g) {
            if (!box_hit(S->sbox + 6 * g, o, d, t_min, t_max)) continue;
            scan_span(S, y, g, o, d, t_min, &yc);
        }
        if (yc.t < best.t) {
            if (best.t < second) second = best.t;
            best = yc;
        } else if (yc.t < second) {
            second = yc.t;
        }
    }
    for (int k = 0; k < 16; ++k) out[k] = 0.0;
    out[15] = second;
    if (!(best.t <= t_max)) {
        out[0] = INFINITY;
        out[1] = -1;
        out[12] = (double)(flags | ORC_HIT_MISS);
        return;
    }
    int y = best.y;
    int64_t g = best.g;
    int seg = (int)(g - S->span_off[y]);
    const d3* p = span_cp(S, y, g);
    double R = S->R[y];
    if ((seg == 0 && best.s <= 0.0) || (g == S->span_off[y + 1] - 1 && best.s >= 1.0))
        flags |= ORC_HIT_CAP;
    if (best.depth < 1e-3) flags |= ORC_HIT_GRAZING;
    /* an entry right after t_min: the balls nearest the origin lie behind
     * t_min, so the first ball ahead sits on the t_min level set and its
     * parameter is not well defined */
    if (best.t - t_min < 1e-2 * R) flags |= ORC_HIT_ORIGIN_EDGE;
    if (second - best.t < 1e-7 * (best.t > 1.0 ? best.t : 1.0)) flags |= ORC_HIT_TIE;
    double fr[10];
    orc_scene_frame(S, y, seg, best.s, fr);
    d3 T = mk(fr[0], fr[1], fr[2]), N = mk(fr[3], fr[4], fr[5]);
    d3 Bv = cross(T, N);
    d3 hp = add(o, scl(d, best.t));
    d3 q = scl(sub(hp, bs_pos(p, best.s)), 1.0 / R);
    double qn = dot(q, N), qb = dot(q, Bv);
    double ql = sqrt(qn * qn + qb * qb);
    d3 wi = scl(d, -1.0);
    double wn = dot(wi, N), wb = dot(wi, Bv);
    double wl = sqrt(wn * wn + wb * wb);
    double h = (ql > 0.0 && wl > 0.0) ? (qb * wn - qn * wb) / (ql * wl) : 0.0;
    if (h > 1.0) h = 1.0;
    if (h < -1.0) h = -1.0;
    out[0] = best.t;
    out[1] = y;
    out[2] = seg;
    out[3] = best.s;
    out[4] = h;
    out[5] = fr[6];
    out[6] = T.x; out[7] = T.y; out[8] = T.z;
    out[9] = N.x; out[10] = N.y; out[11] = N.z;
    out[12] = (double)flags;
    out[13] = best.depth;
    out[14] = 0.0;
}

void orc_intersect(const void* scene, int64_t n, const float* o, const float* d, const float* t_max,
                   double t_min, double* out, int nthreads)
{
    const scene_t* S = (const scene_t*)scene;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < n; ++i) {
        d3 oo = mk(o[3 * i], o[3 * i + 1], o[3 * i + 2]);
        d3 dd = unit(mk(d[3 * i], d[3 * i + 1], d[3 * i + 2]));
        intersect_one(S, oo, dd, (double)t_max[i], t_min, -1, out + 16 * i);
    }
}

void orc_intersect_one(const void* scene, const double o[3], const double d[3], double t_min,
                       double t_max, int32_t skip_yarn, double out[16])
{
    intersect_one((const scene_t*)scene, mk(o[0], o[1], o[2]), unit(mk(d[0], d[1], d[2])), t_max,
                  t_min, skip_yarn, out);
}

double orc_scene_radius(const void* scene, int32_t yarn) { return ((const scene_t*)scene)->R[yarn]; }
