// yarn_tube.hpp -- device side of ray / yarn-tube intersection.
//
// A yarn is a uniform cubic B-spline centreline (the explicit yarn curves
// of Sec. 3.3) with radius R; its tube is the union of the balls of radius
// R centred on the curve.  Entering through the ball at C(s) happens at
// ray parameter T(s) = z(s) - sqrt(R^2 - r^2(s)), with z the distance of
// C(s) along the ray and r its distance from the ray, so the entry into a
// span is the minimum of T over s (an interior minimum is where the ray
// meets the tube surface, the closest-point condition).  Per span: T is
// sampled at a few points, the best sample is bracketed and polished by
// safeguarded Newton on dT/ds in double precision.
//
// The BVH is built binary (binned SAH) and collapsed to four children per
// node: a node holds its four child boxes as structure of arrays and the
// child codes in one 128-byte line, so a ray fetches half as many nodes
// one after another as in the binary tree.  Hit children are visited near
// first, and the per-thread stack lives in LDS.  The closest-hit traversal
// runs nodes and span scans in separate loops, with postponed leaves, so
// the span scans of a wavefront run together; the point query for tubes
// holding the origin stops each span's distance test as soon as a sample
// decides it.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/bysdf.h"
#include "bysdf_math.hpp"

namespace yarn {

constexpr int kStack = 64;        // binary BVH depth bound enforced by the builder
constexpr int kWideDepthMax = 40; // depth bound of the 4-wide tree (LDS stack: 123 entries)
// Entries of a lane's traversal stack for a 4-wide BVH whose deepest node
// sits at the given depth (root 0): a visit pushes at most three siblings,
// and a path holds depth + 1 nodes, so 3 (depth + 1) entries never
// overflow.  The traversal kernels size their LDS stacks with this at
// launch, which leaves LDS for more wavefronts per CU on shallow trees.
inline int stack_entries(int depth) { return 3 * (depth + 1); }
constexpr int kMaxExcluded = 4;   // yarns holding the ray origin
constexpr double kExcludeFrac = 1e-3;

// hit flags
constexpr uint32_t HIT_MISS = 1u << 0;
constexpr uint32_t HIT_CAP = 1u << 1;
constexpr uint32_t HIT_EXCLUDED = 1u << 2;
constexpr uint32_t HIT_BAD_INPUT = 1u << 9;

// binary node of the build: child boxes lo0 hi0 lo1 hi1 packed, child codes
// (>= 0 node, < 0 leaf: -(first*4 + count-1) - 1)
struct BNode {
    float4 a, b, c;
    int4 d;
};
// node of the traversed 4-wide tree: bounds of child c in component c of
// each float4; an unused slot has an empty box (lo +inf, hi -inf)
struct WNode {
    float4 lox, loy, loz, hix, hiy, hiz;
    int4 code;  // child codes as above (node codes index the wide nodes)
    int4 pad;   // to 128 bytes
};

// span record (leaf order): first control point, yarn, index in the
// yarn, samples | first-span bit 16 | last-span bit 17
struct SpanRec {
    int cp0, yarn, seg, info;
};

struct SceneView {
    const float4* cp;       // x y z R per control point
    const SpanRec* span;    // leaf order
    const float4* frame;    // per span (leaf order): RMF normal at s = 0, arc length at s = 0
    const WNode* node;
    const float* yarn_phase;
    const int* yarn_type;
    int n_nodes;
};

struct D3 {
    double x, y, z;
};
__host__ __device__ inline D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__host__ __device__ inline D3 operator+(D3 a, D3 b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline D3 operator-(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline D3 operator*(D3 a, double s) { return d3(a.x * s, a.y * s, a.z * s); }
__host__ __device__ inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline D3 cross(D3 a, D3 b)
{
    return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline D3 unit(D3 a) { return a * bysdf::rsqrt_(dot(a, a)); }

// uniform cubic B-spline basis and its first two derivatives
__host__ __device__ inline void basis(double s, double* b)
{
    double u = 1.0 - s, s2 = s * s, s3 = s2 * s;
    b[0] = u * u * u * (1.0 / 6.0);
    b[1] = (3.0 * s3 - 6.0 * s2 + 4.0) * (1.0 / 6.0);
    b[2] = (-3.0 * s3 + 3.0 * s2 + 3.0 * s + 1.0) * (1.0 / 6.0);
    b[3] = s3 * (1.0 / 6.0);
}
__host__ __device__ inline void basis1(double s, double* b)
{
    double u = 1.0 - s;
    b[0] = -0.5 * u * u;
    b[1] = 1.5 * s * s - 2.0 * s;
    b[2] = -1.5 * s * s + s + 0.5;
    b[3] = 0.5 * s * s;
}
__host__ __device__ inline void basis2(double s, double* b)
{
    b[0] = 1.0 - s;
    b[1] = 3.0 * s - 2.0;
    b[2] = -3.0 * s + 1.0;
    b[3] = s;
}
__host__ __device__ inline D3 comb(const D3* c, const double* b)
{
    return d3(b[0] * c[0].x + b[1] * c[1].x + b[2] * c[2].x + b[3] * c[3].x,
              b[0] * c[0].y + b[1] * c[1].y + b[2] * c[2].y + b[3] * c[3].y,
              b[0] * c[0].z + b[1] * c[1].z + b[2] * c[2].z + b[3] * c[3].z);
}

// Ray-space view of one span: control points relative to the origin.
struct SpanGeo {
    D3 c[4];
    double R;
};

// Power-form coefficients a0 + a1 s + a2 s^2 + a3 s^3 of a uniform cubic
// B-spline coordinate with control values c0..c3 (the basis above, expanded).
__host__ __device__ inline void spline_power(const double* c, double* a)
{
    a[0] = (c[0] + 4.0 * c[1] + c[2]) * (1.0 / 6.0);
    a[1] = (c[2] - c[0]) * 0.5;
    a[2] = (c[0] - 2.0 * c[1] + c[2]) * 0.5;
    a[3] = (c[3] - c[0] + 3.0 * (c[1] - c[2])) * (1.0 / 6.0);
}

// A span seen from the ray: the centreline's offset (u, w) from the ray
// and its position z along it, each a cubic in s in power form.
struct RayCubic {
    double u[4], w[4], z[4];
};

__host__ __device__ inline double horner3(const double* a, double s)
{
    return fma(fma(fma(a[3], s, a[2]), s, a[1]), s, a[0]);
}

// entry T(s) = z - sqrt(R^2 - u^2 - w^2) if above t_min, else +inf
__host__ __device__ inline double entry_at(const RayCubic& rc, double R, double s, double t_min)
{
    const double u = horner3(rc.u, s), w = horner3(rc.w, s);
    const double q2 = R * R - (u * u + w * w);
    if (!(q2 > 0.0)) return INFINITY;
    const double t = horner3(rc.z, s) - bysdf::sqrt_(q2);
    return t > t_min ? t : INFINITY;
}

// dT/ds and d2T/ds2 at s; returns false where the ball misses the ray
__host__ __device__ inline bool entry_slope(const RayCubic& rc, double R, double s, double* g1, double* g2)
{
    double u = horner3(rc.u, s), w = horner3(rc.w, s);
    double q2 = R * R - (u * u + w * w);
    if (!(q2 > 0.0)) return false;
    // first and second derivatives of the three cubics
    auto d1 = [s](const double* a) { return fma(fma(3.0 * a[3], s, 2.0 * a[2]), s, a[1]); };
    auto d2 = [s](const double* a) { return fma(6.0 * a[3], s, 2.0 * a[2]); };
    const double u1 = d1(rc.u), w1 = d1(rc.w), z1 = d1(rc.z);
    const double u2 = d2(rc.u), w2 = d2(rc.w), z2 = d2(rc.z);
    const double q = bysdf::sqrt_(q2), iq = bysdf::rcp_(q);
    const double h = u * u1 + w * w1;  // (r^2)' / 2
    *g1 = z1 + h * iq;
    const double hp = u1 * u1 + w1 * w1 + u * u2 + w * w2;
    *g2 = z2 + (hp + h * h / q2) * iq;
    return true;
}

// Sampled scan of one span: the smallest entry T(s_i) > t_min over the
// nsamp + 1 samples, if it is at most t_lim (and the control-point hull
// reaches the ray's R-slab within [t_min, t_lim + R]).
__host__ __device__ inline bool span_scan(const SpanGeo& g, D3 d, D3 e1, D3 e2, double t_min, double t_lim,
                                          int nsamp, double* t_out, int* i_out)
{
    const double R = g.R;
    bool all_pu = true, all_nu = true, all_pw = true, all_nw = true, all_b = true, all_f = true;
    double pu[4], pw[4], pz[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double u = dot(g.c[k], e1), w = dot(g.c[k], e2), z = dot(g.c[k], d);
        pu[k] = u;
        pw[k] = w;
        pz[k] = z;
        all_pu &= u > R;
        all_nu &= u < -R;
        all_pw &= w > R;
        all_nw &= w < -R;
        all_b &= z + R < t_min;
        all_f &= z - R > t_lim;
    }
    if (all_pu || all_nu || all_pw || all_nw || all_b || all_f) return false;
    // the curve lies in the hull of its control points: in the plane across
    // the ray, a hull entirely more than R to one side of the line through
    // the outer two points' direction (the span's chord) misses the ray
    {
        double cx = pu[3] - pu[0], cy = pw[3] - pw[0];
        double cl = bysdf::sqrt_(cx * cx + cy * cy);
        if (cl > 1e-12 * R) {
            const double icl = bysdf::rcp_(cl);
            double nx = -cy * icl, ny = cx * icl;
            bool all_p = true, all_n = true;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double sd = nx * pu[k] + ny * pw[k];
                all_p &= sd > R;
                all_n &= sd < -R;
            }
            if (all_p || all_n) return false;
        }
    }
    // the samples in the ray's frame (e1, e2, d): the centreline's offset
    // (u, w) from the ray and its position z along it are cubics in s, in
    // power form from the projected control points, so a sample costs three
    // Horner steps per coordinate and r^2 = u^2 + w^2 has no cancellation
    RayCubic rc;
    spline_power(pu, rc.u);
    spline_power(pw, rc.w);
    spline_power(pz, rc.z);
    const double inv = 1.0 / nsamp;
    double bt = INFINITY;
    int bi = -1;
    for (int i = 0; i <= nsamp; ++i) {
        const double t = entry_at(rc, R, i * inv, t_min);
        if (t < bt) {
            bt = t;
            bi = i;
        }
    }
    if (bi < 0 || bt > t_lim) return false;
    *t_out = bt;
    *i_out = bi;
    return true;
}

// Minimum of T in the bracket of sample bi (best sampled value bt):
// safeguarded Newton on dT/ds in double precision.
__host__ __device__ inline void span_refine(const SpanGeo& g, D3 d, D3 e1, D3 e2, double t_min, int nsamp, int bi,
                                            double bt, double* t_out, double* s_out)
{
    RayCubic rc;
    {
        double pu[4], pw[4], pz[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            pu[k] = dot(g.c[k], e1);
            pw[k] = dot(g.c[k], e2);
            pz[k] = dot(g.c[k], d);
        }
        spline_power(pu, rc.u);
        spline_power(pw, rc.w);
        spline_power(pz, rc.z);
    }
    const double R = g.R;
    const double inv = 1.0 / nsamp;
    double lo = bi > 0 ? (bi - 1) * inv : 0.0, hi = bi < nsamp ? (bi + 1) * inv : 1.0;
    double s = bi * inv, g1, g2;
    // slope at the bracket ends (a ball that misses the ray reads as a
    // steep wall: -inf on the left, +inf on the right)
    double glo = entry_slope(rc, R, lo, &g1, &g2) ? g1 : -INFINITY;
    double ghi = entry_slope(rc, R, hi, &g1, &g2) ? g1 : INFINITY;
    double sb = s;
    if (glo >= 0.0) {
        sb = lo;
    } else if (ghi <= 0.0) {
        sb = hi;
    } else {
        for (int it = 0; it < 24; ++it) {
            double sn;
            if (entry_slope(rc, R, s, &g1, &g2)) {
                if (g1 < 0.0)
                    lo = s;
                else
                    hi = s;
                sn = s - g1 * bysdf::rcp_(g2);
                if (!(g2 > 0.0) || !(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
            } else {
                sn = 0.5 * (lo + hi);
            }
            bool done = fabs(sn - s) < 1e-15 || hi - lo < 1e-15;
            s = sn;
            if (done) break;
        }
        sb = s;
    }
    double t = entry_at(rc, R, sb, t_min);
    // where T is flat the refined value ties the best sample to rounding:
    // keep the refined parameter
    if (t <= bt + 1e-12 * fmax(1.0, fabs(bt))) {
        *t_out = fmin(t, bt);
        *s_out = sb;
    } else {
        *t_out = bt;
        *s_out = bi * inv;
    }
}

__host__ __device__ inline void load_span(const SceneView& S, const SpanRec& r, D3 o, SpanGeo* g)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float4 p = S.cp[r.cp0 + k];
        g->c[k] = d3((double)p.x - o.x, (double)p.y - o.y, (double)p.z - o.z);
        if (k == 0) g->R = (double)p.w;
    }
}

// Whether the curve comes closer than lim to the origin of the span view,
// as the squared distance from the samples refined by safeguarded Newton on
// the derivative of |C(s)|^2 decides it.  Two exits skip the refinement
// without changing the answer: a sample already closer than lim (the
// refinement only lowers the minimum), and samples all farther than
// lim + L / (2 nsamp), with L = max_k |c_{k+1} - c_k| bounding the speed
// |C'(s)| (the derivative of a uniform cubic B-spline segment is a convex
// combination of its control-point differences), so that no point of the
// curve, being within 1 / (2 nsamp) of a sample, can come closer than lim.
__host__ __device__ inline bool span_within(const SpanGeo& g, int nsamp, double lim)
{
    // the centreline relative to the point, a cubic per coordinate
    double cx[4], cy[4], cz[4], ax[4], ay[4], az[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cx[k] = g.c[k].x;
        cy[k] = g.c[k].y;
        cz[k] = g.c[k].z;
    }
    spline_power(cx, ax);
    spline_power(cy, ay);
    spline_power(cz, az);
    auto at = [&](double s) { return d3(horner3(ax, s), horner3(ay, s), horner3(az, s)); };
    double inv = 1.0 / nsamp, bv = INFINITY;
    int bi = 0;
    for (int i = 0; i <= nsamp; ++i) {
        D3 p = at(i * inv);
        double v = dot(p, p);
        if (v < bv) {
            bv = v;
            bi = i;
        }
    }
    const double lim2 = lim * lim;
    if (bv < lim2) return true;
    double L2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const D3 dc = g.c[k + 1] - g.c[k];
        L2 = fmax(L2, dot(dc, dc));
    }
    // the relative margin covers the rounding of the samples and of L
    const double m = lim + 0.5 * bysdf::sqrt_(L2) * inv;
    if (bv > m * m * (1.0 + 1e-9)) return false;
    double lo = bi > 0 ? (bi - 1) * inv : 0.0, hi = bi < nsamp ? (bi + 1) * inv : 1.0, s = bi * inv;
    for (int it = 0; it < 20; ++it) {
        D3 p = at(s);
        auto d1 = [s](const double* a) { return fma(fma(3.0 * a[3], s, 2.0 * a[2]), s, a[1]); };
        auto d2 = [s](const double* a) { return fma(6.0 * a[3], s, 2.0 * a[2]); };
        D3 p1 = d3(d1(ax), d1(ay), d1(az)), p2 = d3(d2(ax), d2(ay), d2(az));
        double f1 = dot(p, p1), f2 = dot(p1, p1) + dot(p, p2);
        double v = dot(p, p);
        if (v < bv) bv = v;
        if (f1 < 0.0)
            lo = s;
        else
            hi = s;
        double sn = s - f1 * bysdf::rcp_(f2);
        if (!(f2 > 0.0) || !(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
        if (fabs(sn - s) < 1e-15) break;
        s = sn;
    }
    D3 p = at(s);
    double v = dot(p, p);
    return (v < bv ? v : bv) < lim2;
}
// True when the span is certainly farther than lim from the origin of the
// span view: the curve lies in the hull of its control points, which lies
// within the slab of the chord direction they span and within the
// cylinder around the chord line that holds them.
__host__ __device__ inline bool span_far(const SpanGeo& g, double lim)
{
    D3 ch = g.c[3] - g.c[0];
    double cl2 = dot(ch, ch);
    if (!(cl2 > 0.0)) return false;
    D3 t = ch * bysdf::rsqrt_(cl2);
    bool all_p = true, all_n = true;
    double rho2 = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double a = dot(g.c[k], t);
        all_p &= a > lim;
        all_n &= a < -lim;
        D3 q = g.c[k] - g.c[0];
        D3 pq = q - t * dot(q, t);
        rho2 = fmax(rho2, dot(pq, pq));
    }
    if (all_p || all_n) return true;
    D3 p0 = g.c[0] - t * dot(g.c[0], t);  // origin to the chord line
    double dl = bysdf::sqrt_(dot(p0, p0)) - bysdf::sqrt_(rho2);
    return dl > lim;
}

__host__ __device__ inline void decode_leaf(int code, int* first, int* count)
{
    int c = -code - 1;
    *first = c >> 2;
    *count = (c & 3) + 1;
}
__host__ __device__ inline int leaf_code(int first, int count) { return -((first << 2) | (count - 1)) - 1; }
// end of a traversal: below every leaf code of a scene of fewer than 2^29 spans
constexpr int kTraceDone = INT32_MIN;

// Whether the predicate holds on any active lane of the wavefront (on the
// host, a single lane: the predicate itself).
__host__ __device__ inline bool wave_any(bool p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __any((int)p) != 0;
#else
    return p;
#endif
}

// box of child c (0..3) of a wide node
__host__ __device__ inline float comp4(const float4& v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}
__host__ __device__ inline int comp4i(const int4& v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

__host__ __device__ inline bool box_ray(float3 lo, float3 hi, float3 o, float3 inv, float t0, float t1, float* tn)
{
    float ax = (lo.x - o.x) * inv.x, bx = (hi.x - o.x) * inv.x;
    float ay = (lo.y - o.y) * inv.y, by = (hi.y - o.y) * inv.y;
    float az = (lo.z - o.z) * inv.z, bz = (hi.z - o.z) * inv.z;
    float tmin = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), t0));
    float tmax = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), t1));
    // conservative against the rounding of the slab distances
    tmax *= 1.0000004f;
    *tn = tmin;
    return tmin <= tmax;
}

__host__ __device__ inline bool box_point(float3 lo, float3 hi, float3 p)
{
    return p.x >= lo.x && p.x <= hi.x && p.y >= lo.y && p.y <= hi.y && p.z >= lo.z && p.z <= hi.z;
}

// Yarns whose tube holds the origin (distance to the centreline below
// R (1 - 1e-3)).  Point query through the BVH; stack at stk[k * stride].
// Yarn `skip` (-1: none) is left out of the query and comes first in ex:
// a ray leaving a yarn skips that yarn whatever its origin.
__host__ __device__ inline int excluded_yarns(const SceneView& S, D3 o, int* stk, int stride, int* ex,
                                              int skip = -1)
{
    float3 of = make_float3((float)o.x, (float)o.y, (float)o.z);
    int nex = 0, sp = 0, code = 0;
    if (skip >= 0) ex[nex++] = skip;
    while (true) {
        if (code >= 0) {
            const WNode n = S.node[code];
            // the float origin may sit a rounding step outside a box that
            // holds the double origin: grow the test box by a relative ulp
            float3 e = make_float3(fabsf(of.x) * 2.4e-7f + 1e-30f, fabsf(of.y) * 2.4e-7f + 1e-30f,
                                   fabsf(of.z) * 2.4e-7f + 1e-30f);
            int next = 0, nh = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float3 lo = make_float3(comp4(n.lox, c) - e.x, comp4(n.loy, c) - e.y, comp4(n.loz, c) - e.z);
                float3 hi = make_float3(comp4(n.hix, c) + e.x, comp4(n.hiy, c) + e.y, comp4(n.hiz, c) + e.z);
                if (box_point(lo, hi, of)) {
                    // the first hit child is visited next, the others pushed
                    if (nh > 0) stk[sp++ * stride] = next;
                    next = comp4i(n.code, c);
                    ++nh;
                }
            }
            if (nh > 0) {
                code = next;
                continue;
            }
        } else {
            int first, count;
            decode_leaf(code, &first, &count);
            for (int k = 0; k < count; ++k) {
                SpanRec r = S.span[first + k];
                bool seen = false;
                for (int j = 0; j < nex; ++j) seen |= ex[j] == r.yarn;
                if (seen || nex >= kMaxExcluded + (skip >= 0 ? 1 : 0)) continue;
                SpanGeo g;
                load_span(S, r, o, &g);
                double lim = g.R * (1.0 - kExcludeFrac);
                if (span_far(g, lim)) continue;
                if (span_within(g, r.info & 0xffff, lim)) ex[nex++] = r.yarn;
            }
        }
        if (sp == 0) break;
        code = stk[--sp * stride];
    }
    return nex;
}

struct RayHit {
    double t, s;
    int span;  // leaf-order span index, -1 for a miss
};

// Candidates kept for refinement: spans whose best sample lies within
// kCandMargin R of the best sample so far.  A minimum between samples
// undershoots its bracket's best sample by far less than that unless the
// ray only grazes the tube (samples are at most 0.05 R apart along the
// curve), so the true first entry is among them.
constexpr int kCand = 6;
constexpr double kCandMargin = 0.1;

// Closest entering hit with t_min < t <= t_max.  Traversal ranks spans by
// their sampled entries (an upper bound of the true entry, so it is safe
// for culling); only the candidates are refined, once, at the end.
__host__ __device__ inline RayHit closest_hit(const SceneView& S, D3 o, D3 d, double t_min, double t_max,
                                              const int* ex, int nex, int* stk, int stride)
{
    float3 of = make_float3((float)o.x, (float)o.y, (float)o.z);
    float3 inv = make_float3(1.0f / (fabs(d.x) > 1e-30 ? (float)d.x : 1e-30f),
                             1.0f / (fabs(d.y) > 1e-30 ? (float)d.y : 1e-30f),
                             1.0f / (fabs(d.z) > 1e-30 ? (float)d.z : 1e-30f));
    // the float origin is within a relative ulp of the double one: widen
    // the slab interval by that much along the ray
    float slack = 2.4e-7f * (fabsf(of.x) + fabsf(of.y) + fabsf(of.z)) + 1e-30f;
    // basis of the plane across the ray (for the span hull test)
    D3 a = fabs(d.x) < 0.9 ? d3(1, 0, 0) : d3(0, 1, 0);
    D3 e1 = unit(cross(d, a)), e2 = cross(d, e1);
    // candidates sorted by sampled entry (static indices: registers)
    double ct[kCand];
    int cs[kCand], ci[kCand];
#pragma unroll
    for (int k = 0; k < kCand; ++k) {
        ct[k] = INFINITY;
        cs[k] = -1;
        ci[k] = 0;
    }
    double tb = t_max;  // best sampled entry (bounds the true first entry)
    int sp = 0, code = 0;
    float t0 = (float)t_min - slack;
    // Two inner loops (the while-while form of Aila and Laine, HPG 2009,
    // with their postponed leaves): a lane that reaches a leaf holds it and
    // goes on through nodes until every lane of the wavefront holds a leaf
    // or is done; then the held leaves are scanned one span per step, with
    // the leaves met meanwhile.  The expensive span scans so run with most
    // lanes active.  A lane may visit nodes before scanning a leaf it holds,
    // with the larger bound tb of that moment: that costs only pruning.  A
    // span that survives the final filter of the candidates (sampled entry
    // within kCandMargin R of the final tb) passes the scan limit whenever
    // it is scanned, and the candidate list keeps the smallest entries, so
    // the refined candidates, and the hit, do not depend on the order.
    int leaf = 0;  // the held leaf's code, 0 for none
    while (code != kTraceDone || leaf != 0) {
        while (code >= 0) {
            const float t1 = (float)tb + slack;
            const WNode n = S.node[code];
            float tn[4];
            int cc[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float3 lo = make_float3(comp4(n.lox, c), comp4(n.loy, c), comp4(n.loz, c));
                float3 hi = make_float3(comp4(n.hix, c), comp4(n.hiy, c), comp4(n.hiz, c));
                float t;
                tn[c] = box_ray(lo, hi, of, inv, t0, t1, &t) ? t : INFINITY;
                cc[c] = comp4i(n.code, c);
            }
            // hit children near first (a sorting network; misses sort last)
#define YARN_CSWAP(a, b)                                      \
    do {                                                      \
        const bool sw_ = tn[b] < tn[a];                       \
        const float ta_ = tn[a];                              \
        const int ca_ = cc[a];                                \
        tn[a] = sw_ ? tn[b] : tn[a];                          \
        tn[b] = sw_ ? ta_ : tn[b];                            \
        cc[a] = sw_ ? cc[b] : cc[a];                          \
        cc[b] = sw_ ? ca_ : cc[b];                            \
    } while (0)
            YARN_CSWAP(0, 1);
            YARN_CSWAP(2, 3);
            YARN_CSWAP(0, 2);
            YARN_CSWAP(1, 3);
            YARN_CSWAP(1, 2);
#undef YARN_CSWAP
            if (tn[0] < INFINITY) {
                // push the farther hits, farthest first
                if (tn[3] < INFINITY) stk[sp++ * stride] = cc[3];
                if (tn[2] < INFINITY) stk[sp++ * stride] = cc[2];
                if (tn[1] < INFINITY) stk[sp++ * stride] = cc[1];
                code = cc[0];
            } else {
                code = sp > 0 ? stk[--sp * stride] : kTraceDone;
            }
            if (leaf == 0 && code < 0 && code != kTraceDone) {
                leaf = code;
                code = sp > 0 ? stk[--sp * stride] : kTraceDone;
            }
            if (!wave_any(leaf == 0 && code != kTraceDone)) break;
        }
        while (leaf != 0) {
            int first, count;
            decode_leaf(leaf, &first, &count);
            SpanRec r = S.span[first];
            bool skip = false;
            for (int j = 0; j < nex; ++j) skip |= ex[j] == r.yarn;
            if (!skip) {
                SpanGeo g;
                load_span(S, r, o, &g);
                double t;
                int bi;
                double lim = fmin(t_max, tb + kCandMargin * g.R);
                if (span_scan(g, d, e1, e2, t_min, lim, r.info & 0xffff, &t, &bi)) {
                    tb = fmin(tb, t);
                    double nt = t;
                    int nsp = first, nbi = bi;
#pragma unroll
                    for (int q = 0; q < kCand; ++q) {
                        if (nt < ct[q]) {
                            double tt = ct[q];
                            int ts = cs[q], tq = ci[q];
                            ct[q] = nt;
                            cs[q] = nsp;
                            ci[q] = nbi;
                            nt = tt;
                            nsp = ts;
                            nbi = tq;
                        }
                    }
                }
            }
            // the leaf's next span, else a leaf met meanwhile (and the next
            // entry of the stack behind it)
            if (count > 1) {
                leaf = leaf_code(first + 1, count - 1);
            } else if (code < 0 && code != kTraceDone) {
                leaf = code;
                code = sp > 0 ? stk[--sp * stride] : kTraceDone;
            } else {
                leaf = 0;
            }
        }
    }
    RayHit best{t_max, 0.0, -1};
#pragma unroll
    for (int q = 0; q < kCand; ++q) {
        if (cs[q] < 0) continue;
        SpanRec r = S.span[cs[q]];
        SpanGeo g;
        load_span(S, r, o, &g);
        if (ct[q] > tb + kCandMargin * g.R) continue;
        double t, s;
        span_refine(g, d, e1, e2, t_min, r.info & 0xffff, ci[q], ct[q], &t, &s);
        if (t < best.t || (t == best.t && best.span < 0)) {
            best.t = t;
            best.s = s;
            best.span = cs[q];
        }
    }
    if (!(best.t <= t_max)) best.span = -1;
    return best;
}

// Frame, h and arc length at a hit.
struct HitFrame {
    D3 T, N, B, c;  // tangent, reference normal, binormal, centreline point
    double v;       // arc length from the yarn start
};

__host__ __device__ inline HitFrame hit_frame(const SceneView& S, int span, double s)
{
    SpanRec r = S.span[span];
    D3 c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float4 p = S.cp[r.cp0 + k];
        c[k] = d3(p.x, p.y, p.z);
    }
    double b[4];
    basis(0.0, b);
    D3 x0 = comb(c, b);
    basis1(0.0, b);
    D3 t0 = unit(comb(c, b));
    basis(s, b);
    D3 x1 = comb(c, b);
    basis1(s, b);
    D3 t1 = unit(comb(c, b));
    float4 f = S.frame[span];
    D3 n0 = d3(f.x, f.y, f.z);
    // one double-reflection step of the rotation-minimising frame
    // (Wang, Juettler, Zheng and Liu 2008) from the span start to s
    // a chord at rounding level has a random direction; its limit for a
    // vanishing step is the tangent
    D3 v1 = x1 - x0;
    double c1 = dot(v1, v1);
    if (!(c1 > 1e-16 * (dot(x0, x0) + dot(x1, x1)))) {
        v1 = t0;
        c1 = 1.0;
    }
    D3 nl = n0 - v1 * (2.0 * dot(v1, n0) / c1);
    D3 tl = t0 - v1 * (2.0 * dot(v1, t0) / c1);
    D3 v2 = t1 - tl;
    double c2 = dot(v2, v2);
    if (c2 > 0.0) nl = nl - v2 * (2.0 * dot(v2, nl) / c2);
    HitFrame h;
    h.T = t1;
    h.N = unit(nl - t1 * dot(nl, t1));
    h.B = cross(h.T, h.N);
    h.c = x1;
    // arc length inside the span: 5-point Gauss-Legendre on [0, s]
    const double gx[5] = {0.0, -0.5384693101056831, 0.5384693101056831, -0.9061798459386640,
                          0.9061798459386640};
    const double gw[5] = {0.5688888888888889, 0.4786286704993665, 0.4786286704993665,
                          0.2369268850561891, 0.2369268850561891};
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        basis1(0.5 * s * (1.0 + gx[k]), b);
        D3 dd = comb(c, b);
        acc += gw[k] * bysdf::sqrt_(dot(dd, dd));
    }
    h.v = (double)f.w + 0.5 * s * acc;
    return h;
}

// One ray: exclusion point query, closest entering hit, hit frame, h, v.
// stk: this lane's stack entries at stk[k * stride].
__host__ __device__ inline void intersect_ray(const SceneView& S, int64_t i, const yarn_ray_soa& R,
                                              double t_min, const yarn_hit_soa& H, int* stk, int stride)
{
    D3 o = d3(R.o_x[i], R.o_y[i], R.o_z[i]);
    D3 dr = d3(R.d_x[i], R.d_y[i], R.d_z[i]);
    double tm = R.t_max[i];
    double l2 = dot(dr, dr);
    uint32_t flags = 0;
    bool ok = __builtin_isfinite(o.x) && __builtin_isfinite(o.y) && __builtin_isfinite(o.z) &&
              __builtin_isfinite(l2) && l2 > 0.0 && !__builtin_isnan(tm);
    if (ok) {
        D3 d = dr * (1.0 / sqrt(l2));
        int ex[kMaxExcluded];
        int nex = excluded_yarns(S, o, stk, stride, ex);
        if (nex) flags |= HIT_EXCLUDED;
        RayHit hit = closest_hit(S, o, d, t_min, tm, ex, nex, stk, stride);
        if (hit.span >= 0) {
            SpanRec r = S.span[hit.span];
            HitFrame f = hit_frame(S, hit.span, hit.s);
            D3 p = o + d * hit.t;
            D3 q = p - f.c;
            double qn = dot(q, f.N), qb = dot(q, f.B);
            double wn = -dot(d, f.N), wb = -dot(d, f.B);
            double ql = sqrt(qn * qn + qb * qb), wl = sqrt(wn * wn + wb * wb);
            double h = (ql > 0.0 && wl > 0.0) ? (qb * wn - qn * wb) / (ql * wl) : 0.0;
            h = fmin(1.0, fmax(-1.0, h));
            if (((r.info >> 16) & 1) && hit.s <= 0.0) flags |= HIT_CAP;
            if (((r.info >> 17) & 1) && hit.s >= 1.0) flags |= HIT_CAP;
            H.t[i] = (float)hit.t;
            H.yarn[i] = r.yarn;
            H.seg[i] = r.seg;
            H.s[i] = (float)hit.s;
            H.h[i] = (float)h;
            H.u[i] = S.yarn_phase[r.yarn];
            H.v[i] = (float)f.v;
            H.tan_x[i] = (float)f.T.x;
            H.tan_y[i] = (float)f.T.y;
            H.tan_z[i] = (float)f.T.z;
            H.nrm_x[i] = (float)f.N.x;
            H.nrm_y[i] = (float)f.N.y;
            H.nrm_z[i] = (float)f.N.z;
            H.flags[i] = flags;
            return;
        }
    } else {
        flags |= HIT_BAD_INPUT;
    }
    H.t[i] = INFINITY;
    H.yarn[i] = -1;
    H.seg[i] = -1;
    H.s[i] = 0.f;
    H.h[i] = 0.f;
    H.u[i] = 0.f;
    H.v[i] = 0.f;
    H.tan_x[i] = H.tan_y[i] = H.tan_z[i] = 0.f;
    H.nrm_x[i] = H.nrm_y[i] = H.nrm_z[i] = 0.f;
    H.flags[i] = flags | HIT_MISS;
}

}  // namespace yarn
