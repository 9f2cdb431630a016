// yarn_build.hpp -- host side of a yarn scene build (see yarn_scene.hip):
// validation, per-span records, rotation-minimising frames and arc lengths,
// the binned-SAH BVH collapsed to four children per node, spans in leaf
// order.  No device call; the library uploads the result.  The per-yarn
// frames and the top levels of the tree are built on host threads; the
// result does not depend on their number.
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <exception>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/bysdf.h"
#include "yarn_tube.hpp"

namespace yarn {

inline int build_fail(std::string* err, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (err) *err = buf;
    return code;
}

// Host threads a build may use (0: the hardware's count, at most 16).
inline std::atomic<int>& build_threads_setting()
{
    static std::atomic<int> n{0};
    return n;
}

// host-side arrays of a scene, as uploaded
struct HostScene {
    std::vector<float4> cp;
    std::vector<SpanRec> span;
    std::vector<float4> frame;
    std::vector<WNode> node;  // the 4-wide tree
    std::vector<float> phase;
    std::vector<int> type;
    int depth = 0;
    int32_t n_yarns = 0;
};

// ------------------------------------------------------------ host build
namespace detail {

struct H3 {
    double x, y, z;
};
H3 operator+(H3 a, H3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
H3 operator-(H3 a, H3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
H3 operator*(H3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
double hdot(H3 a, H3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
H3 hunit(H3 a) { return a * (1.0 / std::sqrt(hdot(a, a))); }

H3 hpos(const H3* p, double s)
{
    double u = 1.0 - s, s2 = s * s, s3 = s2 * s;
    return p[0] * (u * u * u / 6.0) + p[1] * ((3 * s3 - 6 * s2 + 4) / 6.0) +
           p[2] * ((-3 * s3 + 3 * s2 + 3 * s + 1) / 6.0) + p[3] * (s3 / 6.0);
}
H3 hder(const H3* p, double s)
{
    double u = 1.0 - s;
    return p[0] * (-0.5 * u * u) + p[1] * (1.5 * s * s - 2 * s) + p[2] * (-1.5 * s * s + s + 0.5) +
           p[3] * (0.5 * s * s);
}
H3 reflect_step(H3 x0, H3 t0, H3 n0, H3 x1, H3 t1)
{
    H3 v1 = x1 - x0;
    double c1 = hdot(v1, v1);
    if (!(c1 > 1e-16 * (hdot(x0, x0) + hdot(x1, x1)))) {
        v1 = t0;  // the chord's limit for a vanishing step
        c1 = 1.0;
    }
    H3 nl = n0 - v1 * (2 * hdot(v1, n0) / c1);
    H3 tl = t0 - v1 * (2 * hdot(v1, t0) / c1);
    H3 v2 = t1 - tl;
    double c2 = hdot(v2, v2);
    if (c2 > 0) nl = nl - v2 * (2 * hdot(v2, nl) / c2);
    return nl;
}
double span_length(const H3* p)
{
    static const double gx[5] = {0.0, -0.5384693101056831, 0.5384693101056831, -0.9061798459386640,
                                 0.9061798459386640};
    static const double gw[5] = {0.5688888888888889, 0.4786286704993665, 0.4786286704993665,
                                 0.2369268850561891, 0.2369268850561891};
    double acc = 0;
    for (int k = 0; k < 5; ++k) {
        H3 d = hder(p, 0.5 * (1 + gx[k]));
        acc += gw[k] * std::sqrt(hdot(d, d));
    }
    return 0.5 * acc;
}

struct Prim {
    float lo[3], hi[3], c[3];
    int id;
};

struct Builder {
    std::vector<Prim>& prims;
    std::vector<BNode> nodes;
    int max_depth = 0;
    static constexpr int kLeafMax = 4;
    static constexpr int kBins = 16;
    static constexpr int kMedianDepth = 40;

    explicit Builder(std::vector<Prim>& p) : prims(p) {}

    static float area(const float* lo, const float* hi)
    {
        float dx = std::max(0.f, hi[0] - lo[0]), dy = std::max(0.f, hi[1] - lo[1]),
              dz = std::max(0.f, hi[2] - lo[2]);
        return 2.f * (dx * dy + dy * dz + dz * dx);
    }
    void bounds(int b, int e, float* lo, float* hi) const
    {
        for (int k = 0; k < 3; ++k) {
            lo[k] = INFINITY;
            hi[k] = -INFINITY;
        }
        for (int i = b; i < e; ++i)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], prims[i].lo[k]);
                hi[k] = std::max(hi[k], prims[i].hi[k]);
            }
    }
    static int leaf_code(int first, int count) { return -((first << 2) | (count - 1)) - 1; }

    // returns the child code for prims [b, e)
    int build(int b, int e, int depth)
    {
        max_depth = std::max(max_depth, depth);
        int n = e - b;
        if (n <= kLeafMax && depth > 0) return leaf_code(b, n);
        const int mid = split(b, e, depth);
        int self = (int)nodes.size();
        nodes.push_back(BNode{});
        int c0 = build(b, mid, depth + 1);
        int c1 = build(mid, e, depth + 1);
        set_node(self, b, mid, e, c0, c1);
        return self;
    }

    // As build, with the subtree of the upper half of each of the top
    // `levels` splits built by its own builder on another thread, its
    // nodes appended afterwards.  The prims of the two halves are disjoint
    // ranges, and each split sees the same range as in build, so the tree
    // (and its collapse, which renumbers nodes in its own order) is the same.
    int build_par(int b, int e, int depth, int levels)
    {
        if (levels <= 0 || e - b < 8192) return build(b, e, depth);
        max_depth = std::max(max_depth, depth);
        const int mid = split(b, e, depth);
        int self = (int)nodes.size();
        nodes.push_back(BNode{});
        Builder up(prims);
        int c1 = 0;
        std::exception_ptr up_fail, lo_fail;
        auto upper = [&] {
            try {
                c1 = up.build_par(mid, e, depth + 1, levels - 1);
            } catch (...) {
                up_fail = std::current_exception();
            }
        };
        // a thread that cannot be started leaves its half to this one
        std::thread th;
        try {
            th = std::thread(upper);
        } catch (const std::system_error&) {
        }
        int c0 = 0;
        try {
            c0 = build_par(b, mid, depth + 1, levels - 1);
        } catch (...) {
            lo_fail = std::current_exception();
        }
        if (th.joinable())
            th.join();
        else if (!lo_fail)
            upper();
        if (lo_fail) std::rethrow_exception(lo_fail);
        if (up_fail) std::rethrow_exception(up_fail);
        const int base = (int)nodes.size();
        for (BNode nd : up.nodes) {
            if (nd.d.x >= 0) nd.d.x += base;
            if (nd.d.y >= 0) nd.d.y += base;
            nodes.push_back(nd);
        }
        if (c1 >= 0) c1 += base;
        max_depth = std::max(max_depth, up.max_depth);
        set_node(self, b, mid, e, c0, c1);
        return self;
    }

    void set_node(int self, int b, int mid, int e, int c0, int c1)
    {
        float lo0[3], hi0[3], lo1[3], hi1[3];
        bounds(b, mid, lo0, hi0);
        bounds(mid, e, lo1, hi1);
        BNode& nd = nodes[self];
        nd.a = make_float4(lo0[0], lo0[1], lo0[2], hi0[0]);
        nd.b = make_float4(hi0[1], hi0[2], lo1[0], lo1[1]);
        nd.c = make_float4(lo1[2], hi1[0], hi1[1], hi1[2]);
        nd.d = make_int4(c0, c1, 0, 0);
    }

    // the split of prims [b, e) (n > kLeafMax or the root): binned SAH over
    // the three axes, else the object median along the widest centroid
    // axis; the prims are partitioned and the first of the upper part returned
    int split(int b, int e, int depth)
    {
        const int n = e - b;
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = b; i < e; ++i)
            for (int k = 0; k < 3; ++k) {
                clo[k] = std::min(clo[k], prims[i].c[k]);
                chi[k] = std::max(chi[k], prims[i].c[k]);
            }
        int axis = 0;
        for (int k = 1; k < 3; ++k)
            if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
        int mid = -1;
        if (depth < kMedianDepth && chi[axis] > clo[axis] && n > kLeafMax) {
            // binned SAH over the three axes
            float best = INFINITY;
            int bax = -1, bsplit = -1;
            for (int k = 0; k < 3; ++k) {
                if (!(chi[k] > clo[k])) continue;
                int cnt[kBins] = {};
                float blo[kBins][3], bhi[kBins][3];
                for (int j = 0; j < kBins; ++j)
                    for (int q = 0; q < 3; ++q) {
                        blo[j][q] = INFINITY;
                        bhi[j][q] = -INFINITY;
                    }
                float sc = kBins / (chi[k] - clo[k]);
                for (int i = b; i < e; ++i) {
                    int j = std::min(kBins - 1, (int)((prims[i].c[k] - clo[k]) * sc));
                    cnt[j]++;
                    for (int q = 0; q < 3; ++q) {
                        blo[j][q] = std::min(blo[j][q], prims[i].lo[q]);
                        bhi[j][q] = std::max(bhi[j][q], prims[i].hi[q]);
                    }
                }
                float rlo[3] = {INFINITY, INFINITY, INFINITY}, rhi[3] = {-INFINITY, -INFINITY, -INFINITY};
                float rarea[kBins];
                int rcnt[kBins];
                int acc = 0;
                for (int j = kBins - 1; j > 0; --j) {
                    for (int q = 0; q < 3; ++q) {
                        rlo[q] = std::min(rlo[q], blo[j][q]);
                        rhi[q] = std::max(rhi[q], bhi[j][q]);
                    }
                    acc += cnt[j];
                    rcnt[j] = acc;
                    rarea[j] = area(rlo, rhi);
                }
                float llo[3] = {INFINITY, INFINITY, INFINITY}, lhi[3] = {-INFINITY, -INFINITY, -INFINITY};
                int lc = 0;
                for (int j = 0; j < kBins - 1; ++j) {
                    for (int q = 0; q < 3; ++q) {
                        llo[q] = std::min(llo[q], blo[j][q]);
                        lhi[q] = std::max(lhi[q], bhi[j][q]);
                    }
                    lc += cnt[j];
                    if (lc == 0 || rcnt[j + 1] == 0) continue;
                    float cost = area(llo, lhi) * lc + rarea[j + 1] * rcnt[j + 1];
                    if (cost < best) {
                        best = cost;
                        bax = k;
                        bsplit = j;
                    }
                }
            }
            if (bax >= 0) {
                float sc = kBins / (chi[bax] - clo[bax]);
                float cl = clo[bax];
                Prim* m = std::partition(prims.data() + b, prims.data() + e, [&](const Prim& p) {
                    return std::min(kBins - 1, (int)((p.c[bax] - cl) * sc)) <= bsplit;
                });
                mid = (int)(m - prims.data());
                if (mid <= b || mid >= e) mid = -1;
            }
        }
        if (mid < 0) {
            // object median along the widest centroid axis
            mid = b + n / 2;
            std::nth_element(prims.begin() + b, prims.begin() + mid, prims.begin() + e,
                             [axis](const Prim& p, const Prim& q) { return p.c[axis] < q.c[axis]; });
        }
        return mid;
    }
};

// Collapse of the binary tree to four children per node: a node takes its
// binary children and, while it has fewer than four, replaces the internal
// child with the largest box surface by that child's two children.  Leaf
// codes are kept; node codes are renumbered in the wide array (root 0).
struct Collapse {
    const std::vector<BNode>& bin;
    std::vector<WNode> wide;
    int max_depth = 0;
    struct Child {
        float lo[3], hi[3];
        int code;
    };

    explicit Collapse(const std::vector<BNode>& b) : bin(b) {}

    static void children(const BNode& n, Child* c)
    {
        const float v[12] = {n.a.x, n.a.y, n.a.z, n.a.w, n.b.x, n.b.y, n.b.z, n.b.w, n.c.x, n.c.y, n.c.z, n.c.w};
        for (int k = 0; k < 2; ++k) {
            for (int q = 0; q < 3; ++q) {
                c[k].lo[q] = v[6 * k + q];
                c[k].hi[q] = v[6 * k + 3 + q];
            }
        }
        c[0].code = n.d.x;
        c[1].code = n.d.y;
    }
    static float area(const Child& c)
    {
        float dx = std::max(0.f, c.hi[0] - c.lo[0]), dy = std::max(0.f, c.hi[1] - c.lo[1]),
              dz = std::max(0.f, c.hi[2] - c.lo[2]);
        return 2.f * (dx * dy + dy * dz + dz * dx);
    }

    int run(int bcode, int depth)
    {
        max_depth = std::max(max_depth, depth);
        Child ch[4];
        children(bin[bcode], ch);
        int nch = 2;
        while (nch < 4) {
            int pick = -1;
            float best = -1.f;
            for (int k = 0; k < nch; ++k)
                if (ch[k].code >= 0 && area(ch[k]) > best) {
                    best = area(ch[k]);
                    pick = k;
                }
            if (pick < 0) break;
            Child two[2];
            children(bin[ch[pick].code], two);
            ch[pick] = two[0];
            ch[nch++] = two[1];
        }
        const int self = (int)wide.size();
        wide.push_back(WNode{});
        int code[4];
        for (int k = 0; k < nch; ++k) code[k] = ch[k].code >= 0 ? run(ch[k].code, depth + 1) : ch[k].code;
        WNode& w = wide[self];
        float lo[3][4], hi[3][4];
        int cw[4];
        for (int k = 0; k < 4; ++k) {
            // an unused slot, or a slot with an inverted box, is never entered
            bool empty = k >= nch;
            for (int q = 0; q < 3 && !empty; ++q) empty = !(ch[k].lo[q] <= ch[k].hi[q]);
            for (int q = 0; q < 3; ++q) {
                lo[q][k] = empty ? INFINITY : ch[k].lo[q];
                hi[q][k] = empty ? INFINITY : ch[k].hi[q];
            }
            cw[k] = empty ? 0 : code[k];
        }
        w.lox = make_float4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
        w.loy = make_float4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
        w.loz = make_float4(lo[2][0], lo[2][1], lo[2][2], lo[2][3]);
        w.hix = make_float4(hi[0][0], hi[0][1], hi[0][2], hi[0][3]);
        w.hiy = make_float4(hi[1][0], hi[1][1], hi[1][2], hi[1][3]);
        w.hiz = make_float4(hi[2][0], hi[2][1], hi[2][2], hi[2][3]);
        w.code = make_int4(cw[0], cw[1], cw[2], cw[3]);
        w.pad = make_int4(0, 0, 0, 0);
        return self;
    }
};

}  // namespace detail

using namespace detail;

// Host part of the scene build: validation, per-span records, frames and
// arc lengths, the BVH, spans in leaf order.  No device call.
inline int yarn_scene_build_host(const float* ctrl, const int64_t* off, int32_t n_yarns,
                                 const int32_t* yarn_type, const float* yarn_phase, HostScene* hs,
                                 std::string* err)
{
    if (!ctrl || !off || n_yarns < 1) return build_fail(err, BYSDF_ERR_INVALID_ARG, "need ctrl, offsets and n_yarns >= 1");
    if (off[0] != 0) return build_fail(err, BYSDF_ERR_INVALID_ARG, "yarn_offsets[0] must be 0");
    int64_t n_spans = 0;
    for (int y = 0; y < n_yarns; ++y) {
        int64_t m = off[y + 1] - off[y];
        if (m < 4) return build_fail(err, BYSDF_ERR_INVALID_PARAM, "yarn %d has %lld control points (need >= 4)", y, (long long)m);
        n_spans += m - 3;
    }
    int64_t n_cp = off[n_yarns];
    if (n_spans >= (1 << 29)) return build_fail(err, BYSDF_ERR_INVALID_PARAM, "too many spans (%lld)", (long long)n_spans);
    for (int64_t i = 0; i < 4 * n_cp; ++i)
        if (!std::isfinite(ctrl[i])) return build_fail(err, BYSDF_ERR_INVALID_PARAM, "non-finite control point value at %lld", (long long)i);
    for (int y = 0; y < n_yarns; ++y) {
        if (!(ctrl[4 * off[y] + 3] > 0.f)) return build_fail(err, BYSDF_ERR_INVALID_PARAM, "yarn %d has radius <= 0", y);
        if (yarn_type && yarn_type[y] < 0) return build_fail(err, BYSDF_ERR_INVALID_PARAM, "yarn %d has type %d < 0", y, yarn_type[y]);
    }
    // per span: record, frame at the start, box
    std::vector<SpanRec> rec(n_spans);
    std::vector<float4> frame(n_spans);
    std::vector<Prim> prims(n_spans);
    // yarns are independent: each thread takes every nt-th yarn
    std::vector<int64_t> first_span(n_yarns + 1, 0);
    for (int y = 0; y < n_yarns; ++y) first_span[y + 1] = first_span[y] + (off[y + 1] - off[y] - 3);
    const int set = build_threads_setting().load();
    const int nt = set > 0 ? set : (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto yarn_spans = [&](int y) {
        double R = ctrl[4 * off[y] + 3];
        int64_t m = off[y + 1] - off[y];
        H3 n{0, 0, 0};
        double v = 0.0;
        int64_t g = first_span[y];
        for (int64_t j = 0; j + 3 < m; ++j, ++g) {
            int64_t c0 = off[y] + j;
            H3 p[4];
            for (int k = 0; k < 4; ++k)
                p[k] = {ctrl[4 * (c0 + k)], ctrl[4 * (c0 + k) + 1], ctrl[4 * (c0 + k) + 2]};
            if (j == 0) {
                H3 t = hunit(hder(p, 0.0));
                H3 up = std::fabs(t.z) > std::cos(25.0 * 3.14159265358979323846 / 180.0) ? H3{1, 0, 0} : H3{0, 0, 1};
                n = hunit(up - t * hdot(up, t));
            }
            frame[g] = make_float4((float)n.x, (float)n.y, (float)n.z, (float)v);
            double len = span_length(p);
            // samples per span: spacing at most 0.05 R along the curve, so a
            // ray dipping 1e-3 R into a crossing tube meets a sample
            int ns = (int)std::ceil(len / (0.05 * R));
            ns = std::max(4, std::min(64, ns));
            int info = ns | (j == 0 ? 1 << 16 : 0) | (j + 4 == m ? 1 << 17 : 0);
            rec[g] = SpanRec{(int)c0, y, (int)j, info};
            // transport the frame to the next span start
            const int steps = 16;
            H3 x = hpos(p, 0.0), t = hunit(hder(p, 0.0));
            for (int k = 1; k <= steps; ++k) {
                double s = (double)k / steps;
                H3 x1 = hpos(p, s), t1 = hunit(hder(p, s));
                n = reflect_step(x, t, n, x1, t1);
                x = x1;
                t = t1;
            }
            n = hunit(n - t * hdot(n, t));
            v += len;
            Prim& pr = prims[g];
            for (int q = 0; q < 3; ++q) {
                pr.lo[q] = INFINITY;
                pr.hi[q] = -INFINITY;
            }
            for (int k = 0; k < 4; ++k) {
                double c[3] = {p[k].x, p[k].y, p[k].z};
                for (int q = 0; q < 3; ++q) {
                    pr.lo[q] = std::min(pr.lo[q], std::nextafter((float)(c[q] - R), -INFINITY));
                    pr.hi[q] = std::max(pr.hi[q], std::nextafter((float)(c[q] + R), INFINITY));
                }
            }
            for (int q = 0; q < 3; ++q) pr.c[q] = 0.5f * (pr.lo[q] + pr.hi[q]);
            pr.id = (int)g;
        }
    };
    {
        // (the per-yarn work allocates nothing and cannot throw; a worker
        // that cannot be started leaves its yarns to this thread)
        std::vector<std::thread> pool;
        int started = 1;
        try {
            pool.reserve(nt);
            for (; started < nt; ++started)
                pool.emplace_back([&, w = started] {
                    for (int y = w; y < n_yarns; y += nt) yarn_spans(y);
                });
        } catch (const std::exception&) {
        }
        for (int w = 0; w < nt; ++w)
            if (w == 0 || w >= started)
                for (int y = w; y < n_yarns; y += nt) yarn_spans(y);
        for (std::thread& th : pool) th.join();
    }
    Builder B(prims);
    B.nodes.reserve(n_spans);
    if (n_spans == 1) {
        // a root with the single leaf and an empty box
        BNode nd;
        nd.a = make_float4(prims[0].lo[0], prims[0].lo[1], prims[0].lo[2], prims[0].hi[0]);
        nd.b = make_float4(prims[0].hi[1], prims[0].hi[2], INFINITY, INFINITY);
        nd.c = make_float4(INFINITY, -INFINITY, -INFINITY, -INFINITY);
        nd.d = make_int4(Builder::leaf_code(0, 1), Builder::leaf_code(0, 1), 0, 0);
        B.nodes.push_back(nd);
        B.max_depth = 1;
    } else {
        int levels = 0;
        while ((1 << levels) < nt) ++levels;
        B.build_par(0, (int)n_spans, 0, levels);
    }
    if (B.max_depth > kStack)
        return build_fail(err, BYSDF_ERR_INVALID_PARAM, "BVH depth %d exceeds %d", B.max_depth, kStack);
    // spans in leaf order
    std::vector<SpanRec>& rec_o = hs->span;
    std::vector<float4>& frame_o = hs->frame;
    rec_o.resize(n_spans);
    frame_o.resize(n_spans);
    for (int64_t i = 0; i < n_spans; ++i) {
        rec_o[i] = rec[prims[i].id];
        frame_o[i] = frame[prims[i].id];
    }
    std::vector<float4>& cp = hs->cp;
    cp.resize(n_cp);
    for (int64_t i = 0; i < n_cp; ++i) {
        // the radius of every point is its yarn's (the first point's r)
        cp[i] = make_float4(ctrl[4 * i], ctrl[4 * i + 1], ctrl[4 * i + 2], 0.f);
    }
    for (int y = 0; y < n_yarns; ++y)
        for (int64_t i = off[y]; i < off[y + 1]; ++i) cp[i].w = ctrl[4 * off[y] + 3];
    std::vector<float>& phase = hs->phase;
    std::vector<int>& type = hs->type;
    phase.assign(n_yarns, 0.f);
    type.assign(n_yarns, 0);
    for (int y = 0; y < n_yarns; ++y) {
        if (yarn_phase) phase[y] = yarn_phase[y];
        if (yarn_type) type[y] = yarn_type[y];
    }

    Collapse W(B.nodes);
    W.wide.reserve(B.nodes.size() / 2 + 1);
    W.run(0, 0);
    if (W.max_depth > kWideDepthMax)
        return build_fail(err, BYSDF_ERR_INVALID_PARAM, "4-wide BVH depth %d exceeds %d", W.max_depth,
                          kWideDepthMax);
    hs->node = std::move(W.wide);
    hs->depth = W.max_depth;
    hs->n_yarns = n_yarns;
    return 0;
}

}  // namespace yarn
