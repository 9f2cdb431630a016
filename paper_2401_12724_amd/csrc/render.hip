// render.hip -- wavefront path tracer of BYSDF-shaded yarn scenes
// (shade_wavefront, see include/bysdf.h).
//
// One wavefront pass renders spp_batch samples of every pixel of the crop;
// each path owns a radiance slot for the whole pass.  Per bounce:
//   k_r_extend  one ray per lane (LDS traversal stack): yarn BVH, the light
//               rectangle, the environment; light / environment hits add
//               their radiance to the path's slot and end it
//   k_r_shade   BYSDF at the hit (wave-uniform type): one state at x and one
//               set of forward nodes serve the next-event evaluation and
//               the sample; far field by the LOD rule, or the
//               multi-scale model over the pixel footprint of a camera
//               hit; appends a shadow ray and the continued path
//               (wave-aggregated atomics: compaction)
//   k_r_shadow  shadow rays; a yarn whose implicit plies are missed is
//               passed through; an unblocked ray adds its contribution
// then k_r_accum averages the slots of each pixel in a fixed order.  A
// slot is written by at most one kernel per bounce, so the image does not
// depend on the queue order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "../../include/bysdf.h"
#include "bysdf_model.hpp"
#include "bysdf_multi.hpp"
#include "lib_internal.hpp"
#include "philox.hpp"
#include "yarn_tube.hpp"

using bysdf::Derived;
using bysdf::EvalOut;
using bysdf::NodesComputed;
using bysdf::PlyHit;
using bysdf::SampleOut;
using bysdf::TypeRec;
using bysdf::V3;
using bysdf::XState;
using yarn::D3;
using yarn::SceneView;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return bysdf_set_error(code, buf);
}

namespace {

constexpr int kTraceBlock = 128;
constexpr int kShadeBlock = 256;
constexpr int kMaxPassThrough = 16;
constexpr uint32_t kSampleFail = 1u << 6;

struct RView {
    SceneView S;
    const TypeRec* types;
    const float4* tables;
    double eye[3], f[3], r[3], u[3];
    double th, aspect, pix_angle;
    double lc[3], leu[3], lev[3], ln[3];
    double area, eu2, ev2;
    float Le[3], env[3];
    int W, H, cx, cy, cw, ch, spp, max_depth, n_h;
    int multiscale;
    int grad_type;  // -1: no image gradient
    float lod_px;
    double eps;
    uint32_t key0, key1;
};

// Gradient mode: per path, D[(3c + p) cap + i] is d ln(throughput_c) / d
// theta_p for theta = (r, k^B_c, sigma_t) of the gradient type; per shadow
// ray, G[(3c + p) cap + i] is d(contribution_c) / d theta_p.  NULL otherwise.
constexpr int kGrad = 9;

struct PathQ {
    float *ox, *oy, *oz, *dx, *dy, *dz, *tr, *tg, *tb, *pdf, *line0;
    int *skip, *lid;
    float* D;
};
struct HitQ {
    float *t, *s, *h, *v, *R, *Tx, *Ty, *Tz, *Nx, *Ny, *Nz;
    int *yarn, *seg;
};
struct ShadowQ {
    float *ox, *oy, *oz, *dx, *dy, *dz, *tmax, *cr, *cg, *cb;
    int *skip, *lid;
    float* G;
};

__device__ inline D3 dv(const double* a) { return yarn::d3(a[0], a[1], a[2]); }

__device__ inline void rnd(const RView& V, uint64_t slot, uint32_t depth, uint32_t stream, float u[4])
{
    uint32_t o[4];
    rng::philox4x32_10((uint32_t)slot, (uint32_t)(slot >> 32), depth, stream, V.key0, V.key1, o);
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = rng::u01(o[k]);
}

// index of this lane's item in a queue, one atomic per wavefront
__device__ inline int wave_append(bool want, int* counter)
{
    unsigned long long m = __ballot(want);
    if (!m) return -1;
    int lane = __lane_id();
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    return want ? base + __popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// local BYSDF direction (x = N, y = T x N, z = T), single precision
__device__ inline V3<float> to_loc(D3 T, D3 N, D3 w)
{
    D3 B = yarn::cross(T, N);
    return bysdf::mk3<float>((float)yarn::dot(w, N), (float)yarn::dot(w, B), (float)yarn::dot(w, T));
}

// ------------------------------------------------------------ kernels

__global__ __launch_bounds__(256) void k_r_fill(float* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_r_counters(int* cnt, int a, int b, int c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (a >= 0) cnt[a] = 0;
        if (b >= 0) cnt[b] = 0;
        if (c >= 0) cnt[c] = 0;
    }
}

__global__ void k_r_tally(const int* cnt, int idx, unsigned long long* stats, int which)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) stats[which] += (unsigned long long)cnt[idx];
}

__global__ __launch_bounds__(256) void k_r_camera(RView V, PathQ A, float* L, int cap, int spp_batch, int j0,
                                                  int* cnt)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[0] = cap;
    for (int lid = blockIdx.x * blockDim.x + threadIdx.x; lid < cap; lid += gridDim.x * blockDim.x) {
        int pix = lid / spp_batch, j = j0 + lid % spp_batch;
        uint64_t slot = (uint64_t)pix * V.spp + j;
        int px = V.cx + pix % V.cw, py = V.cy + pix / V.cw;
        float u0[4];
        rnd(V, slot, 0, 0, u0);
        double sx = (2.0 * (px + (double)u0[0]) / V.W - 1.0) * V.th * V.aspect;
        double sy = (1.0 - 2.0 * (py + (double)u0[1]) / V.H) * V.th;
        D3 d = yarn::unit(dv(V.f) + dv(V.r) * sx + dv(V.u) * sy);
        A.ox[lid] = (float)V.eye[0];
        A.oy[lid] = (float)V.eye[1];
        A.oz[lid] = (float)V.eye[2];
        A.dx[lid] = (float)d.x;
        A.dy[lid] = (float)d.y;
        A.dz[lid] = (float)d.z;
        A.tr[lid] = A.tg[lid] = A.tb[lid] = 1.0f;
        A.pdf[lid] = -1.0f;
        A.line0[lid] = 0.0f;
        A.skip[lid] = -1;
        A.lid[lid] = lid;
        L[lid] = L[cap + lid] = L[2 * cap + lid] = 0.0f;
        if (A.D)
            for (int k = 0; k < kGrad; ++k) {
                A.D[k * cap + lid] = 0.0f;
                L[(3 + k) * cap + lid] = 0.0f;
            }
    }
}

#ifndef RENDER_TRACE_MIN_WAVES
#define RENDER_TRACE_MIN_WAVES 3
#endif
__global__ __launch_bounds__(kTraceBlock, RENDER_TRACE_MIN_WAVES) void k_r_extend(RView V, PathQ Q,
                                                                                  const int* cnt_in, HitQ H,
                                                                                  float* L, int cap, int depth)
{
    extern __shared__ int stk[];  // yarn::stack_entries(BVH depth) x kTraceBlock
    int* my = stk + threadIdx.x;
    const int n = *cnt_in;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        D3 o = yarn::d3(Q.ox[i], Q.oy[i], Q.oz[i]);
        D3 d = yarn::unit(yarn::d3(Q.dx[i], Q.dy[i], Q.dz[i]));
        const double tmin = depth == 0 ? 0.0 : V.eps;
        const int lid = Q.lid[i], skip = Q.skip[i];
        int ex[yarn::kMaxExcluded + 1];
        int nex = yarn::excluded_yarns(V.S, o, my, kTraceBlock, ex, skip);
        yarn::RayHit hit = yarn::closest_hit(V.S, o, d, tmin, 1e30, ex, nex, my, kTraceBlock);
        // the light: one-sided rectangle
        D3 ln = dv(V.ln);
        double den = yarn::dot(d, ln), tl = INFINITY;
        if (den < 0.0) {
            double t = yarn::dot(dv(V.lc) - o, ln) / den;
            if (t > tmin) {
                D3 q = o + d * t - dv(V.lc);
                double a = yarn::dot(q, dv(V.leu)) / V.eu2, b = yarn::dot(q, dv(V.lev)) / V.ev2;
                if (a >= 0.0 && a <= 1.0 && b >= 0.0 && b <= 1.0) tl = t;
            }
        }
        const bool miss = hit.span < 0;
        float thr[3] = {Q.tr[i], Q.tg[i], Q.tb[i]};
        if (tl < INFINITY && (miss || tl < hit.t)) {
            double w = 1.0;
            float pdf = Q.pdf[i];
            if (pdf > 0.0f) {
                double dl = (double)Q.line0[i] + tl;
                double pl = dl * dl / (V.area * fabs(den));
                w = (double)pdf * pdf / ((double)pdf * pdf + pl * pl);
            }
            float wf = (float)w;
            for (int c = 0; c < 3; ++c) L[c * cap + lid] += thr[c] * V.Le[c] * wf;
            if (Q.D)
                for (int k = 0; k < kGrad; ++k) L[(3 + k) * cap + lid] += thr[k / 3] * V.Le[k / 3] * wf * Q.D[k * cap + i];
            H.yarn[i] = -1;
            continue;
        }
        if (miss) {
            for (int c = 0; c < 3; ++c) L[c * cap + lid] += thr[c] * V.env[c];
            if (Q.D)
                for (int k = 0; k < kGrad; ++k) L[(3 + k) * cap + lid] += thr[k / 3] * V.env[k / 3] * Q.D[k * cap + i];
            H.yarn[i] = -1;
            continue;
        }
        if (depth == V.max_depth) {
            H.yarn[i] = -1;
            continue;
        }
        yarn::SpanRec r = V.S.span[hit.span];
        yarn::HitFrame fr = yarn::hit_frame(V.S, hit.span, hit.s);
        D3 p = o + d * hit.t;
        D3 q = p - fr.c;
        double qn = yarn::dot(q, fr.N), qb = yarn::dot(q, fr.B);
        double wn = -yarn::dot(d, fr.N), wb = -yarn::dot(d, fr.B);
        double ql = sqrt(qn * qn + qb * qb), wl = sqrt(wn * wn + wb * wb);
        double h = (ql > 0.0 && wl > 0.0) ? (qb * wn - qn * wb) / (ql * wl) : 0.0;
        h = fmin(1.0, fmax(-1.0, h));
        H.t[i] = (float)hit.t;
        H.s[i] = (float)hit.s;
        H.h[i] = (float)h;
        H.v[i] = (float)fr.v;
        H.R[i] = V.S.cp[r.cp0].w;
        H.Tx[i] = (float)fr.T.x;
        H.Ty[i] = (float)fr.T.y;
        H.Tz[i] = (float)fr.T.z;
        H.Nx[i] = (float)fr.N.x;
        H.Ny[i] = (float)fr.N.y;
        H.Nz[i] = (float)fr.N.z;
        H.yarn[i] = r.yarn;
        H.seg[i] = r.seg;
    }
}


// far field (Eq. 7, W = 1): mean value and mean pdf over n_h strata of h
template <int MP>
__device__ inline void far_eval(const Derived<double, float>& P, const TabPtr& tab, float u, float v,
                                const V3<float>& wi, const V3<float>& wo, int n_h, float zeta, double E[3],
                                double* pdf, const double* disk)
{
    E[0] = E[1] = E[2] = 0.0;
    *pdf = 0.0;
    V3<double> wo_g = bysdf::mk3<double>(wo.x, wo.y, wo.z);
    for (int j = 0; j < n_h; ++j) {
        float hj = (float)(-1.0 + 2.0 * (j + (double)zeta) / n_h);
        XState<double, float, MP> X;
        bysdf::state_at_x(P, tab, hj, u, v, wi, X);
        if (X.ph.pass) continue;
        EvalOut<float> e;
        bysdf::lobes(P, tab, X, wo_g, 0.0f, 0.0f, false, e, disk);
        for (int c = 0; c < 3; ++c) E[c] += e.E[c];
        *pdf += e.pdf;
    }
    for (int c = 0; c < 3; ++c) E[c] /= n_h;
    *pdf /= n_h;
}

// Custom ray differentials (Sec. 5.3): the azimuthal offsets covered by the
// pixel of a camera hit.  The yarn is taken as the straight tube of radius R
// along T through the hit's axis point c (the hit lies at azimuth
// psi = atan2(wi) + asin h from c in the (N, T x N) plane), and a ray's
// offset is its signed distance from that axis over R, the h of the
// intersection.  The offsets of the rays one pixel to the right and one
// pixel up give the screen-space gradient of h; the rays one pixel along and
// against that gradient give the two ends, cut at +-1; h0 lies between.
__device__ inline void camera_footprint(const RView& V, D3 o, D3 d, double t, D3 T, D3 N, double R,
                                        float h0, float* h1, float* h2)
{
    const D3 B = yarn::cross(T, N);
    const D3 p = o + d * t;
    const double psi = atan2(-yarn::dot(d, B), -yarn::dot(d, N)) + asin((double)h0);
    const D3 c = p - (N * cos(psi) + B * sin(psi)) * R;
    const D3 e = o - c;
    const double ex = yarn::dot(e, N), ey = yarn::dot(e, B);
    const D3 f = dv(V.f), r = dv(V.r), u = dv(V.u);
    const double df = yarn::dot(d, f);
    const double sx = yarn::dot(d, r) / df, sy = yarn::dot(d, u) / df;
    const double px = 2.0 * V.th * V.aspect / V.W, py = 2.0 * V.th / V.H;
    auto offset = [&](double a, double b) {
        const D3 dd = yarn::unit(f + r * (sx + a * px) + u * (sy + b * py));
        const double dx = yarn::dot(dd, N), dy = yarn::dot(dd, B);
        const double l = sqrt(dx * dx + dy * dy);
        return l > 1e-12 ? (ex * dy - ey * dx) / (l * R) : (double)h0;
    };
    const double gx = offset(1.0, 0.0) - h0, gy = offset(0.0, 1.0) - h0;
    const double gl = sqrt(gx * gx + gy * gy);
    double lo = h0, hi = h0;
    if (gl > 0.0) {
        const double hp = offset(gx / gl, gy / gl), hm = offset(-gx / gl, -gy / gl);
        lo = fmin(lo, fmax(-1.0, fmin(hp, hm)));
        hi = fmax(hi, fmin(1.0, fmax(hp, hm)));
    }
    *h1 = (float)lo;
    *h2 = (float)hi;
}

// dE_c / d theta for theta = (r, k^B_c, sigma_t): the reflected body lobe
// is linear in r and the transmitted one in 1 - r, both in k^B_c, and only
// the forward specular lobe sees sigma_t (ds = dEyS / dsigma_t).
__device__ inline void bysdf_grad(const Derived<double, float>& P, const EvalOut<float>& e, float ds, float dE[kGrad])
{
    for (int c = 0; c < 3; ++c) {
        dE[3 * c] = (P.r > 0.0f ? e.ExB[c] / P.r : 0.0f) - (P.r < 1.0f ? e.EyB[c] / (1.0f - P.r) : 0.0f);
        dE[3 * c + 1] = P.alb[c] > 0.0f ? (e.ExB[c] + e.EyB[c]) / P.alb[c] : 0.0f;
        dE[3 * c + 2] = ds;
    }
}

template <int MP, bool MS, bool GRAD>
#ifndef RENDER_SHADE_MIN_WAVES
#define RENDER_SHADE_MIN_WAVES 1
#endif
__global__ __launch_bounds__(kShadeBlock, RENDER_SHADE_MIN_WAVES) void k_r_shade(RView V, PathQ Q, const int* cnt_in, HitQ H, PathQ O,
                                                            int* cnt_out, ShadowQ SQ, int* cnt_sh, int cap,
                                                            int depth, int j0, int spp_batch)
{
    bysdf::stage_math_tables();
    __syncthreads();
    const int n = *cnt_in;
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int i = base + threadIdx.x;
        const bool act = i < n && H.yarn[i] >= 0;
        int yarn_id = act ? H.yarn[i] : 0;
        int type = act ? V.S.yarn_type[yarn_id] : 0;
        // the path and its hit are read again after the BYSDF (below), so
        // that only the BYSDF's inputs and outputs stay live through it
        auto path_at = [&](D3& o, D3& d, D3& T, D3& N, float& t, float& R) {
            o = yarn::d3(0, 0, 0), d = yarn::d3(0, 0, 1), T = yarn::d3(0, 0, 1), N = yarn::d3(1, 0, 0);
            t = 0.f;
            R = 0.f;
            if (act) {
                o = yarn::d3(Q.ox[i], Q.oy[i], Q.oz[i]);
                d = yarn::unit(yarn::d3(Q.dx[i], Q.dy[i], Q.dz[i]));
                t = H.t[i];
                R = H.R[i];
                T = yarn::d3(H.Tx[i], H.Ty[i], H.Tz[i]);
                N = yarn::d3(H.Nx[i], H.Ny[i], H.Nz[i]);
            }
        };
        // next-event estimation: a uniform point of the light
        auto light_at = [&](D3 p, const float* u1, D3& wl, double& dist2, double& cosl) {
            D3 yl = dv(V.lc) + dv(V.leu) * (double)u1[0] + dv(V.lev) * (double)u1[1];
            D3 lv = yl - p;
            dist2 = yarn::dot(lv, lv);
            wl = lv * (1.0 / sqrt(dist2));
            cosl = -yarn::dot(wl, dv(V.ln));
        };
        const int lid = act ? Q.lid[i] : 0;
        const uint64_t slot = (uint64_t)(lid / spp_batch) * V.spp + j0 + lid % spp_batch;
        float u1[4] = {0, 0, 0, 0}, u2[4] = {0, 0, 0, 0};
        if (act) {
            rnd(V, slot, (uint32_t)depth, 1, u1);
            rnd(V, slot, (uint32_t)depth, 2, u2);
        }
        // multi-scale: the camera hits use their pixel footprint, later
        // bounces the near field; otherwise the far field by the LOD rule
        const bool msx = MS && depth == 0;
        bool far;
        float hq = 0.f, uq = 0.f, vl = 0.f, fh1, fh2;
        V3<float> wi, wol;
        bool lit;
        {
            D3 o, d, T, N;
            float t, R;
            path_at(o, d, T, N, t, R);
            if (act) {
                hq = H.h[i];
                vl = (float)((double)H.v[i] / (double)R);
                uq = V.S.yarn_phase[yarn_id];
            }
            const D3 p = o + d * (double)t;
            wi = to_loc(T, N, d * -1.0);
            const D3 pe = p - dv(V.eye);
            far = !MS && !GRAD && 2.0 * R / (sqrt(yarn::dot(pe, pe)) * V.pix_angle) < V.lod_px;
            fh1 = hq;
            fh2 = hq;
            if (msx && act) camera_footprint(V, o, d, (double)t, T, N, (double)R, hq, &fh1, &fh2);
            D3 wl;
            double dist2, cosl;
            light_at(p, u1, wl, dist2, cosl);
            wol = to_loc(T, N, wl);
            lit = cosl > 0.0;
        }
        // gradient mode: path log-derivatives in, BYSDF derivatives at the
        // light direction and at the drawn one
        // (Dp: into this hit; Dn: out of it along the drawn direction)
        float Dp[GRAD ? kGrad : 1], Dn[GRAD ? kGrad : 1], dEn[GRAD ? kGrad : 1], dEs[GRAD ? kGrad : 1];
        float Es[3] = {0.f, 0.f, 0.f};
        if (GRAD)
            for (int k = 0; k < kGrad; ++k) {
                Dp[k] = Dn[k] = act ? Q.D[k * cap + i] : 0.0f;
                dEn[k] = dEs[k] = 0.0f;
            }
        double En[3] = {0, 0, 0}, pb = 0.0;
        // the BYSDF's continuation: 0 none, 1 straight through the yarn,
        // 2 a drawn direction wo with weight wgt and density pdf_s
        int mode = 0;
        float wo_s[3] = {0.f, 0.f, 0.f}, wgt[3] = {1.f, 1.f, 1.f};
        double pdf_s = 0.0;
        for_each_wave_type(type, act, [&](int tu) {
            const Derived<double, float>& P = V.types[tu].d;
            TabPtr tab{V.tables + V.types[tu].table_off};
            SampleOut<float> so;
            uint32_t sf = 0;
            if (GRAD) {
                XState<double, float, MP> X;
                bysdf::state_at_x(P, tab, hq, uq, vl, wi, X);
                NodesComputed<double, float, MP, TabPtr> nf{P, tab, X, 0.0f, 0.0f, false,
                                                            V.types[tu].node_disk};
                V3<double> ws;
                bool ok;
                sf = bysdf::sample_draw(P, X, wi, u1[2], u1[3], u2[0], nf, so, ws, ok);
                if (!X.ph.pass) {
                    EvalOut<float> en, es;
                    float dsn = 0.0f, dss = 0.0f;
                    bysdf::lobes_nodes2_dsigma(P, X, bysdf::mk3<double>(wol.x, wol.y, wol.z), lit, ws, ok,
                                               nf, en, es, dsn, dss);
                    const bool mine = tu == V.grad_type;
                    if (lit) {
                        for (int c = 0; c < 3; ++c) En[c] = en.E[c];
                        pb = en.pdf;
                        if (mine) bysdf_grad(P, en, dsn, dEn);
                    }
                    if (ok) {
                        sf = bysdf::sample_finish(es, ws, sf, so);
                        for (int c = 0; c < 3; ++c) Es[c] = es.E[c];
                        if (mine) bysdf_grad(P, es, dss, dEs);
                    }
                }
            } else if (msx) {
                const TypeRec& Rt = V.types[tu];
                bysdf::Footprint fp;
                bysdf::make_footprint(hq, fh1, fh2, u2[2], V.n_h, fp);
                const Derived<double, float> Pm = bysdf::widened(P, Rt.beta, Rt.aniso, fp);
                if (lit) {
                    EvalOut<float> e;
                    bysdf::eval_multi<double, float, MP>(Pm, tab, fp, uq, vl, wi, wol, 0.0f, 0.0f, false, e);
                    for (int c = 0; c < 3; ++c) En[c] = e.E[c];
                    pb = e.pdf;
                }
                sf = bysdf::sample_multi<double, float, MP>(Pm, tab, fp, u2[1], uq, vl, wi, u1[2], u1[3],
                                                            u2[0], 0.0f, 0.0f, false, so);
            } else if (!far) {
                // the light direction and the drawn one share the state at x
                // and the forward nodes
                XState<double, float, MP> X;
                bysdf::state_at_x(P, tab, hq, uq, vl, wi, X);
                NodesComputed<double, float, MP, TabPtr> nf{P, tab, X, 0.0f, 0.0f, false,
                                                            V.types[tu].node_disk};
                EvalOut<float> e;
                for (int c = 0; c < 3; ++c) e.E[c] = 0.0f;
                e.pdf = 0.0f;
                sf = bysdf::eval_sample_from_x(P, X, wi, bysdf::mk3<double>(wol.x, wol.y, wol.z), lit, u1[2],
                                               u1[3], u2[0], nf, e, so);
                if (!X.ph.pass && lit) {
                    for (int c = 0; c < 3; ++c) En[c] = e.E[c];
                    pb = e.pdf;
                }
            } else {
                if (lit) far_eval<MP>(P, tab, uq, vl, wi, wol, V.n_h, u2[2], En, &pb, V.types[tu].node_disk);
                int js = (int)floorf(u2[1] * V.n_h);
                js = js > V.n_h - 1 ? V.n_h - 1 : js;
                float hs = (float)(-1.0 + 2.0 * (js + (double)u2[2]) / V.n_h);
                XState<double, float, MP> X;
                bysdf::state_at_x(P, tab, hs, uq, vl, wi, X);
                NodesComputed<double, float, MP, TabPtr> nf{P, tab, X, 0.0f, 0.0f, false,
                                                            V.types[tu].node_disk};
                sf = bysdf::sample_from_x(P, X, wi, u1[2], u1[3], u2[0], nf, so);
            }
            if (depth == V.max_depth) return;
            if (so.lobe == 4) {
                mode = 1;
            } else if (so.lobe >= 0 && !(sf & kSampleFail) && so.pdf > 0.0f) {
                V3<float> wo = bysdf::mk3<float>(so.wo[0], so.wo[1], so.wo[2]);
                double pdf = so.pdf;
                bool ok = true;
                if (far) {
                    double E[3];
                    far_eval<MP>(P, tab, uq, vl, wi, wo, V.n_h, u2[2], E, &pdf, V.types[tu].node_disk);
                    ok = pdf > 0.0;
                    for (int c = 0; c < 3; ++c) wgt[c] = ok ? (float)(E[c] / pdf) : 0.0f;
                } else {
                    for (int c = 0; c < 3; ++c) wgt[c] = so.wgt[c];
                }
                if (ok) {
                    mode = 2;
                    wo_s[0] = wo.x;
                    wo_s[1] = wo.y;
                    wo_s[2] = wo.z;
                    pdf_s = pdf;
                }
            }
        });
        D3 o, d, T, N;
        float t, R;
        path_at(o, d, T, N, t, R);
        const D3 p = o + d * (double)t;
        float thr[3] = {0.f, 0.f, 0.f}, line0 = 0.f;
        if (act) {
            thr[0] = Q.tr[i];
            thr[1] = Q.tg[i];
            thr[2] = Q.tb[i];
            line0 = Q.line0[i];
        }
        // the continued path
        bool cont = false;
        D3 dnew = d;
        float pdf_new = act ? Q.pdf[i] : -1.0f;
        float line_new = line0;
        if (mode == 1) {
            // straight through the yarn: the last scattering event stays in force
            cont = true;
            line_new = line0 + t;
        } else if (mode == 2) {
            D3 B = yarn::cross(T, N);
            dnew = yarn::unit(N * (double)wo_s[0] + B * (double)wo_s[1] + T * (double)wo_s[2]);
            pdf_new = (float)pdf_s;
            line_new = 0.0f;
            float nt[3];
            for (int c = 0; c < 3; ++c) nt[c] = thr[c] * wgt[c];
            if (GRAD)
                for (int k = 0; k < kGrad; ++k)
                    if (Es[k / 3] > 0.0f) Dn[k] = Dp[k] + dEs[k] / Es[k / 3];
            cont = nt[0] > 0.f || nt[1] > 0.f || nt[2] > 0.f;
            for (int c = 0; c < 3; ++c) thr[c] = nt[c];
        }
        // shadow ray
        D3 wl;
        double dist2, cosl;
        light_at(p, u1, wl, dist2, cosl);
        bool want_sh = act && cosl > 0.0 && (En[0] > 0.0 || En[1] > 0.0 || En[2] > 0.0);
        float ct[3] = {0, 0, 0};
        if (want_sh) {
            double pl = dist2 / (V.area * cosl);
            double w = pl * pl / (pl * pl + pb * pb);
            float fac = (float)(w / pl);
            float th0[3] = {act ? Q.tr[i] : 0.f, act ? Q.tg[i] : 0.f, act ? Q.tb[i] : 0.f};
            for (int c = 0; c < 3; ++c) ct[c] = th0[c] * (float)En[c] * V.Le[c] * fac;
            if (GRAD)
                for (int k = 0; k < kGrad; ++k) {
                    const int c = k / 3;
                    dEn[k] = th0[c] * V.Le[c] * fac * (dEn[k] + (float)En[c] * Dp[k]);
                }
        }
        int js = wave_append(want_sh, cnt_sh);
        if (want_sh) {
            D3 ds = yarn::unit(yarn::d3((float)wl.x, (float)wl.y, (float)wl.z));
            SQ.ox[js] = (float)p.x;
            SQ.oy[js] = (float)p.y;
            SQ.oz[js] = (float)p.z;
            SQ.dx[js] = (float)ds.x;
            SQ.dy[js] = (float)ds.y;
            SQ.dz[js] = (float)ds.z;
            SQ.tmax[js] = (float)(sqrt(dist2) * (1.0 - 1e-5));
            SQ.cr[js] = ct[0];
            SQ.cg[js] = ct[1];
            SQ.cb[js] = ct[2];
            SQ.skip[js] = yarn_id;
            SQ.lid[js] = lid;
            if (GRAD)
                for (int k = 0; k < kGrad; ++k) SQ.G[k * cap + js] = dEn[k];
        }
        // continued path: from the hit point, past its own yarn
        bool want = act && cont;
        int jo = wave_append(want, cnt_out);
        if (want) {
            O.ox[jo] = (float)p.x;
            O.oy[jo] = (float)p.y;
            O.oz[jo] = (float)p.z;
            O.dx[jo] = (float)dnew.x;
            O.dy[jo] = (float)dnew.y;
            O.dz[jo] = (float)dnew.z;
            O.tr[jo] = thr[0];
            O.tg[jo] = thr[1];
            O.tb[jo] = thr[2];
            O.pdf[jo] = pdf_new;
            O.line0[jo] = line_new;
            O.skip[jo] = yarn_id;
            O.lid[jo] = lid;
            if (GRAD)
                for (int k = 0; k < kGrad; ++k) O.D[k * cap + jo] = Dn[k];
        }
        (void)cap;
    }
}

template <int MP>
__global__ __launch_bounds__(kTraceBlock, RENDER_TRACE_MIN_WAVES) void k_r_shadow(RView V, ShadowQ SQ,
                                                                                  const int* cnt, float* L,
                                                                                  int cap)
{
    bysdf::stage_math_tables();
    __syncthreads();
    extern __shared__ int stk[];  // yarn::stack_entries(BVH depth) x kTraceBlock
    int* my = stk + threadIdx.x;
    const int n = *cnt;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        D3 o = yarn::d3(SQ.ox[i], SQ.oy[i], SQ.oz[i]);
        D3 d = yarn::unit(yarn::d3(SQ.dx[i], SQ.dy[i], SQ.dz[i]));
        double tmax = SQ.tmax[i];
        int skip = SQ.skip[i];
        bool visible = false;
        for (int k = 0; k < kMaxPassThrough; ++k) {
            int ex[yarn::kMaxExcluded + 1];
            int nex = yarn::excluded_yarns(V.S, o, my, kTraceBlock, ex, skip);
            yarn::RayHit hit = yarn::closest_hit(V.S, o, d, V.eps, tmax, ex, nex, my, kTraceBlock);
            if (hit.span < 0) {
                visible = true;
                break;
            }
            yarn::SpanRec r = V.S.span[hit.span];
            yarn::HitFrame fr = yarn::hit_frame(V.S, hit.span, hit.s);
            float th = (float)hit.t;
            D3 p = o + d * (double)th;
            D3 q = o + d * hit.t - fr.c;
            double qn = yarn::dot(q, fr.N), qb = yarn::dot(q, fr.B);
            double wn = -yarn::dot(d, fr.N), wb = -yarn::dot(d, fr.B);
            double ql = sqrt(qn * qn + qb * qb), wlen = sqrt(wn * wn + wb * wb);
            double hh = (ql > 0.0 && wlen > 0.0) ? (qb * wn - qn * wb) / (ql * wlen) : 0.0;
            float h = (float)fmin(1.0, fmax(-1.0, hh));
            float R = V.S.cp[r.cp0].w;
            D3 Tf = yarn::d3((float)fr.T.x, (float)fr.T.y, (float)fr.T.z);
            D3 Nf = yarn::d3((float)fr.N.x, (float)fr.N.y, (float)fr.N.z);
            V3<float> wi = to_loc(Tf, Nf, d * -1.0);
            float vl = (float)((double)(float)fr.v / (double)R);
            const Derived<double, float>& P = V.types[V.S.yarn_type[r.yarn]].d;
            PlyHit<double, MP> ph;
            bysdf::trace_plies(P, h, V.S.yarn_phase[r.yarn], vl, wi, ph);
            if (!ph.pass) break;
            double sxy = sqrt((double)wi.x * wi.x + (double)wi.y * wi.y);
            double ch = 2.0 * R * sqrt(fmax(0.0, 1.0 - (double)h * h)) / fmax(sxy, 1e-12);
            D3 on = p + d * ch;
            o = yarn::d3((float)on.x, (float)on.y, (float)on.z);
            tmax -= (double)th + ch;
            if (tmax <= 0.0) {
                visible = true;
                break;
            }
            skip = r.yarn;
        }
        if (visible) {
            const int lid = SQ.lid[i];
            L[lid] += SQ.cr[i];
            L[cap + lid] += SQ.cg[i];
            L[2 * cap + lid] += SQ.cb[i];
            if (SQ.G)
                for (int k = 0; k < kGrad; ++k) L[(3 + k) * cap + lid] += SQ.G[k * cap + i];
        }
    }
}

__global__ __launch_bounds__(256) void k_r_accum(const float* L, float* fb, float* grad, int npix, int spp_batch,
                                                 int cap, float inv_spp)
{
    for (int pix = blockIdx.x * blockDim.x + threadIdx.x; pix < npix; pix += gridDim.x * blockDim.x) {
        for (int c = 0; c < 3; ++c) {
            float s = 0.0f;
            for (int j = 0; j < spp_batch; ++j) s += L[c * cap + pix * spp_batch + j];
            fb[3 * pix + c] += s * inv_spp;
        }
        if (grad)
            for (int k = 0; k < kGrad; ++k) {
                float s = 0.0f;
                for (int j = 0; j < spp_batch; ++j) s += L[(3 + k) * cap + pix * spp_batch + j];
                grad[kGrad * pix + k] += s * inv_spp;
            }
    }
}

// ------------------------------------------------------------ host side

constexpr int kPathArrays = 13, kHitArrays = 13, kShadowArrays = 12;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_settings(const render_settings* rs)
{
    if (!rs) return fail(BYSDF_ERR_INVALID_ARG, "settings are NULL");
    if (rs->width < 1 || rs->height < 1 || rs->crop_w < 1 || rs->crop_h < 1 || rs->crop_x < 0 || rs->crop_y < 0 ||
        rs->crop_x + rs->crop_w > rs->width || rs->crop_y + rs->crop_h > rs->height)
        return fail(BYSDF_ERR_INVALID_PARAM, "crop %d,%d %dx%d outside the %dx%d image", rs->crop_x, rs->crop_y,
                    rs->crop_w, rs->crop_h, rs->width, rs->height);
    if (rs->spp < 1 || rs->max_depth < 0 || rs->max_depth > 64 || rs->n_h < 1 || rs->n_h > 64)
        return fail(BYSDF_ERR_INVALID_PARAM, "need spp >= 1, 0 <= max_depth <= 64, 1 <= n_h <= 64");
    if (rs->spp_batch < 0 || rs->spp_batch > rs->spp)
        return fail(BYSDF_ERR_INVALID_PARAM, "spp_batch must be in [0, spp]");
    if (rs->multiscale != 0 && rs->multiscale != 1)
        return fail(BYSDF_ERR_INVALID_PARAM, "multiscale must be 0 or 1");
    if (rs->multiscale && rs->n_h > bysdf::kMaxStrata)
        return fail(BYSDF_ERR_INVALID_PARAM, "multi-scale rendering needs n_h <= 16");
    if (!(rs->vfov > 0.f && rs->vfov < 3.1f) || !(rs->ray_eps >= 0.f) || !(rs->lod_px >= 0.f))
        return fail(BYSDF_ERR_INVALID_PARAM, "need 0 < vfov < 3.1, ray_eps >= 0, lod_px >= 0");
    int b = rs->spp_batch ? rs->spp_batch : rs->spp;
    if ((int64_t)rs->crop_w * rs->crop_h * b >= (int64_t)1 << 30)
        return fail(BYSDF_ERR_INVALID_PARAM, "crop x spp_batch exceeds 2^30 paths per pass");
    const float* v[] = {rs->eye, rs->look_at, rs->up, rs->light_corner, rs->light_u, rs->light_v,
                        rs->light_radiance, rs->env_radiance};
    for (const float* a : v)
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(a[k])) return fail(BYSDF_ERR_INVALID_PARAM, "non-finite setting");
    return 0;
}

size_t workspace_bytes(int64_t cap, bool grad)
{
    size_t arr = align256(sizeof(float) * cap);
    // gradient mode: path log-derivatives in both queues, shadow-ray
    // derivatives and the gradient slots
    const int extra = grad ? 4 * kGrad : 0;
    return arr * (2 * kPathArrays + kHitArrays + kShadowArrays + 3 + extra) + 256;
}

struct HD {
    double x, y, z;
};
HD hd(const float* a) { return HD{a[0], a[1], a[2]}; }
HD hsub(HD a, HD b) { return HD{a.x - b.x, a.y - b.y, a.z - b.z}; }
HD hcross(HD a, HD b) { return HD{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double hdot(HD a, HD b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
HD hunit(HD a)
{
    double l = std::sqrt(hdot(a, a));
    return HD{a.x / l, a.y / l, a.z / l};
}
void put(double* dst, HD a)
{
    dst[0] = a.x;
    dst[1] = a.y;
    dst[2] = a.z;
}

}  // namespace

extern "C" size_t shade_wavefront_workspace_size(const render_settings* rs)
{
    if (check_settings(rs)) return 0;
    int b = rs->spp_batch ? rs->spp_batch : rs->spp;
    return workspace_bytes((int64_t)rs->crop_w * rs->crop_h * b, false);
}

extern "C" size_t shade_wavefront_grad_workspace_size(const render_settings* rs)
{
    if (check_settings(rs)) return 0;
    int b = rs->spp_batch ? rs->spp_batch : rs->spp;
    return workspace_bytes((int64_t)rs->crop_w * rs->crop_h * b, true);
}

extern "C" void bysdf_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    rng::philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1], out);
}

static int render(const yarn_scene_t* scene, const bysdf_types_t* types, const render_settings* rs, float* fb,
                  float* grad, int grad_type, void* ws, size_t ws_bytes, int64_t* ray_counts, hipStream_t stream)
{
    if (!scene || !types || !fb || !ws) return fail(BYSDF_ERR_INVALID_ARG, "scene, types, framebuffer and workspace must be non-NULL");
    int rc = check_settings(rs);
    if (rc) return rc;
    if (((uintptr_t)ws & 255u) || ((uintptr_t)fb & 3u) || ((uintptr_t)grad & 3u))
        return fail(BYSDF_ERR_INVALID_ARG, "workspace must be 256-byte aligned, framebuffer and gradient 4-byte aligned");
    const bool g = grad != nullptr;
    const int spp_batch = rs->spp_batch ? rs->spp_batch : rs->spp;
    const int npix = rs->crop_w * rs->crop_h;
    const int cap = npix * spp_batch;
    if (ws_bytes < workspace_bytes(cap, g))
        return fail(BYSDF_ERR_INVALID_ARG, "workspace of %zu bytes, need %zu", ws_bytes, workspace_bytes(cap, g));
    BysdfTypesView tv = bysdf_types_view(types);
    if (yarn_scene_max_type(scene) >= tv.n_types)
        return fail(BYSDF_ERR_INVALID_PARAM, "the scene uses type %d, the handle has %d types", yarn_scene_max_type(scene),
                    tv.n_types);
    if (g && (grad_type < 0 || grad_type >= tv.n_types))
        return fail(BYSDF_ERR_INVALID_ARG, "grad_type %d outside the handle's %d types", grad_type, tv.n_types);
    if (g && rs->multiscale) return fail(BYSDF_ERR_INVALID_PARAM, "the image gradient is of the near-field render");
    RView V;
    V.S = yarn_scene_view(scene);
    V.types = tv.types;
    V.tables = tv.tables;
    HD eye = hd(rs->eye), f = hunit(hsub(hd(rs->look_at), eye));
    HD r = hunit(hcross(f, hd(rs->up)));
    HD u = hcross(r, f);
    put(V.eye, eye);
    put(V.f, f);
    put(V.r, r);
    put(V.u, u);
    V.th = std::tan(0.5 * (double)rs->vfov);
    V.aspect = (double)rs->width / rs->height;
    V.pix_angle = 2.0 * V.th / rs->height;
    HD leu = hd(rs->light_u), lev = hd(rs->light_v), lx = hcross(leu, lev);
    V.area = std::sqrt(hdot(lx, lx));
    if (!(V.area > 0.0)) return fail(BYSDF_ERR_INVALID_PARAM, "the light has zero area");
    put(V.lc, hd(rs->light_corner));
    put(V.leu, leu);
    put(V.lev, lev);
    put(V.ln, HD{lx.x / V.area, lx.y / V.area, lx.z / V.area});
    V.eu2 = hdot(leu, leu);
    V.ev2 = hdot(lev, lev);
    for (int c = 0; c < 3; ++c) {
        V.Le[c] = rs->light_radiance[c];
        V.env[c] = rs->env_radiance[c];
    }
    V.W = rs->width;
    V.H = rs->height;
    V.cx = rs->crop_x;
    V.cy = rs->crop_y;
    V.cw = rs->crop_w;
    V.ch = rs->crop_h;
    V.spp = rs->spp;
    V.max_depth = rs->max_depth;
    V.n_h = rs->n_h;
    V.lod_px = rs->lod_px;
    V.multiscale = rs->multiscale;
    V.grad_type = g ? grad_type : -1;
    V.eps = rs->ray_eps;
    V.key0 = (uint32_t)rs->seed;
    V.key1 = (uint32_t)(rs->seed >> 32);

    // workspace carve-up
    char* w = (char*)ws;
    const size_t arr = align256(sizeof(float) * cap);
    auto take = [&]() {
        char* p = w;
        w += arr;
        return p;
    };
    PathQ Qs[2];
    for (int k = 0; k < 2; ++k) {
        float** fp[] = {&Qs[k].ox, &Qs[k].oy, &Qs[k].oz, &Qs[k].dx, &Qs[k].dy, &Qs[k].dz, &Qs[k].tr,
                        &Qs[k].tg, &Qs[k].tb, &Qs[k].pdf, &Qs[k].line0};
        for (float** q : fp) *q = (float*)take();
        Qs[k].skip = (int*)take();
        Qs[k].lid = (int*)take();
        Qs[k].D = nullptr;
    }
    HitQ Hh;
    {
        float** fp[] = {&Hh.t, &Hh.s, &Hh.h, &Hh.v, &Hh.R, &Hh.Tx, &Hh.Ty, &Hh.Tz, &Hh.Nx, &Hh.Ny, &Hh.Nz};
        for (float** q : fp) *q = (float*)take();
        Hh.yarn = (int*)take();
        Hh.seg = (int*)take();
    }
    ShadowQ SQ;
    {
        float** fp[] = {&SQ.ox, &SQ.oy, &SQ.oz, &SQ.dx, &SQ.dy, &SQ.dz, &SQ.tmax, &SQ.cr, &SQ.cg, &SQ.cb};
        for (float** q : fp) *q = (float*)take();
        SQ.skip = (int*)take();
        SQ.lid = (int*)take();
        SQ.G = nullptr;
    }
    if (g) {
        for (int k = 0; k < 2; ++k) {
            Qs[k].D = (float*)w;
            w += kGrad * arr;
        }
        SQ.G = (float*)w;
        w += kGrad * arr;
    }
    float* L = (float*)w;
    w += (g ? 3 + kGrad : 3) * arr;
    int* cnt = (int*)w;                                       // [0], [1]: path queues, [2]: shadow rays
    unsigned long long* stats = (unsigned long long*)(w + 64);  // extension, shadow rays

    auto grid_for = [](int64_t n, int block, int cap_blocks) {
        int64_t g = (n + block - 1) / block;
        return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap_blocks));
    };
    hipLaunchKernelGGL(k_r_fill, dim3(grid_for(3 * (int64_t)npix, 256, 4096)), dim3(256), 0, stream, fb,
                       3 * (int64_t)npix);
    if (g)
        hipLaunchKernelGGL(k_r_fill, dim3(grid_for(kGrad * (int64_t)npix, 256, 4096)), dim3(256), 0, stream, grad,
                           kGrad * (int64_t)npix);
    hipLaunchKernelGGL(k_r_fill, dim3(1), dim3(256), 0, stream, (float*)stats, (int64_t)4);
    const bool mp4 = tv.max_plies <= 4;
    int64_t sinfo[6];
    if (int rc = yarn_scene_info(scene, sinfo)) return rc;
    const size_t stk_bytes = sizeof(int) * yarn::stack_entries((int)sinfo[4]) * kTraceBlock;
    for (int j0 = 0; j0 < rs->spp; j0 += spp_batch) {
        const int nb = std::min(spp_batch, rs->spp - j0);
        const int n = npix * nb;
        hipLaunchKernelGGL(k_r_camera, dim3(grid_for(n, 256, 8192)), dim3(256), 0, stream, V, Qs[0], L, n, nb, j0,
                           cnt);
        for (int depth = 0; depth <= rs->max_depth; ++depth) {
            const int a = depth & 1, b = a ^ 1;
            hipLaunchKernelGGL(k_r_tally, dim3(1), dim3(64), 0, stream, cnt, a, stats, 0);
            hipLaunchKernelGGL(k_r_extend, dim3(grid_for(n, kTraceBlock, 16384)), dim3(kTraceBlock), stk_bytes,
                               stream, V, Qs[a], cnt + a, Hh, L, n, depth);
            if (depth == rs->max_depth) break;
            hipLaunchKernelGGL(k_r_counters, dim3(1), dim3(64), 0, stream, cnt, b, 2, -1);
            // multi-scale mode: only the camera hits (depth 0) take the
            // footprint; later bounces are near field, which the plain
            // kernel computes when its view disables the far-field rule
            const bool ms0 = rs->multiscale && depth == 0;
            auto shade = g ? (mp4 ? k_r_shade<4, false, true> : k_r_shade<8, false, true>)
                           : ms0 ? (mp4 ? k_r_shade<4, true, false> : k_r_shade<8, true, false>)
                                 : (mp4 ? k_r_shade<4, false, false> : k_r_shade<8, false, false>);
            RView Vs = V;
            if (rs->multiscale && !ms0) Vs.lod_px = 0.0f;
            hipLaunchKernelGGL(shade, dim3(grid_for(n, kShadeBlock, 8192)), dim3(kShadeBlock), 0, stream, Vs,
                               Qs[a], cnt + a, Hh, Qs[b], cnt + b, SQ, cnt + 2, n, depth, j0, nb);
            hipLaunchKernelGGL(k_r_tally, dim3(1), dim3(64), 0, stream, cnt, 2, stats, 1);
            hipLaunchKernelGGL(mp4 ? k_r_shadow<4> : k_r_shadow<8>, dim3(grid_for(n, kTraceBlock, 16384)),
                               dim3(kTraceBlock), stk_bytes, stream, V, SQ, cnt + 2, L, n);
        }
        hipLaunchKernelGGL(k_r_accum, dim3(grid_for(npix, 256, 4096)), dim3(256), 0, stream, L, fb, grad, npix, nb,
                           n, 1.0f / rs->spp);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BYSDF_ERR_LAUNCH, "shade_wavefront: %s", hipGetErrorString(e));
    if (ray_counts) {
        unsigned long long h[2];
        e = hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(BYSDF_ERR_LAUNCH, "ray counts: %s", hipGetErrorString(e));
        ray_counts[0] = (int64_t)h[0];
        ray_counts[1] = (int64_t)h[1];
    }
    return 0;
}

extern "C" int shade_wavefront(const yarn_scene_t* scene, const bysdf_types_t* types, const render_settings* rs,
                               float* fb, void* ws, size_t ws_bytes, int64_t* ray_counts, hipStream_t stream)
{
    return render(scene, types, rs, fb, nullptr, -1, ws, ws_bytes, ray_counts, stream);
}

extern "C" int shade_wavefront_grad(const yarn_scene_t* scene, const bysdf_types_t* types,
                                    const render_settings* rs, int32_t grad_type, float* fb, float* grad,
                                    void* ws, size_t ws_bytes, int64_t* ray_counts, hipStream_t stream)
{
    if (!grad) return fail(BYSDF_ERR_INVALID_ARG, "gradient buffer must be non-NULL");
    return render(scene, types, rs, fb, grad, grad_type, ws, ws_bytes, ray_counts, stream);
}
