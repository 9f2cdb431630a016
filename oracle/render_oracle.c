/*
 * render_oracle.c -- plain CPU path tracer of BYSDF-shaded yarn scenes.
 * TEST INFRASTRUCTURE ONLY; the algorithm is stated in render_oracle.h.
 */
#include "render_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "yarn_oracle.h"

typedef struct { double x, y, z; } r3;

static r3 R3(double x, double y, double z) { r3 r = {x, y, z}; return r; }
static r3 radd(r3 a, r3 b) { return R3(a.x + b.x, a.y + b.y, a.z + b.z); }
static r3 rsub(r3 a, r3 b) { return R3(a.x - b.x, a.y - b.y, a.z - b.z); }
static r3 rscl(r3 a, double s) { return R3(a.x * s, a.y * s, a.z * s); }
static double rdot(r3 a, r3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static r3 rcross(r3 a, r3 b) { return R3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static r3 runit(r3 a) { return rscl(a, 1.0 / sqrt(rdot(a, a))); }
static double f32(double x) { return (double)(float)x; }
static r3 r3f(r3 a) { return R3(f32(a.x), f32(a.y), f32(a.z)); }
static r3 r3v(const float* p) { return R3(p[0], p[1], p[2]); }

static void rnd(uint64_t seed, uint64_t slot, uint32_t depth, uint32_t stream, double u[4])
{
    uint32_t ctr[4] = {(uint32_t)slot, (uint32_t)(slot >> 32), depth, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = (double)(o[i] >> 8) * (1.0 / 16777216.0);
}

/* hit record as the device keeps it: single precision fields */
typedef struct {
    int miss, yarn, seg;
    double t, s, h, v;
    r3 T, N;
} hitrec;

static void trace(const void* scene, r3 o, r3 d, double t_min, double t_max, int skip, hitrec* hr)
{
    double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z}, out[16];
    orc_intersect_one(scene, oo, dd, t_min, t_max, skip, out);
    hr->miss = ((unsigned)out[12] & ORC_HIT_MISS) != 0;
    if (hr->miss) return;
    hr->yarn = (int)out[1];
    hr->seg = (int)out[2];
    hr->t = f32(out[0]);
    hr->s = f32(out[3]);
    hr->h = f32(out[4]);
    hr->v = f32(out[5]);
    hr->T = r3f(R3(out[6], out[7], out[8]));
    hr->N = r3f(R3(out[9], out[10], out[11]));
}

/* local BYSDF direction of a world direction at a hit (x = N, y = T x N,
 * z = T), rounded to single precision */
static void to_loc(const hitrec* hr, r3 w, double l[3])
{
    r3 B = rcross(hr->T, hr->N);
    l[0] = f32(rdot(w, hr->N));
    l[1] = f32(rdot(w, B));
    l[2] = f32(rdot(w, hr->T));
}

typedef struct {
    const void* scene;
    const orc_params* types;
    const double* const* tables;
    const int32_t* yarn_type;
    const float* yarn_phase;
} ctx_t;

/* chord of the tube cross-section crossed by a ray with offset h */
static double chord_len(double R, double h, const double wi[3])
{
    double sxy = sqrt(wi[0] * wi[0] + wi[1] * wi[1]);
    double c = 1.0 - h * h;
    return 2.0 * R * sqrt(c > 0.0 ? c : 0.0) / (sxy > 1e-12 ? sxy : 1e-12);
}

static int unoccluded(const ctx_t* C, r3 o, r3 d, double t_max, int skip, double eps)
{
    for (int k = 0; k < 16; ++k) {
        hitrec hr;
        trace(C->scene, o, d, eps, t_max, skip, &hr);
        if (hr.miss) return 1;
        int y = hr.yarn;
        const orc_params* P = &C->types[C->yarn_type[y]];
        double R = orc_scene_radius(C->scene, y);
        double wi[3];
        to_loc(&hr, rscl(d, -1.0), wi);
        double vl = f32(hr.v / R);
        double tmp[10 + ORC_MAX_PLIES];
        uint32_t f = orc_ply_hit(P, hr.h, (double)C->yarn_phase[y], vl, wi, tmp);
        if (!(f & ORC_PASS_THROUGH)) return 0;
        double ch = chord_len(R, hr.h, wi);
        r3 p = radd(o, rscl(d, hr.t));
        o = r3f(radd(p, rscl(d, ch)));
        t_max -= hr.t + ch;
        if (t_max <= 0.0) return 1;
        skip = y;
    }
    return 0;
}

/* far field (Eq. 7, W = 1): mean value and mean pdf over n_h strata */
static void far_eval(const ctx_t* C, const orc_params* P, const double* tab, double u, double v,
                     const double wi[3], const double wo[3], int n_h, double zeta, double E[3],
                     double* pdf)
{
    E[0] = E[1] = E[2] = 0.0;
    *pdf = 0.0;
    for (int j = 0; j < n_h; ++j) {
        double hj = f32(-1.0 + 2.0 * (j + zeta) / n_h);
        double out[13];
        orc_eval_query(P, tab, hj, u, v, wi, wo, out);
        for (int c = 0; c < 3; ++c) E[c] += f32(out[c]);
        *pdf += f32(out[11]);
    }
    for (int c = 0; c < 3; ++c) E[c] /= n_h;
    *pdf /= n_h;
    (void)C;
}

/* Pixel footprint of a camera hit in azimuthal offsets (custom ray
 * differentials, Sec. 5.3).  Locally the yarn is the straight tube of radius
 * R about the axis through c along T, where c lies R from the hit p against
 * the surface normal at azimuth atan2(wi) + asin h in the (N, T x N) plane;
 * a camera ray through screen point (sx, sy) then has offset
 * cross(o - c, d) / (|d| R) in that plane.  One-pixel steps right and up
 * give the gradient of h on the screen; the rays one pixel along and
 * against it give the ends h1 <= h2, cut at -1 and 1 and widened to contain
 * h0.  FP32 results, as the query's h. */
static void camera_footprint(r3 o, r3 f, r3 rr, r3 uu, double th, double aspect, int width,
                             int height, r3 du, double t, const hitrec* hr, double R, double* h1,
                             double* h2)
{
    double h0 = hr->h;
    r3 B = rcross(hr->T, hr->N);
    r3 p = radd(o, rscl(du, t));
    double ang = atan2(-rdot(du, B), -rdot(du, hr->N)) + asin(h0);
    r3 c = rsub(p, rscl(radd(rscl(hr->N, cos(ang)), rscl(B, sin(ang))), R));
    r3 e = rsub(o, c);
    double e1 = rdot(e, hr->N), e2 = rdot(e, B);
    double fd = rdot(du, f);
    double sx = rdot(du, rr) / fd, sy = rdot(du, uu) / fd;
    double stepx = 2.0 * th * aspect / width, stepy = 2.0 * th / height;
    double hx[4];
    double dirs[4][2] = {{1, 0}, {0, 1}, {0, 0}, {0, 0}};
    for (int k = 0; k < 4; ++k) {
        if (k == 2) {
            double gx = hx[0] - h0, gy = hx[1] - h0, gl = sqrt(gx * gx + gy * gy);
            if (!(gl > 0.0)) {
                *h1 = *h2 = h0;
                return;
            }
            dirs[2][0] = gx / gl; dirs[2][1] = gy / gl;
            dirs[3][0] = -gx / gl; dirs[3][1] = -gy / gl;
        }
        r3 dd = runit(radd(f, radd(rscl(rr, sx + dirs[k][0] * stepx), rscl(uu, sy + dirs[k][1] * stepy))));
        double a = rdot(dd, hr->N), b = rdot(dd, B), l = sqrt(a * a + b * b);
        hx[k] = l > 1e-12 ? (e1 * b - e2 * a) / (l * R) : h0;
    }
    double lo = hx[2] < hx[3] ? hx[2] : hx[3], hi = hx[2] < hx[3] ? hx[3] : hx[2];
    lo = lo < -1.0 ? -1.0 : lo;
    hi = hi > 1.0 ? 1.0 : hi;
    *h1 = f32(lo < h0 ? lo : h0);
    *h2 = f32(hi > h0 ? hi : h0);
}

/* The footprint of the camera ray through continuous pixel position (px, py)
 * (test access): out = h0, h1, h2 of its first yarn hit; returns the yarn or
 * -1 on a miss. */
int orc_camera_footprint(const void* scene, const orc_render_settings* rs, double px, double py,
                         double out[3])
{
    r3 eye = r3v(rs->eye);
    r3 f = runit(rsub(r3v(rs->look_at), eye));
    r3 rr = runit(rcross(f, r3v(rs->up)));
    r3 uu = rcross(rr, f);
    double th = tan(0.5 * rs->vfov);
    double aspect = (double)rs->width / rs->height;
    double sx = (2.0 * px / rs->width - 1.0) * th * aspect;
    double sy = (1.0 - 2.0 * py / rs->height) * th;
    r3 o = r3f(eye);
    r3 du = runit(r3f(runit(radd(f, radd(rscl(rr, sx), rscl(uu, sy))))));
    hitrec hr;
    trace(scene, o, du, 0.0, 1e30, -1, &hr);
    if (hr.miss) return -1;
    double R = orc_scene_radius(scene, hr.yarn);
    out[0] = hr.h;
    camera_footprint(o, f, rr, uu, th, aspect, rs->width, rs->height, du, hr.t, &hr, f32(R), &out[1],
                     &out[2]);
    return hr.yarn;
}

/* dE_c / d theta_p at one direction, theta = (r, k^B_c, sigma_t) (image
 * fitting, Sec. 5.2): out[13] is the query's evaluation; the reflected body
 * lobe is r times an r-free term and the transmitted one (1 - r) times one,
 * both linear in k^B_c; sigma_t by central differences of the evaluation
 * (only E_yS depends on it). */
static void bysdf_derivs(const orc_params* P, const double* tab, double h, double u, double v,
                         const double wi[3], const double wo[3], const double out[13], double dE[9])
{
    orc_params q = *P;
    double hs = 1e-4 * (P->sigma_t > 1e-3 ? P->sigma_t : 1e-3);
    double ep[13], em[13];
    q.sigma_t = P->sigma_t + hs;
    orc_eval_query(&q, tab, h, u, v, wi, wo, ep);
    q.sigma_t = P->sigma_t - hs;
    orc_eval_query(&q, tab, h, u, v, wi, wo, em);
    double ds = (ep[4] - em[4]) / (2.0 * hs);
    for (int c = 0; c < 3; ++c) {
        double xb = out[5 + c], yb = out[8 + c];
        dE[3 * c] = (P->r > 0.0 ? xb / P->r : 0.0) - (P->r < 1.0 ? yb / (1.0 - P->r) : 0.0);
        dE[3 * c + 1] = P->albedo[c] > 0.0 ? (xb + yb) / P->albedo[c] : 0.0;
        dE[3 * c + 2] = ds;
    }
}

int orc_render(const void* scene, const orc_params* types, const double* const* tables,
               int32_t n_types, const int32_t* yarn_type, const float* yarn_phase,
               const orc_render_settings* rs, double* fb, double* sq, double* grad, int nthreads)
{
    (void)n_types;
    ctx_t C = {scene, types, tables, yarn_type, yarn_phase};
    r3 eye = r3v(rs->eye);
    r3 f = runit(rsub(r3v(rs->look_at), eye));
    r3 rr = runit(rcross(f, r3v(rs->up)));
    r3 uu = rcross(rr, f);
    double th = tan(0.5 * rs->vfov);
    double aspect = (double)rs->width / rs->height;
    double pix_angle = 2.0 * th / rs->height;
    r3 lc = r3v(rs->light_corner), leu = r3v(rs->light_u), lev = r3v(rs->light_v);
    r3 lx = rcross(leu, lev);
    double area = sqrt(rdot(lx, lx));
    r3 ln = rscl(lx, 1.0 / area);
    double eu2 = rdot(leu, leu), ev2 = rdot(lev, lev);
    int64_t npix = (int64_t)rs->crop_w * rs->crop_h;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t pix = 0; pix < npix; ++pix) {
        int pxc = (int)(pix % rs->crop_w), pyc = (int)(pix / rs->crop_w);
        int px = rs->crop_x + pxc, py = rs->crop_y + pyc;
        double acc[3] = {0, 0, 0}, acc2[3] = {0, 0, 0}, gacc[9] = {0};
        for (int j = 0; j < rs->spp; ++j) {
            uint64_t slot = (uint64_t)pix * rs->spp + j;
            double u0[4];
            rnd(rs->seed, slot, 0, 0, u0);
            double sx = (2.0 * (px + u0[0]) / rs->width - 1.0) * th * aspect;
            double sy = (1.0 - 2.0 * (py + u0[1]) / rs->height) * th;
            r3 o = r3f(eye);
            r3 d = r3f(runit(radd(f, radd(rscl(rr, sx), rscl(uu, sy)))));
            float thr[3] = {1.f, 1.f, 1.f}, L[3] = {0.f, 0.f, 0.f};
            /* gradient mode: D = d ln(throughput_c) / d theta_p, g = the
             * path's d(radiance_c) / d theta_p, index 3c + p */
            double D[9] = {0}, g[9] = {0};
            double last_pdf = -1.0;
            /* distance from the last scattering event to the ray origin
             * along the straight line (pass-through keeps the line) */
            double line0 = 0.0;
            int skip = -1;
            /* up to max_depth scattering events; the ray leaving the last
             * one is still traced for the light or the environment */
            for (int depth = 0; depth <= rs->max_depth; ++depth) {
                r3 du = runit(d);
                double tmin = depth == 0 ? 0.0 : rs->ray_eps;
                hitrec hr;
                trace(scene, o, du, tmin, 1e30, skip, &hr);
                /* the light: one-sided rectangle emitting along ln */
                double den = rdot(du, ln), tl = INFINITY;
                if (den < 0.0) {
                    double t = rdot(rsub(lc, o), ln) / den;
                    if (t > tmin) {
                        r3 q = rsub(radd(o, rscl(du, t)), lc);
                        double a = rdot(q, leu) / eu2, b = rdot(q, lev) / ev2;
                        if (a >= 0.0 && a <= 1.0 && b >= 0.0 && b <= 1.0) tl = t;
                    }
                }
                if (tl < INFINITY && (hr.miss || tl < hr.t)) {
                    double w = 1.0;
                    if (last_pdf > 0.0 && rs->nee) {
                        double dl = line0 + tl;
                        double pl = dl * dl / (area * fabs(den));
                        w = last_pdf * last_pdf / (last_pdf * last_pdf + pl * pl);
                    }
                    float wf = (float)w;
                    for (int c = 0; c < 3; ++c) L[c] += thr[c] * rs->light_radiance[c] * wf;
                    for (int k = 0; k < 9; ++k) g[k] += (double)thr[k / 3] * rs->light_radiance[k / 3] * wf * D[k];
                    break;
                }
                if (hr.miss) {
                    for (int c = 0; c < 3; ++c) L[c] += thr[c] * rs->env_radiance[c];
                    for (int k = 0; k < 9; ++k) g[k] += (double)thr[k / 3] * rs->env_radiance[k / 3] * D[k];
                    break;
                }
                if (depth == rs->max_depth) break;
                int y = hr.yarn;
                const orc_params* P = &types[yarn_type[y]];
                const double* tab = tables[yarn_type[y]];
                double R = orc_scene_radius(scene, y);
                r3 p = radd(o, rscl(du, hr.t));
                double wi[3];
                to_loc(&hr, rscl(du, -1.0), wi);
                double uq = (double)yarn_phase[y];
                double vl = f32(hr.v / R);
                double dist_cam = sqrt(rdot(rsub(p, eye), rsub(p, eye)));
                /* multi-scale: camera hits over their pixel footprint, later
                 * bounces near field; otherwise the LOD rule picks the far field */
                int ms = rs->multiscale && depth == 0;
                int far = !rs->multiscale && !grad && 2.0 * R / (dist_cam * pix_angle) < rs->lod_px;
                int gt = grad && yarn_type[y] == rs->grad_type;
                double fh1 = hr.h, fh2 = hr.h;
                if (ms)
                    camera_footprint(o, f, rr, uu, th, aspect, rs->width, rs->height, du, hr.t, &hr,
                                     f32(R), &fh1, &fh2);
                double u1[4], u2[4];
                rnd(rs->seed, slot, (uint32_t)depth, 1, u1);
                rnd(rs->seed, slot, (uint32_t)depth, 2, u2);
                /* next-event estimation */
                r3 yl = radd(lc, radd(rscl(leu, u1[0]), rscl(lev, u1[1])));
                r3 lv = rsub(yl, p);
                double dist2 = rdot(lv, lv);
                r3 wl = rscl(lv, 1.0 / sqrt(dist2));
                double cosl = -rdot(wl, ln);
                if (cosl > 0.0 && rs->nee) {
                    double wo[3];
                    to_loc(&hr, wl, wo);
                    double E[3], pb, dEn[9] = {0};
                    if (ms) {
                        double out[13];
                        orc_eval_multi_query(P, tab, hr.h, fh1, fh2, u2[2], rs->n_h, uq, vl, wi, wo,
                                             out);
                        for (int c = 0; c < 3; ++c) E[c] = f32(out[c]);
                        pb = f32(out[11]);
                    } else if (far) {
                        far_eval(&C, P, tab, uq, vl, wi, wo, rs->n_h, u2[2], E, &pb);
                    } else {
                        double out[13];
                        orc_eval_query(P, tab, hr.h, uq, vl, wi, wo, out);
                        for (int c = 0; c < 3; ++c) E[c] = f32(out[c]);
                        pb = f32(out[11]);
                        if (gt) bysdf_derivs(P, tab, hr.h, uq, vl, wi, wo, out, dEn);
                    }
                    if (E[0] > 0.0 || E[1] > 0.0 || E[2] > 0.0) {
                        double pl = dist2 / (area * cosl);
                        double w = pl * pl / (pl * pl + pb * pb);
                        float fac = (float)(w / pl);
                        float ct[3];
                        for (int c = 0; c < 3; ++c)
                            ct[c] = thr[c] * (float)E[c] * rs->light_radiance[c] * fac;
                        r3 os = r3f(p), ds = runit(r3f(wl));
                        if (unoccluded(&C, os, ds, sqrt(dist2) * (1.0 - 1e-5), y, rs->ray_eps)) {
                            for (int c = 0; c < 3; ++c) L[c] += ct[c];
                            if (grad)
                                for (int k = 0; k < 9; ++k)
                                    g[k] += (double)thr[k / 3] * rs->light_radiance[k / 3] * fac *
                                            (dEn[k] + E[k / 3] * D[k]);
                        }
                    }
                }
                /* continue the path with a BYSDF sample */
                double xi[3] = {u1[2], u1[3], u2[0]};
                double so[12];
                uint32_t sf;
                double hq = hr.h;
                if (far) {
                    int js = (int)floor(u2[1] * rs->n_h);
                    if (js > rs->n_h - 1) js = rs->n_h - 1;
                    hq = f32(-1.0 + 2.0 * (js + u2[2]) / rs->n_h);
                }
                if (ms) {
                    double sm[13];
                    sf = orc_sample_multi_query(P, tab, hr.h, fh1, fh2, u2[2], u2[1], rs->n_h, uq, vl,
                                                wi, xi, sm);
                    memcpy(so, sm, sizeof(so));
                } else {
                    sf = orc_sample_query(P, tab, hq, uq, vl, wi, xi, so);
                }
                int lobe = (int)so[10];
                r3 dnew;
                if (lobe == 4) {
                    /* straight through the yarn: the last scattering event
                     * and its pdf stay in force */
                    dnew = du;
                    line0 += hr.t;
                } else {
                    if (lobe < 0 || (sf & ORC_SAMPLE_FAIL) || !(f32(so[6]) > 0.0)) break;
                    double wo[3] = {f32(so[0]), f32(so[1]), f32(so[2])};
                    float wgt[3];
                    double pdf;
                    if (far) {
                        double E[3];
                        far_eval(&C, P, tab, uq, vl, wi, wo, rs->n_h, u2[2], E, &pdf);
                        if (!(pdf > 0.0)) break;
                        for (int c = 0; c < 3; ++c) wgt[c] = (float)(E[c] / pdf);
                    } else {
                        for (int c = 0; c < 3; ++c) wgt[c] = (float)so[3 + c];
                        pdf = f32(so[6]);
                    }
                    r3 B = rcross(hr.T, hr.N);
                    dnew = runit(radd(radd(rscl(hr.N, wo[0]), rscl(B, wo[1])), rscl(hr.T, wo[2])));
                    if (gt) {
                        /* the value at the drawn (unrounded) direction */
                        double es[13], dEs[9];
                        orc_eval_query(P, tab, hq, uq, vl, wi, so, es);
                        bysdf_derivs(P, tab, hq, uq, vl, wi, so, es, dEs);
                        for (int k = 0; k < 9; ++k)
                            if (es[k / 3] > 0.0) D[k] += dEs[k] / es[k / 3];
                    }
                    for (int c = 0; c < 3; ++c) thr[c] *= wgt[c];
                    last_pdf = pdf;
                    line0 = 0.0;
                    if (!(thr[0] > 0.f || thr[1] > 0.f || thr[2] > 0.f)) break;
                }
                /* the BYSDF is located at the yarn hit: the path continues
                 * from there, past its own yarn */
                r3 onew = p;
                o = r3f(onew);
                d = r3f(dnew);
                skip = y;
            }
            for (int c = 0; c < 3; ++c) {
                acc[c] += L[c];
                acc2[c] += (double)L[c] * L[c];
            }
            for (int k = 0; k < 9; ++k) gacc[k] += g[k];
        }
        for (int c = 0; c < 3; ++c) {
            fb[3 * pix + c] = acc[c] / rs->spp;
            if (sq) sq[3 * pix + c] = acc2[c] / rs->spp;
        }
        if (grad)
            for (int k = 0; k < 9; ++k) grad[9 * pix + k] = gacc[k] / rs->spp;
    }
    return 0;
}
