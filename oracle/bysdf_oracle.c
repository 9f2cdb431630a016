/*
 * bysdf_oracle.c -- plain FP64 CPU oracle of the BYSDF (arXiv 2401.12724).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  The product library never includes, links or
 * calls it, and it shares no code with the HIP path.
 *
 * Structure follows the paper:
 *   yarn hit (Sec. 3.3)          -> hit point x2 on the yarn circle
 *   implicit plies (Sec. 3.4)    -> fixed-point update of the ply centre on
 *                                   the ray's ellipse plane, 2D ray tracing,
 *                                   closest ply, ply frame
 *   implicit fibers (Sec. 3.5.1) -> 1D fiber table, fiber frame
 *   self-shadowing (Sec. 4.1.4)  -> G_p (ply horizon), G_f (fiber table)
 *   lobes (Sec. 4.1, Eq. 1-6)    -> f_x^S, f_x^B, f_y^S, f_y^B
 *   importance sampling (4.1.5)  -> lobe selection, GGX / cosine sampling
 *   far field (Sec. 4.2, Eq. 7)  -> stratified average over h
 *   energy test (Sec. 4.3)       -> white-furnace blocks
 */
#include "bysdf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define TWO_PI (2.0 * PI)

/* Margins of the oracle-only flags.  A query within these distances of a
 * discrete decision is flagged; see the parity rule in the tests. */
static double g_margin_geo = 1e-7;   /* decisions on O(1) geometric quantities */
static double g_margin_shade = 2e-6; /* decisions on shading cosines */
static double g_amplify_max = 1e5;   /* ply fixed point: max_k A_k * max(1, |kappa|) */
static double g_margin_tir = 1e-6;   /* 1 - sin^2 of the transmitted angle at exit */
static double g_margin_xi = 1e-6;    /* lobe / node selection edges */

void orc_set_margins(double geo, double shade, double amplify, double tir, double xi)
{
    g_margin_geo = geo;
    g_margin_shade = shade;
    g_amplify_max = amplify;
    g_margin_tir = tir;
    g_margin_xi = xi;
}

/* ------------------------------------------------------------------ */
/* small vector algebra                                                */
/* ------------------------------------------------------------------ */
typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
static v3 vadd(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vsub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vscl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 vcross(v3 a, v3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double vlen(v3 a) { return sqrt(vdot(a, a)); }
static v3 vnorm(v3 a) { return vscl(a, 1.0 / vlen(a)); }

typedef struct { v3 t, b, n; } frame; /* tangent, bitangent, normal */

static v3 to_local(const frame* f, v3 w) { return mk(vdot(w, f->t), vdot(w, f->b), vdot(w, f->n)); }
static v3 to_world(const frame* f, v3 l)
{
    return vadd(vadd(vscl(f->t, l.x), vscl(f->b, l.y)), vscl(f->n, l.z));
}

/* ------------------------------------------------------------------ */
/* microfacet ingredients (Walter et al. 2007; Heitz 2018)             */
/* ------------------------------------------------------------------ */

/* Unpolarised dielectric Fresnel reflectance for light arriving with
 * cosine cos_i >= 0 on the side of index 1 of an interface of relative
 * index eta_rel (transmitted side / incident side).  Total internal
 * reflection returns 1. */
double orc_fresnel(double cos_i, double eta_rel)
{
    double s2t = (1.0 - cos_i * cos_i) / (eta_rel * eta_rel);
    if (s2t >= 1.0) return 1.0;
    double ct = sqrt(1.0 - s2t);
    double rs = (cos_i - eta_rel * ct) / (cos_i + eta_rel * ct);
    double rp = (eta_rel * cos_i - ct) / (eta_rel * cos_i + ct);
    return 0.5 * (rs * rs + rp * rp);
}

/* Anisotropic GGX normal distribution; m in the local frame (z = normal). */
double orc_ggx_D(const double m[3], double ax, double ay)
{
    if (m[2] <= 0.0) return 0.0;
    double t = m[0] * m[0] / (ax * ax) + m[1] * m[1] / (ay * ay) + m[2] * m[2];
    return 1.0 / (PI * ax * ay * t * t);
}

/* Smith masking G1 for GGX with the sidedness test chi+((w.m)(w.n)). */
double orc_smith_G1(const double w[3], const double m[3], double ax, double ay)
{
    double wm = w[0] * m[0] + w[1] * m[1] + w[2] * m[2];
    if (wm * w[2] <= 0.0) return 0.0;
    double z2 = w[2] * w[2];
    double a2t2 = (ax * ax * w[0] * w[0] + ay * ay * w[1] * w[1]) / z2;
    return 2.0 / (1.0 + sqrt(1.0 + a2t2));
}

/* Visible-normal sampling of GGX (Heitz 2018, JCGT 7(4)): stretch the view
 * direction to the unit-roughness configuration, sample the projected
 * disc of the hemisphere seen from it with the disc half warped towards
 * the view, lift to the hemisphere, unstretch. wi local, wi.z > 0. */
void orc_vndf(const double wi[3], double ax, double ay, double u1, double u2, double m[3])
{
    v3 vh = vnorm(mk(ax * wi[0], ay * wi[1], wi[2]));
    double lensq = vh.x * vh.x + vh.y * vh.y;
    v3 t1 = lensq > 0.0 ? vscl(mk(-vh.y, vh.x, 0.0), 1.0 / sqrt(lensq)) : mk(1.0, 0.0, 0.0);
    v3 t2 = vcross(vh, t1);
    double rad = sqrt(u1);
    double phi = TWO_PI * u2;
    double p1 = rad * cos(phi);
    double p2 = rad * sin(phi);
    double s = 0.5 * (1.0 + vh.z);
    p2 = (1.0 - s) * sqrt(1.0 - p1 * p1) + s * p2;
    double lift = 1.0 - p1 * p1 - p2 * p2;
    v3 nh = vadd(vadd(vscl(t1, p1), vscl(t2, p2)), vscl(vh, sqrt(lift > 0.0 ? lift : 0.0)));
    v3 ne = vnorm(mk(ax * nh.x, ay * nh.y, nh.z > 0.0 ? nh.z : 0.0));
    m[0] = ne.x; m[1] = ne.y; m[2] = ne.z;
}

static double D_l(v3 m, double ax, double ay) { double a[3] = {m.x, m.y, m.z}; return orc_ggx_D(a, ax, ay); }
static double G1_l(v3 w, v3 m, double ax, double ay)
{
    double a[3] = {w.x, w.y, w.z}, b[3] = {m.x, m.y, m.z};
    return orc_smith_G1(a, b, ax, ay);
}

/* Albedo of the single-scattering Lommel-Seeliger lobe 1/(4 pi (mu_i+mu_o))
 * times mu_o over the hemisphere: 1/2 [1 - mu ln(1 + 1/mu)]. */
double orc_ls_albedo(double mu)
{
    if (mu <= 0.0) return 0.5;
    return 0.5 * (1.0 - mu * log(1.0 + 1.0 / mu));
}

/* ------------------------------------------------------------------ */
/* implicit fibers: the 1D fiber table (Sec. 3.5.1)                    */
/* ------------------------------------------------------------------ */

/* Fiber centres of one ply cross-section, in ply radii: a Vogel spiral of
 * M centres inside radius 1 - rho (deterministic, uniform density). */
static void fiber_centres(int M, double rho, double* fx, double* fy)
{
    double g = PI * (3.0 - sqrt(5.0));
    for (int j = 0; j < M; ++j) {
        double rj = (1.0 - rho) * sqrt((j + 0.5) / M);
        fx[j] = rj * cos(j * g);
        fy[j] = rj * sin(j * g);
    }
}

typedef struct { double lo, hi; } ival;

static int ival_cmp(const void* a, const void* b)
{
    double x = ((const ival*)a)->lo, y = ((const ival*)b)->lo;
    return (x > y) - (x < y);
}

/* Total length of the union of intervals (sorted and merged). */
static double union_length(ival* iv, int n)
{
    if (n == 0) return 0.0;
    qsort(iv, n, sizeof(ival), ival_cmp);
    double tot = 0.0, lo = iv[0].lo, hi = iv[0].hi;
    for (int i = 1; i < n; ++i) {
        if (iv[i].lo > hi) { tot += hi - lo; lo = iv[i].lo; hi = iv[i].hi; }
        else if (iv[i].hi > hi) hi = iv[i].hi;
    }
    return tot + (hi - lo);
}

/* Cosine-weighted measure 1/2 * sum(sin hi - sin lo) of the union. */
static double union_cos_measure(ival* iv, int n)
{
    if (n == 0) return 0.0;
    qsort(iv, n, sizeof(ival), ival_cmp);
    double tot = 0.0, lo = iv[0].lo, hi = iv[0].hi;
    for (int i = 1; i < n; ++i) {
        if (iv[i].lo > hi) { tot += sin(hi) - sin(lo); lo = iv[i].lo; hi = iv[i].hi; }
        else if (iv[i].hi > hi) hi = iv[i].hi;
    }
    tot += sin(hi) - sin(lo);
    return 0.5 * tot;
}

/* Number of fiber tables of a type (fiber migration off: one). */
static int mig_count(const orc_params* p) { return p->mig_tables > 1 ? p->mig_tables : 1; }

/* Uniform in [0, 1) from the top 24 bits of a Philox output word. */
static double u01_24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* Fiber migration draws: Philox4x32-10 with key (mig_seed, "FIBR"). */
static void mig_philox(const orc_params* p, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                       uint32_t out[4])
{
    const uint32_t ctr[4] = {c0, c1, c2, c3};
    const uint32_t key[2] = {p->mig_seed, 0x46494252u};
    orc_philox4x32_10(ctr, key, out);
}

/* Fiber centres of table m: the regular layout for m = 0; for m > 0 every
 * fiber j moves towards the ply centre by the factor
 * min(1, 1 + spread (2 xi_j - 1)), xi_j from the counter (j, m, "MIGR", 0). */
static void fiber_centres_m(const orc_params* p, int m, double* fx, double* fy)
{
    int M = p->fibers_per_ply;
    fiber_centres(M, p->fiber_radius, fx, fy);
    if (m == 0) return;
    for (int j = 0; j < M; ++j) {
        uint32_t o[4];
        mig_philox(p, (uint32_t)j, (uint32_t)m, 0x4d494752u, 0u, o);
        double f = 1.0 + p->mig_spread * (2.0 * u01_24(o[0]) - 1.0);
        if (f > 1.0) f = 1.0;
        fx[j] *= f;
        fy[j] *= f;
    }
}

/* Texel i looks radially inwards from the ply boundary at angle
 * zeta_i = 2 pi (i + 1/2) / N_u.  The first fiber hit gives the normal
 * perturbation dn (signed angle from the ply's radial normal to the fiber
 * normal), the normalised radius of that fiber, and the cosine-weighted
 * unoccluded fraction of the fiber hemisphere at the hit point. */
static void table_of_centres(const orc_params* p, const double* fx, const double* fy, ival* iv,
                             double* tab);

int orc_table(const orc_params* p, double* tab)
{
    int M = p->fibers_per_ply, Nu = p->tex_size;
    double rho = p->fiber_radius;
    if (M < 1 || Nu < 2 || !(rho > 0.0 && rho < 1.0)) return -1;
    if (p->mig_tables > 1 && !(p->mig_spread >= 0.0 && p->mig_spread < 1.0)) return -1;
    double* fx = (double*)malloc(sizeof(double) * M);
    double* fy = (double*)malloc(sizeof(double) * M);
    ival* iv = (ival*)malloc(sizeof(ival) * (M > 1 ? M : 1));
    for (int m = 0; m < mig_count(p); ++m) {
        fiber_centres_m(p, m, fx, fy);
        table_of_centres(p, fx, fy, iv, tab + (size_t)3 * Nu * m);
    }
    free(fx); free(fy); free(iv);
    return 0;
}

/* One table from the fiber centres fx, fy (ply radii). */
static void table_of_centres(const orc_params* p, const double* fx, const double* fy, ival* iv,
                             double* tab)
{
    int M = p->fibers_per_ply, Nu = p->tex_size;
    double rho = p->fiber_radius;
    for (int i = 0; i < Nu; ++i) {
        double zeta = TWO_PI * (i + 0.5) / Nu;
        double ex = cos(zeta), ey = sin(zeta);
        double ox = (1.0 + 1e-9) * ex, oy = (1.0 + 1e-9) * ey;
        double dx = -ex, dy = -ey;
        int best = -1;
        double sbest = 0.0;
        for (int j = 0; j < M; ++j) {
            double wx = ox - fx[j], wy = oy - fy[j];
            double b = wx * dx + wy * dy;
            double c = wx * wx + wy * wy - rho * rho;
            double disc = b * b - c;
            if (disc < 0.0) continue;
            double s = -b - sqrt(disc);
            if (s < 0.0) continue;
            if (best < 0 || s < sbest) { best = j; sbest = s; }
        }
        if (best < 0) {
            tab[3 * i + 0] = 0.0;
            tab[3 * i + 1] = 0.0;
            tab[3 * i + 2] = 1.0;
            continue;
        }
        double qx = ox + sbest * dx, qy = oy + sbest * dy;
        double nx = (qx - fx[best]) / rho, ny = (qy - fy[best]) / rho;
        double dn = atan2(ex * ny - ey * nx, ex * nx + ey * ny);
        double rh = sqrt(fx[best] * fx[best] + fy[best] * fy[best]) / (1.0 - rho);
        int n = 0;
        for (int l = 0; l < M; ++l) {
            if (l == best) continue;
            double wx = fx[l] - qx, wy = fy[l] - qy;
            double dist = sqrt(wx * wx + wy * wy);
            double beta = atan2(nx * wy - ny * wx, nx * wx + ny * wy);
            double ratio = rho / dist;
            double gam = asin(ratio < 1.0 ? ratio : 1.0);
            double lo = beta - gam, hi = beta + gam;
            if (lo < -0.5 * PI) lo = -0.5 * PI;
            if (hi > 0.5 * PI) hi = 0.5 * PI;
            if (hi > lo) { iv[n].lo = lo; iv[n].hi = hi; ++n; }
        }
        double blocked = union_cos_measure(iv, n);
        /* the texture stores single-precision texels (Sec. 3.5.1 keeps these
         * values in a 1D texture): compute in double, store rounded */
        tab[3 * i + 0] = (double)(float)dn;
        tab[3 * i + 1] = (double)(float)rh;
        tab[3 * i + 2] = (double)(float)(blocked < 1.0 ? 1.0 - blocked : 0.0);
    }
}

/* Periodic linear interpolation between texel centres. */
static void tab_lookup(const double* tab, int Nu, double uf, double out[3])
{
    double x = uf / TWO_PI * Nu - 0.5;
    double fl = floor(x);
    double f = x - fl;
    long i0 = (long)fmod(fl, (double)Nu);
    if (i0 < 0) i0 += Nu;
    long i1 = (i0 + 1) % Nu;
    for (int c = 0; c < 3; ++c) out[c] = (1.0 - f) * tab[3 * i0 + c] + f * tab[3 * i1 + c];
}

/* Table of ply k in migration period q: Philox counter (q low, q high,
 * k, "SELT"), first word modulo the table count. */
static int mig_table(const orc_params* p, int64_t q, int k)
{
    uint32_t o[4];
    uint64_t uq = (uint64_t)q;
    mig_philox(p, (uint32_t)(uq & 0xffffffffu), (uint32_t)(uq >> 32), (uint32_t)k, 0x53454c54u, o);
    return (int)(o[0] % (uint32_t)mig_count(p));
}

/* Fiber-table values at fiber phase uf on ply k at ply arc length vply
 * (Sec. 3.5.1; with migration, Sec. 3.5.2: the period's table, blended
 * linearly into the next period's over the period's last mig_blend share,
 * so the values are continuous along the ply). */
static void fiber_lookup(const orc_params* p, const double* tab, double uf, double vply, int k,
                         double out[3])
{
    int Nu = p->tex_size;
    if (mig_count(p) == 1) {
        tab_lookup(tab, Nu, uf, out);
        return;
    }
    double t = vply / p->mig_period;
    double fl = floor(t), ph = t - fl;
    int64_t q = (int64_t)fl;
    double b = p->mig_blend;
    double w = (b > 0.0 && ph > 1.0 - b) ? (ph - (1.0 - b)) / b : 0.0;
    double o0[3], o1[3];
    tab_lookup(tab + (size_t)3 * Nu * mig_table(p, q, k), Nu, uf, o0);
    tab_lookup(tab + (size_t)3 * Nu * mig_table(p, q + 1, k), Nu, uf, o1);
    for (int c = 0; c < 3; ++c) out[c] = (1.0 - w) * o0[c] + w * o1[c];
}

int orc_mig_table(const orc_params* p, int64_t q, int k) { return mig_table(p, q, k); }

void orc_fiber_lookup(const orc_params* p, const double* tab, double uf, double vply, int k,
                      double out[3])
{
    fiber_lookup(p, tab, uf, vply, k, out);
}

/* ------------------------------------------------------------------ */
/* self-shadowing: ply horizon (Sec. 4.1.4)                            */
/* ------------------------------------------------------------------ */

/* Raw ply visibility at angle a around ply 0 of the nominal symmetric
 * cross-section, for incident 2D angle phi measured from the local ply
 * normal: 1 - |window ∩ occluded| / |window| with a box window of
 * half-width Delta_p.  Occluded directions are those below the ply's own
 * tangent line and those towards the other plies' discs. */
double orc_ply_shadow_raw(const orc_params* p, double a, double phi)
{
    int Np = p->n_plies;
    double rp = p->ply_radius, Rpc = p->ply_center_radius, dlt = p->shadow_halfwidth;
    double nax = cos(a), nay = sin(a);
    double Px = Rpc + rp * nax, Py = rp * nay;
    ival sets[ORC_MAX_PLIES + 1];
    int ns = 0;
    sets[ns].lo = 0.5 * PI; sets[ns].hi = 1.5 * PI; ++ns;
    for (int j = 1; j < Np; ++j) {
        double cx = Rpc * cos(TWO_PI * j / Np), cy = Rpc * sin(TWO_PI * j / Np);
        double wx = cx - Px, wy = cy - Py;
        double dist = sqrt(wx * wx + wy * wy);
        double beta = atan2(nax * wy - nay * wx, nax * wx + nay * wy);
        double ratio = rp / dist;
        double gam = asin(ratio < 1.0 ? ratio : 1.0);
        sets[ns].lo = beta - gam; sets[ns].hi = beta + gam; ++ns;
    }
    double wlo = phi - dlt, whi = phi + dlt;
    ival pieces[3 * (ORC_MAX_PLIES + 1)];
    int np = 0;
    for (int s = 0; s < ns; ++s) {
        for (int sh = -1; sh <= 1; ++sh) {
            double lo = sets[s].lo + sh * TWO_PI, hi = sets[s].hi + sh * TWO_PI;
            if (lo < wlo) lo = wlo;
            if (hi > whi) hi = whi;
            if (hi > lo) { pieces[np].lo = lo; pieces[np].hi = hi; ++np; }
        }
    }
    double occ = union_length(pieces, np);
    double vis = 1.0 - occ / (2.0 * dlt);
    /* exact visibility lies in [0, 1]; clamp away rounding */
    return vis < 0.0 ? 0.0 : (vis > 1.0 ? 1.0 : vis);
}

/* ------------------------------------------------------------------ */
/* implicit plies (Sec. 3.4)                                           */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t flags;
    int pass;
    double x2[2], dh[2], kappa, s_exit;
    double cst[ORC_MAX_PLIES][2], th[ORC_MAX_PLIES], amp[ORC_MAX_PLIES];
    int kstar;
    double sstar, p2[2], n2[2], vhit, a;
} plyhit;

static double helix_rate(const orc_params* p)
{
    return p->ply_center_radius > 0.0 ? tan(p->ply_twist) / p->ply_center_radius : 0.0;
}

/* Yarn hit (Sec. 3.3) and ply hit (Sec. 3.4) of one query. */
static void trace_plies(const orc_params* p, double h, double u, double v, v3 wi, plyhit* g)
{
    memset(g, 0, sizeof(*g));
    int Np = p->n_plies;
    double rp = p->ply_radius, Rpc = p->ply_center_radius;
    double wp = helix_rate(p);
    double sxy = sqrt(wi.x * wi.x + wi.y * wi.y);
    if (sxy < 1e-6) {
        g->flags |= ORC_AXIAL | ORC_PASS_THROUGH;
        g->pass = 1;
        return;
    }
    /* incident ray d = -wi; hit on the unit yarn circle at offset h:
     * x2 = the direction of wi_xy rotated by gamma = asin h. */
    double cx = wi.x / sxy, cy = wi.y / sxy;
    double hc = h > 1.0 ? 1.0 : (h < -1.0 ? -1.0 : h);
    double cg = sqrt(1.0 - hc * hc), sg = hc;
    g->x2[0] = cx * cg - cy * sg;
    g->x2[1] = cy * cg + cx * sg;
    g->dh[0] = -cx;
    g->dh[1] = -cy;
    g->kappa = -wi.z / sxy;
    g->s_exit = -2.0 * (g->x2[0] * g->dh[0] + g->x2[1] * g->dh[1]);

    double sk[ORC_MAX_PLIES];
    int hit[ORC_MAX_PLIES];
    double mg = g_margin_geo;
    for (int k = 0; k < Np; ++k) {
        /* ply-centre helix: theta_k(z) = u + 2 pi k / N_p + w_p z.  The
         * ellipse plane holds the ray and the horizontal normal to it; a
         * cross-section point q at height z lies on it iff
         * z = v + kappa (q - x2).dh.  Update the height from the ply
         * centre of the current cross-section (the paper's heuristic). */
        double vj = v;
        double amp_tail = 1.0, amp = 1.0; /* suffix-product error bound */
        double gprime[32];
        int nit = p->n_iter;
        for (int j = 0; j < nit; ++j) {
            double th = u + TWO_PI * k / Np + wp * vj;
            double ccx = Rpc * cos(th), ccy = Rpc * sin(th);
            gprime[j] = g->kappa * wp * Rpc * (-sin(th) * g->dh[0] + cos(th) * g->dh[1]);
            vj = v + g->kappa * ((ccx - g->x2[0]) * g->dh[0] + (ccy - g->x2[1]) * g->dh[1]);
        }
        for (int j = nit - 1; j >= 0; --j) {
            amp_tail *= fabs(gprime[j]);
            amp += amp_tail;
        }
        double th = u + TWO_PI * k / Np + wp * vj;
        g->th[k] = th;
        g->cst[k][0] = Rpc * cos(th);
        g->cst[k][1] = Rpc * sin(th);
        g->amp[k] = amp;
        /* 2D ray against the ply disc, inside the yarn chord */
        double wx = g->x2[0] - g->cst[k][0], wy = g->x2[1] - g->cst[k][1];
        double b = wx * g->dh[0] + wy * g->dh[1];
        double c = wx * wx + wy * wy - rp * rp;
        double disc = b * b - c;
        double m = mg * (amp > 1.0 ? amp : 1.0);
        hit[k] = 0;
        if (fabs(disc) < m * rp * rp) g->flags |= ORC_NEARTIE;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double slo = -b - sq, shi = -b + sq;
            if (shi >= 0.0 && slo <= g->s_exit) {
                hit[k] = 1;
                sk[k] = slo > 0.0 ? slo : 0.0;
                /* s* = max(s_lo, 0) is continuous: only the hit/miss ends
                 * (s_hi = 0, s_lo = s_exit) and ties are decisions */
                if (fabs(shi) < m || fabs(slo - g->s_exit) < m) g->flags |= ORC_NEARTIE;
            } else if (fabs(shi) < m || fabs(slo - g->s_exit) < m) {
                g->flags |= ORC_NEARTIE;
            }
        }
    }
    int ks = -1;
    for (int k = 0; k < Np; ++k)
        if (hit[k] && (ks < 0 || sk[k] < sk[ks])) ks = k;
    if (ks < 0) {
        g->flags |= ORC_PASS_THROUGH;
        g->pass = 1;
        return;
    }
    for (int k = 0; k < Np; ++k) {
        if (k == ks || !hit[k]) continue;
        double m = mg * (g->amp[k] > g->amp[ks] ? g->amp[k] : g->amp[ks]);
        if (fabs(sk[k] - sk[ks]) < (m > mg ? m : mg)) g->flags |= ORC_NEARTIE;
    }
    /* Rounding of the phase (relative 1e-16 of up to ~50 rad) reaches v*
     * amplified by A |kappa|; the steep fiber table then turns an error in
     * v* into a value error a few thousand times larger.  The table is
     * interpolated linearly between texels (Sec. 3.5.1), so its steepest
     * slope grows with the texel count: the bound is priced per texel,
     * relative to the 512-texel table at which the limit was set. */
    double amax = 0.0;
    for (int k = 0; k < Np; ++k) amax = g->amp[k] > amax ? g->amp[k] : amax;
    double ak = fabs(g->kappa);
    double texel_scale = p->tex_size > 512 ? p->tex_size / 512.0 : 1.0;
    if (amax * (ak > 1.0 ? ak : 1.0) * texel_scale > g_amplify_max) g->flags |= ORC_ILLCOND;
    g->kstar = ks;
    g->sstar = sk[ks];
    g->p2[0] = g->x2[0] + g->sstar * g->dh[0];
    g->p2[1] = g->x2[1] + g->sstar * g->dh[1];
    double nx = g->p2[0] - g->cst[ks][0], ny = g->p2[1] - g->cst[ks][1];
    double nl = sqrt(nx * nx + ny * ny);
    g->n2[0] = nx / nl;
    g->n2[1] = ny / nl;
    g->vhit = v + g->kappa * g->sstar;
}

/* Ply frame and fiber frame on disc k at 2D outward normal n2 and
 * yarn-axis height z (Sec. 3.4 last paragraph, Sec. 3.5.1). */
static void fiber_frame(const orc_params* p, const double* tab, double th, int k, double n2x,
                        double n2y, double z, frame* f, double* gf_tab, double* a_out)
{
    double wp = helix_rate(p);
    double slope = p->ply_center_radius * wp;
    double chx = cos(th), chy = sin(th);
    v3 tp = vnorm(mk(-slope * chy, slope * chx, 1.0));
    v3 n23 = mk(n2x, n2y, 0.0);
    v3 np = vnorm(vsub(n23, vscl(tp, vdot(n23, tp))));
    double a = atan2(chx * n2y - chy * n2x, chx * n2x + chy * n2y);
    double vply = z * sqrt(1.0 + slope * slope);
    double rho = p->fiber_radius;
    double wf = tan(p->fiber_twist) / ((1.0 - rho) * p->ply_radius);
    double tv[3];
    fiber_lookup(p, tab, a + wf * vply, vply, k, tv);
    v3 bp = vcross(tp, np);
    v3 npr = vadd(vscl(np, cos(tv[0])), vscl(bp, sin(tv[0])));
    double tfa = tv[1] * tan(p->fiber_twist);
    double ca = 1.0 / sqrt(1.0 + tfa * tfa), sa = tfa * ca;
    v3 t = vsub(vscl(tp, ca), vscl(bp, sa));
    v3 n = vnorm(vsub(npr, vscl(t, vdot(npr, t))));
    f->t = t;
    f->n = n;
    f->b = vcross(n, t);
    if (gf_tab) *gf_tab = tv[2];
    if (a_out) *a_out = a;
}

uint32_t orc_ply_hit(const orc_params* p, double h, double u, double v, const double wi[3],
                     double* out)
{
    plyhit g;
    trace_plies(p, h, u, v, mk(wi[0], wi[1], wi[2]), &g);
    out[0] = g.pass;
    out[1] = g.pass ? -1 : g.kstar;
    out[2] = g.sstar;
    out[3] = g.p2[0]; out[4] = g.p2[1];
    out[5] = g.n2[0]; out[6] = g.n2[1];
    out[7] = g.vhit;
    out[8] = g.pass ? 0.0 : g.amp[g.kstar];
    out[9] = 0.0;
    if (!g.pass) {
        double th = g.th[g.kstar], chx = cos(th), chy = sin(th);
        out[9] = atan2(chx * g.n2[1] - chy * g.n2[0], chx * g.n2[0] + chy * g.n2[1]);
    }
    for (int k = 0; k < p->n_plies; ++k) out[10 + k] = g.pass ? 0.0 : g.th[k];
    return g.flags;
}

/* ------------------------------------------------------------------ */
/* everything that depends on wi only                                  */
/* ------------------------------------------------------------------ */

typedef struct {
    int kind;     /* 0 chord through the plies, 1 thin sheet */
    double T;     /* (1 - F) G1 of the refraction at x */
    double att;   /* tau^N (Eq. 4) */
    v3 wt;        /* refracted direction at x */
    frame fy;     /* shading frame at the exit point y */
    v3 y;         /* exit point (x2, z) in yarn coordinates */
    int N;        /* plies entered by the chord */
    double ell;   /* 3D chord length |x - y| */
} fnode;

typedef struct {
    plyhit ph;
    frame fx;
    double Gp, Gf, mu_i, w[4];
    v3 x3;
    int K;
    fnode nd[ORC_MAX_NODES];
} xgeom;

static double frac(double x) { return x - floor(x); }

/* The hit at x: ply hit, fiber frame and the two shadowing terms. */
static void geom_hit(const orc_params* p, const double* tab, double h, double u, double v, v3 wi,
                     xgeom* g)
{
    memset(g, 0, sizeof(*g));
    trace_plies(p, h, u, v, wi, &g->ph);
    if (g->ph.pass) return;
    plyhit* ph = &g->ph;
    int ks = ph->kstar;
    double gft, a;
    fiber_frame(p, tab, ph->th[ks], ks, ph->n2[0], ph->n2[1], ph->vhit, &g->fx, &gft, &a);
    ph->a = a;
    g->x3 = mk(ph->p2[0], ph->p2[1], ph->vhit);

    /* shadowing: G_p from the ply horizon at the hit, G_f from the table */
    double phi = atan2(ph->n2[0] * wi.y - ph->n2[1] * wi.x, ph->n2[0] * wi.x + ph->n2[1] * wi.y);
    double gpr = orc_ply_shadow_raw(p, a, phi);
    g->Gp = 1.0 - p->ply_density * (1.0 - gpr);
    g->Gf = 1.0 - p->fiber_density * (1.0 - gft);
}

/* Everything else that depends on wi only, from the frame at x: lobe
 * weights and the forward quadrature nodes. */
static void geom_shade(const orc_params* p, const double* tab, v3 wi, const double* shift,
                       xgeom* g)
{
    if (g->ph.pass) return;
    plyhit* ph = &g->ph;
    int ks = ph->kstar;
    double ax = p->beta, ay = p->beta * p->aniso, eta = p->eta;
    g->mu_i = vdot(wi, g->fx.n);
    if (fabs(g->mu_i) < g_margin_shade) ph->flags |= ORC_NEARTIE;
    double PR = orc_fresnel(g->mu_i > 0.0 ? g->mu_i : 0.0, eta);
    g->w[0] = (1.0 - p->B) * PR;
    g->w[1] = (1.0 - p->B) * (1.0 - PR);
    g->w[2] = p->B * p->r;
    g->w[3] = p->B * (1.0 - p->r);

    /* forward quadrature nodes of the integral over exit points (Eq. 1) */
    int K = p->K;
    g->K = K;
    double sh0 = shift ? shift[0] : 0.0, sh1 = shift ? shift[1] : 0.0;
    double phig = 0.5 * (sqrt(5.0) - 1.0);
    for (int k = 0; k < K; ++k) {
        fnode* nd = &g->nd[k];
        if (g->mu_i <= 0.0) {
            ph->flags |= ORC_BACKFACING;
            nd->kind = 1;
            nd->T = 0.0;
            nd->att = 1.0;
            nd->fy.t = g->fx.t;
            nd->fy.n = vscl(g->fx.n, -1.0);
            nd->fy.b = vcross(nd->fy.n, nd->fy.t);
            nd->y = g->x3;
            continue;
        }
        double a1 = (k + 0.5) / K + sh0, a2 = (k + 0.5) * phig + sh1;
        if (shift && (fabs(a1 - floor(a1 + 0.5)) < g_margin_xi || fabs(a2 - floor(a2 + 0.5)) < g_margin_xi))
            ph->flags |= ORC_NEAR_LOBE_BOUNDARY;
        double xi1 = frac(a1), xi2 = frac(a2);
        v3 wl = to_local(&g->fx, wi);
        double ml[3], wla[3] = {wl.x, wl.y, wl.z};
        orc_vndf(wla, ax, ay, xi1, xi2, ml);
        v3 m = to_world(&g->fx, mk(ml[0], ml[1], ml[2]));
        double c = vdot(wi, m);
        if (c < 0.0) c = 0.0;
        double s2t = (1.0 - c * c) / (eta * eta);
        double ct = sqrt(1.0 - s2t);
        v3 wt = vadd(vscl(wi, -1.0 / eta), vscl(m, c / eta - ct));
        nd->wt = wt;
        nd->T = (1.0 - orc_fresnel(c, eta)) * G1_l(to_local(&g->fx, wt), mk(ml[0], ml[1], ml[2]), ax, ay);
        /* chord through the projected cross-section (the paper's
         * elliptical cross-section seen along the yarn axis) */
        double e2x = wt.x, e2y = wt.y;
        double le = sqrt(e2x * e2x + e2y * e2y);
        double en = e2x * ph->n2[0] + e2y * ph->n2[1];
        if (fabs(le - 1e-6) < g_margin_geo || fabs(en) < g_margin_geo * (le > 1e-6 ? le : 1e-6))
            ph->flags |= ORC_NEARTANGENT;
        if (le < 1e-6 || en >= 0.0) {
            nd->kind = 1;
            nd->att = 1.0;
            nd->fy.t = g->fx.t;
            nd->fy.n = vscl(g->fx.n, -1.0);
            nd->fy.b = vcross(nd->fy.n, nd->fy.t);
            nd->y = g->x3;
            continue;
        }
        double ex = e2x / le, ey = e2y / le;
        double bq = ph->p2[0] * ex + ph->p2[1] * ey;
        double cq = ph->p2[0] * ph->p2[0] + ph->p2[1] * ph->p2[1] - 1.0;
        double dq = bq * bq - cq;
        double syarn = -bq + sqrt(dq > 0.0 ? dq : 0.0);
        int Np = p->n_plies, N = 0, jL = -1;
        double sout[ORC_MAX_PLIES];
        int ent[ORC_MAX_PLIES];
        double rp = p->ply_radius;
        for (int j = 0; j < Np; ++j) {
            ent[j] = 0;
            if (j == ks) {
                double sx = -2.0 * rp * en / le;
                ent[j] = 1;
                sout[j] = sx < syarn ? sx : syarn;
                continue;
            }
            double wx = ph->p2[0] - ph->cst[j][0], wy = ph->p2[1] - ph->cst[j][1];
            double b = wx * ex + wy * ey;
            double cc = wx * wx + wy * wy - rp * rp;
            double disc = b * b - cc;
            double mg = g_margin_geo * (ph->amp[j] > 1.0 ? ph->amp[j] : 1.0);
            if (fabs(disc) < mg * rp * rp) ph->flags |= ORC_NEARTANGENT;
            if (disc <= 0.0) continue;
            double sq = sqrt(disc);
            double slo = -b - sq, shi = -b + sq;
            if (fabs(shi) < mg || fabs(slo - syarn) < mg) ph->flags |= ORC_NEARTANGENT;
            if (shi > 0.0 && slo < syarn) {
                ent[j] = 1;
                sout[j] = shi < syarn ? shi : syarn;
                if (fabs(shi - syarn) < mg) ph->flags |= ORC_NEARTANGENT;
            }
        }
        for (int j = 0; j < Np; ++j) {
            if (!ent[j]) continue;
            ++N;
            if (jL < 0 || sout[j] > sout[jL]) jL = j;
        }
        for (int j = 0; j < Np; ++j) {
            if (!ent[j] || j == jL) continue;
            double mg = g_margin_geo * (ph->amp[j] > ph->amp[jL] ? ph->amp[j] : ph->amp[jL]);
            if (fabs(sout[j] - sout[jL]) < (mg > g_margin_geo ? mg : g_margin_geo)) ph->flags |= ORC_NEARTANGENT;
        }
        double so = sout[jL];
        double y2x = ph->p2[0] + so * ex, y2y = ph->p2[1] + so * ey;
        double ell = so / le;
        double zy = ph->vhit + wt.z * ell;
        double nyx = y2x - ph->cst[jL][0], nyy = y2y - ph->cst[jL][1];
        double nyl = sqrt(nyx * nyx + nyy * nyy);
        nd->kind = 0;
        nd->N = N;
        nd->ell = ell;
        nd->att = exp(-p->sigma_t * ell * N);
        fiber_frame(p, tab, ph->th[jL], jL, nyx / nyl, nyy / nyl, zy, &nd->fy, NULL, NULL);
        nd->y = mk(y2x, y2y, zy);
    }
}

static void geom_x(const orc_params* p, const double* tab, double h, double u, double v,
                   v3 wi, const double* shift, xgeom* g)
{
    geom_hit(p, tab, h, u, v, wi, g);
    geom_shade(p, tab, wi, shift, g);
}

/* ------------------------------------------------------------------ */
/* lobes and pdf for one wo (Eq. 1-6, Sec. 4.1.5)                      */
/* ------------------------------------------------------------------ */

/* Exit refraction at y of node k: Walter's BTDF from inside (index eta)
 * to outside, for wi' = -wt.  Returns f_t * |wo.n_y| in *val and the
 * solid-angle pdf of sampling wo through that node in *pdf. */
static void exit_btdf(const orc_params* p, const fnode* nd, v3 wo, double* val, double* pdf,
                      uint32_t* flags)
{
    *val = 0.0;
    *pdf = 0.0;
    double ax = p->beta, ay = p->beta * p->aniso, eta = p->eta;
    v3 wip = vscl(nd->wt, -1.0);
    double ci = vdot(wip, nd->fy.n), co = vdot(wo, nd->fy.n);
    if (!(ci < 0.0 && co > 0.0)) return;
    v3 mh = vscl(vadd(vscl(wip, eta), wo), -1.0);
    double ml = vlen(mh);
    if (ml == 0.0) return;
    mh = vscl(mh, 1.0 / ml);
    if (vdot(mh, nd->fy.n) < 0.0) mh = vscl(mh, -1.0);
    double im = vdot(wip, mh), om = vdot(wo, mh);
    if (!(im < 0.0 && om > 0.0)) return;
    double den = eta * im + om;
    /* near the critical angle the transmittance falls like the cosine of
     * the transmitted angle, whose derivative is unbounded */
    double s2t_in = eta * eta * (1.0 - im * im);
    if (1.0 - s2t_in < g_margin_tir) *flags |= ORC_NEAR_TIR;
    v3 ml3 = to_local(&nd->fy, mh);
    double D = D_l(ml3, ax, ay);
    double g1i = G1_l(to_local(&nd->fy, wip), ml3, ax, ay);
    double g1o = G1_l(to_local(&nd->fy, wo), ml3, ax, ay);
    double F = orc_fresnel(-im, 1.0 / eta);
    double jac = fabs(om) / (den * den);
    *val = fabs(im) * (1.0 - F) * g1i * g1o * D * jac / fabs(ci);
    *pdf = g1i * fabs(im) * D / fabs(ci) * jac;
}

/* The implicit ply hit with the ply's own frame (Sec. 3.4), for the
 * cross-section study.  out: pass, ply, hit point (x, y, v), ply tangent
 * (3, derivative of the centre helix), ply normal (3, the 2D outward normal
 * made orthogonal to the tangent). */
uint32_t orc_ply_frame(const orc_params* p, double h, double u, double v, const double wi[3],
                       double out[11])
{
    plyhit g;
    for (int i = 0; i < 11; ++i) out[i] = 0.0;
    trace_plies(p, h, u, v, mk(wi[0], wi[1], wi[2]), &g);
    out[0] = g.pass;
    out[1] = -1;
    if (g.pass) return g.flags;
    int k = g.kstar;
    double slope = p->ply_center_radius * helix_rate(p);
    double chx = cos(g.th[k]), chy = sin(g.th[k]);
    v3 tp = vnorm(mk(-slope * chy, slope * chx, 1.0));
    v3 n23 = mk(g.n2[0], g.n2[1], 0.0);
    v3 np = vnorm(vsub(n23, vscl(tp, vdot(n23, tp))));
    out[1] = k;
    out[2] = g.p2[0]; out[3] = g.p2[1]; out[4] = g.vhit;
    out[5] = tp.x; out[6] = tp.y; out[7] = tp.z;
    out[8] = np.x; out[9] = np.y; out[10] = np.z;
    return g.flags;
}

/* Explicit helical plies around a yarn whose centreline is a circular arc
 * of curvature kappa (per yarn radius; 0: straight), the reference of the
 * cross-section study.  Coordinates are the query frame at the yarn hit
 * (N, T x N, T) = (x, y, z).  The centreline bends towards +x:
 * c(s) = ((1 - cos ks)/k, 0, sin(ks)/k), T(s) = (sin ks, 0, cos ks),
 * N(s) = (cos ks, 0, -sin ks), B = y (the rotation-minimising frame of a
 * planar arc).  Ply j's centre at arc length s is
 * c(s) + R_pc (cos th N(s) + sin th B), th = u + 2 pi j / N_p + w_p (v + s),
 * and the ply is the disc of radius r_p about it in the plane normal to
 * T(s).  The ray enters the unit yarn tube at x2 (the query's hit, in the
 * cross-section at s = 0) going along -wi; a point belongs to the cross
 * section of its nearest centreline point.  The first point inside a ply
 * (marching by `step`, then bisection) is the hit.  out: ply (-1: none),
 * hit point (3), unit tangent of the ply's centre curve there (3).
 * Returns 0 when the ray meets the tube before x2 (x2 is then not the yarn
 * hit), else 1. */
static void arc_section(double kappa, const double q[3], double* s, double c[3], double N[3])
{
    if (kappa == 0.0) {
        *s = q[2];
        c[0] = 0.0; c[1] = 0.0; c[2] = q[2];
        N[0] = 1.0; N[1] = 0.0; N[2] = 0.0;
        return;
    }
    double rc = 1.0 / kappa;
    double a = atan2(q[2], rc - q[0]);
    *s = a * rc;
    c[0] = rc * (1.0 - cos(a)); c[1] = 0.0; c[2] = rc * sin(a);
    N[0] = cos(a); N[1] = 0.0; N[2] = -sin(a);
}

/* -1: outside the tube, otherwise the index of a ply containing q, or
 * `n_plies` when inside the tube but in no ply */
static int explicit_inside(const orc_params* p, double kappa, double u, double v, const double q[3])
{
    double s, c[3], N[3];
    arc_section(kappa, q, &s, c, N);
    double d[3] = {q[0] - c[0], q[1] - c[1], q[2] - c[2]};
    double x = d[0] * N[0] + d[1] * N[1] + d[2] * N[2], y = d[1];
    if (x * x + y * y > 1.0) return -1;
    double wp = helix_rate(p), rp = p->ply_radius, Rpc = p->ply_center_radius;
    for (int j = 0; j < p->n_plies; ++j) {
        double th = u + TWO_PI * j / p->n_plies + wp * (v + s);
        double ex = x - Rpc * cos(th), ey = y - Rpc * sin(th);
        if (ex * ex + ey * ey <= rp * rp) return j;
    }
    return p->n_plies;
}

int orc_explicit_ply(const orc_params* p, double kappa, double h, double u, double v,
                     const double wi[3], double step, double out[7])
{
    for (int i = 0; i < 7; ++i) out[i] = 0.0;
    out[0] = -1;
    double sxy = sqrt(wi[0] * wi[0] + wi[1] * wi[1]);
    if (!(sxy > 1e-9)) return 0;
    double cx = wi[0] / sxy, cy = wi[1] / sxy, g = asin(h);
    double x2[3] = {cx * cos(g) - cy * sin(g), cy * cos(g) + cx * sin(g), 0.0};
    /* nothing of the tube before x2 along the ray */
    for (double t = step; t < 4.0; t += step) {
        double q[3] = {x2[0] + t * wi[0], x2[1] + t * wi[1], x2[2] + t * wi[2]};
        if (explicit_inside(p, kappa, u, v, q) >= 0) return 0;
    }
    double tmax = 2.5 / sxy, tprev = 0.0;
    for (double t = 0.0; t <= tmax; t += step) {
        double q[3] = {x2[0] - t * wi[0], x2[1] - t * wi[1], x2[2] - t * wi[2]};
        int j = explicit_inside(p, kappa, u, v, q);
        if (j >= 0 && j < p->n_plies) {
            double lo = tprev, hi = t;
            for (int it = 0; it < 40; ++it) {
                double mid = 0.5 * (lo + hi);
                double qm[3] = {x2[0] - mid * wi[0], x2[1] - mid * wi[1], x2[2] - mid * wi[2]};
                int jm = explicit_inside(p, kappa, u, v, qm);
                if (jm >= 0 && jm < p->n_plies) hi = mid; else lo = mid;
            }
            double qh[3] = {x2[0] - hi * wi[0], x2[1] - hi * wi[1], x2[2] - hi * wi[2]};
            j = explicit_inside(p, kappa, u, v, qh);
            double s, c[3], N[3];
            arc_section(kappa, qh, &s, c, N);
            double T[3] = {kappa == 0.0 ? 0.0 : sin(kappa * s), 0.0, kappa == 0.0 ? 1.0 : cos(kappa * s)};
            double wp = helix_rate(p), Rpc = p->ply_center_radius;
            double th = u + TWO_PI * j / p->n_plies + wp * (v + s);
            /* d/ds of c + R_pc (cos th N + sin th B), with dN/ds = -kappa T */
            double a = 1.0 - kappa * Rpc * cos(th), bn = -Rpc * wp * sin(th), bb = Rpc * wp * cos(th);
            double tg[3] = {a * T[0] + bn * N[0], bb, a * T[2] + bn * N[2]};
            double l = sqrt(tg[0] * tg[0] + tg[1] * tg[1] + tg[2] * tg[2]);
            out[0] = j;
            out[1] = qh[0]; out[2] = qh[1]; out[3] = qh[2];
            out[4] = tg[0] / l; out[5] = tg[1] / l; out[6] = tg[2] / l;
            return 1;
        }
        if (j < 0 && t > 2.0 * step) break; /* left the tube */
        tprev = t;
    }
    return 1;
}

static void lobes(const orc_params* p, const xgeom* g, v3 wi, v3 wo, double out[13],
                  uint32_t* flags)
{
    for (int i = 0; i < 13; ++i) out[i] = 0.0;
    if (g->ph.pass) return;
    double ax = p->beta, ay = p->beta * p->aniso, eta = p->eta;
    double mu_i = g->mu_i, mu_o = vdot(wo, g->fx.n);
    if (fabs(mu_o) < g_margin_shade) *flags |= ORC_NEARTIE;
    double ExS = 0.0, pxS = 0.0;
    if (mu_i > 0.0 && mu_o > 0.0) {
        v3 hv = vnorm(vadd(wi, wo));
        v3 hl = to_local(&g->fx, hv);
        double D = D_l(hl, ax, ay);
        double g1i = G1_l(to_local(&g->fx, wi), hl, ax, ay);
        double g1o = G1_l(to_local(&g->fx, wo), hl, ax, ay);
        double ih = vdot(wi, hv), oh = vdot(wo, hv);
        ExS = (1.0 - p->B) * p->k_spec * orc_fresnel(ih, eta) * g1i * g1o * D / (4.0 * mu_i);
        if (oh > 0.0) pxS = g1i * (ih > 0.0 ? ih : 0.0) * D / mu_i / (4.0 * oh);
    }
    double bx = 0.0, pxB = 0.0;
    if (mu_o > 0.0) {
        double mp = mu_i > 0.0 ? mu_i : 0.0;
        double fls = 1.0 / (4.0 * PI * (mp + mu_o));
        bx = p->B * p->r * g->Gp * g->Gf * (fls + 1.0 / PI) * mu_o / (1.0 + orc_ls_albedo(mp));
        pxB = mu_o / PI;
    }
    double EyS = 0.0, pyS = 0.0, by = 0.0, pyB = 0.0;
    for (int k = 0; k < g->K; ++k) {
        const fnode* nd = &g->nd[k];
        double cy = vdot(wo, nd->fy.n);
        if (cy > 0.0) { by += cy / PI; pyB += cy / PI; }
        if (mu_i > 0.0) {
            double val, pd;
            exit_btdf(p, nd, wo, &val, &pd, flags);
            EyS += nd->T * nd->att * val;
            pyS += pd;
        }
    }
    EyS *= (1.0 - p->B) * p->k_spec / g->K;
    pyS /= g->K;
    by *= p->B * (1.0 - p->r) * g->Gp * g->Gf / g->K;
    pyB /= g->K;
    out[3] = ExS;
    out[4] = EyS;
    for (int c = 0; c < 3; ++c) {
        out[5 + c] = bx * p->albedo[c];
        out[8 + c] = by * p->albedo[c];
        out[c] = ExS + EyS + out[5 + c] + out[8 + c];
    }
    out[11] = g->w[0] * pxS + g->w[1] * pyS + g->w[2] * pxB + g->w[3] * pyB;
}

/* ------------------------------------------------------------------ */
/* per-query drivers                                                   */
/* ------------------------------------------------------------------ */

static uint32_t check_dir(v3 w)
{
    if (!isfinite(w.x) || !isfinite(w.y) || !isfinite(w.z)) return ORC_BAD_INPUT;
    if (fabs(vlen(w) - 1.0) > 1e-3) return ORC_BAD_INPUT;
    return 0;
}

static int valid_type(int32_t t, int32_t n_types) { return t >= 0 && t < n_types; }

static void eval_one(const orc_params* p, const double* tab, double h, double u, double v,
                     v3 wi, v3 wo, const double* shift, double out[13], uint32_t* fl)
{
    uint32_t bad = check_dir(wi) | check_dir(wo);
    if (!isfinite(h) || fabs(h) > 1.0 || !isfinite(u) || !isfinite(v)) bad |= ORC_BAD_INPUT;
    if (bad) {
        for (int i = 0; i < 13; ++i) out[i] = 0.0;
        *fl = bad;
        return;
    }
    xgeom g;
    geom_x(p, tab, h, u, v, wi, shift, &g);
    uint32_t f = g.ph.flags;
    lobes(p, &g, wi, wo, out, &f);
    *fl = f;
}

#define Q_H(i) ((double)h[i])
#define Q_WI(i) mk(wi[i], wi[n + (i)], wi[2 * n + (i)])
#define Q_WO(i) mk(wo[i], wo[n + (i)], wo[2 * n + (i)])

int orc_eval(const orc_params* types, const double* const* tables, int32_t n_types,
             int64_t n, const int32_t* type, const float* h, const float* u, const float* v,
             const float* wi, const float* wo, const float* shift, double* out_eval,
             uint32_t* flags, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int32_t t = type[i];
        if (!valid_type(t, n_types)) {
            for (int c = 0; c < 13; ++c) out_eval[13 * i + c] = 0.0;
            flags[i] = ORC_BAD_INPUT;
            continue;
        }
        double sh[2];
        if (shift) { sh[0] = shift[i]; sh[1] = shift[n + i]; }
        eval_one(&types[t], tables[t], Q_H(i), u[i], v[i], Q_WI(i), Q_WO(i),
                 shift ? sh : NULL, &out_eval[13 * i], &flags[i]);
    }
    return 0;
}


/* One query of eval (single type, its table): out[13] as orc_eval. */
uint32_t orc_eval_query(const orc_params* p, const double* tab, double h, double u, double v,
                        const double wi[3], const double wo[3], double out[13])
{
    uint32_t f;
    eval_one(p, tab, h, u, v, mk(wi[0], wi[1], wi[2]), mk(wo[0], wo[1], wo[2]), NULL, out, &f);
    return f;
}

/* Draw one direction (Sec. 4.1.5): pick a lobe with the energy weights,
 * then GGX visible normals for the specular lobes and a cosine lobe for
 * the body lobes; the forward lobes also pick one quadrature node.
 * out: wo(3) weight(3) pdf exit(3) lobe node.  Lobes: 0 x-specular,
 * 1 y-specular, 2 x-body, 3 y-body, 4 pass-through. */
static int draw_from(const orc_params* p, const xgeom* gp, v3 wi, const double xi[3], v3* wo_out,
                     double out[12], uint32_t* fl);

static void sample_one(const orc_params* p, const double* tab, double h, double u, double v,
                       v3 wi, const double xi[3], const double* shift, double out[12],
                       uint32_t* fl)
{
    for (int i = 0; i < 12; ++i) out[i] = 0.0;
    uint32_t bad = check_dir(wi);
    if (!isfinite(h) || fabs(h) > 1.0 || !isfinite(u) || !isfinite(v)) bad |= ORC_BAD_INPUT;
    if (bad) { *fl = bad; out[10] = -1; return; }
    xgeom g;
    geom_x(p, tab, h, u, v, wi, shift, &g);
    uint32_t f = g.ph.flags;
    if (g.ph.pass) {
        /* no ply hit: the ray continues through the yarn unchanged */
        out[0] = -wi.x; out[1] = -wi.y; out[2] = -wi.z;
        out[3] = out[4] = out[5] = 1.0;
        out[10] = 4;
        *fl = f;
        return;
    }
    v3 wo;
    if (!draw_from(p, &g, wi, xi, &wo, out, &f)) { *fl = f | ORC_SAMPLE_FAIL; return; }
    double e[13];
    lobes(p, &g, wi, wo, e, &f);
    double pdf = e[11];
    if (!(pdf > 0.0)) { *fl = f | ORC_SAMPLE_FAIL; return; }
    out[0] = wo.x; out[1] = wo.y; out[2] = wo.z;
    for (int c = 0; c < 3; ++c) out[3 + c] = e[c] / pdf;
    out[6] = pdf;
    *fl = f;
}

/* The draw of sample_one from the state at x of a hit (not a
 * pass-through): lobe and node from xi[0], the direction from xi[1],
 * xi[2].  Sets the exit point, lobe and node in out[7..11] and returns 1
 * with the unit direction in *wo_out, or 0 when no valid direction. */
static int draw_from(const orc_params* p, const xgeom* gp, v3 wi, const double xi[3], v3* wo_out,
                     double out[12], uint32_t* fl)
{
    const xgeom g = *gp;
    uint32_t f = *fl;
    double ax = p->beta, ay = p->beta * p->aniso, eta = p->eta;
    double cum[3];
    cum[0] = g.w[0];
    cum[1] = cum[0] + g.w[1];
    cum[2] = cum[1] + g.w[2];
    int lobe = 3;
    for (int l = 0; l < 3; ++l)
        if (xi[0] < cum[l]) { lobe = l; break; }
    for (int l = 0; l < 3; ++l)
        if (fabs(xi[0] - cum[l]) < g_margin_xi) f |= ORC_NEAR_LOBE_BOUNDARY;
    int node = 0;
    if (lobe == 1 || lobe == 3) {
        double lo = cum[lobe - 1];
        double xk = (xi[0] - lo) / g.w[lobe] * g.K;
        node = (int)floor(xk);
        if (node > g.K - 1) node = g.K - 1;
        if (node < 0) node = 0;
        double nearest = floor(xk + 0.5);
        if (nearest > 0.0 && nearest < g.K && fabs(xk - nearest) < g_margin_xi * g.K / g.w[lobe])
            f |= ORC_NEAR_LOBE_BOUNDARY;
    }
    v3 wo = mk(0, 0, 0);
    int ok = 0;
    if (lobe == 0) {
        v3 wl = to_local(&g.fx, wi);
        if (wl.z > 0.0) {
            double ml[3], wla[3] = {wl.x, wl.y, wl.z};
            orc_vndf(wla, ax, ay, xi[1], xi[2], ml);
            v3 m = to_world(&g.fx, mk(ml[0], ml[1], ml[2]));
            wo = vsub(vscl(m, 2.0 * vdot(wi, m)), wi);
            double mo = vdot(wo, g.fx.n);
            if (fabs(mo) < g_margin_shade) f |= ORC_NEARTIE;
            ok = mo > 0.0;
        }
    } else if (lobe == 1) {
        const fnode* nd = &g.nd[node];
        v3 wip = vscl(nd->wt, -1.0);
        frame fi; /* inside-facing frame at y */
        fi.t = nd->fy.t;
        fi.n = vscl(nd->fy.n, -1.0);
        fi.b = vcross(fi.n, fi.t);
        v3 wl = to_local(&fi, wip);
        if (fabs(wl.z) < g_margin_shade) f |= ORC_NEARTIE;
        if (wl.z > 0.0 && g.mu_i > 0.0) {
            double ml[3], wla[3] = {wl.x, wl.y, wl.z};
            orc_vndf(wla, ax, ay, xi[1], xi[2], ml);
            v3 m = to_world(&fi, mk(ml[0], ml[1], ml[2]));
            double c = vdot(wip, m);
            if (c < 0.0) c = 0.0;
            double s2t = eta * eta * (1.0 - c * c);
            if (fabs(1.0 - s2t) < g_margin_tir) f |= ORC_NEAR_TIR;
            if (s2t < 1.0) {
                double ct = sqrt(1.0 - s2t);
                wo = vadd(vscl(wip, -eta), vscl(m, eta * c - ct));
                double co = vdot(wo, nd->fy.n);
                if (fabs(co) < g_margin_shade) f |= ORC_NEARTIE;
                ok = co > 0.0;
            }
        }
    } else {
        const frame* fr = lobe == 2 ? &g.fx : &g.nd[node].fy;
        double rad = sqrt(xi[1]), ph = TWO_PI * xi[2];
        double z = 1.0 - xi[1];
        wo = to_world(fr, mk(rad * cos(ph), rad * sin(ph), sqrt(z > 0.0 ? z : 0.0)));
        ok = 1;
    }
    v3 ex = (lobe == 1 || lobe == 3) ? g.nd[node].y : g.x3;
    out[7] = ex.x; out[8] = ex.y; out[9] = ex.z;
    out[10] = lobe;
    out[11] = node;
    *fl = f;
    if (!ok) return 0;
    *wo_out = vnorm(wo);
    return 1;
}

/* One query of the sampler (single type, its table): out[12] as orc_sample. */
uint32_t orc_sample_query(const orc_params* p, const double* tab, double h, double u, double v,
                          const double wi[3], const double xi[3], double out[12])
{
    uint32_t f;
    sample_one(p, tab, h, u, v, mk(wi[0], wi[1], wi[2]), xi, NULL, out, &f);
    return f;
}

int orc_sample(const orc_params* types, const double* const* tables, int32_t n_types,
               int64_t n, const int32_t* type, const float* h, const float* u, const float* v,
               const float* wi, const float* xi, const float* shift, double* out,
               uint32_t* flags, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int32_t t = type[i];
        if (!valid_type(t, n_types)) {
            for (int c = 0; c < 12; ++c) out[12 * i + c] = 0.0;
            out[12 * i + 10] = -1;
            flags[i] = ORC_BAD_INPUT;
            continue;
        }
        double x3[3] = {xi[i], xi[n + i], xi[2 * n + i]};
        double sh[2];
        if (shift) { sh[0] = shift[i]; sh[1] = shift[n + i]; }
        sample_one(&types[t], tables[t], Q_H(i), u[i], v[i], Q_WI(i), x3, shift ? sh : NULL,
                   &out[12 * i], &flags[i]);
    }
    return 0;
}

/* White furnace per block (Sec. 4.3): mean and sample variance of the
 * sampling weights E/pdf of `block` draws for the block's first query. */
int orc_furnace(const orc_params* types, const double* const* tables, int32_t n_types,
                int64_t n, int32_t block, const int32_t* type, const float* h,
                const float* u, const float* v, const float* wi, const float* xi,
                const float* shift, double* mean, double* var, int nthreads)
{
    if (block < 2) return -1;
    int64_t nb = n / block;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t b = 0; b < nb; ++b) {
        int64_t q0 = b * block;
        int32_t t = type[q0];
        double s[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
        double sh[2];
        if (shift) { sh[0] = shift[q0]; sh[1] = shift[n + q0]; }
        double wts[3 * 1024];
        double* w = block <= 1024 ? wts : (double*)malloc(sizeof(double) * 3 * block);
        for (int j = 0; j < block; ++j) {
            int64_t q = q0 + j;
            double x3[3] = {xi[q], xi[n + q], xi[2 * n + q]};
            double o[12];
            uint32_t fl = 0;
            if (valid_type(t, n_types))
                sample_one(&types[t], tables[t], Q_H(q0), u[q0], v[q0], Q_WI(q0), x3,
                           shift ? sh : NULL, o, &fl);
            else
                memset(o, 0, sizeof(o));
            for (int c = 0; c < 3; ++c) {
                w[3 * j + c] = o[3 + c];
                s[c] += o[3 + c];
            }
        }
        for (int c = 0; c < 3; ++c) {
            double m = s[c] / block;
            for (int j = 0; j < block; ++j) {
                double d = w[3 * j + c] - m;
                s2[c] += d * d;
            }
            mean[3 * b + c] = m;
            var[3 * b + c] = s2[c] / (block - 1);
        }
        if (w != wts) free(w);
    }
    return 0;
}

/* Far field (Eq. 7) with W = 1 and N_h stratified offsets. */
int orc_eval_far(const orc_params* types, const double* const* tables, int32_t n_types,
                 int64_t n, int32_t n_h, double zeta, const int32_t* type, const float* u,
                 const float* v, const float* wi, const float* wo, double* out_E, int nthreads)
{
    if (n_h < 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int32_t t = type[i];
        double acc[3] = {0, 0, 0};
        if (valid_type(t, n_types)) {
            for (int j = 0; j < n_h; ++j) {
                double hj = -1.0 + 2.0 * (j + zeta) / n_h;
                double o[13];
                uint32_t fl;
                eval_one(&types[t], tables[t], hj, u[i], v[i], Q_WI(i), Q_WO(i), NULL, o, &fl);
                for (int c = 0; c < 3; ++c) acc[c] += o[c];
            }
        }
        for (int c = 0; c < 3; ++c) out_E[3 * i + c] = acc[c] / n_h;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* multi-scale BYSDF (Sec. 4.2, Eq. 8-11; footprint as in Sec. 5.3)    */
/* ------------------------------------------------------------------ */

/* The pixel footprint on the yarn: offsets h1 <= h0 <= h2 from the ray
 * differentials, n strata of [h1, h2] at the shared offset zeta, each with
 * the weight W of a tent that is 1 at h0 and 0 at h1 and h2 (the weight
 * falls with the distance to h0).  The number of strata grows with the
 * covered share of the yarn, n = ceil(n_max (h2 - h1) / 2) in [1, n_max];
 * a single stratum carries weight 1.  Stratum offsets are rounded to FP32,
 * the precision of a query's h. */
typedef struct {
    int n;
    double h[ORC_MAX_STRATA], w[ORC_MAX_STRATA];
    double wsum;
} footprint;

static int footprint_make(double h0, double h1, double h2, double zeta, int n_max, footprint* fp)
{
    if (!(h1 >= -1.0 && h1 <= h0 && h0 <= h2 && h2 <= 1.0) || !(zeta >= 0.0 && zeta < 1.0))
        return -1;
    int n = (int)ceil(n_max * (h2 - h1) * 0.5);
    n = n < 1 ? 1 : (n > n_max ? n_max : n);
    fp->n = n;
    fp->wsum = 0.0;
    for (int j = 0; j < n; ++j) {
        double hj = (double)(float)fma(h2 - h1, (j + zeta) / n, h1);
        double w = 1.0;
        if (n > 1) {
            if (hj < h0)
                w = 1.0 - (h0 - hj) / (h0 - h1);
            else if (h2 > h0)
                w = 1.0 - (hj - h0) / (h2 - h0);
        }
        fp->h[j] = hj;
        fp->w[j] = w;
        fp->wsum += w;
    }
    return 0;
}

/* Aggregated geometry of the footprint (Eq. 9-11): the W-weighted means of
 * the fiber normal, the fiber tangent and the fiber shadowing G_f over the
 * strata that hit a ply.  The mean normal is normalised, the mean tangent
 * made orthogonal to it and normalised; a single contributing stratum
 * keeps its own frame.  Returns 0 when no stratum of positive weight hits
 * a ply. */
static int footprint_geometry(const orc_params* p, const double* tab, double u, double v, v3 wi,
                              const footprint* fp, frame* F, double* Gm, uint32_t* flags)
{
    v3 sn = mk(0, 0, 0), st = mk(0, 0, 0);
    double sg = 0.0, sw = 0.0;
    frame first;
    int have = 0;
    double g1 = 0.0;
    for (int j = 0; j < fp->n; ++j) {
        xgeom g;
        geom_hit(p, tab, fp->h[j], u, v, wi, &g);
        *flags |= g.ph.flags & ~ORC_PASS_THROUGH;
        if (g.ph.pass || !(fp->w[j] > 0.0)) continue;
        sn = vadd(sn, vscl(g.fx.n, fp->w[j]));
        st = vadd(st, vscl(g.fx.t, fp->w[j]));
        sg += fp->w[j] * g.Gf;
        sw += fp->w[j];
        if (!have) { first = g.fx; g1 = g.Gf; }
        ++have;
    }
    if (!have) return 0;
    if (have == 1) {
        /* one stratum: its own frame and shadowing, unrounded */
        *F = first;
        *Gm = g1;
        return 1;
    }
    *Gm = sg / sw;
    double ln = vlen(sn);
    if (ln < 1e-6 * sw) *flags |= ORC_ILLCOND;
    if (!(ln > 1e-12 * sw)) {
        *F = first;
        return 1;
    }
    v3 n = vscl(sn, 1.0 / ln);
    v3 t = vsub(st, vscl(n, vdot(st, n)));
    double lt = vlen(t);
    if (lt < 1e-6 * sw) *flags |= ORC_ILLCOND;
    if (!(lt > 1e-12 * sw)) {
        *F = first;
        return 1;
    }
    F->n = n;
    F->t = vscl(t, 1.0 / lt);
    F->b = vcross(F->n, F->t);
    return 1;
}

/* The near-field model at one stratum with the footprint's aggregated
 * frame, shadowing and roughness (Eq. 8 integrand): the ply hit and the
 * chords through the plies are the stratum's own. */
static int stratum_state(const orc_params* pm, const double* tab, double hj, double u, double v,
                         v3 wi, const frame* F, double Gm, const double* shift, xgeom* g,
                         uint32_t* flags)
{
    geom_hit(pm, tab, hj, u, v, wi, g);
    if (g->ph.pass) return 0;
    g->fx = *F;
    g->Gf = Gm;
    geom_shade(pm, tab, wi, shift, g);
    *flags |= g->ph.flags & ~ORC_PASS_THROUGH;
    return 1;
}

static int footprint_inputs_ok(double h0, double h1, double h2, double zeta)
{
    return isfinite(h1) && isfinite(h2) && isfinite(zeta) && h1 >= -1.0 && h1 <= h0 && h0 <= h2 &&
           h2 <= 1.0 && zeta >= 0.0 && zeta < 1.0;
}

/* f_multi of Eq. 8 at wo with the tent weights: out[13] as eval_one, each
 * entry the W-weighted mean over the strata (pass-through strata count
 * with value 0).  The specular roughness is beta_multi = beta + (h2 - h1)/2
 * along the fiber (the linear widening of Sec. 4.2 normalised by the
 * full-range C = 2 of the far field). */
static void eval_multi_one(const orc_params* p, const double* tab, double h0, double h1,
                           double h2, double zeta, int n_max, double u, double v, v3 wi, v3 wo,
                           const double* shift, double out[13], uint32_t* fl)
{
    for (int i = 0; i < 13; ++i) out[i] = 0.0;
    uint32_t bad = check_dir(wi) | check_dir(wo);
    if (!isfinite(h0) || !isfinite(u) || !isfinite(v) || !footprint_inputs_ok(h0, h1, h2, zeta))
        bad |= ORC_BAD_INPUT;
    if (bad) { *fl = bad; return; }
    footprint fp;
    footprint_make(h0, h1, h2, zeta, n_max, &fp);
    orc_params pm = *p;
    pm.beta = p->beta + (h2 - h1) * 0.5;
    uint32_t f = 0;
    frame F;
    double Gm;
    if (!footprint_geometry(&pm, tab, u, v, wi, &fp, &F, &Gm, &f)) {
        *fl = f | ORC_PASS_THROUGH;
        return;
    }
    for (int j = 0; j < fp.n; ++j) {
        xgeom g;
        if (!stratum_state(&pm, tab, fp.h[j], u, v, wi, &F, Gm, shift, &g, &f)) continue;
        double e[13];
        lobes(&pm, &g, wi, wo, e, &f);
        for (int i = 0; i < 12; ++i) out[i] += fp.w[j] * e[i];
    }
    for (int i = 0; i < 12; ++i) out[i] /= fp.wsum;
    *fl = f;
}

/* The multi-scale sampler: a stratum drawn with probability W / sum W from
 * xi_s, a pass-through stratum passes the ray through (lobe 4), otherwise
 * the stratum's aggregated state draws the direction as sample_one does,
 * and the weight and pdf are those of f_multi at it.  out[13]: wo(3)
 * weight(3) pdf exit(3) lobe node stratum. */
static void sample_multi_one(const orc_params* p, const double* tab, double h0, double h1,
                             double h2, double zeta, double xis, int n_max, double u, double v,
                             v3 wi, const double xi[3], const double* shift, double out[13],
                             uint32_t* fl)
{
    for (int i = 0; i < 13; ++i) out[i] = 0.0;
    uint32_t bad = check_dir(wi);
    if (!isfinite(h0) || !isfinite(u) || !isfinite(v) || !footprint_inputs_ok(h0, h1, h2, zeta) ||
        !(xis >= 0.0 && xis < 1.0))
        bad |= ORC_BAD_INPUT;
    if (bad) { *fl = bad; out[10] = -1; return; }
    footprint fp;
    footprint_make(h0, h1, h2, zeta, n_max, &fp);
    orc_params pm = *p;
    pm.beta = p->beta + (h2 - h1) * 0.5;
    uint32_t f = 0;
    /* the stratum */
    int s = fp.n - 1;
    double cum = 0.0, xw = xis * fp.wsum;
    for (int j = 0; j < fp.n; ++j) {
        cum += fp.w[j];
        if (j < fp.n - 1 && fabs(xw - cum) < g_margin_xi * fp.wsum) f |= ORC_NEAR_LOBE_BOUNDARY;
        if (xw < cum) { s = j; break; }
    }
    out[12] = s;
    frame F;
    double Gm;
    int any = footprint_geometry(&pm, tab, u, v, wi, &fp, &F, &Gm, &f);
    xgeom g;
    if (!any || !stratum_state(&pm, tab, fp.h[s], u, v, wi, &F, Gm, shift, &g, &f)) {
        out[0] = -wi.x; out[1] = -wi.y; out[2] = -wi.z;
        out[3] = out[4] = out[5] = 1.0;
        out[10] = 4;
        *fl = f | ORC_PASS_THROUGH;
        return;
    }
    v3 wo;
    if (!draw_from(&pm, &g, wi, xi, &wo, out, &f)) { *fl = f | ORC_SAMPLE_FAIL; return; }
    double E[3] = {0, 0, 0}, pdf = 0.0;
    for (int j = 0; j < fp.n; ++j) {
        xgeom gj;
        if (!stratum_state(&pm, tab, fp.h[j], u, v, wi, &F, Gm, shift, &gj, &f)) continue;
        double e[13];
        lobes(&pm, &gj, wi, wo, e, &f);
        for (int c = 0; c < 3; ++c) E[c] += fp.w[j] * e[c];
        pdf += fp.w[j] * e[11];
    }
    for (int c = 0; c < 3; ++c) E[c] /= fp.wsum;
    pdf /= fp.wsum;
    if (!(pdf > 0.0)) { *fl = f | ORC_SAMPLE_FAIL; return; }
    out[0] = wo.x; out[1] = wo.y; out[2] = wo.z;
    for (int c = 0; c < 3; ++c) out[3 + c] = E[c] / pdf;
    out[6] = pdf;
    *fl = f;
}

int orc_eval_multi(const orc_params* types, const double* const* tables, int32_t n_types,
                   int64_t n, int32_t n_max, const int32_t* type, const float* h, const float* h1,
                   const float* h2, const float* zeta, const float* u, const float* v,
                   const float* wi, const float* wo, const float* shift, double* out,
                   uint32_t* flags, int nthreads)
{
    if (n_max < 1 || n_max > ORC_MAX_STRATA) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int32_t t = type[i];
        if (!valid_type(t, n_types)) {
            for (int c = 0; c < 13; ++c) out[13 * i + c] = 0.0;
            flags[i] = ORC_BAD_INPUT;
            continue;
        }
        double sh[2];
        if (shift) { sh[0] = shift[i]; sh[1] = shift[n + i]; }
        eval_multi_one(&types[t], tables[t], h[i], h1[i], h2[i], zeta[i], n_max, u[i], v[i], Q_WI(i),
                       Q_WO(i), shift ? sh : NULL, &out[13 * i], &flags[i]);
    }
    return 0;
}

int orc_sample_multi(const orc_params* types, const double* const* tables, int32_t n_types,
                     int64_t n, int32_t n_max, const int32_t* type, const float* h,
                     const float* h1, const float* h2, const float* zeta, const float* xi_s,
                     const float* u, const float* v, const float* wi, const float* xi,
                     const float* shift, double* out, uint32_t* flags, int nthreads)
{
    if (n_max < 1 || n_max > ORC_MAX_STRATA) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int32_t t = type[i];
        if (!valid_type(t, n_types)) {
            for (int c = 0; c < 13; ++c) out[13 * i + c] = 0.0;
            out[13 * i + 10] = -1;
            flags[i] = ORC_BAD_INPUT;
            continue;
        }
        double x3[3] = {xi[i], xi[n + i], xi[2 * n + i]};
        double sh[2];
        if (shift) { sh[0] = shift[i]; sh[1] = shift[n + i]; }
        sample_multi_one(&types[t], tables[t], h[i], h1[i], h2[i], zeta[i], xi_s[i], n_max, u[i],
                         v[i], Q_WI(i), x3, shift ? sh : NULL, &out[13 * i], &flags[i]);
    }
    return 0;
}

/* One multi-scale query (single type, its table): out[13] as orc_eval_multi. */
uint32_t orc_eval_multi_query(const orc_params* p, const double* tab, double h0, double h1,
                              double h2, double zeta, int32_t n_max, double u, double v,
                              const double wi[3], const double wo[3], double out[13])
{
    uint32_t f;
    eval_multi_one(p, tab, h0, h1, h2, zeta, n_max, u, v, mk(wi[0], wi[1], wi[2]),
                   mk(wo[0], wo[1], wo[2]), NULL, out, &f);
    return f;
}

/* One multi-scale draw (single type, its table): out[13] as orc_sample_multi. */
uint32_t orc_sample_multi_query(const orc_params* p, const double* tab, double h0, double h1,
                                double h2, double zeta, double xi_s, int32_t n_max, double u,
                                double v, const double wi[3], const double xi[3], double out[13])
{
    uint32_t f;
    sample_multi_one(p, tab, h0, h1, h2, zeta, xi_s, n_max, u, v, mk(wi[0], wi[1], wi[2]), xi, NULL,
                     out, &f);
    return f;
}

/* Strata of one footprint (test access): offsets and weights, returns n. */
int orc_footprint(double h0, double h1, double h2, double zeta, int32_t n_max, double* hs,
                  double* ws)
{
    if (n_max < 1 || n_max > ORC_MAX_STRATA) return -1;
    footprint fp;
    if (footprint_make(h0, h1, h2, zeta, n_max, &fp)) return -1;
    for (int j = 0; j < fp.n; ++j) { hs[j] = fp.h[j]; ws[j] = fp.w[j]; }
    return fp.n;
}

/* theta index -> parameter slot */
static double* theta_slot(orc_params* p, int k)
{
    switch (k) {
    case 0: return &p->albedo[0];
    case 1: return &p->albedo[1];
    case 2: return &p->albedo[2];
    case 3: return &p->beta;
    case 4: return &p->ply_twist;
    case 5: return &p->fiber_twist;
    case 6: return &p->ply_density;
    default: return &p->fiber_density;
    }
}

int orc_grad_fd(const orc_params* types, const double* const* tables, int32_t n_types,
                int64_t n, const int32_t* type, const float* h, const float* u, const float* v,
                const float* wi, const float* wo, const float* gE, double rel_step,
                double* grad, double* per_query, int nthreads)
{
    for (int64_t i = 0; i < (int64_t)n_types * 8; ++i) grad[i] = 0.0;
    double* pq = per_query ? per_query : (double*)malloc(sizeof(double) * 8 * (n > 0 ? n : 1));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int32_t t = type[i];
        for (int k = 0; k < 8; ++k) pq[8 * i + k] = 0.0;
        if (!valid_type(t, n_types)) continue;
        for (int k = 0; k < 8; ++k) {
            orc_params pp = types[t], pm = types[t];
            double* sp = theta_slot(&pp, k);
            double* sm = theta_slot(&pm, k);
            double hstep = rel_step * (fabs(*sp) > 1e-3 ? fabs(*sp) : 1e-3);
            *sp += hstep;
            *sm -= hstep;
            double op[13], om[13];
            uint32_t fp, fm;
            eval_one(&pp, tables[t], Q_H(i), u[i], v[i], Q_WI(i), Q_WO(i), NULL, op, &fp);
            eval_one(&pm, tables[t], Q_H(i), u[i], v[i], Q_WI(i), Q_WO(i), NULL, om, &fm);
            double d = 0.0;
            for (int c = 0; c < 3; ++c) d += gE[3 * i + c] * (op[c] - om[c]) / (2.0 * hstep);
            pq[8 * i + k] = d;
        }
    }
    /* fixed-order per-type sums */
    for (int64_t i = 0; i < n; ++i) {
        int32_t t = type[i];
        if (!valid_type(t, n_types)) continue;
        for (int k = 0; k < 8; ++k) grad[8 * t + k] += pq[8 * i + k];
    }
    if (!per_query) free(pq);
    return 0;
}

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplies with the published multipliers and Weyl key bumps. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Probe of the forward nodes of one query (for the brute-force pins).
 * Per node 16 doubles: kind N ell att T wt(3) y(3) n_y(3) p2x p2y.
 * Returns the flags; nodes are written only when the ply is hit. */
uint32_t orc_nodes(const orc_params* p, const double* tab, double h, double u, double v,
                   const double wi[3], const double* shift, double* out)
{
    xgeom g;
    geom_x(p, tab, h, u, v, mk(wi[0], wi[1], wi[2]), shift, &g);
    if (g.ph.pass) return g.ph.flags;
    for (int k = 0; k < g.K; ++k) {
        const fnode* nd = &g.nd[k];
        double* o = out + 16 * k;
        o[0] = nd->kind; o[1] = nd->N; o[2] = nd->ell; o[3] = nd->att; o[4] = nd->T;
        o[5] = nd->wt.x; o[6] = nd->wt.y; o[7] = nd->wt.z;
        o[8] = nd->y.x; o[9] = nd->y.y; o[10] = nd->y.z;
        o[11] = nd->fy.n.x; o[12] = nd->fy.n.y; o[13] = nd->fy.n.z;
        o[14] = g.ph.p2[0]; o[15] = g.ph.p2[1];
    }
    return g.ph.flags;
}

/* Probe of the shading frame at x: t(3) b(3) n(3) Gp Gf mu_i w(4). */
uint32_t orc_frame_x(const orc_params* p, const double* tab, double h, double u, double v,
                     const double wi[3], double* out)
{
    xgeom g;
    geom_x(p, tab, h, u, v, mk(wi[0], wi[1], wi[2]), NULL, &g);
    if (g.ph.pass) return g.ph.flags;
    out[0] = g.fx.t.x; out[1] = g.fx.t.y; out[2] = g.fx.t.z;
    out[3] = g.fx.b.x; out[4] = g.fx.b.y; out[5] = g.fx.b.z;
    out[6] = g.fx.n.x; out[7] = g.fx.n.y; out[8] = g.fx.n.z;
    out[9] = g.Gp; out[10] = g.Gf; out[11] = g.mu_i;
    for (int l = 0; l < 4; ++l) out[12 + l] = g.w[l];
    return g.ph.flags;
}
