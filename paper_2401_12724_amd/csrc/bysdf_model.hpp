// bysdf_model.hpp -- per-query BYSDF model (arXiv 2401.12724, Sec. 3-4) for
// one lane of a gfx950 wavefront.
//
// Precision split: the geometry chain (yarn hit, ply-centre fixed point,
// phases, frames, forward chords) runs in the geometry scalar G, the lobes
// in the shading scalar S.  The fiber normal turns by ~pi across one fiber,
// so the specular lobes amplify a phase error by a few hundred; phases of
// scene-scale v (hundreds of yarn radii) must not be rounded to float.
//
// Per-ply state lives in register arrays indexed by compile-time constants
// (fully unrolled loops up to kMaxPlies with a runtime guard).
#pragma once

#include "bysdf_math.hpp"
#include "philox.hpp"

namespace bysdf {

constexpr int kMaxPlies = 8;
constexpr int kMaxNodes = 16;
constexpr int kMaxMigTables = 8;  // fiber tables of one type with migration

// flag bits (public numbering; see include/bysdf.h)
constexpr uint32_t F_PASS_THROUGH = 1u << 0;
constexpr uint32_t F_AXIAL = 1u << 4;
constexpr uint32_t F_BACKFACING = 1u << 5;
constexpr uint32_t F_SAMPLE_FAIL = 1u << 6;
constexpr uint32_t F_BAD_INPUT = 1u << 9;

// Stages of the geometry chain.  A scope of the model names the stage it
// belongs to with a StageMark of the geometry scalar.  For the kernels'
// scalars the mark is empty and compiles to nothing; a host-side
// measurement scalar specialises it to change the arithmetic of one stage
// at a time (the precision audit).
enum GeomStage : int {
    kStagePlies = 0,  // yarn hit, ply-centre fixed point, ray/disc tests (Sec. 3.3-3.4)
    kStageFrame,      // fiber table lookup and fiber frame (Sec. 3.5)
    kStageShadow,     // ply horizon G_p (Sec. 4.1.4)
    kStageRefract,    // visible normal and refraction into the yarn at x (Sec. 4.1.1)
    kStageChord,      // chord through the cross-section, exit ply and point (Sec. 4.1.1)
    kStageHalfX,      // half vector and cosines of the lobes at x (Eq. 2, 5)
    kStageExit,       // half vector, cosines and transmittance of the exit (Eq. 3)
    kStageSample,     // drawn directions (Sec. 4.1.5)
    kStageRest,       // everything else in the geometry scalar
    kNumStages
};
template <class G> struct StageMark {
    __host__ __device__ explicit StageMark(int) {}
};

// Scalars one query needs, in the kernel's scalar types.
template <class G, class S> struct Derived {
    int Np, K, N_it, Nu;
    double inv_np;
    G rp, Rpc, slope, wp_turns, tnorm_inv, vply_scale, wf_turns, tan_af;
    G ax_g, ay_g, eta_g, inv_eta_g;
    S ax, ay, eta, kS, B, r, sigma_t, rho_p, rho_f, dP;
    S alb[3];
    S rp_s, Rpc_s;
    // fiber migration (Sec. 3.5.2): n_mig tables switched per period of
    // mig_period along the ply, blended over the period's last mig_blend
    int n_mig;
    uint32_t mig_seed;
    double mig_period, mig_blend;
    // directions of the ply centres of the nominal cross-section,
    // (cos, sin)(2 pi k / N_p), k < N_p
    double ply_c[kMaxPlies], ply_s[kMaxPlies];
};

// Per-type record resident in device memory: the primary parameters and
// everything derived from them, ready to be read with scalar loads when a
// wavefront serves one type.
struct TypeRec {
    int32_t n_plies, K, n_iter, tex_size, table_off, table_texels;  // table_texels: all migration tables
    // primary parameters
    double rp, Rpc, ply_twist, fiber_twist, rho_f_geom;  // rho_f_geom = r_f / r_p
    double beta, aniso, eta;
    float albedo[3], k_spec, B, r, sigma_t, ply_density, fiber_density, shadow_hw;
    int32_t mig_tables;
    uint32_t mig_seed;
    double mig_period, mig_blend, mig_spread;
    Derived<double, float> d;
    // disk points (d1, d2) of the visible-normal samples of the K forward
    // nodes without a lattice shift: they depend on K alone, so they are
    // formed once at creation and read with scalar loads
    double node_disk[2 * kMaxNodes];
};

// Fill the derived scalars of a record (host at creation, device when the
// differentiable parameters change).
__host__ __device__ inline void fill_derived(TypeRec& t)
{
    Derived<double, float>& d = t.d;
    double wp = t.Rpc > 0.0 ? tan(t.ply_twist) / t.Rpc : 0.0;
    d.Np = t.n_plies; d.K = t.K; d.N_it = t.n_iter; d.Nu = t.tex_size;
    d.inv_np = 1.0 / t.n_plies;
    d.rp = t.rp;
    d.Rpc = t.Rpc;
    d.slope = t.Rpc * wp;                        // tan(alpha_p), 0 without a helix
    d.vply_scale = sqrt(1.0 + d.slope * d.slope); // ply arc length per yarn length
    d.tnorm_inv = 1.0 / d.vply_scale;
    d.wp_turns = wp * kInvTwoPi;                 // helix turns per unit length
    d.tan_af = tan(t.fiber_twist);
    d.wf_turns = d.tan_af / ((1.0 - t.rho_f_geom) * t.rp) * kInvTwoPi;
    d.ax_g = t.beta;
    d.ay_g = t.beta * t.aniso;
    d.eta_g = t.eta;
    d.inv_eta_g = 1.0 / t.eta;
    d.ax = (float)t.beta;
    d.ay = (float)(t.beta * t.aniso);
    d.eta = (float)t.eta;
    d.kS = t.k_spec; d.B = t.B; d.r = t.r; d.sigma_t = t.sigma_t;
    d.rho_p = t.ply_density; d.rho_f = t.fiber_density; d.dP = t.shadow_hw;
    for (int c = 0; c < 3; ++c) d.alb[c] = t.albedo[c];
    d.rp_s = (float)t.rp;
    d.Rpc_s = (float)t.Rpc;
    d.n_mig = t.mig_tables > 1 ? t.mig_tables : 1;
    d.mig_seed = t.mig_seed;
    d.mig_period = t.mig_period;
    d.mig_blend = t.mig_blend;
    for (int k = 0; k < kMaxPlies; ++k) {
        d.ply_c[k] = 1.0;
        d.ply_s[k] = 0.0;
        if (k < t.n_plies) sincos_turns(k * d.inv_np, &d.ply_s[k], &d.ply_c[k]);
    }
}

__host__ __device__ inline Derived<double, float> derive(const TypeRec& t) { return t.d; }

// The derived scalars in other scalar types (host-side tools: the op counter
// and the precision audit).
template <class G2, class S2> inline Derived<G2, S2> rebind(const Derived<double, float>& f)
{
    Derived<G2, S2> d;
    d.Np = f.Np; d.K = f.K; d.N_it = f.N_it; d.Nu = f.Nu; d.inv_np = f.inv_np;
    d.rp = G2(f.rp); d.Rpc = G2(f.Rpc); d.slope = G2(f.slope); d.wp_turns = G2(f.wp_turns);
    d.tnorm_inv = G2(f.tnorm_inv); d.vply_scale = G2(f.vply_scale); d.wf_turns = G2(f.wf_turns);
    d.tan_af = G2(f.tan_af); d.ax_g = G2(f.ax_g); d.ay_g = G2(f.ay_g); d.eta_g = G2(f.eta_g);
    d.inv_eta_g = G2(f.inv_eta_g);
    d.ax = S2(f.ax); d.ay = S2(f.ay); d.eta = S2(f.eta); d.kS = S2(f.kS); d.B = S2(f.B); d.r = S2(f.r);
    d.sigma_t = S2(f.sigma_t); d.rho_p = S2(f.rho_p); d.rho_f = S2(f.rho_f); d.dP = S2(f.dP);
    for (int c = 0; c < 3; ++c) d.alb[c] = S2(f.alb[c]);
    d.rp_s = S2(f.rp_s); d.Rpc_s = S2(f.Rpc_s);
    d.n_mig = f.n_mig; d.mig_seed = f.mig_seed; d.mig_period = f.mig_period; d.mig_blend = f.mig_blend;
    for (int k = 0; k < kMaxPlies; ++k) {
        d.ply_c[k] = f.ply_c[k];
        d.ply_s[k] = f.ply_s[k];
    }
    return d;
}

// sin and cos of 2 pi t (t in turns) for the geometry scalar
template <class G> __host__ __device__ inline void sincos_turns_g(const G& t, G* s, G* c);
template <> __host__ __device__ inline void sincos_turns_g<double>(const double& t, double* s, double* c)
{
    sincos_turns(t, s, c);
}

// ---------------------------------------------------------------- microfacets

// Dielectric Fresnel for cosine c >= 0 on the index-1 side of an interface
// of relative index e; total internal reflection returns 1.
template <class S> __host__ __device__ inline S fresnel(S c, S e)
{
    S s2t = (S(1) - c * c) * rcp_(e * e);
    if (val(s2t) >= 1.0f) return S(1);
    S ct = sqrt_(S(1) - s2t);
    S rs = (c - e * ct) * rcp_(c + e * ct);
    S rpp = (e * c - ct) * rcp_(e * c + ct);
    return S(0.5f) * (rs * rs + rpp * rpp);
}

// Fresnel transmittance 1 - F written without the cancellation of 1 - F
// near total internal reflection: 1 - r^2 = 4 c e c_t / (c + e c_t)^2 per
// polarisation.
template <class S> __host__ __device__ inline S fresnel_T(S c, S e)
{
    S s2t = (S(1) - c * c) * rcp_(e * e);
    if (val(s2t) >= 1.0f) return S(0);
    S ct = sqrt_(S(1) - s2t);
    S a = c + e * ct, b = e * c + ct;
    return S(2) * e * c * ct * (rcp_(a * a) + rcp_(b * b));
}

template <class S> __host__ __device__ inline S ggx_D(const V3<S>& m, S ax, S ay)
{
    if (!(val(m.z) > 0.0f)) return S(0);
    S qx = m.x * rcp_(ax), qy = m.y * rcp_(ay);
    S t = qx * qx + qy * qy + m.z * m.z;
    return rcp_(S(float(kPi)) * ax * ay * t * t);
}

template <class S> __host__ __device__ inline S smith_G1(const V3<S>& w, const V3<S>& m, S ax, S ay)
{
    S wm = dot(w, m);
    if (!(val(wm) * val(w.z) > 0.0f)) return S(0);
    S tx = ax * w.x, ty = ay * w.y;
    S a2t2 = (tx * tx + ty * ty) * rcp_(w.z * w.z);
    return S(2) * rcp_(S(1) + sqrt_(S(1) + a2t2));
}

// Isotropic roughness (alpha_x = alpha_y = a): D and G1 depend on the
// microfacet and the directions through their cosines with the normal only.
// mz = m.n, ms2 = 1 - mz^2 (formed before narrowing, where it does not
// cancel); wm = w.m (the sign test), wz = w.n, ws2 = 1 - wz^2.
template <class S> __host__ __device__ inline S ggx_D_iso(S mz, S ms2, S a)
{
    if (!(val(mz) > 0.0f)) return S(0);
    const S ia2 = rcp_(a * a);
    S t = ms2 * ia2 + mz * mz;
    return rcp_(S(float(kPi)) * a * a * t * t);
}
template <class S> __host__ __device__ inline S smith_G1_iso(S wm, S wz, S ws2, S a)
{
    if (!(val(wm) * val(wz) > 0.0f)) return S(0);
    S a2t2 = a * a * ws2 * rcp_(wz * wz);
    return S(2) * rcp_(S(1) + sqrt_(S(1) + a2t2));
}
template <class G> __host__ __device__ inline G one_minus_sq(const G& z) { return G(1) - z * z; }

// Visible-normal sampling of GGX (Heitz 2018): stretch the view to unit
// roughness, build a basis around it, sample the projected hemisphere disc
// with its far half compressed according to the view elevation, lift,
// unstretch.  w local with w.z > 0; u1, u2 in [0, 1).
// The uniform point (d1, d2) of the unit disc for the uniforms u1, u2.
template <class T> __host__ __device__ inline void vndf_disk(T u1, T u2, T& d1, T& d2)
{
    T rad = sqrt_(u1);
    T su, cu;
    sincos_turns_g(u2, &su, &cu);
    d1 = rad * cu;
    d2 = rad * su;
}
// The visible normal for the disc point (d1, d2).
template <class T> __host__ __device__ inline V3<T> sample_vndf_disk(const V3<T>& w, T ax, T ay, T d1, T d2)
{
    V3<T> vh = normalize(mk3<T>(ax * w.x, ay * w.y, w.z));
    T l2 = vh.x * vh.x + vh.y * vh.y;
    V3<T> b1 = val(l2) > 0.0 ? mk3<T>(-vh.y, vh.x, T(0)) * rsqrt_(l2)
                             : mk3<T>(T(1), T(0), T(0));
    V3<T> b2 = cross(vh, b1);
    T blend = T(0.5) * (T(1) + vh.z);
    d2 = (T(1) - blend) * sqrt_(T(1) - d1 * d1) + blend * d2;
    T h2 = T(1) - d1 * d1 - d2 * d2;
    T hz = val(h2) > 0.0 ? sqrt_(h2) : T(0);
    V3<T> nh = b1 * d1 + b2 * d2 + vh * hz;
    T nz = val(nh.z) > 0.0 ? nh.z : T(0);
    return normalize(mk3<T>(ax * nh.x, ay * nh.y, nz));
}
template <class T> __host__ __device__ inline V3<T> sample_vndf(const V3<T>& w, T ax, T ay, T u1, T u2)
{
    T d1, d2;
    vndf_disk(u1, u2, d1, d2);
    return sample_vndf_disk(w, ax, ay, d1, d2);
}

// Lommel-Seeliger single-scatter albedo 1/2 [1 - mu ln(1 + 1/mu)].
template <class S> __host__ __device__ inline S ls_albedo(S mu)
{
    if (!(val(mu) > 0.0f)) return S(0.5f);
    return S(0.5f) * (S(1) - mu * log_(S(1) + rcp_(mu)));
}

// ---------------------------------------------------------------- ply hit

// MP: compile-time bound on the plies of the types a kernel serves
template <class G, int MP> struct PlyHit {
    bool pass;
    uint32_t flags;
    G x2x, x2y, dhx, dhy, kappa;
    G cth[MP], sth[MP];  // converged phase of each ply centre (centre = R_pc (cth, sth))
    int ks;
    G p2x, p2y, n2x, n2y, vhit;
};


// Yarn hit (Sec. 3.3) and implicit plies (Sec. 3.4): hit point x2 on the
// unit yarn circle at offset h, then for each ply the fixed-point update of
// the height at which the ply-centre helix crosses the ray's ellipse plane,
// a 2D ray/disc test in the projected cross-section, and the closest ply.
template <class G, class S, int MP>
__host__ __device__ inline void trace_plies(const Derived<G, S>& P, float h, float u, float v,
                                            const V3<float>& wi, PlyHit<G, MP>& g)
{
    StageMark<G> mark(kStagePlies);
    g.pass = false;
    g.flags = 0;
    g.ks = -1;
    double sxy = sqrt((double)wi.x * wi.x + (double)wi.y * wi.y);
    if (sxy < 1e-6) {
        g.pass = true;
        g.flags = F_AXIAL | F_PASS_THROUGH;
        return;
    }
    double cx0 = wi.x / sxy, cy0 = wi.y / sxy;
    double hh = h > 1.0f ? 1.0 : (h < -1.0f ? -1.0 : (double)h);
    double cg = sqrt(1.0 - hh * hh);
    g.x2x = G(cx0 * cg - cy0 * hh);
    g.x2y = G(cy0 * cg + cx0 * hh);
    g.dhx = G(-cx0);
    g.dhy = G(-cy0);
    g.kappa = G(-(double)wi.z / sxy);
    G sexit = G(-2) * (g.x2x * g.dhx + g.x2y * g.dhy);
    double u_turn = (double)u * kInvTwoPi;
    G vv = G((double)v);
    G best_s = G(0);
    int best = -1;
    // every update starts from the hit height, where the ply centres are
    // ply 0's turned by 2 pi k / N_p
    G s0, c0;
    sincos_turns_g(G(u_turn) + P.wp_turns * vv, &s0, &c0);
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        if (k >= P.Np) break;
        G base = G(u_turn + k * P.inv_np);
        G vj = vv;
        const G ck = G(P.ply_c[k]), sk = G(P.ply_s[k]);
        G c = c0 * ck - s0 * sk, s = s0 * ck + c0 * sk;
        for (int j = 0; j < P.N_it; ++j) {
            if (j > 0) sincos_turns_g(base + P.wp_turns * vj, &s, &c);
            vj = vv + g.kappa * ((P.Rpc * c - g.x2x) * g.dhx + (P.Rpc * s - g.x2y) * g.dhy);
        }
        sincos_turns_g(base + P.wp_turns * vj, &s, &c);
        g.cth[k] = c;
        g.sth[k] = s;
        G wx = g.x2x - P.Rpc * c, wy = g.x2y - P.Rpc * s;
        G b = wx * g.dhx + wy * g.dhy;
        G cc = wx * wx + wy * wy - P.rp * P.rp;
        G disc = b * b - cc;
        if (val(disc) >= 0.0) {
            G sq = sqrt_(disc);
            G slo = -b - sq, shi = -b + sq;
            if (val(shi) >= 0.0 && val(slo) <= val(sexit)) {
                G sk = val(slo) > 0.0 ? slo : G(0);
                if (best < 0 || val(sk) < val(best_s)) {
                    best = k;
                    best_s = sk;
                }
            }
        }
    }
    if (best < 0) {
        g.pass = true;
        g.flags |= F_PASS_THROUGH;
        return;
    }
    g.ks = best;
    G ccx = G(0), ccy = G(0);
#pragma unroll
    for (int k = 0; k < MP; ++k)
        if (k == best) { ccx = P.Rpc * g.cth[k]; ccy = P.Rpc * g.sth[k]; }
    g.p2x = g.x2x + best_s * g.dhx;
    g.p2y = g.x2y + best_s * g.dhy;
    G nx = g.p2x - ccx, ny = g.p2y - ccy;
    G inv = rsqrt_(nx * nx + ny * ny);
    g.n2x = nx * inv;
    g.n2y = ny * inv;
    g.vhit = vv + g.kappa * best_s;
}

// ---------------------------------------------------------------- fibers

template <class G> __host__ __device__ inline G floor_g(const G& x);
template <> __host__ __device__ inline double floor_g<double>(const double& x) { return floor(x); }

// Fiber-migration draws (Sec. 3.5.2): Philox4x32-10 with key (seed, "FIBR").
// Table of ply k in period q: counter (q low, q high, k, "SELT"), first word
// modulo the number of tables.
__host__ __device__ inline int mig_table(uint32_t seed, int n_mig, int64_t q, int k)
{
    uint32_t o[4];
    const uint64_t uq = (uint64_t)q;
    rng::philox4x32_10((uint32_t)(uq & 0xffffffffu), (uint32_t)(uq >> 32), (uint32_t)k, 0x53454c54u, seed,
                       0x46494252u, o);
    return (int)(o[0] % (uint32_t)n_mig);
}

// Periodic linear interpolation between the texel centres of the table at
// texel offset base, at a phase given in turns.
template <class G, class Tab>
__host__ __device__ inline void table_at(const Tab& tab, int Nu, int base, const G& turns, G& dn, G& rh,
                                         G& gf)
{
    G fl = floor_g(turns);
    G x = (turns - fl) * G((double)Nu) - G(0.5);
    G xf = floor_g(x);
    G f = x - xf;
    // texel index in [0, Nu): x lies in [-1/2, Nu - 1/2) for a finite phase;
    // anything else (a non-finite phase) reads texel 0
    double xi0 = val(xf) < 0.0 ? val(xf) + Nu : val(xf);
    int i0 = (xi0 >= 0.0 && xi0 < (double)Nu) ? (int)xi0 : 0;
    int i1 = i0 + 1 == Nu ? 0 : i0 + 1;
    float4 t0 = tab(base + i0), t1 = tab(base + i1);
    G omf = G(1) - f;
    dn = omf * G((double)t0.x) + f * G((double)t1.x);
    rh = omf * G((double)t0.y) + f * G((double)t1.y);
    gf = omf * G((double)t0.z) + f * G((double)t1.z);
}

// Ply frame on the disc k with phase (cth, sth) at 2D outward normal (n2x,
// n2y) and yarn height z, then the fiber frame from the 1D fiber table
// (Sec. 3.5.1): normal rotated about the ply tangent by dn, tangent tilted
// against the ply twist by atan(rho_hat tan(alpha_f)).  With fiber
// migration (Sec. 3.5.2) the table is the one drawn for ply k in the
// current period of the ply arc length, blended linearly into the next
// period's table over the period's last mig_blend share.
template <class G, class S, class Tab>
__host__ __device__ inline Frame<G> fiber_frame(const Derived<G, S>& P, const Tab& tab, G cth, G sth, int k,
                                                G n2x, G n2y, G z, G* gf_out, G* a_out)
{
    StageMark<G> mark(kStageFrame);
    V3<G> tp = mk3<G>(-P.slope * sth * P.tnorm_inv, P.slope * cth * P.tnorm_inv, P.tnorm_inv);
    V3<G> n23 = mk3<G>(n2x, n2y, G(0));
    V3<G> np = normalize(n23 - tp * dot(n23, tp));
    G a = atan2_(cth * n2y - sth * n2x, cth * n2x + sth * n2y);
    const G vply = z * P.vply_scale;
    G turns = a * G(kInvTwoPi) + P.wf_turns * vply;
    G dn, rh, gfv;
    if (Tab::kMigration && P.n_mig > 1) {
        G t = vply / G(P.mig_period);
        G fq = floor_g(t);
        G ph = t - fq;
        const int64_t q = (int64_t)val(fq);
        const double b = P.mig_blend;
        G w = (b > 0.0 && val(ph) > 1.0 - b) ? (ph - G(1.0 - b)) / G(b) : G(0);
        const int m0 = mig_table(P.mig_seed, P.n_mig, q, k), m1 = mig_table(P.mig_seed, P.n_mig, q + 1, k);
        G d0, r0, g0, d1, r1, g1;
        table_at(tab, P.Nu, m0 * P.Nu, turns, d0, r0, g0);
        table_at(tab, P.Nu, m1 * P.Nu, turns, d1, r1, g1);
        G omw = G(1) - w;
        dn = omw * d0 + w * d1;
        rh = omw * r0 + w * r1;
        gfv = omw * g0 + w * g1;
    } else {
        table_at(tab, P.Nu, 0, turns, dn, rh, gfv);
    }
    V3<G> bp = cross(tp, np);
    G sdn, cdn;
    sincos_turns_g(dn * G(kInvTwoPi), &sdn, &cdn);
    V3<G> npr = np * cdn + bp * sdn;
    G tfa = rh * P.tan_af;
    G ca = rsqrt_(G(1) + tfa * tfa);
    G sa = tfa * ca;
    Frame<G> fr;
    fr.t = tp * ca - bp * sa;
    fr.n = normalize(npr - fr.t * dot(npr, fr.t));
    fr.b = cross(fr.n, fr.t);
    if (gf_out) *gf_out = gfv;
    if (a_out) *a_out = a;
    return fr;
}

// ---------------------------------------------------------------- shadowing

// Raw ply visibility (Sec. 4.1.4): at angle a around ply 0 of the nominal
// cross-section, the share of the window [phi - dP, phi + dP] of incident
// 2D directions (measured from the local normal) that is neither below the
// ply's tangent line nor towards another ply's disc.  Each occluded set
// meets the window in at most one piece (the window is shorter than the
// gap between a set's 2 pi copies); the union length uses a sorting network.
template <class G, int MP>
__host__ __device__ inline G ply_shadow_raw(int Np, G rp, G Rpc, G dP, G a, G phi, const double* ply_c,
                                            const double* ply_s)
{
    G lo[MP], hi[MP];
    G wlo = phi - dP, whi = phi + dP;
    G na_x, na_y;
    sincos_turns_g(a * G(kInvTwoPi), &na_y, &na_x);
    G Px = Rpc + rp * na_x, Py = rp * na_y;
    const G big = G(1e30);
#pragma unroll
    for (int s = 0; s < MP; ++s) {
        G cen, half;
        bool live = s < Np;
        if (s == 0) {
            cen = G(kPi);
            half = G(0.5 * kPi);
        } else if (live) {
            G wx = Rpc * G(ply_c[s]) - Px, wy = Rpc * G(ply_s[s]) - Py;
            G d2 = wx * wx + wy * wy;
            cen = atan2_(na_x * wy - na_y * wx, na_x * wx + na_y * wy);
            // asin(r_p / d) = atan2(r_p, sqrt(d^2 - r_p^2)); inside the disc: pi/2
            G e2 = d2 - rp * rp;
            half = val(e2) > 0.0 ? atan2_(rp, sqrt_(e2)) : G(0.5 * kPi);
        } else {
            cen = G(0);
            half = G(0);
        }
        // copy of the set closest to the window
        G shift = G(kTwoPi * rint(val((cen - phi) * G(kInvTwoPi))));
        G l = cen - half - shift, h2 = cen + half - shift;
        l = val(l) > val(wlo) ? l : wlo;
        h2 = val(h2) < val(whi) ? h2 : whi;
        bool ok = live && val(h2) > val(l);
        lo[s] = ok ? l : big;
        hi[s] = ok ? h2 : big;
    }
    // sort by lower end (odd-even transposition network, MP passes)
#pragma unroll
    for (int pass = 0; pass < MP; ++pass) {
#pragma unroll
        for (int i = pass & 1; i + 1 < MP; i += 2) {
            bool sw = val(lo[i + 1]) < val(lo[i]);
            G a0 = sw ? lo[i + 1] : lo[i], a1 = sw ? lo[i] : lo[i + 1];
            G b0 = sw ? hi[i + 1] : hi[i], b1 = sw ? hi[i] : hi[i + 1];
            lo[i] = a0; lo[i + 1] = a1; hi[i] = b0; hi[i + 1] = b1;
        }
    }
    G occ = G(0), cl = lo[0], ch = hi[0];
    bool any = val(lo[0]) < 1e29;
#pragma unroll
    for (int i = 1; i < MP; ++i) {
        bool live = val(lo[i]) < 1e29;
        if (live && val(lo[i]) > val(ch)) {
            occ = occ + (ch - cl);
            cl = lo[i];
            ch = hi[i];
        } else if (live && val(hi[i]) > val(ch)) {
            ch = hi[i];
        }
    }
    if (any) occ = occ + (ch - cl);
    G vis = G(1) - occ / (G(2) * dP);
    return val(vis) < 0.0 ? G(0) : (val(vis) > 1.0 ? G(1) : vis);
}

// ---------------------------------------------------------------- state at x

template <class G, class S, int MP> struct XState {
    PlyHit<G, MP> ph;
    Frame<G> fx;      // fiber frame at x (geometry precision)
    Frame<S> fxs;     // the same, shading precision
    V3<G> wi_g;
    V3<S> wi_s;
    S Gp, Gf, mu_i;
    S w[4];           // lobe selection weights
    G a;
    G rawp, rawf;     // visibilities before the density blends
};

// The cosine at x and the lobe selection weights from the frame at x.
template <class G, class S, int MP>
__host__ __device__ inline void lobe_weights(const Derived<G, S>& P, XState<G, S, MP>& X)
{
    X.mu_i = Narrow<S>::from(dot(X.wi_g, X.fx.n));
    S PR = fresnel<S>(val(X.mu_i) > 0.0f ? X.mu_i : S(0), P.eta);
    X.w[0] = (S(1) - P.B) * PR;
    X.w[1] = (S(1) - P.B) * (S(1) - PR);
    X.w[2] = P.B * P.r;
    X.w[3] = P.B * (S(1) - P.r);
}

template <class G, class S, int MP, class Tab>
__host__ __device__ inline void state_after_plies(const Derived<G, S>& P, const Tab& tab, const V3<float>& wi,
                                                  XState<G, S, MP>& X)
{
    X.wi_g = mk3<G>(G((double)wi.x), G((double)wi.y), G((double)wi.z));
    X.wi_s = mk3<S>(S(wi.x), S(wi.y), S(wi.z));
    if (X.ph.pass) return;
    G cth = G(0), sth = G(0);
#pragma unroll
    for (int k = 0; k < MP; ++k)
        if (k == X.ph.ks) { cth = X.ph.cth[k]; sth = X.ph.sth[k]; }
    G gft;
    X.fx = fiber_frame(P, tab, cth, sth, X.ph.ks, X.ph.n2x, X.ph.n2y, X.ph.vhit, &gft, &X.a);
    X.fxs = narrowf<S>(X.fx);
    // shadowing in the geometry scalar: a mostly occluded window leaves a
    // small visible share that single precision cannot resolve
    G raw;
    {
        StageMark<G> mark(kStageShadow);
        G phi = atan2_(X.ph.n2x * X.wi_g.y - X.ph.n2y * X.wi_g.x, X.ph.n2x * X.wi_g.x + X.ph.n2y * X.wi_g.y);
        raw = ply_shadow_raw<G, MP>(P.Np, P.rp, P.Rpc, G(val(P.dP)), X.a, phi, P.ply_c, P.ply_s);
    }
    X.rawp = raw;
    X.rawf = gft;
    X.Gp = Narrow<S>::from(G(1) - G(val(P.rho_p)) * (G(1) - raw));
    X.Gf = Narrow<S>::from(G(1) - G(val(P.rho_f)) * (G(1) - gft));
    lobe_weights(P, X);
}

// Everything at x that does not depend on wo: ply hit, fiber frame,
// shadowing, lobe weights.
template <class G, class S, int MP, class Tab>
__host__ __device__ inline void state_at_x(const Derived<G, S>& P, const Tab& tab, float h, float u,
                                           float v, const V3<float>& wi, XState<G, S, MP>& X)
{
    trace_plies(P, h, u, v, wi, X.ph);
    state_after_plies(P, tab, wi, X);
}

// ---------------------------------------------------------------- forward nodes

// Point k of the rank-1 lattice of the forward-node integral (Eq. 1):
// ((k + 1/2) / K, (k + 1/2) (sqrt 5 - 1) / 2) modulo 1, shifted by (s0, s1)
// when the query carries a shift.
__host__ __device__ inline void node_lattice(int k, int K, float s0, float s1, bool has_shift, double& xi1,
                                             double& xi2)
{
    const double phig = 0.61803398874989484820;
    double a1 = (k + 0.5) / K, a2 = (k + 0.5) * phig;
    if (has_shift) {
        a1 += s0;
        a2 += s1;
    }
    xi1 = a1 - floor(a1);
    xi2 = a2 - floor(a2);
}

// The unshifted nodes' disc points of a record (host, at creation).
inline void fill_node_disk(TypeRec& t)
{
    for (int k = 0; k < kMaxNodes; ++k) {
        double d1 = 0.0, d2 = 0.0;
        if (k < t.K) {
            double xi1, xi2;
            node_lattice(k, t.K, 0.0f, 0.0f, false, xi1, xi2);
            vndf_disk<double>(xi1, xi2, d1, d2);
        }
        t.node_disk[2 * k] = d1;
        t.node_disk[2 * k + 1] = d2;
    }
}

template <class G, class S> struct Node {
    S T, att;        // refraction weight at x, tau^N
    V3<G> wt;        // refracted direction
    Frame<G> fy;     // fiber frame at the exit point
    V3<G> y;         // exit point (x, y, height)
};

// Node k of the integral over exit points (Eq. 1): a visible normal at x
// from a rank-1 lattice point, refraction into the yarn, the chord through
// the projected cross-section, the plies it enters, the exit ply and the
// fiber frame there (Eq. 3-4).
template <class G, class S, int MP, class Tab>
__host__ __device__ inline void forward_node(const Derived<G, S>& P, const Tab& tab,
                                             const XState<G, S, MP>& X, int k, float s0, float s1,
                                             bool has_shift, Node<G, S>& nd,
                                             const double* disk = nullptr)
{
    // The node is assembled in a local and stored once: partial stores on
    // several return paths get merged by the optimiser into stores through a
    // selected stack address, which pins the node in scratch memory.
    const PlyHit<G, MP>& ph = X.ph;
    Node<G, S> r;
    // no refraction into the yarn, or a chord that leaves at once: the exit
    // is the entry point x with the fiber frame flipped (thin-sheet exit)
    r.T = S(0);
    r.att = S(1);
    r.wt = mk3<G>(G(0), G(0), G(0));
    r.fy.t = X.fx.t;
    r.fy.n = -X.fx.n;
    r.fy.b = cross(r.fy.n, r.fy.t);
    r.y = mk3<G>(ph.p2x, ph.p2y, ph.vhit);
    if (val(X.mu_i) > 0.0f) {
        StageMark<G> mark(kStageRefract);
        V3<G> wl = to_local(X.fx, X.wi_g);
        G d1, d2;
        if (disk && !has_shift) {
            d1 = G(disk[2 * k]);
            d2 = G(disk[2 * k + 1]);
        } else {
            double xi1, xi2;
            node_lattice(k, P.K, s0, s1, has_shift, xi1, xi2);
            vndf_disk<G>(G(xi1), G(xi2), d1, d2);
        }
        V3<G> ml = sample_vndf_disk<G>(wl, P.ax_g, P.ay_g, d1, d2);
        V3<G> m = to_world(X.fx, ml);
        G c = dot(X.wi_g, m);
        c = val(c) > 0.0 ? c : G(0);
        G ie = P.inv_eta_g;
        G s2t = (G(1) - c * c) * ie * ie;
        G ct = sqrt_(G(1) - s2t);
        V3<G> wt = X.wi_g * (-ie) + m * (c * ie - ct);
        r.wt = wt;
        S cs = Narrow<S>::from(c);
        S g1t;
        if (val(P.ax) == val(P.ay)) {
            const G tz = dot(wt, X.fx.n);
            g1t = smith_G1_iso<S>(Narrow<S>::from(dot(wt, m)), Narrow<S>::from(tz),
                                  Narrow<S>::from(one_minus_sq(tz)), P.ax);
        } else {
            g1t = smith_G1<S>(narrow3<S>(to_local(X.fx, wt)), narrow3<S>(ml), P.ax, P.ay);
        }
        r.T = fresnel_T<S>(cs, P.eta) * g1t;
        // chord in the projected cross-section, starting at the ply hit
        StageMark<G> chord_mark(kStageChord);
        G le2 = wt.x * wt.x + wt.y * wt.y;
        G il = val(le2) > 0.0 ? rsqrt_(le2) : G(0);
        G le = le2 * il;
        G en = wt.x * ph.n2x + wt.y * ph.n2y;
        if (!(val(le) < 1e-6 || val(en) >= 0.0)) {
            G ex = wt.x * il, ey = wt.y * il;
            G bq = ph.p2x * ex + ph.p2y * ey;
            G cq = ph.p2x * ph.p2x + ph.p2y * ph.p2y - G(1);
            G dq = bq * bq - cq;
            G syarn = -bq + (val(dq) > 0.0 ? sqrt_(dq) : G(0));
            int N = 0, jl = -1;
            G sbest = G(0), cxl = G(0), cyl = G(0), cthl = G(0), sthl = G(0);
#pragma unroll
            for (int j = 0; j < MP; ++j) {
                if (j >= P.Np) break;
                bool ent = false;
                G so = G(0);
                if (j == ph.ks) {
                    // the chord starts on this disc's rim and heads inside
                    G sx = G(-2) * P.rp * en * il;
                    so = val(sx) < val(syarn) ? sx : syarn;
                    ent = true;
                } else {
                    G wx = ph.p2x - P.Rpc * ph.cth[j], wy = ph.p2y - P.Rpc * ph.sth[j];
                    G b = wx * ex + wy * ey;
                    G cc = wx * wx + wy * wy - P.rp * P.rp;
                    G disc = b * b - cc;
                    if (val(disc) > 0.0) {
                        G sq = sqrt_(disc);
                        G slo = -b - sq, shi = -b + sq;
                        if (val(shi) > 0.0 && val(slo) < val(syarn)) {
                            ent = true;
                            so = val(shi) < val(syarn) ? shi : syarn;
                        }
                    }
                }
                if (ent) {
                    ++N;
                    if (jl < 0 || val(so) > val(sbest)) {
                        jl = j;
                        sbest = so;
                        cxl = P.Rpc * ph.cth[j];
                        cyl = P.Rpc * ph.sth[j];
                        cthl = ph.cth[j];
                        sthl = ph.sth[j];
                    }
                }
            }
            G y2x = ph.p2x + sbest * ex, y2y = ph.p2y + sbest * ey;
            G ell = sbest * il;
            G zy = ph.vhit + wt.z * ell;
            G nyx = y2x - cxl, nyy = y2y - cyl;
            G ninv = rsqrt_(nyx * nyx + nyy * nyy);
            r.att = exp_(-P.sigma_t * Narrow<S>::from(ell) * S(float(N)));
            r.fy = fiber_frame<G, S, Tab>(P, tab, cthl, sthl, jl, nyx * ninv, nyy * ninv, zy, nullptr,
                                          nullptr);
            r.y = mk3<G>(y2x, y2y, zy);
        }
    }
    nd = r;
}

// Exit refraction at y (Eq. 3): Walter's BTDF from inside (index eta) to
// outside for wi' = -wt, times |wo.n_y|, and the solid-angle pdf of drawing
// wo through this node.  The half vector, the cosines and the transmittance
// use the geometry scalar: next to the critical angle the transmittance
// falls like the transmitted cosine, whose derivative is unbounded.
template <class G, class S>
__host__ __device__ inline void exit_btdf(const Derived<G, S>& P, const V3<G>& wt, const Frame<G>& fy,
                                          const V3<G>& wo, S* val_out, S* pdf_out)
{
    StageMark<G> mark(kStageExit);
    *val_out = S(0);
    *pdf_out = S(0);
    V3<G> wip = -wt;
    G ci = dot(wip, fy.n), co = dot(wo, fy.n);
    if (!(val(ci) < 0.0 && val(co) > 0.0)) return;
    V3<G> mh = -(wip * P.eta_g + wo);
    G ml2 = dot(mh, mh);
    if (!(val(ml2) > 0.0)) return;
    mh = mh * rsqrt_(ml2);
    G mz = dot(mh, fy.n);
    if (val(mz) < 0.0) {
        mh = -mh;
        mz = -mz;
    }
    G im = dot(wip, mh), om = dot(wo, mh);
    if (!(val(im) < 0.0 && val(om) > 0.0)) return;
    G den = P.eta_g * im + om;
    G Ft = fresnel_T<G>(-im, P.inv_eta_g);
    S D, g1i, g1o;
    if (val(P.ax) == val(P.ay)) {
        D = ggx_D_iso<S>(Narrow<S>::from(mz), Narrow<S>::from(one_minus_sq(mz)), P.ax);
        g1i = smith_G1_iso<S>(Narrow<S>::from(im), Narrow<S>::from(ci), Narrow<S>::from(one_minus_sq(ci)),
                              P.ax);
        g1o = smith_G1_iso<S>(Narrow<S>::from(om), Narrow<S>::from(co), Narrow<S>::from(one_minus_sq(co)),
                              P.ax);
    } else {
        V3<S> ml = narrow3<S>(to_local(fy, mh));
        D = ggx_D<S>(ml, P.ax, P.ay);
        g1i = smith_G1<S>(narrow3<S>(to_local(fy, wip)), ml, P.ax, P.ay);
        g1o = smith_G1<S>(narrow3<S>(to_local(fy, wo)), ml, P.ax, P.ay);
    }
    // |wi'.m| |wo.m| / (|wi'.n| |wo.n|) * Jacobian / (eta wi'.m + wo.m)^2,
    // times |wo.n| for the returned value
    S geo = Narrow<S>::from((im * om) * rcp_(ci * (den * den)));
    *val_out = geo * Narrow<S>::from(Ft) * g1i * g1o * D;
    *pdf_out = geo * g1i * D;
}

// ---------------------------------------------------------------- lobes

template <class S> struct EvalOut {
    S E[3], ExS, EyS, ExB[3], EyB[3], pdf;
    S body0;  // body lobes per unit albedo without G_p G_f (closed-form derivatives)
};

// Running sums of the lobes at one direction wo: the terms at x and the
// sums over the forward nodes.
template <class S> struct LobeAcc {
    S ExS, pxS, bxu, pxB;  // specular and body at x (body per unit albedo, before G_p G_f)
    S EyS, pyS, by, pyB;   // sums over the nodes
};

// The four lobes of Eq. 1 and the mixture pdf of Sec. 4.1.5 at wo, in three
// steps: the terms at x, one step per forward node, and the combination.
// Dot products, the half vector and local coordinates are formed in the
// geometry scalar (a grazing cosine or a near-opposite pair cancels), the
// lobe formulas then run in the shading scalar.
template <class G, class S, int MP>
__host__ __device__ inline void lobes_at_x(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                           const V3<G>& wo_g, LobeAcc<S>& a)
{
    StageMark<G> mark(kStageHalfX);
    S mu_i = X.mu_i;
    G mu_o_g = dot(wo_g, X.fx.n);
    S mu_o = Narrow<S>::from(mu_o_g);
    S ExS = S(0), pxS = S(0);
    bool front_i = val(mu_i) > 0.0f;
    if (front_i && val(mu_o_g) > 0.0) {
        V3<G> hv = normalize(X.wi_g + wo_g);
        const G ih_g = dot(X.wi_g, hv), oh_g = dot(wo_g, hv);
        S D, g1i, g1o;
        if (val(P.ax) == val(P.ay)) {
            const G hz = dot(hv, X.fx.n), iz = dot(X.wi_g, X.fx.n);
            D = ggx_D_iso<S>(Narrow<S>::from(hz), Narrow<S>::from(one_minus_sq(hz)), P.ax);
            g1i = smith_G1_iso<S>(Narrow<S>::from(ih_g), Narrow<S>::from(iz), Narrow<S>::from(one_minus_sq(iz)),
                                  P.ax);
            g1o = smith_G1_iso<S>(Narrow<S>::from(oh_g), mu_o, Narrow<S>::from(one_minus_sq(mu_o_g)), P.ax);
        } else {
            V3<S> hl = narrow3<S>(to_local(X.fx, hv));
            D = ggx_D<S>(hl, P.ax, P.ay);
            g1i = smith_G1<S>(narrow3<S>(to_local(X.fx, X.wi_g)), hl, P.ax, P.ay);
            g1o = smith_G1<S>(narrow3<S>(to_local(X.fx, wo_g)), hl, P.ax, P.ay);
        }
        S ih = Narrow<S>::from(ih_g), oh = Narrow<S>::from(oh_g);
        S ihp = val(ih) > 0.0f ? ih : S(0);
        const S q4 = rcp_(S(4) * mu_i);
        ExS = (S(1) - P.B) * P.kS * fresnel<S>(ihp, P.eta) * g1i * g1o * D * q4;
        if (val(oh) > 0.0f) pxS = g1i * ihp * D * q4 * rcp_(oh);
    }
    S bxu = S(0), pxB = S(0);
    if (val(mu_o_g) > 0.0) {
        S mp = front_i ? mu_i : S(0);
        S fls = rcp_(S(float(4.0 * kPi)) * (mp + mu_o));
        bxu = P.B * P.r * (fls + S(float(1.0 / kPi))) * mu_o * rcp_(S(1) + ls_albedo<S>(mp));
        pxB = mu_o * S(float(1.0 / kPi));
    }
    a.ExS = ExS;
    a.pxS = pxS;
    a.bxu = bxu;
    a.pxB = pxB;
    a.EyS = a.pyS = a.by = a.pyB = S(0);
}

// dsig (nullable): accumulates the node sum of EyS with each term times
// ln(tau^N) = -sigma_t l N, from which dEyS / dsigma_t follows.
template <class G, class S>
__host__ __device__ inline void lobes_node_step(const Derived<G, S>& P, bool front_i, const Node<G, S>& nd,
                                                const V3<G>& wo_g, LobeAcc<S>& a, S* dsig = nullptr)
{
    G cyg = dot(wo_g, nd.fy.n);
    if (val(cyg) > 0.0) {
        S c = Narrow<S>::from(cyg) * S(float(1.0 / kPi));
        a.by = a.by + c;
        a.pyB = a.pyB + c;
    }
    if (front_i) {
        S vv, pd;
        exit_btdf(P, nd.wt, nd.fy, wo_g, &vv, &pd);
        a.EyS = a.EyS + nd.T * nd.att * vv;
        a.pyS = a.pyS + pd;
        if (dsig && val(nd.att) > 0.0f) *dsig = *dsig + nd.T * nd.att * vv * log_(nd.att);
    }
}

template <class G, class S, int MP>
__host__ __device__ inline void lobes_finish(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                             const LobeAcc<S>& a, EvalOut<S>& o)
{
    S invK = rcp_(S(float(P.K)));
    S EyS = a.EyS * (S(1) - P.B) * P.kS * invK;
    S pyS = a.pyS * invK;
    S byu = a.by * P.B * (S(1) - P.r) * invK;
    S pyB = a.pyB * invK;
    S gg = X.Gp * X.Gf;
    S bx = a.bxu * gg, byg = byu * gg;
    o.body0 = a.bxu + byu;
    o.ExS = a.ExS;
    o.EyS = EyS;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o.ExB[c] = bx * P.alb[c];
        o.EyB[c] = byg * P.alb[c];
        o.E[c] = a.ExS + EyS + o.ExB[c] + o.EyB[c];
    }
    o.pdf = X.w[0] * a.pxS + X.w[1] * pyS + X.w[2] * a.pxB + X.w[3] * pyB;
}

template <class G, class S, int MP, class NodeFn>
__host__ __device__ inline void lobes_nodes(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                            const V3<G>& wo_g, const NodeFn& node_of, EvalOut<S>& o)
{
    LobeAcc<S> a;
    lobes_at_x(P, X, wo_g, a);
    const bool front_i = val(X.mu_i) > 0.0f;
    for (int k = 0; k < P.K; ++k) {
        Node<G, S> nd;
        node_of(k, nd);
        lobes_node_step(P, front_i, nd, wo_g, a);
    }
    lobes_finish(P, X, a, o);
}

// The lobes at two directions of one hit (a given direction and a sampled
// one, say): the forward nodes depend on wi only, so each is computed once
// and serves both.  A direction whose flag is false is skipped and its
// output left untouched.
template <class G, class S, int MP, class NodeFn>
__host__ __device__ inline void lobes_nodes2(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                             const V3<G>& wo_a, bool use_a, const V3<G>& wo_b,
                                             bool use_b, const NodeFn& node_of, EvalOut<S>& oa,
                                             EvalOut<S>& ob)
{
    LobeAcc<S> a, b;
    if (use_a) lobes_at_x(P, X, wo_a, a);
    if (use_b) lobes_at_x(P, X, wo_b, b);
    const bool front_i = val(X.mu_i) > 0.0f;
    if (use_a || use_b) {
        for (int k = 0; k < P.K; ++k) {
            Node<G, S> nd;
            node_of(k, nd);
            if (use_a) lobes_node_step(P, front_i, nd, wo_a, a);
            if (use_b) lobes_node_step(P, front_i, nd, wo_b, b);
        }
    }
    if (use_a) lobes_finish(P, X, a, oa);
    if (use_b) lobes_finish(P, X, b, ob);
}

// lobes_nodes2 with, per direction, the derivative of E_yS with respect to
// sigma_t (Eq. 4: each node's term carries tau^N = exp(-sigma_t l N)):
// dEyS / dsigma_t = (1 - B) k_S / K sum_k T att f ln(att) / sigma_t.
template <class G, class S, int MP, class NodeFn>
__host__ __device__ inline void lobes_nodes2_dsigma(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                                    const V3<G>& wo_a, bool use_a, const V3<G>& wo_b,
                                                    bool use_b, const NodeFn& node_of, EvalOut<S>& oa,
                                                    EvalOut<S>& ob, S& dsa, S& dsb)
{
    LobeAcc<S> a, b;
    S ga = S(0), gb = S(0);
    if (use_a) lobes_at_x(P, X, wo_a, a);
    if (use_b) lobes_at_x(P, X, wo_b, b);
    const bool front_i = val(X.mu_i) > 0.0f;
    if (use_a || use_b) {
        for (int k = 0; k < P.K; ++k) {
            Node<G, S> nd;
            node_of(k, nd);
            if (use_a) lobes_node_step(P, front_i, nd, wo_a, a, &ga);
            if (use_b) lobes_node_step(P, front_i, nd, wo_b, b, &gb);
        }
    }
    if (use_a) lobes_finish(P, X, a, oa);
    if (use_b) lobes_finish(P, X, b, ob);
    const S f = val(P.sigma_t) > 0.0f ? (S(1) - P.B) * P.kS * rcp_(S(float(P.K)) * P.sigma_t) : S(0);
    dsa = ga * f;
    dsb = gb * f;
}

// node providers: compute node k from the state at x, or read it from an
// array filled beforehand (hits shared by many directions)
// disk: the record's node_disk (nullable: the disc points are then formed
// per node)
template <class G, class S, int MP, class Tab> struct NodesComputed {
    const Derived<G, S>& P;
    const Tab& tab;
    const XState<G, S, MP>& X;
    float s0, s1;
    bool has_shift;
    const double* disk = nullptr;
    __host__ __device__ void operator()(int k, Node<G, S>& nd) const
    {
        forward_node(P, tab, X, k, s0, s1, has_shift, nd, disk);
    }
};
template <class G, class S> struct NodesStored {
    const Node<G, S>* nodes;
    __host__ __device__ void operator()(int k, Node<G, S>& nd) const { nd = nodes[k]; }
};

template <class G, class S, int MP, class Tab>
__host__ __device__ inline void lobes(const Derived<G, S>& P, const Tab& tab, const XState<G, S, MP>& X,
                                      const V3<G>& wo_g, float s0, float s1, bool has_shift,
                                      EvalOut<S>& o, const double* disk = nullptr)
{
    NodesComputed<G, S, MP, Tab> nf{P, tab, X, s0, s1, has_shift, disk};
    lobes_nodes(P, X, wo_g, nf, o);
}

__host__ __device__ inline uint32_t check_inputs(float h, float u, float v, const V3<float>& a)
{
    bool bad = !(h >= -1.0f && h <= 1.0f) || !__builtin_isfinite(u) || !__builtin_isfinite(v);
    bad = bad || !__builtin_isfinite(a.x) || !__builtin_isfinite(a.y) || !__builtin_isfinite(a.z);
    if (!bad) {
        float l = sqrtf(a.x * a.x + a.y * a.y + a.z * a.z);
        bad = fabsf(l - 1.0f) > 1e-3f;
    }
    return bad ? F_BAD_INPUT : 0u;
}

__host__ __device__ inline uint32_t check_dir(const V3<float>& a)
{
    bool bad = !__builtin_isfinite(a.x) || !__builtin_isfinite(a.y) || !__builtin_isfinite(a.z);
    if (!bad) bad = fabsf(sqrtf(a.x * a.x + a.y * a.y + a.z * a.z) - 1.0f) > 1e-3f;
    return bad ? F_BAD_INPUT : 0u;
}


// ---------------------------------------------------------------- sampler

template <class S> struct SampleOut {
    S wo[3], wgt[3], pdf, ex[3];
    int lobe, node;
};

// Importance sampling (Sec. 4.1.5): xi0 picks a lobe with the selection
// weights (and, for the forward lobes, a node); visible-normal GGX samples
// the specular lobes (reflection at x, refraction out of the yarn at y),
// cosine lobes the body lobes.  The weight is the full value over the full
// mixture pdf at the drawn direction.  Lobes: 0 x-specular, 1 y-specular,
// 2 x-body, 3 y-body, 4 pass-through.
//
// First step: the lobe and node from xi0 (so.lobe, so.node; a pass-through
// fills the whole output).  Returns the flags.
template <class G, class S, int MP>
__host__ __device__ inline uint32_t sample_pick(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                                const V3<float>& wi, float xi0, SampleOut<S>& so)
{
    for (int c = 0; c < 3; ++c) {
        so.wo[c] = S(0); so.wgt[c] = S(0); so.ex[c] = S(0);
    }
    so.pdf = S(0);
    so.lobe = -1;
    so.node = 0;
    uint32_t flags = X.ph.flags;
    if (X.ph.pass) {
        so.wo[0] = S(-wi.x); so.wo[1] = S(-wi.y); so.wo[2] = S(-wi.z);
        so.wgt[0] = so.wgt[1] = so.wgt[2] = S(1);
        so.lobe = 4;
        return flags;
    }
    if (!(val(X.mu_i) > 0.0f)) flags |= F_BACKFACING;
    S c0 = X.w[0], c1 = c0 + X.w[1], c2 = c1 + X.w[2];
    float x0 = xi0;
    int lobe = x0 < val(c0) ? 0 : (x0 < val(c1) ? 1 : (x0 < val(c2) ? 2 : 3));
    int node = 0;
    if (lobe == 1 || lobe == 3) {
        S lo = lobe == 1 ? c0 : c2;
        S wl = lobe == 1 ? X.w[1] : X.w[3];
        S xk = (S(x0) - lo) / wl * S(float(P.K));
        int nk = (int)floorf(val(xk));
        node = nk > P.K - 1 ? P.K - 1 : (nk < 0 ? 0 : nk);
    }
    so.lobe = lobe;
    so.node = node;
    return flags;
}

// Second step: the direction of the picked lobe.  nd is the picked node
// (read for the forward lobes only).  Each step below runs once per
// wavefront whatever mix of lobes its lanes drew: one visible-normal sample
// (specular lobes: the frame at x or the node's inside-facing exit frame),
// one cosine sample (body lobes).  Sets the exit point and returns whether a
// direction was drawn (wo normalised).
template <class G, class S, int MP>
__host__ __device__ inline bool sample_dir(const Derived<G, S>& P, const XState<G, S, MP>& X, int lobe,
                                           const Node<G, S>& nd, float xi1, float xi2, SampleOut<S>& so,
                                           V3<G>& wo)
{
    StageMark<G> mark(kStageSample);
    bool ok = false;
    wo = mk3<G>(G(0), G(0), G(0));
    const bool fwd = lobe == 1 || lobe == 3;
    V3<G> ex = fwd ? nd.y : mk3<G>(X.ph.p2x, X.ph.p2y, X.ph.vhit);
    const G gx1 = G((double)xi1), gx2 = G((double)xi2);
    if (lobe <= 1) {
        // reflection at x, or refraction out of the yarn at the node's
        // exit point (visible normals seen from inside, up = -n_y)
        Frame<G> F;
        V3<G> w;
        if (lobe == 0) {
            F = X.fx;
            w = X.wi_g;
        } else {
            F.t = nd.fy.t;
            F.n = -nd.fy.n;
            F.b = cross(F.n, F.t);
            w = -nd.wt;
        }
        V3<G> wl = to_local(F, w);
        if (val(wl.z) > 0.0 && (lobe == 0 || val(X.mu_i) > 0.0f)) {
            V3<G> ml = sample_vndf<G>(wl, P.ax_g, P.ay_g, gx1, gx2);
            V3<G> mw = to_world(F, ml);
            if (lobe == 0) {
                wo = mw * (G(2) * dot(X.wi_g, mw)) - X.wi_g;
                ok = val(dot(wo, X.fx.n)) > 0.0;
            } else {
                G c = dot(w, mw);
                c = val(c) > 0.0 ? c : G(0);
                G s2t = P.eta_g * P.eta_g * (G(1) - c * c);
                if (val(s2t) < 1.0) {
                    G ct = sqrt_(G(1) - s2t);
                    wo = w * (-P.eta_g) + mw * (P.eta_g * c - ct);
                    ok = val(dot(wo, nd.fy.n)) > 0.0;
                }
            }
        }
    } else {
        // cosine lobe about the fiber normal at x or at the node's exit
        Frame<G> fr = lobe == 2 ? X.fx : nd.fy;
        G rad = sqrt_(gx1);
        G su, cu;
        sincos_turns_g(gx2, &su, &cu);
        G z = G(1) - gx1;
        wo = to_world(fr, mk3<G>(rad * cu, rad * su, val(z) > 0.0 ? sqrt_(z) : G(0)));
        ok = true;
    }
    so.ex[0] = Narrow<S>::from(ex.x);
    so.ex[1] = Narrow<S>::from(ex.y);
    so.ex[2] = Narrow<S>::from(ex.z);
    if (ok) wo = normalize(wo);
    return ok;
}

// Both steps: the drawn direction in wo, ok when a direction was drawn.
template <class G, class S, int MP, class NodeFn>
__host__ __device__ inline uint32_t sample_draw(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                                const V3<float>& wi, float xi0, float xi1, float xi2,
                                                const NodeFn& node_of, SampleOut<S>& so, V3<G>& wo,
                                                bool& ok)
{
    wo = mk3<G>(G(0), G(0), G(0));
    ok = false;
    uint32_t flags = sample_pick(P, X, wi, xi0, so);
    if (X.ph.pass) return flags;
    Node<G, S> nd;
    if (so.lobe == 1 || so.lobe == 3) node_of(so.node, nd);
    ok = sample_dir(P, X, so.lobe, nd, xi1, xi2, so, wo);
    return ok ? flags : flags | F_SAMPLE_FAIL;
}

// Last step of the sampler: weight and pdf from the lobes at the drawn
// direction; a direction of zero density counts as a failed draw.
template <class G, class S>
__host__ __device__ inline uint32_t sample_finish(const EvalOut<S>& e, const V3<G>& wo, uint32_t flags,
                                                  SampleOut<S>& so)
{
    if (!(val(e.pdf) > 0.0f)) return flags | F_SAMPLE_FAIL;
    so.wo[0] = Narrow<S>::from(wo.x);
    so.wo[1] = Narrow<S>::from(wo.y);
    so.wo[2] = Narrow<S>::from(wo.z);
    S ip = rcp_(e.pdf);
    for (int c = 0; c < 3; ++c) so.wgt[c] = e.E[c] * ip;
    so.pdf = e.pdf;
    return flags;
}

// A drawn direction and, optionally, a given one on the same hit, with the
// forward nodes computed once.  The node loop starts at the node the draw
// picked (node 0 for the lobes at x), so the draw takes its frame from the
// first iteration and every node serves both directions: K nodes per query,
// summed in the rotated order.  The given direction's output is written only
// when eval_ok and the hit is not a pass-through; returns the sampler's flags.
template <class G, class S, int MP, class NodeFn>
__host__ __device__ inline uint32_t sample_eval_nodes(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                                      const V3<float>& wi, const V3<G>& wo_q, bool eval_ok,
                                                      float xi0, float xi1, float xi2, const NodeFn& node_of,
                                                      EvalOut<S>& eo, SampleOut<S>& so)
{
    uint32_t flags = sample_pick(P, X, wi, xi0, so);
    if (X.ph.pass) return flags;
    const int lobe = so.lobe;
    const int k0 = (lobe == 1 || lobe == 3) ? so.node : 0;
    LobeAcc<S> a, b;
    if (eval_ok) lobes_at_x(P, X, wo_q, a);
    const bool front_i = val(X.mu_i) > 0.0f;
    V3<G> ws;
    bool ok;
    {
        Node<G, S> nd;
        node_of(k0, nd);
        ok = sample_dir(P, X, lobe, nd, xi1, xi2, so, ws);
        if (ok) lobes_at_x(P, X, ws, b);
        if (eval_ok) lobes_node_step(P, front_i, nd, wo_q, a);
        if (ok) lobes_node_step(P, front_i, nd, ws, b);
    }
    for (int j = 1; j < P.K; ++j) {
        int k = k0 + j;
        k = k >= P.K ? k - P.K : k;
        Node<G, S> nd;
        node_of(k, nd);
        if (eval_ok) lobes_node_step(P, front_i, nd, wo_q, a);
        if (ok) lobes_node_step(P, front_i, nd, ws, b);
    }
    if (eval_ok) lobes_finish(P, X, a, eo);
    if (!ok) return flags | F_SAMPLE_FAIL;
    EvalOut<S> es;
    lobes_finish(P, X, b, es);
    return sample_finish(es, ws, flags, so);
}

template <class G, class S, int MP, class NodeFn>
__host__ __device__ inline uint32_t sample_from_x(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                                  const V3<float>& wi, float xi0, float xi1,
                                                  float xi2, const NodeFn& node_of,
                                                  SampleOut<S>& so)
{
    EvalOut<S> unused;
    return sample_eval_nodes(P, X, wi, mk3<G>(G(0), G(0), G(0)), false, xi0, xi1, xi2, node_of, unused, so);
}

// Evaluation at a given direction wo_q and one sampled direction for the
// same hit, sharing the state at x and the forward nodes.  The eval output
// is written only when eval_ok (the given direction is valid) and the hit is
// not a pass-through; returns the sampler's flags.
template <class G, class S, int MP, class NodeFn>
__host__ __device__ inline uint32_t eval_sample_from_x(const Derived<G, S>& P, const XState<G, S, MP>& X,
                                                       const V3<float>& wi, const V3<G>& wo_q,
                                                       bool eval_ok, float xi0, float xi1, float xi2,
                                                       const NodeFn& node_of, EvalOut<S>& eo,
                                                       SampleOut<S>& so)
{
    return sample_eval_nodes(P, X, wi, wo_q, eval_ok, xi0, xi1, xi2, node_of, eo, so);
}

template <class G, class S, int MP, class Tab>
__host__ __device__ inline uint32_t sample_query(const Derived<G, S>& P, const Tab& tab, float h,
                                                 float u, float v, const V3<float>& wi, float xi0,
                                                 float xi1, float xi2, float s0, float s1,
                                                 bool has_shift, SampleOut<S>& so,
                                                 const double* disk = nullptr)
{
    uint32_t bad = check_inputs(h, u, v, wi);
    if (bad) {
        for (int c = 0; c < 3; ++c) {
            so.wo[c] = S(0); so.wgt[c] = S(0); so.ex[c] = S(0);
        }
        so.pdf = S(0);
        so.lobe = -1;
        so.node = 0;
        return bad;
    }
    XState<G, S, MP> X;
    state_at_x(P, tab, h, u, v, wi, X);
    NodesComputed<G, S, MP, Tab> nf{P, tab, X, s0, s1, has_shift, disk};
    return sample_from_x(P, X, wi, xi0, xi1, xi2, nf, so);
}

}  // namespace bysdf
