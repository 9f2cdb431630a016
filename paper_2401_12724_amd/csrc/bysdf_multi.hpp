// bysdf_multi.hpp -- the multi-scale BYSDF (Sec. 4.2, Eq. 8-11) on top of
// the near-field model of bysdf_model.hpp.
//
// A query carries the pixel footprint on the yarn: the azimuthal offsets
// h1 <= h0 <= h2 of the ray differentials around the hit offset h0
// (Sec. 5.3) and a strata offset zeta.  The footprint is cut into
// n = ceil(n_max (h2 - h1) / 2) strata h_j = h1 + (h2 - h1)(j + zeta)/n
// (rounded to FP32, the precision of a query's h), each weighted by a tent
// W that is 1 at h0 and falls to 0 at h1 and at h2 (a single stratum
// weighs 1).  Over the strata that hit a ply:
//   - the fiber normal and tangent at x are averaged with W (Eq. 9-10);
//     the mean normal is normalised and the mean tangent made orthogonal
//     to it, and a single contributing stratum keeps its own frame;
//   - the fiber shadowing G_f is averaged with W (Eq. 11);
//   - the specular roughness widens to beta + (h2 - h1) / 2: linear in the
//     covered range, normalised by the full range of the far field.
// f_multi (Eq. 8) is the W-weighted mean over all strata of the near-field
// model at each stratum's own ply hit, evaluated with that aggregated frame
// and shadowing; a stratum that passes between the plies contributes 0.
// The sampler draws a stratum with probability W / sum W, passes the ray
// through if that stratum does, and otherwise draws from the stratum's
// aggregated state; its weight and pdf are those of f_multi.
#pragma once

#include "bysdf_model.hpp"

namespace bysdf {

constexpr int kMaxStrata = 16;

struct Footprint {
    double h0, h1, h2, zeta;
    int n;
    double wsum;
};

__host__ __device__ inline uint32_t check_footprint(float h0, float h1, float h2, float zeta)
{
    // false for NaN as well
    const bool ok = h1 >= -1.0f && h1 <= h0 && h0 <= h2 && h2 <= 1.0f && zeta >= 0.0f && zeta < 1.0f;
    return ok ? 0u : F_BAD_INPUT;
}

// stratum offset: one FMA and an IEEE quotient in FP64, then FP32
__host__ __device__ inline float stratum_h(const Footprint& f, int j)
{
    return (float)fma(f.h2 - f.h1, ((double)j + f.zeta) / (double)f.n, f.h1);
}

__host__ __device__ inline double stratum_w(const Footprint& f, double hj)
{
    if (f.n == 1) return 1.0;
    if (hj < f.h0) return 1.0 - (f.h0 - hj) / (f.h0 - f.h1);
    if (f.h2 > f.h0) return 1.0 - (hj - f.h0) / (f.h2 - f.h0);
    return 1.0;
}

__host__ __device__ inline void make_footprint(float h0, float h1, float h2, float zeta, int n_max,
                                               Footprint& f)
{
    f.h0 = h0;
    f.h1 = h1;
    f.h2 = h2;
    f.zeta = zeta;
    // exact in FP64: a difference of two FP32 values times a small integer
    const int n = (int)ceil((double)n_max * (f.h2 - f.h1) * 0.5);
    f.n = n < 1 ? 1 : (n > n_max ? n_max : n);
    f.wsum = 0.0;
    for (int j = 0; j < f.n; ++j) f.wsum += stratum_w(f, (double)stratum_h(f, j));
}

// The type's scalars with the footprint's widened roughness.
template <class G, class S>
__host__ __device__ inline Derived<G, S> widened(const Derived<G, S>& P, double beta, double aniso,
                                                 const Footprint& f)
{
    Derived<G, S> Pm = P;
    const double bm = beta + (f.h2 - f.h1) * 0.5;
    Pm.ax_g = G(bm);
    Pm.ay_g = G(bm * aniso);
    Pm.ax = S(float(bm));
    Pm.ay = S(float(bm * aniso));
    return Pm;
}

// What the aggregation needs of a stratum: the ply hit, the fiber frame and
// the raw fiber visibility (the values state_at_x computes for them; the
// ply horizon and the lobe weights are left out).
template <class G, class S, int MP, class Tab>
__host__ __device__ inline bool stratum_frame(const Derived<G, S>& P, const Tab& tab, float h, float u, float v,
                                              const V3<float>& wi, Frame<G>& fx, G& rawf, uint32_t& flags)
{
    PlyHit<G, MP> ph;
    trace_plies(P, h, u, v, wi, ph);
    flags = ph.flags;
    if (ph.pass) return false;
    G cth = G(0), sth = G(0);
#pragma unroll
    for (int k = 0; k < MP; ++k)
        if (k == ph.ks) {
            cth = ph.cth[k];
            sth = ph.sth[k];
        }
    G a;
    fx = fiber_frame(P, tab, cth, sth, ph.ks, ph.n2x, ph.n2y, ph.vhit, &rawf, &a);
    return true;
}

// The aggregated frame and fiber shadowing of the footprint (Eq. 9-11).
// Returns false when no stratum of positive weight hits a ply.  Flags of
// the strata's ply traces (but pass-through) are or-ed into `flags`.
template <class G, class S, int MP, class Tab>
__host__ __device__ inline bool footprint_geometry(const Derived<G, S>& P, const Tab& tab,
                                                   const Footprint& f, float u, float v,
                                                   const V3<float>& wi, Frame<G>& F, S& Gm,
                                                   uint32_t& flags)
{
    V3<G> sn = mk3<G>(G(0), G(0), G(0)), st = sn;
    G sg = G(0);
    double sw = 0.0;
    int have = 0;
    for (int j = 0; j < f.n; ++j) {
        const float hj = stratum_h(f, j);
        const double w = stratum_w(f, (double)hj);
        Frame<G> fx;
        G rawf;
        uint32_t sfl;
        const bool hit = stratum_frame<G, S, MP>(P, tab, hj, u, v, wi, fx, rawf, sfl);
        flags |= sfl & ~F_PASS_THROUGH;
        if (!hit || !(w > 0.0)) continue;
        const G gf = G(1) - G(val(P.rho_f)) * (G(1) - rawf);
        if (have == 0) {
            F = fx;
            Gm = Narrow<S>::from(gf);
        }
        const G gw = G(w);
        sn = sn + fx.n * gw;
        st = st + fx.t * gw;
        sg = sg + gf * gw;
        sw += w;
        ++have;
    }
    if (have == 0) return false;
    if (have == 1) return true;
    Gm = Narrow<S>::from(sg / G(sw));
    const G ln2 = dot(sn, sn);
    if (!(val(ln2) > 1e-24 * sw * sw)) return true;
    const V3<G> n = sn * rsqrt_(ln2);
    const V3<G> t = st - n * dot(st, n);
    const G lt2 = dot(t, t);
    if (!(val(lt2) > 1e-24 * sw * sw)) return true;
    F.n = n;
    F.t = t * rsqrt_(lt2);
    F.b = cross(F.n, F.t);
    return true;
}

// A stratum's state at x with the footprint's aggregated frame and shadowing.
template <class G, class S, int MP>
__host__ __device__ inline void apply_aggregate(const Derived<G, S>& P, XState<G, S, MP>& X,
                                                const Frame<G>& F, S Gm)
{
    X.fx = F;
    X.fxs = narrowf<S>(F);
    X.Gf = Gm;
    lobe_weights(P, X);
}

// f_multi and its pdf at wo (Eq. 8); the outputs are laid out as the
// near-field evaluation's.  Returns the flags.
template <class G, class S, int MP, class Tab>
__host__ __device__ inline uint32_t eval_multi(const Derived<G, S>& Pm, const Tab& tab, const Footprint& f,
                                               float u, float v, const V3<float>& wi,
                                               const V3<float>& wo, float s0, float s1, bool has_shift,
                                               EvalOut<S>& o)
{
    for (int c = 0; c < 3; ++c) o.E[c] = o.ExB[c] = o.EyB[c] = S(0);
    o.ExS = o.EyS = o.pdf = S(0);
    uint32_t fl = 0;
    Frame<G> F;
    S Gm;
    if (!footprint_geometry<G, S, MP>(Pm, tab, f, u, v, wi, F, Gm, fl)) return fl | F_PASS_THROUGH;
    const V3<G> wo_g = mk3<G>(G((double)wo.x), G((double)wo.y), G((double)wo.z));
    for (int j = 0; j < f.n; ++j) {
        const float hj = stratum_h(f, j);
        XState<G, S, MP> X;
        state_at_x(Pm, tab, hj, u, v, wi, X);
        if (X.ph.pass) continue;
        apply_aggregate(Pm, X, F, Gm);
        if (!(val(X.mu_i) > 0.0f)) fl |= F_BACKFACING;
        EvalOut<S> e;
        lobes(Pm, tab, X, wo_g, s0, s1, has_shift, e);
        const S w = S(float(stratum_w(f, (double)hj)));
        for (int c = 0; c < 3; ++c) {
            o.E[c] = o.E[c] + w * e.E[c];
            o.ExB[c] = o.ExB[c] + w * e.ExB[c];
            o.EyB[c] = o.EyB[c] + w * e.EyB[c];
        }
        o.ExS = o.ExS + w * e.ExS;
        o.EyS = o.EyS + w * e.EyS;
        o.pdf = o.pdf + w * e.pdf;
    }
    const S iw = S(float(1.0 / f.wsum));
    for (int c = 0; c < 3; ++c) {
        o.E[c] = o.E[c] * iw;
        o.ExB[c] = o.ExB[c] * iw;
        o.EyB[c] = o.EyB[c] * iw;
    }
    o.ExS = o.ExS * iw;
    o.EyS = o.EyS * iw;
    o.pdf = o.pdf * iw;
    return fl;
}

// The multi-scale sampler.  so.node holds node + 16 x stratum.
template <class G, class S, int MP, class Tab>
__host__ __device__ inline uint32_t sample_multi(const Derived<G, S>& Pm, const Tab& tab,
                                                 const Footprint& f, float xi_s, float u, float v,
                                                 const V3<float>& wi, float xi0, float xi1, float xi2,
                                                 float s0, float s1, bool has_shift, SampleOut<S>& so)
{
    for (int c = 0; c < 3; ++c) so.wo[c] = so.wgt[c] = so.ex[c] = S(0);
    so.pdf = S(0);
    so.lobe = -1;
    so.node = 0;
    // the stratum: the first whose cumulative weight exceeds xi_s sum W
    int s = f.n - 1;
    {
        const double xw = (double)xi_s * f.wsum;
        double cum = 0.0;
        for (int j = 0; j < f.n - 1; ++j) {
            cum += stratum_w(f, (double)stratum_h(f, j));
            if (xw < cum) {
                s = j;
                break;
            }
        }
    }
    uint32_t fl = 0;
    Frame<G> F;
    S Gm;
    const bool any = footprint_geometry<G, S, MP>(Pm, tab, f, u, v, wi, F, Gm, fl);
    V3<G> wo;
    bool ok = false;
    bool pass = !any;
    if (any) {
        XState<G, S, MP> X;
        state_at_x(Pm, tab, stratum_h(f, s), u, v, wi, X);
        pass = X.ph.pass;
        if (!pass) {
            apply_aggregate(Pm, X, F, Gm);
            NodesComputed<G, S, MP, Tab> nf{Pm, tab, X, s0, s1, has_shift};
            fl |= sample_draw(Pm, X, wi, xi0, xi1, xi2, nf, so, wo, ok);
        }
    }
    if (pass) {
        so.wo[0] = S(-wi.x);
        so.wo[1] = S(-wi.y);
        so.wo[2] = S(-wi.z);
        so.wgt[0] = so.wgt[1] = so.wgt[2] = S(1);
        so.lobe = 4;
        so.node = 16 * s;
        return fl | F_PASS_THROUGH;
    }
    so.node += 16 * s;
    if (!ok) return fl;
    // f_multi and its pdf at the drawn direction
    EvalOut<S> em;
    em.E[0] = em.E[1] = em.E[2] = S(0);
    em.pdf = S(0);
    for (int j = 0; j < f.n; ++j) {
        const float hj = stratum_h(f, j);
        XState<G, S, MP> X;
        state_at_x(Pm, tab, hj, u, v, wi, X);
        if (X.ph.pass) continue;
        apply_aggregate(Pm, X, F, Gm);
        EvalOut<S> e;
        lobes(Pm, tab, X, wo, s0, s1, has_shift, e);
        const S w = S(float(stratum_w(f, (double)hj)));
        for (int c = 0; c < 3; ++c) em.E[c] = em.E[c] + w * e.E[c];
        em.pdf = em.pdf + w * e.pdf;
    }
    const S iw = S(float(1.0 / f.wsum));
    for (int c = 0; c < 3; ++c) em.E[c] = em.E[c] * iw;
    em.pdf = em.pdf * iw;
    return sample_finish(em, wo, fl, so);
}

}  // namespace bysdf
