// bysdf_dual.hpp -- forward-mode dual scalars for the adjoint kernel.
//
// A Dual<T> carries a value and one tangent.  Running the per-query model
// with Dual<double> geometry and Dual<float> shading, seeded on one
// parameter, yields the derivative of every output with respect to that
// parameter; branch decisions use the value only (the derivative of the
// piecewise-smooth model away from its decision boundaries).
#pragma once

#include "bysdf_model.hpp"

namespace bysdf {

template <class T> struct Dual {
    T v, d;
    __host__ __device__ Dual() = default;
    __host__ __device__ Dual(double x) : v((T)x), d((T)0) {}
    __host__ __device__ Dual(float x) : v((T)x), d((T)0) {}
    __host__ __device__ Dual(int x) : v((T)x), d((T)0) {}
    __host__ __device__ static Dual make(T v, T d)
    {
        Dual r;
        r.v = v;
        r.d = d;
        return r;
    }
};

template <class T> __host__ __device__ inline Dual<T> operator+(Dual<T> a, Dual<T> b)
{
    return Dual<T>::make(a.v + b.v, a.d + b.d);
}
template <class T> __host__ __device__ inline Dual<T> operator-(Dual<T> a, Dual<T> b)
{
    return Dual<T>::make(a.v - b.v, a.d - b.d);
}
template <class T> __host__ __device__ inline Dual<T> operator-(Dual<T> a)
{
    return Dual<T>::make(-a.v, -a.d);
}
template <class T> __host__ __device__ inline Dual<T> operator*(Dual<T> a, Dual<T> b)
{
    return Dual<T>::make(a.v * b.v, a.d * b.v + a.v * b.d);
}
template <class T> __host__ __device__ inline Dual<T> operator/(Dual<T> a, Dual<T> b)
{
    T q = a.v / b.v;
    return Dual<T>::make(q, (a.d - q * b.d) / b.v);
}

using DD = Dual<double>;
using DF = Dual<float>;

__host__ __device__ inline double val(DD x) { return x.v; }
__host__ __device__ inline float val(DF x) { return x.v; }

template <class T> __host__ __device__ inline Dual<T> sqrt_(Dual<T> x)
{
    T s = sqrt_(x.v);
    return Dual<T>::make(s, s > (T)0 ? x.d / ((T)2 * s) : (T)0);
}
template <class T> __host__ __device__ inline Dual<T> rcp_(Dual<T> x)
{
    T r = rcp_(x.v);
    return Dual<T>::make(r, -x.d * r * r);
}
template <class T> __host__ __device__ inline Dual<T> rsqrt_(Dual<T> x)
{
    T r = rsqrt_(x.v);
    return Dual<T>::make(r, (T)(-0.5) * r * r * r * x.d);
}
template <class T> __host__ __device__ inline Dual<T> sin_(Dual<T> x)
{
    return Dual<T>::make(sin_(x.v), cos_(x.v) * x.d);
}
template <class T> __host__ __device__ inline Dual<T> cos_(Dual<T> x)
{
    return Dual<T>::make(cos_(x.v), -sin_(x.v) * x.d);
}
template <class T> __host__ __device__ inline Dual<T> exp_(Dual<T> x)
{
    T e = exp_(x.v);
    return Dual<T>::make(e, e * x.d);
}
template <class T> __host__ __device__ inline Dual<T> log_(Dual<T> x)
{
    return Dual<T>::make(log_(x.v), x.d / x.v);
}
template <class T> __host__ __device__ inline Dual<T> asin_(Dual<T> x)
{
    T c = sqrt_((T)1 - x.v * x.v);
    return Dual<T>::make(asin_(x.v), c > (T)0 ? x.d / c : (T)0);
}
template <class T> __host__ __device__ inline Dual<T> atan2_(Dual<T> y, Dual<T> x)
{
    T r2 = x.v * x.v + y.v * y.v;
    return Dual<T>::make(atan2_(y.v, x.v), r2 > (T)0 ? (x.v * y.d - y.v * x.d) / r2 : (T)0);
}
__host__ __device__ inline DD tan_(DD x)
{
    double t = tan(x.v);
    return DD::make(t, (1.0 + t * t) * x.d);
}

template <> __host__ __device__ inline DD floor_g<DD>(const DD& x) { return DD::make(floor(x.v), 0.0); }
template <> __host__ __device__ inline void sincos_turns_g<DD>(const DD& t, DD* s, DD* c)
{
    double sv, cv;
    sincos_turns(t.v, &sv, &cv);
    *s = DD::make(sv, kTwoPi * cv * t.d);
    *c = DD::make(cv, -kTwoPi * sv * t.d);
}
template <> struct Narrow<DF> {
    __host__ __device__ static DF from(DD x) { return DF::make((float)x.v, (float)x.d); }
    __host__ __device__ static DF from(DF x) { return x; }
    __host__ __device__ static DF from(double x) { return DF::make((float)x, 0.0f); }
    __host__ __device__ static DF from(float x) { return DF::make(x, 0.0f); }
};

// Plain values as duals with zero tangents (parts of the model that do not
// depend on the seeded parameter are computed in plain arithmetic).
__host__ __device__ inline V3<DD> promote(const V3<double>& a) { return mk3<DD>(DD(a.x), DD(a.y), DD(a.z)); }
__host__ __device__ inline V3<DF> promote(const V3<float>& a) { return mk3<DF>(DF(a.x), DF(a.y), DF(a.z)); }
template <class T> __host__ __device__ inline Frame<Dual<T>> promote(const Frame<T>& f)
{
    Frame<Dual<T>> g;
    g.t = promote(f.t);
    g.b = promote(f.b);
    g.n = promote(f.n);
    return g;
}
template <int MP> __host__ __device__ inline void promote(const PlyHit<double, MP>& a, PlyHit<DD, MP>& b)
{
    b.pass = a.pass;
    b.flags = a.flags;
    b.x2x = DD(a.x2x); b.x2y = DD(a.x2y); b.dhx = DD(a.dhx); b.dhy = DD(a.dhy);
    b.kappa = DD(a.kappa);
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        b.cth[k] = DD(a.cth[k]);
        b.sth[k] = DD(a.sth[k]);
    }
    b.ks = a.ks;
    b.p2x = DD(a.p2x); b.p2y = DD(a.p2y); b.n2x = DD(a.n2x); b.n2y = DD(a.n2y);
    b.vhit = DD(a.vhit);
}
template <int MP>
__host__ __device__ inline void promote(const XState<double, float, MP>& a, XState<DD, DF, MP>& b)
{
    promote(a.ph, b.ph);
    b.fx = promote(a.fx);
    b.fxs = promote(a.fxs);
    b.wi_g = promote(a.wi_g);
    b.wi_s = promote(a.wi_s);
    b.Gp = DF(a.Gp);
    b.Gf = DF(a.Gf);
    b.mu_i = DF(a.mu_i);
    for (int k = 0; k < 4; ++k) b.w[k] = DF(a.w[k]);
    b.a = DD(a.a);
    b.rawp = DD(a.rawp);
    b.rawf = DD(a.rawf);
}

// Scalars of one type with the tangent seeded on one differentiable
// parameter: 0 beta, 1 ply twist, 2 fiber twist.
__host__ __device__ inline Derived<DD, DF> derive_dual(const TypeRec& t, int seed)
{
    const Derived<double, float>& f = t.d;
    Derived<DD, DF> d;
    d.Np = f.Np; d.K = f.K; d.N_it = f.N_it; d.Nu = f.Nu; d.inv_np = f.inv_np;
    DD beta = DD::make(t.beta, seed == 0 ? 1.0 : 0.0);
    DD ap = DD::make(t.ply_twist, seed == 1 ? 1.0 : 0.0);
    DD af = DD::make(t.fiber_twist, seed == 2 ? 1.0 : 0.0);
    d.rp = DD(t.rp);
    d.Rpc = DD(t.Rpc);
    DD tap = tan_(ap);
    DD wp = t.Rpc > 0.0 ? tap / DD(t.Rpc) : DD(0.0);
    d.slope = DD(t.Rpc) * wp;
    d.vply_scale = sqrt_(DD(1.0) + d.slope * d.slope);
    d.tnorm_inv = DD(1.0) / d.vply_scale;
    d.wp_turns = wp * DD(kInvTwoPi);
    d.tan_af = tan_(af);
    d.wf_turns = d.tan_af / DD((1.0 - t.rho_f_geom) * t.rp) * DD(kInvTwoPi);
    d.ax_g = beta;
    d.ay_g = beta * DD(t.aniso);
    d.eta_g = DD(t.eta);
    d.inv_eta_g = DD(1.0 / t.eta);
    d.ax = Narrow<DF>::from(d.ax_g);
    d.ay = Narrow<DF>::from(d.ay_g);
    d.eta = DF(f.eta);
    d.kS = DF(f.kS); d.B = DF(f.B); d.r = DF(f.r); d.sigma_t = DF(f.sigma_t);
    d.rho_p = DF(f.rho_p); d.rho_f = DF(f.rho_f); d.dP = DF(f.dP);
    for (int c = 0; c < 3; ++c) d.alb[c] = DF(f.alb[c]);
    d.rp_s = DF(f.rp_s);
    d.Rpc_s = DF(f.Rpc_s);
    d.n_mig = f.n_mig; d.mig_seed = f.mig_seed; d.mig_period = f.mig_period; d.mig_blend = f.mig_blend;
    for (int k = 0; k < kMaxPlies; ++k) {
        d.ply_c[k] = f.ply_c[k];
        d.ply_s[k] = f.ply_s[k];
    }
    return d;
}

}  // namespace bysdf
