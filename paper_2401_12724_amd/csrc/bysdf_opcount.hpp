// bysdf_opcount.hpp -- counting scalars: running the per-query model on the
// host with these in place of double / float tallies the algorithmic
// operations of the kernels' formulation (one query at a time).
#pragma once

#include "bysdf_model.hpp"

namespace bysdf {

struct OpTally {
    // [0] geometry scalar (FP64), [1] shading scalar (FP32)
    double add[2], mul[2], div[2], sqrt[2], trans[2];
};

extern thread_local OpTally* g_tally;

template <class T, int P> struct Cnt {
    T v;
    Cnt() = default;
    Cnt(double x) : v((T)x) {}
    Cnt(float x) : v((T)x) {}
    Cnt(int x) : v((T)x) {}
    static void add() { if (g_tally) g_tally->add[P] += 1; }
    static void mul() { if (g_tally) g_tally->mul[P] += 1; }
    static void div() { if (g_tally) g_tally->div[P] += 1; }
};
template <class T, int P> inline Cnt<T, P> mkc(T x) { Cnt<T, P> r; r.v = x; return r; }
template <class T, int P> inline Cnt<T, P> operator+(Cnt<T, P> a, Cnt<T, P> b) { Cnt<T, P>::add(); return mkc<T, P>(a.v + b.v); }
template <class T, int P> inline Cnt<T, P> operator-(Cnt<T, P> a, Cnt<T, P> b) { Cnt<T, P>::add(); return mkc<T, P>(a.v - b.v); }
template <class T, int P> inline Cnt<T, P> operator*(Cnt<T, P> a, Cnt<T, P> b) { Cnt<T, P>::mul(); return mkc<T, P>(a.v * b.v); }
template <class T, int P> inline Cnt<T, P> operator/(Cnt<T, P> a, Cnt<T, P> b) { Cnt<T, P>::div(); return mkc<T, P>(a.v / b.v); }
template <class T, int P> inline Cnt<T, P> operator-(Cnt<T, P> a) { return mkc<T, P>(-a.v); }

using CD = Cnt<double, 0>;
using CF = Cnt<float, 1>;

inline double val(CD x) { return x.v; }
inline float val(CF x) { return x.v; }
#define BYSDF_CNT_FN1(name, fn, kind)                                                  \
    inline CD name(CD x) { if (g_tally) g_tally->kind[0] += 1; return mkc<double, 0>(fn(x.v)); } \
    inline CF name(CF x) { if (g_tally) g_tally->kind[1] += 1; return mkc<float, 1>((float)fn(x.v)); }
BYSDF_CNT_FN1(sqrt_, std::sqrt, sqrt)
BYSDF_CNT_FN1(sin_, std::sin, trans)
BYSDF_CNT_FN1(cos_, std::cos, trans)
BYSDF_CNT_FN1(asin_, std::asin, trans)
BYSDF_CNT_FN1(exp_, std::exp, trans)
BYSDF_CNT_FN1(log_, std::log, trans)
#undef BYSDF_CNT_FN1
inline CD rcp_(CD x) { if (g_tally) g_tally->div[0] += 1; return mkc<double, 0>(1.0 / x.v); }
inline CF rcp_(CF x) { if (g_tally) g_tally->div[1] += 1; return mkc<float, 1>(1.0f / x.v); }
inline CD rsqrt_(CD x) { if (g_tally) g_tally->sqrt[0] += 1; return mkc<double, 0>(1.0 / std::sqrt(x.v)); }
inline CF rsqrt_(CF x) { if (g_tally) g_tally->sqrt[1] += 1; return mkc<float, 1>(1.0f / std::sqrt(x.v)); }
inline CD atan2_(CD y, CD x) { if (g_tally) g_tally->trans[0] += 1; return mkc<double, 0>(std::atan2(y.v, x.v)); }
inline CF atan2_(CF y, CF x) { if (g_tally) g_tally->trans[1] += 1; return mkc<float, 1>(std::atan2(y.v, x.v)); }
template <> __host__ __device__ inline CD floor_g<CD>(const CD& x) { if (g_tally) g_tally->add[0] += 1; return mkc<double, 0>(std::floor(x.v)); }
template <> __host__ __device__ inline void sincos_turns_g<CD>(const CD& t, CD* s, CD* c)
{
    if (g_tally) { g_tally->add[0] += 2; g_tally->mul[0] += 1; g_tally->trans[0] += 2; }
    double ss, cc;
    sincos_turns(t.v, &ss, &cc);
    *s = mkc<double, 0>(ss);
    *c = mkc<double, 0>(cc);
}
template <> struct Narrow<CF> {
    static CF from(CD x) { return mkc<float, 1>((float)x.v); }
    static CF from(CF x) { return x; }
    static CF from(double x) { return mkc<float, 1>((float)x); }
};

inline Derived<CD, CF> derive_counted(const TypeRec& t) { return rebind<CD, CF>(derive(t)); }

}  // namespace bysdf
