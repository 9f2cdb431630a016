// bysdf_precision.hpp -- a host-side geometry scalar for the precision
// audit: the kernels' per-query model run on the host with the arithmetic
// of chosen stages of the geometry chain (GeomStage) rounded to single
// precision.
//
// An Emu holds a double.  Inside a scope whose stage is selected by the
// thread's mask, every operation rounds its operands and its result to the
// nearest float, so the stage computes as a single-precision stage would:
// values entering it are converted to float, every intermediate is a float.
// Elementary functions are evaluated in double on the rounded argument and
// rounded once (correctly rounded single precision; the hardware's FP32
// transcendentals are within a few ulp of that).  Outside selected stages
// an Emu computes in double exactly as the kernels' geometry scalar.
//
// A measurement tool only: nothing on the library's compute path uses it.
#pragma once

#include <cmath>

#include "bysdf_model.hpp"

namespace bysdf {

extern thread_local unsigned g_audit_mask;  // bit s: stage s in single precision
extern thread_local int g_audit_stage;       // stage of the innermost marked scope

inline double emu_round(double x)
{
    return ((g_audit_mask >> g_audit_stage) & 1u) ? (double)(float)x : x;
}

struct Emu {
    double v;
    Emu() = default;
    Emu(double x) : v(x) {}
    Emu(float x) : v(x) {}
    Emu(int x) : v(x) {}
};
inline Emu mke(double x) { Emu r; r.v = emu_round(x); return r; }
inline double ein(Emu a) { return emu_round(a.v); }
inline Emu operator+(Emu a, Emu b) { return mke(ein(a) + ein(b)); }
inline Emu operator-(Emu a, Emu b) { return mke(ein(a) - ein(b)); }
inline Emu operator*(Emu a, Emu b) { return mke(ein(a) * ein(b)); }
inline Emu operator/(Emu a, Emu b) { return mke(ein(a) / ein(b)); }
inline Emu operator-(Emu a) { Emu r; r.v = -a.v; return r; }
inline double val(Emu x) { return x.v; }

inline Emu sqrt_(Emu x) { return mke(std::sqrt(ein(x))); }
inline Emu rsqrt_(Emu x) { return mke(1.0 / std::sqrt(ein(x))); }
inline Emu rcp_(Emu x) { return mke(1.0 / ein(x)); }
inline Emu sin_(Emu x) { return mke(std::sin(ein(x))); }
inline Emu cos_(Emu x) { return mke(std::cos(ein(x))); }
inline Emu asin_(Emu x) { return mke(std::asin(ein(x))); }
inline Emu exp_(Emu x) { return mke(std::exp(ein(x))); }
inline Emu log_(Emu x) { return mke(std::log(ein(x))); }
inline Emu atan2_(Emu y, Emu x) { return mke(std::atan2(ein(y), ein(x))); }
template <> __host__ __device__ inline Emu floor_g<Emu>(const Emu& x) { return mke(std::floor(ein(x))); }
template <> __host__ __device__ inline void sincos_turns_g<Emu>(const Emu& t, Emu* s, Emu* c)
{
    const double a = ein(t);
    if ((g_audit_mask >> g_audit_stage) & 1u) {
        // sin and cos of 2 pi a for the float a: reduce the turn exactly
        // (a - rint(a) is exact), then evaluate in double and round once
        const double r = a - std::rint(a);
        *s = mke(std::sin(kTwoPi * r));
        *c = mke(std::cos(kTwoPi * r));
    } else {
        double ss, cc;
        sincos_turns(a, &ss, &cc);
        s->v = ss;
        c->v = cc;
    }
}

template <> struct StageMark<Emu> {
    int prev;
    explicit StageMark(int s) : prev(g_audit_stage) { g_audit_stage = s; }
    ~StageMark() { g_audit_stage = prev; }
    StageMark(const StageMark&) = delete;
    StageMark& operator=(const StageMark&) = delete;
};

}  // namespace bysdf
