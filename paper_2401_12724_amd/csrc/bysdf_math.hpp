// bysdf_math.hpp -- scalar and vector helpers for the BYSDF kernels (gfx950).
//
// Every routine is a template over its scalar so the same source serves the
// forward kernels (double geometry, float shading) and the adjoint kernel
// (dual numbers carrying parameter tangents).  Branch decisions always use
// the primal value (val()).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bysdf {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kInvTwoPi = 0.15915494309189533577;

// Tables of the FP64 sine/cosine and arctangent below (math_tables.inc,
// written by gen_math_tables.py).  Device code reads them from constant
// memory, host code from an ordinary array.
#include "math_tables.inc"
struct SinCos64 {
    double c, s;
};
static __constant__ SinCos64 kSinCosTurnsDev[64] = {BYSDF_SINCOS_TABLE};
static const SinCos64 kSinCosTurnsHost[64] = {BYSDF_SINCOS_TABLE};
static __constant__ double kAtanDev[65] = {BYSDF_ATAN_TABLE};
static const double kAtanHost[65] = {BYSDF_ATAN_TABLE};
// A kernel reads the tables from LDS: every kernel that evaluates the model
// calls stage_math_tables() and a barrier before anything else (1.5 KB per
// workgroup).  Reading them from constant memory instead costs about 6 %
// of the fused evaluation + sampling (the lookups sit on dependency chains).
static __shared__ SinCos64 s_sincos_turns[64];
static __shared__ double s_atan[65];
__device__ inline void stage_math_tables()
{
    for (int i = threadIdx.x; i < 64; i += blockDim.x) s_sincos_turns[i] = kSinCosTurnsDev[i];
    for (int i = threadIdx.x; i < 65; i += blockDim.x) s_atan[i] = kAtanDev[i];
}
__host__ __device__ inline SinCos64 sincos_table(int j)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return s_sincos_turns[j];
#else
    return kSinCosTurnsHost[j];
#endif
}
__host__ __device__ inline double atan_table(int j)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return s_atan[j];
#else
    return kAtanHost[j];
#endif
}

// ---------------------------------------------------------------- scalars
__host__ __device__ inline float val(float x) { return x; }
__host__ __device__ inline double val(double x) { return x; }

// Single-precision square root, reciprocal, exp and log for the lobe
// formulas: on the device the hardware instructions (about 1 ulp; the
// library's rescaling of denormal arguments is skipped -- the lobes never
// form them), exp and log through exp2 / log2 with one multiply.
__host__ __device__ inline float sqrt_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}
__host__ __device__ inline float rcp_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
__host__ __device__ inline double rcp_(double x);  // after div_ordinary below
// Double-precision square root.  The device path takes the hardware
// reciprocal-root estimate, one Goldschmidt step that refines the root and
// half its reciprocal together, and one Newton correction of the root,
// which leaves it within an ulp of the rounded root.  It skips the
// library's rescaling of arguments below 2^-767 and its infinity fix-up:
// the model only forms arguments that are 0 (returned exactly), negative
// (NaN, as the library), or far above that range.
__host__ __device__ inline double sqrt_(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, hy = 0.5 * y;
    const double r = fma(-hy, g, 0.5);
    g = fma(g, r, g);
    hy = fma(hy, r, hy);
    const double d = fma(-g, g, x);
    g = fma(d, hy, g);
    return x == 0.0 ? 0.0 : g;
#else
    return sqrt(x);
#endif
}
// reciprocal square root (the device uses the hardware estimate refined by
// the math library; the host path only serves host-side tools)
__host__ __device__ inline float rsqrt_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return rsqrtf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}
// Double-precision reciprocal square root: hardware estimate y and one
// third-order correction y (1 + e/2 + 3e^2/8) with e = 1 - x y^2.  Without
// the library's fix-up for 0 and infinity (the model guards zero lengths
// itself).
__host__ __device__ inline double rsqrt_(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
#else
    return 1.0 / sqrt(x);
#endif
}
__host__ __device__ inline float sin_(float x) { return sinf(x); }
__host__ __device__ inline double sin_(double x) { return sin(x); }
__host__ __device__ inline float cos_(float x) { return cosf(x); }
__host__ __device__ inline double cos_(double x) { return cos(x); }
__host__ __device__ inline float atan2_(float y, float x) { return atan2f(y, x); }

// Quotient a / b in double precision from the hardware reciprocal estimate:
// two Newton steps on 1/b, the product, and one residual correction (within
// an ulp).  For b of ordinary magnitude (no overflow or denormal handling).
__host__ __device__ inline double div_ordinary(double a, double b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    r = fma(r, fma(-b, r, 1.0), r);
    const double q = a * r;
    return fma(fma(-b, q, a), r, q);
#else
    return a / b;
#endif
}

// Double-precision reciprocal of an argument of ordinary magnitude: the
// hardware estimate and two Newton steps (within an ulp).
__host__ __device__ inline double rcp_(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}

// atan2 in double precision: fold to the first octant (t = min/max in
// [0, 1]), pick the table point j/64 nearest t from a single-precision
// estimate of the quotient, and add to atan(j/64) (a correctly rounded table
// entry) the arctangent of the remainder d = (t - j/64)/(1 + t j/64), |d| <
// 1/127, from its odd Taylor series to d^7 (remainder below 1e-20).  The
// remainder takes one quotient, (mn - tj mx)/(mx + tj mn).  Then unfold.
__host__ __device__ inline double atan2_(double y, double x)
{
    const double ax = fabs(x), ay = fabs(y);
    const double mx = fmax(ax, ay), mn = fmin(ax, ay);
#if defined(__HIP_DEVICE_COMPILE__)
    const float te = (float)mn * __builtin_amdgcn_rcpf((float)mx);
#else
    const float te = (float)mn / (float)mx;
#endif
    float jf = rintf(64.0f * te);
    jf = jf > 0.0f ? (jf < 64.0f ? jf : 64.0f) : 0.0f;  // also maps a NaN estimate to 0
    const int j = (int)jf;
    const double tj = (double)jf * (1.0 / 64.0);
    const double num = fma(-tj, mx, mn), den = fma(tj, mn, mx);
    const double d = mx > 0.0 ? div_ordinary(num, den) : 0.0;
    const double d2 = d * d;
    const double p = fma(d * d2, fma(fma(-1.0 / 7.0, d2, 1.0 / 5.0), d2, -1.0 / 3.0), d);
    double a = atan_table(j) + p;
    if (ay > ax) a = 0.5 * kPi - a;
    if (x < 0.0) a = kPi - a;
    return y < 0.0 ? -a : a;
}
__host__ __device__ inline float asin_(float x) { return asinf(x); }
__host__ __device__ inline double asin_(double x) { return asin(x); }
__host__ __device__ inline float exp_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(x * 1.44269504088896340736f);
#else
    return expf(x);
#endif
}
__host__ __device__ inline double exp_(double x) { return exp(x); }
__host__ __device__ inline float log_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_logf(x) * 0.69314718055994530942f;
#else
    return logf(x);
#endif
}
__host__ __device__ inline double log_(double x) { return log(x); }
__host__ __device__ inline float abs_(float x) { return fabsf(x); }
__host__ __device__ inline double abs_(double x) { return fabs(x); }
__host__ __device__ inline float min_(float a, float b) { return a < b ? a : b; }
__host__ __device__ inline double min_(double a, double b) { return a < b ? a : b; }
__host__ __device__ inline float max_(float a, float b) { return a > b ? a : b; }
__host__ __device__ inline double max_(double a, double b) { return a > b ? a : b; }

// sin and cos of 2 pi t for a phase t measured in turns.  The reduction is
// exact: drop whole turns, then the nearest 1/64 turn j, leaving |a| <= pi/64
// rad; sin a and cos a from their Taylor series to a^7 and a^8 (remainders
// below 5e-18), turned by (cos, sin)(2 pi j / 64) from a correctly rounded
// table: about a dozen fused multiply-adds and one table read.
__host__ __device__ inline void sincos_turns(double t, double* s, double* c)
{
    const double r = t - rint(t);
    const double jd = rint(64.0 * r);
    const double a = fma(jd, -1.0 / 64.0, r) * kTwoPi;
    const double a2 = a * a;
    const double sp = fma(fma(fma(-1.0 / 5040.0, a2, 1.0 / 120.0), a2, -1.0 / 6.0), a2 * a, a);
    const double cp = fma(fma(fma(fma(1.0 / 40320.0, a2, -1.0 / 720.0), a2, 1.0 / 24.0), a2, -0.5), a2, 1.0);
    const SinCos64 e = sincos_table((int)jd & 63);
    *s = fma(e.s, cp, e.c * sp);
    *c = fma(e.c, cp, -(e.s * sp));
}

// narrowing to the shading scalar
template <class To> struct Narrow;
template <> struct Narrow<float> {
    __host__ __device__ static float from(double x) { return (float)x; }
    __host__ __device__ static float from(float x) { return x; }
    // other geometry scalars (host-side tools) narrow through their value
    template <class G> static float from(const G& x) { return (float)val(x); }
};
template <> struct Narrow<double> {
    __host__ __device__ static double from(double x) { return x; }
    __host__ __device__ static double from(float x) { return x; }
};

// ---------------------------------------------------------------- vectors
template <class T> struct V3 {
    T x, y, z;
};

template <class T> __host__ __device__ inline V3<T> mk3(T x, T y, T z)
{
    V3<T> r;
    r.x = x; r.y = y; r.z = z;
    return r;
}
template <class T> __host__ __device__ inline V3<T> operator+(const V3<T>& a, const V3<T>& b)
{
    return mk3<T>(a.x + b.x, a.y + b.y, a.z + b.z);
}
template <class T> __host__ __device__ inline V3<T> operator-(const V3<T>& a, const V3<T>& b)
{
    return mk3<T>(a.x - b.x, a.y - b.y, a.z - b.z);
}
template <class T> __host__ __device__ inline V3<T> operator-(const V3<T>& a)
{
    return mk3<T>(-a.x, -a.y, -a.z);
}
template <class T> __host__ __device__ inline V3<T> operator*(const V3<T>& a, const T& s)
{
    return mk3<T>(a.x * s, a.y * s, a.z * s);
}
template <class T> __host__ __device__ inline T dot(const V3<T>& a, const V3<T>& b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class T> __host__ __device__ inline V3<T> cross(const V3<T>& a, const V3<T>& b)
{
    return mk3<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <class T> __host__ __device__ inline V3<T> normalize(const V3<T>& a)
{
    return a * rsqrt_(dot(a, a));
}
template <class To, class From> __host__ __device__ inline V3<To> narrow3(const V3<From>& a)
{
    return mk3<To>(Narrow<To>::from(a.x), Narrow<To>::from(a.y), Narrow<To>::from(a.z));
}

// orthonormal frame: tangent t, bitangent b, normal n
template <class T> struct Frame {
    V3<T> t, b, n;
};
template <class T> __host__ __device__ inline V3<T> to_local(const Frame<T>& f, const V3<T>& w)
{
    return mk3<T>(dot(w, f.t), dot(w, f.b), dot(w, f.n));
}
template <class T> __host__ __device__ inline V3<T> to_world(const Frame<T>& f, const V3<T>& l)
{
    return f.t * l.x + f.b * l.y + f.n * l.z;
}
template <class To, class From> __host__ __device__ inline Frame<To> narrowf(const Frame<From>& f)
{
    Frame<To> r;
    r.t = narrow3<To>(f.t);
    r.b = narrow3<To>(f.b);
    r.n = narrow3<To>(f.n);
    return r;
}

}  // namespace bysdf
