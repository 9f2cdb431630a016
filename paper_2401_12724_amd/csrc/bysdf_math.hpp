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

// ---------------------------------------------------------------- scalars
__host__ __device__ inline float val(float x) { return x; }
__host__ __device__ inline double val(double x) { return x; }

__host__ __device__ inline float sqrt_(float x) { return sqrtf(x); }
__host__ __device__ inline double sqrt_(double x) { return sqrt(x); }
__host__ __device__ inline float sin_(float x) { return sinf(x); }
__host__ __device__ inline double sin_(double x) { return sin(x); }
__host__ __device__ inline float cos_(float x) { return cosf(x); }
__host__ __device__ inline double cos_(double x) { return cos(x); }
__host__ __device__ inline float atan2_(float y, float x) { return atan2f(y, x); }
__host__ __device__ inline double atan2_(double y, double x) { return atan2(y, x); }
__host__ __device__ inline float asin_(float x) { return asinf(x); }
__host__ __device__ inline double asin_(double x) { return asin(x); }
__host__ __device__ inline float exp_(float x) { return expf(x); }
__host__ __device__ inline double exp_(double x) { return exp(x); }
__host__ __device__ inline float log_(float x) { return logf(x); }
__host__ __device__ inline double log_(double x) { return log(x); }
__host__ __device__ inline float abs_(float x) { return fabsf(x); }
__host__ __device__ inline double abs_(double x) { return fabs(x); }
__host__ __device__ inline float min_(float a, float b) { return a < b ? a : b; }
__host__ __device__ inline double min_(double a, double b) { return a < b ? a : b; }
__host__ __device__ inline float max_(float a, float b) { return a > b ? a : b; }
__host__ __device__ inline double max_(double a, double b) { return a > b ? a : b; }

// sin and cos of 2 pi t for a phase t measured in turns: reduce exactly to
// [-1/2, 1/2] turns first so large phases keep their accuracy.
__host__ __device__ inline void sincos_turns(double t, double* s, double* c)
{
    double r = t - rint(t);
    sincos(kTwoPi * r, s, c);
}

// narrowing to the shading scalar
template <class To> struct Narrow;
template <> struct Narrow<float> {
    __host__ __device__ static float from(double x) { return (float)x; }
    __host__ __device__ static float from(float x) { return x; }
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
    T inv = T(1) / sqrt_(dot(a, a));
    return a * inv;
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
