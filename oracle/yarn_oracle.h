/*
 * yarn_oracle.h -- plain FP64 CPU oracle of ray / yarn-tube intersection
 * for scenes of yarns given as uniform cubic B-spline centrelines (the
 * explicit yarn curves of Sec. 3.3 of arXiv 2401.12724).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests and never by the product
 * library; it shares no code with the HIP path.
 *
 * Definitions (all in double precision):
 *   - Yarn Y has control points P_0..P_{n-1} (n >= 4) and n - 3 spans; span
 *     j is the uniform cubic B-spline piece on P_j..P_{j+3}, s in [0, 1].
 *   - Its tube is the set of points within distance R_Y of the centreline:
 *     the union of the balls of radius R_Y centred on every curve point.
 *   - A yarn whose tube contains the ray origin (distance to the centreline
 *     below R_Y (1 - 1e-3)) yields no hit for that ray.
 *   - The hit is the smallest t in (t_min, t_max] at which the ray enters
 *     the tube of a remaining yarn: the minimum over curve points C(s) of
 *     the entry parameter of the ray into the ball at C(s), over balls that
 *     lie ahead of t_min.
 *   - Frame at the hit: tangent T = C'/|C'|, reference normal N from the
 *     rotation-minimising frame transported along the yarn from its first
 *     point, where N starts as the component of +z orthogonal to T (or of
 *     +x if T is within 25 degrees of z); B = T x N.
 *   - h = sine of the hit azimuth measured from the incident direction's
 *     azimuth in the (N, B) plane (the curve-scattering convention, so the
 *     azimuth of the hit is atan2(wi.B, wi.N) + asin h); v = arc length
 *     from the yarn's first curve point.
 */
#ifndef YARN_ORACLE_H
#define YARN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hit flag bits */
#define ORC_HIT_MISS         (1u << 0)  /* no hit in (t_min, t_max] */
#define ORC_HIT_CAP          (1u << 1)  /* entry through a yarn end (ball at its first/last point) */
#define ORC_HIT_EXCLUDED     (1u << 2)  /* some yarn containing the origin was skipped */
#define ORC_HIT_GRAZING      (1u << 3)  /* oracle only: the ray dips less than 1e-3 R into the tube */
#define ORC_HIT_TIE          (1u << 4)  /* oracle only: another yarn's entry within the margin */
#define ORC_HIT_ORIGIN_EDGE  (1u << 5)  /* oracle only: origin within the margin of an exclusion,
                                           or the entry within 1e-2 R of t_min */
#define ORC_HIT_MARGIN_MASK (ORC_HIT_GRAZING | ORC_HIT_TIE | ORC_HIT_ORIGIN_EDGE)

/* Prepared scene: control points (x, y, z, r) as n_cp x 4 floats promoted
 * to double; yarn_off[n_yarns + 1] CSR offsets into the control points.
 * The radius of yarn Y is the r of its first control point. */
void* orc_scene_create(const float* ctrl_xyzr, const int64_t* yarn_off, int32_t n_yarns);
void orc_scene_free(void* scene);

/* Frame along yarn `yarn` at span `seg`, parameter s: out = T(3) N(3) v
 * position(3). */
void orc_scene_frame(const void* scene, int32_t yarn, int32_t seg, double s, double* out);

/* Intersect n rays (origins o[n][3], unit directions d[n][3], t_max[n])
 * with the scene.  out[n][16] = t, yarn, seg, s, h, v, T(3), N(3), flags,
 * depth (how far the ray dips into the tube, in units of R), second-best
 * entry of another yarn (or +inf). */
void orc_intersect(const void* scene, int64_t n, const float* o, const float* d,
                   const float* t_max, double t_min, double* out, int nthreads);

/* One ray (double origin and direction) with yarn `skip_yarn` left out
 * (-1: none); out[16] as orc_intersect. */
void orc_intersect_one(const void* scene, const double o[3], const double d[3], double t_min,
                       double t_max, int32_t skip_yarn, double out[16]);

/* Radius of a yarn. */
double orc_scene_radius(const void* scene, int32_t yarn);

#ifdef __cplusplus
}
#endif
#endif
