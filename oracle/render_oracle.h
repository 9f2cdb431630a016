/*
 * render_oracle.h -- plain CPU path tracer of yarn scenes shaded with the
 * BYSDF (the rendering use of the model, Sec. 4.2 and Sec. 5 of arXiv
 * 2401.12724), for a crop of the image.
 *
 * TEST INFRASTRUCTURE ONLY: it calls the FP64 oracles of the BYSDF and of
 * ray / yarn-tube intersection one ray and one query at a time and shares
 * no code with the HIP path.
 *
 * Per path (slot = pixel index in the crop * spp + sample):
 *   camera ray through the pixel with a jitter; up to max_depth scattering
 *   events, the ray leaving the last one still traced for emission:
 *   the ray meets the first yarn tube or the one-sided rectangular light
 *   (emission weighted by the power heuristic against the previous
 *   BYSDF sample) or leaves the scene (environment radiance);
 *   at a yarn hit: BYSDF query in the rotation-minimising frame (x = N,
 *   y = T x N, z = T; v in yarn radii); far field (Eq. 7, W = 1, N_h
 *   strata with one random offset) when the yarn is narrower than lod_px
 *   pixels at its camera distance, or, in multi-scale mode, the
 *   multi-scale model over the pixel footprint of a camera hit; next-event estimation to a uniform
 *   point of the light with a shadow ray that passes through a yarn where
 *   the implicit plies are missed (Sec. 3.4), weighted by the power
 *   heuristic; then a BYSDF sample continues the path.  At this scale the
 *   BYSDF acts at the yarn hit: shadow rays and continuations leave from
 *   the hit point and skip the yarn they leave (pass-through keeps the
 *   direction), so both estimators of direct light see the same scene.
 *   Random numbers: Philox4x32-10, key = seed, counter = (slot low, slot
 *   high, bounce, stream) with streams 0 (pixel jitter), 1 (light point,
 *   xi0, xi1), 2 (xi2, stratum, stratum offset); u = (x >> 8) * 2^-24.
 * Path state, hit records and query inputs are rounded to single
 * precision where the device kernels keep single precision.
 */
#ifndef RENDER_ORACLE_H
#define RENDER_ORACLE_H

#include <stdint.h>

#include "bysdf_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float eye[3], look_at[3], up[3];
    float vfov;
    int32_t width, height;
    int32_t crop_x, crop_y, crop_w, crop_h;
    float light_corner[3], light_u[3], light_v[3], light_radiance[3];
    float env_radiance[3];
    int32_t spp, max_depth;
    float lod_px;
    int32_t n_h;
    uint64_t seed;
    float ray_eps;
    int32_t nee;   /* oracle-only switch: 0 = no next-event estimation (light
                      reached by BYSDF samples alone, weight 1), for the pin
                      that both estimators agree */
    int32_t multiscale; /* 1: camera hits use the multi-scale model over their
                           pixel footprint (Sec. 4.2, 5.3), later bounces the
                           near field, no LOD switch */
    int32_t grad_type;  /* type whose (r, k^B, sigma_t) the gradient output
                           differentiates (when grad is not NULL) */
} orc_render_settings;

/* Footprint probe: h0, h1, h2 of the camera ray through pixel position
 * (px, py); returns the yarn hit or -1. */
int orc_camera_footprint(const void* scene, const orc_render_settings* rs, double px, double py,
                         double out[3]);

/* fb[crop_h][crop_w][3] receives the mean radiance over spp; if sq is not
 * NULL it receives the mean of the squared per-sample radiance (for the
 * sample variance).  types[yarn_type[y]] and tables[...] describe the
 * yarns' BYSDF types. */
/* grad (nullable): [crop_h][crop_w][3][3], the mean per-pixel derivative
 * d(radiance_c) / d theta_p for theta = (r, k^B_c, sigma_t) of type
 * rs->grad_type, by path derivatives with the sampling densities held
 * fixed; the near field shades every hit (no LOD switch). */
int orc_render(const void* scene, const orc_params* types, const double* const* tables,
               int32_t n_types, const int32_t* yarn_type, const float* yarn_phase,
               const orc_render_settings* rs, double* fb, double* sq, double* grad, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
