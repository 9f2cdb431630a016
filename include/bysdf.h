/*
 * bysdf.h -- C ABI of the MI355X (gfx950) BYSDF library, libbysdf.so.
 *
 * Batched evaluation, importance sampling, white-furnace integration and the
 * adjoint of the bidirectional yarn scattering distribution function of
 * "A Multi-scale Yarn Appearance Model with Fiber Details" (Khattar, Zhu,
 * Montazeri et al., arXiv 2401.12724), plus ray / yarn-tube intersection and
 * a wavefront path tracer that feeds it.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Units: lengths of a query are in yarn radii; angles in radians.  A
 *   query's local frame has the yarn tangent as +z and the yarn's reference
 *   normal (a rotation-minimising frame, Sec. 3.3) as +x.  Directions are
 *   unit vectors pointing away from the hit (towards the camera / light).
 * - A hit is given by (h, u, v) (Sec. 3.3, Sec. 4.2): h in [-1, 1] is the
 *   azimuthal offset of the incident ray from the yarn axis (the hit
 *   azimuth is atan2(wi) + asin h), u the ply-helix phase at the reference
 *   normal, v the longitudinal position along the yarn.
 * - Memory: every query / output pointer is a caller-owned DEVICE pointer
 *   (structure of arrays, one 4-byte element per query, 4-byte aligned).
 *   The library owns opaque handles and the device tables behind them.
 * - Streams: every call is asynchronous on the given hipStream_t (0 = the
 *   null stream); no call synchronises the device except *_create /
 *   *_destroy, which synchronise their stream.
 * - Errors: every function returns 0 on success or a negative
 *   BYSDF_ERR_*; bysdf_last_error() returns a thread-local message.
 *   Per-query problems never fail a call: they set bits in the per-query
 *   flags output and zero the query's outputs.
 */
#ifndef BYSDF_H
#define BYSDF_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ errors */
#define BYSDF_OK 0
#define BYSDF_ERR_INVALID_ARG (-1)      /* null / misaligned pointer, bad size */
#define BYSDF_ERR_INVALID_PARAM (-2)    /* a type parameter out of its range  */
#define BYSDF_ERR_OOM (-3)              /* device (or host) allocation failed  */
#define BYSDF_ERR_LAUNCH (-4)           /* kernel launch or HIP call failed    */
#define BYSDF_ERR_UNSUPPORTED_DEVICE (-5)

/* ------------------------------------------------------- per-query flag bits */
#define BYSDF_FLAG_PASS_THROUGH (1u << 0) /* the ray misses every implicit ply
                                             and continues through the yarn
                                             (Sec. 3.2, Sec. 3.4)             */
#define BYSDF_FLAG_AXIAL (1u << 4)        /* wi (almost) parallel to the yarn
                                             axis: no cross-section hit        */
#define BYSDF_FLAG_BACKFACING (1u << 5)   /* wi below the fiber normal         */
#define BYSDF_FLAG_SAMPLE_FAIL (1u << 6)  /* no valid direction was drawn      */
#define BYSDF_FLAG_BAD_INPUT (1u << 9)    /* non-finite input, |h| > 1, a
                                             direction off unit length by more
                                             than 1e-3, or a bad type id       */

/* --------------------------------------------------------- type parameters */
/* One yarn type.  Geometry follows Sec. 3 (plies as helices around the yarn
 * axis, fibers through a 1D table around each ply), appearance Sec. 4.1
 * (Eq. 2-6) with the shadowing terms of Sec. 4.1.4. */
typedef struct {
    int32_t n_plies;          /* N_p, 1..8                                   */
    int32_t fibers_per_ply;   /* M, 1..256 (fiber table)                      */
    int32_t K;                /* forward quadrature nodes of Eq. 1, 1..16     */
    int32_t n_iter;           /* ply fixed-point updates (Sec. 3.4), 0..16    */
    int32_t tex_size;         /* texels of the fiber table, 2..4096           */
    float ply_radius;         /* r_p in yarn radii, (0, 1]                    */
    float ply_center_radius;  /* R_pc in yarn radii; R_pc + r_p <= 1          */
    float fiber_radius;       /* r_f / r_p, (0, 1)                            */
    float ply_twist;          /* alpha_p, helix angle to the yarn axis        */
    float fiber_twist;        /* alpha_f at the outermost fiber radius        */
    float eta;                /* refractive index, > 1                        */
    float albedo[3];          /* body albedo k^B (RGB), >= 0                  */
    float beta;               /* GGX roughness along the fiber, > 0          */
    float aniso;              /* roughness across / along the fiber, > 0      */
    float k_spec;             /* specular albedo k^S, >= 0                    */
    float B;                  /* body energy share, [0, 1]                    */
    float r;                  /* reflected share of the body energy, [0, 1]   */
    float sigma_t;            /* extinction per yarn radius (Eq. 4), >= 0     */
    float ply_density;        /* rho_p in [0, 1]: G_p = 1 - rho_p (1 - G_raw) */
    float fiber_density;      /* rho_f in [0, 1]: G_f = 1 - rho_f (1 - G_raw) */
    float shadow_halfwidth;   /* half width of the G_p window, (0, pi/2]      */
    /* Fiber migration (Sec. 3.5.2): with mig_tables > 1 the fiber table
     * switches along the ply between that many tables -- table 0 the
     * regular arrangement, table m > 0 with every fiber pulled inwards by
     * min(1, 1 + mig_spread (2 xi - 1)) -- one drawn per ply and period of
     * mig_period yarn radii of ply arc length, blended linearly into the
     * next period's over the period's last mig_blend share.  The draws are
     * Philox4x32-10 keyed by mig_seed.  0 or 1 table: no migration. */
    int32_t mig_tables;       /* 0..8                                          */
    float mig_period;         /* > 0 when mig_tables > 1                       */
    float mig_blend;          /* [0, 1]                                        */
    float mig_spread;         /* [0, 1)                                        */
    uint32_t mig_seed;
} bysdf_type_params;

typedef struct bysdf_types bysdf_types_t; /* opaque: params + fiber tables */

/* Query arrays (device, n elements each).  shift0/shift1 may be NULL: the
 * per-query shift of the forward quadrature lattice (defaults to 0). */
typedef struct {
    const int32_t* type_id;
    const float *h, *u, *v;
    const float *wi_x, *wi_y, *wi_z;
    const float *wo_x, *wo_y, *wo_z;
    const float *shift0, *shift1;
} bysdf_query_soa;

/* Evaluation outputs (device, n elements each).  E is the value times the
 * cosine of wo with each lobe's own normal (f |cos|), in RGB; E_xS / E_yS
 * are the two specular lobes (white), E_xB / E_yB the two body lobes (RGB),
 * pdf the solid-angle density of bysdf_sample_pdf drawing wo. */
typedef struct {
    float *E_r, *E_g, *E_b;
    float *E_xS, *E_yS;
    float *E_xB_r, *E_xB_g, *E_xB_b;
    float *E_yB_r, *E_yB_g, *E_yB_b;
    float* pdf;
    uint32_t* flags;
} bysdf_eval_out_soa;

/* Sampler inputs: like bysdf_query_soa without wo, plus three uniform
 * numbers in [0, 1) per query (xi0 picks the lobe and node, xi1 and xi2 the
 * direction).  With xi0, xi1 and xi2 all NULL the library draws them:
 * Philox4x32-10 (Salmon et al., SC'11) with counter (i mod 2^32, i >> 32,
 * 0, 0x53414d50) for query index i and key (seed mod 2^32, seed >> 32),
 * words 0..2 mapped to [0, 1) as (word >> 8) * 2^-24.  The furnace draws
 * of query index j use the same stream. */
typedef struct {
    const int32_t* type_id;
    const float *h, *u, *v;
    const float *wi_x, *wi_y, *wi_z;
    const float *xi0, *xi1, *xi2;
    const float *shift0, *shift1;
    uint64_t seed;
} bysdf_sample_soa;

/* Sampler outputs.  lobe: 0 specular at x, 1 specular through the yarn to
 * an exit point y, 2 body at x, 3 body at y, 4 pass-through (wo = -wi,
 * weight 1, pdf 0), -1 bad input.  exit_*: the point the path continues
 * from (x for lobes 0/2, the node's exit point y for 1/3), in the query's
 * local frame (x, y in yarn radii, z = height along the yarn). */
typedef struct {
    float *wo_x, *wo_y, *wo_z;
    float *w_r, *w_g, *w_b;   /* E(wo) / pdf(wo), RGB */
    float* pdf;
    float *exit_x, *exit_y, *exit_z;
    int32_t* lobe;
    int32_t* node;
    uint32_t* flags;
} bysdf_sample_out_soa;

/* Library version string. */
const char* bysdf_version(void);

/* Thread-local message of the last failing call on this thread. */
const char* bysdf_last_error(void);

/* Create a handle for n_types yarn types (host array p).  Validates every
 * record, uploads the parameters and builds each distinct fiber table on
 * the device in double precision (Sec. 3.5.1: per texel, the first fiber
 * hit when looking radially inwards from the ply rim, its normal
 * perturbation, normalised radius and unoccluded fraction).  Types with
 * equal (fibers_per_ply, fiber_radius, tex_size) share one table.
 * Synchronises `stream`.  On error *out is left NULL. */
int bysdf_types_create(const bysdf_type_params* p, int32_t n_types, bysdf_types_t** out,
                       hipStream_t stream);

/* Release a handle and its device memory (NULL is accepted). */
int bysdf_types_destroy(bysdf_types_t* types);

/* Number of types in a handle, or a negative error. */
int32_t bysdf_types_count(const bysdf_types_t* types);

/* Copy the fiber tables of type `type_index` to host memory:
 * max(1, mig_tables) x tex_size x 3 floats (dn, rho_hat, G_f; the tables one
 * after the other) into `host_out` (capacity `cap` floats).  Synchronous. */
int bysdf_types_table(const bysdf_types_t* types, int32_t type_index, float* host_out,
                      int64_t cap);

/* Replace the eight differentiable parameters of every type from a DEVICE
 * array theta[n_types][8] = (albedo r, g, b, beta, ply_twist, fiber_twist,
 * ply_density, fiber_density), recomputing the derived constants on the
 * device; tables are untouched (they do not depend on theta).  Values are
 * clamped into their valid ranges.  Asynchronous on `stream`. */
int bysdf_types_set_theta(bysdf_types_t* types, const float* theta, hipStream_t stream);

/* Evaluate the BYSDF (Eq. 1: the four lobes of Eq. 2, 3, 5, 6 with Fresnel,
 * GGX, ply and fiber shadowing, the forward lobes through K quadrature
 * nodes) and the sampling pdf for n queries.  n == 0 is a no-op. */
int bysdf_eval(const bysdf_types_t* types, const bysdf_query_soa* q, int64_t n,
               const bysdf_eval_out_soa* out, hipStream_t stream);

/* Draw one direction per query with the importance sampling of Sec. 4.1.5
 * and return its direction, weight E/pdf, pdf, lobe, node and exit point. */
int bysdf_sample_pdf(const bysdf_types_t* types, const bysdf_sample_soa* q, int64_t n,
                     const bysdf_sample_out_soa* out, hipStream_t stream);

/* Both of the above on the same hits in one pass: per query, the value and
 * pdf at q's wo (as bysdf_eval) and one direction drawn with xi0..xi2 (as
 * bysdf_sample_pdf with the same hit and xi).  The state at the hit point and
 * the K forward quadrature nodes (Sec. 4.1.1) depend on wi only, so they are
 * computed once and serve both directions -- the pattern of a path tracer
 * that evaluates a light direction and draws the next bounce at each hit.
 * xi*: device arrays of n uniforms in [0, 1).  Outputs as for the two calls;
 * a bad wo flags only the eval output.  n == 0 is a no-op. */
int bysdf_eval_sample(const bysdf_types_t* types, const bysdf_query_soa* q, const float* xi0,
                      const float* xi1, const float* xi2, int64_t n,
                      const bysdf_eval_out_soa* eval_out, const bysdf_sample_out_soa* sample_out,
                      hipStream_t stream);

/* ----------------------------------------------------------- ply geometry */
/* Outputs of bysdf_ply_geometry (device, n elements each). */
typedef struct {
    int32_t* ply;             /* hit ply index, -1 when the ray passes through   */
    float *p_x, *p_y, *p_z;   /* ply hit point: projected cross-section (x, y)
                                 and height v along the yarn, yarn radii        */
    float *t_x, *t_y, *t_z;   /* ply tangent at the hit (unit, query frame)      */
    float *n_x, *n_y, *n_z;   /* ply normal at the hit (unit, orthogonal to t)   */
    uint32_t* flags;          /* PASS_THROUGH, AXIAL, BAD_INPUT                  */
} bysdf_ply_out_soa;

/* The implicit ply hit of a query alone (Sec. 3.4): the yarn hit at offset
 * h, the n_iter fixed-point updates that move each ply centre to where its
 * helix crosses the ray's ellipse plane (n_iter = 0: the circular cross
 * section perpendicular to the yarn at the hit), the 2D ray / disc test and
 * the nearest ply, with the ply's tangent (the derivative of its centre
 * helix) and normal there.  q's wo and shift arrays are not read (may be
 * NULL).  For comparing cross-section constructions against explicit
 * helical plies; n == 0 is a no-op. */
int bysdf_ply_geometry(const bysdf_types_t* types, const bysdf_query_soa* q, int64_t n,
                       const bysdf_ply_out_soa* out, hipStream_t stream);

/* ------------------------------------------------------------ multi-scale */
/* The pixel footprint of a multi-scale query (Sec. 4.2 and 5.3): device
 * arrays of n elements.  h1 <= h <= h2 (q's h) in [-1, 1] are the
 * azimuthal offsets of the two ray differentials and of the hit itself;
 * zeta in [0, 1) is the offset of the footprint's strata; xi_s in [0, 1)
 * draws the stratum (sampler only; bysdf_eval_multi ignores it and it may
 * be NULL there).  A query whose footprint breaks these bounds gets
 * BYSDF_FLAG_BAD_INPUT and zero outputs. */
typedef struct {
    const float *h1, *h2;
    const float* zeta;
    const float* xi_s;
} bysdf_footprint_soa;

/* Multi-scale BYSDF f_multi (Sec. 4.2, Eq. 8-11) at q's wo: the footprint
 * [h1, h2] is cut into n = ceil(n_max (h2 - h1) / 2) strata
 * h_j = h1 + (h2 - h1)(j + zeta)/n (FP32), weighted by a tent W that is 1
 * at h and 0 at h1 and h2 (one stratum weighs 1).  Over the strata that hit
 * a ply, the fiber normal and tangent at x (Eq. 9-10, the mean normal
 * normalised, the mean tangent made orthogonal to it) and the fiber
 * shadowing (Eq. 11) are W-weighted means; the roughness along and across
 * the fiber widens to (beta + (h2 - h1)/2)(1, aniso).  Outputs as
 * bysdf_eval, each the W-weighted mean over all strata of the near-field
 * model at that stratum's ply hit with the aggregated frame and shadowing
 * (a stratum between the plies counts 0); BYSDF_FLAG_PASS_THROUGH when no
 * stratum hits.  n_max in 1..16 (BYSDF_ERR_INVALID_ARG otherwise); h1 = h2
 * gives bysdf_eval exactly.  n == 0 is a no-op. */
int bysdf_eval_multi(const bysdf_types_t* types, const bysdf_query_soa* q,
                     const bysdf_footprint_soa* footprint, int64_t n, int32_t n_max,
                     const bysdf_eval_out_soa* out, hipStream_t stream);

/* Importance sampling of f_multi: xi_s picks stratum j with probability
 * W_j / sum W; a stratum between the plies passes the ray through (lobe 4,
 * as bysdf_sample_pdf); otherwise xi0..xi2 draw from that stratum's
 * aggregated state as in bysdf_sample_pdf, and the weight and pdf are those
 * of f_multi at the drawn direction.  Outputs as bysdf_sample_pdf, except
 * node = forward node + 16 x stratum. */
int bysdf_sample_multi(const bysdf_types_t* types, const bysdf_sample_soa* q,
                       const bysdf_footprint_soa* footprint, int64_t n, int32_t n_max,
                       const bysdf_sample_out_soa* out, hipStream_t stream);

/* White-furnace integral per block (Sec. 4.3): block b (n / block blocks)
 * draws `block` directions for the hit of query b*block (type, h, u, v, wi,
 * shift) with the xi of queries b*block .. b*block+block-1, and writes the
 * mean and sample variance of the weights E/pdf (RGB) to mean[3*b + c] and
 * var[3*b + c] (device).  block must be a multiple of 64 in [64, 1024];
 * a trailing partial block is ignored.  Reductions run in a fixed order, so
 * results are bitwise reproducible. */
int bysdf_furnace_blocks(const bysdf_types_t* types, const bysdf_sample_soa* q, int64_t n,
                         int32_t block, float* mean, float* var, hipStream_t stream);

/* Schedule of bysdf_eval_batched (see paper_2401_12724_amd/autotune.py,
 * which picks one by timing candidates on the workload at hand). */
typedef struct {
    int32_t chunk;     /* consecutive tiles a workgroup takes per visit, 1..64 */
    int32_t grid;      /* persistent workgroups (0: 2048)                      */
    int32_t use_lds;   /* stage each tile's fiber table in LDS (when <= 2048
                          texels) instead of reading it through the caches     */
    int32_t block;     /* lanes per workgroup = queries per tile: 128 or 256
                          (0: 256)                                            */
    int32_t min_waves; /* register budget: 1 or 2 wavefronts per SIMD (0: 2);
                          one wavefront keeps every value in registers, two
                          hide more latency but spill                          */
} bysdf_schedule;

/* Bytes of device workspace bysdf_eval_batched needs (0 on bad arguments). */
size_t bysdf_batched_workspace_size(int32_t n_types);

/* bysdf_eval for a heterogeneous batch in one persistent launch: queries
 * grouped by type (type t owns [type_offsets[t], type_offsets[t+1]),
 * DEVICE int64 CSR of n_types + 1 entries, type_offsets[n_types] == n;
 * q->type_id is not read), cut into tiles of at most 256 queries of one
 * type that workgroups take from a device queue.  Same outputs as
 * bysdf_eval.  sched may be NULL (chunk 4, grid 2048, LDS staging, 256
 * lanes, two wavefronts per SIMD).  The
 * launch sequence (a scan, a counter reset, the persistent kernel) contains
 * no memset and no host synchronisation, so it can be captured in a graph;
 * calls sharing one workspace must not overlap.  workspace: DEVICE buffer
 * of bysdf_batched_workspace_size(n_types) bytes, 256-byte aligned. */
int bysdf_eval_batched(const bysdf_types_t* types, const int64_t* type_offsets, int64_t n,
                       const bysdf_query_soa* q, const bysdf_eval_out_soa* out,
                       const bysdf_schedule* sched, void* workspace, size_t ws_bytes,
                       hipStream_t stream);

/* For callers that cannot allocate device memory (code under graph
 * capture, serving loops, harnesses that forbid allocation): bysdf_eval_batched
 * with no workspace argument.  Its workspace (the per-type tile offsets and
 * the queue counter) lives in a static device array of the library, one per
 * GPU, held until the process ends: 4 B per type of up to
 * BYSDF_NOALLOC_MAX_TYPES types plus 256 B (about 64 KB).  The call allocates
 * nothing; its first call on a device looks up that device's copy of the
 * array, so call it with the handle's device current.  The array keeps the
 * last call's contents; every call recomputes the tile offsets and clears
 * the counter with kernels on its stream before use.  Calls that overlap on
 * one GPU (concurrent streams or threads) share the array and race: order
 * them.  Arguments, outputs and errors as bysdf_eval_batched;
 * BYSDF_ERR_INVALID_ARG when the handle holds more than
 * BYSDF_NOALLOC_MAX_TYPES types. */
#define BYSDF_NOALLOC_MAX_TYPES 16384
int bysdf_eval_batched_noalloc(const bysdf_types_t* types, const int64_t* type_offsets, int64_t n,
                               const bysdf_query_soa* q, const bysdf_eval_out_soa* out,
                               const bysdf_schedule* sched, hipStream_t stream);

/* Bytes of device workspace bysdf_eval_backward needs for n queries of a
 * handle with n_types types (0 on bad arguments). */
size_t bysdf_backward_workspace_size(int64_t n, int32_t n_types);

/* Adjoint of bysdf_eval with respect to the eight differentiable parameters
 * theta = (albedo r, g, b, beta, ply_twist, fiber_twist, ply_density,
 * fiber_density) of every type (the parameters a fitting loop adjusts, in
 * the spirit of the differentiable fitting of Sec. 5.2):
 *   grad_theta[t][k] = sum over queries q of type t of
 *                      sum_c grad_E[q][c] * dE_c(q) / d theta_k.
 * Queries are grouped by type: type t owns queries
 * [type_offsets[t], type_offsets[t+1]) (DEVICE int64 array of n_types + 1
 * entries, type_offsets[n_types] == n; q->type_id is not read).  grad_E is
 * a DEVICE float array n x 3 (row-major), grad_theta DEVICE n_types x 8,
 * per_query (nullable) DEVICE n x 8 receives each query's terms.  beta and
 * the twists are differentiated by forward-mode tangents through the whole
 * model (shadowing recomputed, nothing stored by the forward pass); the
 * albedo and the densities enter linearly and use closed forms.  Away from
 * the model's discrete decisions this is the derivative; at a texel centre
 * of the fiber table it is one-sided.  Each tile of at most 256 queries of
 * one type reduces to a partial in a fixed tree order and partials add up
 * per type in tile order: results are bitwise reproducible.  workspace is a
 * DEVICE buffer of bysdf_backward_workspace_size(n, n_types) bytes,
 * 256-byte aligned, owned by the caller. */
int bysdf_eval_backward(const bysdf_types_t* types, const bysdf_query_soa* q, int64_t n,
                        const int64_t* type_offsets, const float* grad_E, float* grad_theta,
                        float* per_query, void* workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------- yarn scenes */
/* A scene of yarns given by their centrelines, uniform cubic B-splines
 * (the explicit yarn curves of Sec. 3.3).  Yarn Y has control points
 * ctrl_xyzr[yarn_offsets[Y] .. yarn_offsets[Y+1]-1] (at least 4; spans
 * j = 0 .. n-4 use points j .. j+3, parameter s in [0, 1]) and radius R_Y =
 * the r of its first control point.  Its tube is the set of points within
 * R_Y of the centreline (the union of balls of radius R_Y on the curve). */
typedef struct yarn_scene yarn_scene_t; /* opaque: curves, frames, BVH on the device */

/* Build a scene from HOST arrays: ctrl_xyzr (n_cp x 4 floats, rows x y z
 * r), yarn_offsets (n_yarns + 1, CSR, yarn_offsets[0] == 0), yarn_type
 * (n_yarns BYSDF type indices, nullable: all 0) and yarn_phase (n_yarns
 * ply-helix phases u in radians, nullable: all 0).  The library computes
 * per span the rotation-minimising frame at its start (double reflection
 * from +z projected off the yarn's first tangent, or +x when that tangent
 * is within 25 degrees of z), the arc length from the yarn start, and a
 * binned-SAH BVH over the spans (depth at most 64), then uploads them.
 * Synchronises `stream`.  Errors: INVALID_ARG for NULL pointers or bad
 * offsets, INVALID_PARAM for fewer than 4 points in a yarn or non-finite
 * / non-positive values, OOM, UNSUPPORTED_DEVICE. */
int yarn_scene_create(const float* ctrl_xyzr, const int64_t* yarn_offsets, int32_t n_yarns,
                      const int32_t* yarn_type, const float* yarn_phase, yarn_scene_t** out,
                      hipStream_t stream);

/* Host threads a scene build (yarn_scene_create) may use: n >= 1, or 0 for
 * the default (the hardware's thread count, at most 16).  The built scene
 * does not depend on it.  Applies to the builds that start afterwards, in
 * every thread of the process.  INVALID_ARG for n < 0 or n > 256. */
int yarn_scene_build_threads(int32_t n);

/* Release a scene (NULL is accepted). */
int yarn_scene_destroy(yarn_scene_t* scene);

/* info[6] = n_yarns, control points, spans, BVH nodes, BVH depth, device
 * bytes held by the scene. */
int yarn_scene_info(const yarn_scene_t* scene, int64_t* info);

/* Rays (DEVICE, n elements each): origins, directions (any non-zero
 * length; normalised inside, t is measured along the unit direction in
 * scene units) and the largest t of interest. */
typedef struct {
    const float *o_x, *o_y, *o_z;
    const float *d_x, *d_y, *d_z;
    const float* t_max;
} yarn_ray_soa;

/* Hits (DEVICE, n elements each).  t: entry parameter (INFINITY on a
 * miss); yarn and seg: yarn index and span within the yarn (-1 on a miss);
 * s: span parameter of the centreline point whose ball the ray enters;
 * h, u, v: the BYSDF hit coordinates (h = sine of the hit azimuth minus the
 * incident azimuth in the (N, B) plane, in [-1, 1]; u = the yarn's phase;
 * v = arc length from the yarn start, scene units); tan / nrm: unit
 * tangent T and reference normal N of the rotation-minimising frame (the
 * binormal is T x N); flags: bit 0 miss, bit 1 entry through a yarn end,
 * bit 2 a yarn holding the origin was skipped, bit 9 bad ray. */
typedef struct {
    float* t;
    int32_t *yarn, *seg;
    float *s, *h, *u, *v;
    float *tan_x, *tan_y, *tan_z;
    float *nrm_x, *nrm_y, *nrm_z;
    uint32_t* flags;
} yarn_hit_soa;

/* First entry of each ray into a yarn tube with t_min < t <= t_max (Sec.
 * 3.3: the explicit yarn curve is the only geometry traced).  A yarn whose
 * tube contains the ray origin (distance to its centreline below
 * R (1 - 1e-3)) is skipped for that ray, so rays leaving a yarn surface do
 * not hit it again.  The search runs in double precision: BVH traversal,
 * then per span a sampled scan of the ball entries and Newton on their
 * slope.  n == 0 is a no-op. */
int yarn_tube_intersect(const yarn_scene_t* scene, const yarn_ray_soa* rays, int64_t n, float t_min,
                        const yarn_hit_soa* hits, hipStream_t stream);

/* ------------------------------------------------------------- rendering */
/* Settings of shade_wavefront.  Camera: pinhole at eye looking at look_at
 * (up vector up), vertical field of view vfov (radians), full image
 * width x height; only the crop [crop_x, crop_x + crop_w) x [crop_y,
 * crop_y + crop_h) is rendered (row 0 at the top).  Light: one-sided
 * rectangle corner + a light_u + b light_v (a, b in [0, 1]) emitting
 * light_radiance (RGB) towards the side of light_u x light_v.  The
 * environment radiance is constant.  spp paths per pixel, at most
 * max_depth scattering events each; yarns narrower than lod_px pixels at
 * their camera distance use the far field (Eq. 7, W = 1) over n_h strata
 * of h.  seed keys the random streams; ray_eps is the t_min of rays that
 * leave a yarn.  spp_batch: samples per pixel per wavefront pass (0 = all
 * at once); it sets the workspace size.  multiscale = 1 replaces the LOD
 * switch by the multi-scale model (Sec. 4.2, as bysdf_eval_multi /
 * bysdf_sample_multi with n_max = n_h <= 16) at camera hits: the footprint
 * [h1, h2] comes from custom ray differentials (Sec. 5.3) -- the offsets,
 * from the hit's local straight yarn axis, of the camera rays one pixel
 * along and against the screen-space gradient of h, cut at +-1 -- and
 * later bounces use the near field. */
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
    int32_t spp_batch;
    int32_t multiscale;
} render_settings;

/* Bytes of device workspace shade_wavefront needs (0 on bad settings). */
size_t shade_wavefront_workspace_size(const render_settings* rs);

/* Path-trace the crop with the BYSDF of each yarn's type (the scene's
 * yarn_type indexes `types`), as a wavefront: camera rays; then per bounce
 * extension rays through the yarn BVH (a light or environment hit adds
 * its radiance, with the power heuristic against the BYSDF pdf for the
 * light), BYSDF shading at the hits (Sec. 4.1, the far field of Sec. 4.2
 * by the LOD rule), next-event estimation to the light with shadow rays
 * that pass through a yarn where its implicit plies are missed (Sec. 3.4),
 * a BYSDF sample to continue, and compaction of the surviving paths.  The
 * BYSDF acts at the yarn hit: rays leave from the hit point and skip the
 * yarn they leave.  Random numbers: Philox4x32-10 keyed by seed, counter
 * (slot, slot >> 32, bounce, stream), slot = (pixel in crop) * spp +
 * sample.  framebuffer: DEVICE float[crop_h][crop_w][3], the mean
 * radiance per pixel (overwritten).  workspace: DEVICE buffer of
 * shade_wavefront_workspace_size(rs) bytes, 256-byte aligned.
 * ray_counts: nullable HOST int64[2] receiving the extension and shadow
 * rays traced; when given, the call synchronises the stream.  Each path
 * writes only its own radiance slot, so the image is a deterministic
 * function of the settings. */
int shade_wavefront(const yarn_scene_t* scene, const bysdf_types_t* types, const render_settings* rs,
                    float* framebuffer, void* workspace, size_t ws_bytes, int64_t* ray_counts,
                    hipStream_t stream);

/* Host utility: the Philox4x32-10 block the renderer draws from, for
 * verification against published known-answer vectors. */
void bysdf_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Workspace bytes of shade_wavefront_grad (the path queues carry the
 * derivatives as well); 0 for invalid settings. */
size_t shade_wavefront_grad_workspace_size(const render_settings* rs);

/* shade_wavefront plus the image's gradient with respect to the body
 * parameters that the paper fits by differentiable rendering (Sec. 5.2):
 * r, the albedo k^B and sigma_t of yarn type grad_type.  grad: DEVICE
 * float[crop_h][crop_w][3][3], grad[y][x][c][p] = d(pixel channel c) /
 * d theta_p for theta = (r, k^B_c, sigma_t) (overwritten).  Each path
 * carries d ln(throughput) / d theta; a hit adds dE/E of the value at the
 * drawn direction, a shadow ray carries d(contribution)/d theta.  The
 * sampling densities are held fixed (the MIS weights and the weights' pdf
 * included), which keeps the estimate unbiased for the derivative of the
 * expected image although the lobe choice depends on r.  The near field
 * shades every hit (lod_px is not used); multiscale must be 0.  The
 * derivatives are exact for r in (0, 1), k^B > 0, sigma_t > 0 (0 is
 * returned for a parameter on its bound).  workspace:
 * shade_wavefront_grad_workspace_size(rs) bytes, 256-byte aligned.  Other
 * arguments and guarantees as shade_wavefront. */
int shade_wavefront_grad(const yarn_scene_t* scene, const bysdf_types_t* types,
                         const render_settings* rs, int32_t grad_type, float* framebuffer, float* grad,
                         void* workspace, size_t ws_bytes, int64_t* ray_counts, hipStream_t stream);

/* Host-only: algorithmic operation count of the kernels' formulation.
 * Runs the per-query model on the host with counting scalars over n
 * queries in HOST arrays (SoA: wi, wo, xi are [3][n]) of the single type
 * *p, whose fiber tables (max(1, mig_tables) x tex_size x 3 floats: dn,
 * rho_hat, G_f, as bysdf_types_table returns them) are given in host memory.
 * mode 0 counts bysdf_eval (wo needed), mode 1 bysdf_sample_pdf (xi
 * needed), mode 2 bysdf_eval_sample (both).  counts[10] receives the mean per query of
 * (add, mul, div, sqrt, transcendental) for the FP64 geometry scalar,
 * then the same five for the FP32 shading scalar.  Touches no device. */
int bysdf_count_ops(const bysdf_type_params* p, const float* table, int64_t n, const float* h,
                    const float* u, const float* v, const float* wi, const float* wo,
                    const float* xi, int32_t mode, double* counts);

#ifdef __cplusplus
}
#endif
#endif
