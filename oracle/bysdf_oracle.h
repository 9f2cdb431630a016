/*
 * bysdf_oracle.h -- plain FP64 CPU oracle of the yarn-level scattering
 * function (BYSDF) of "A Multi-scale Yarn Appearance Model with Fiber
 * Details" (Khattar, Zhu, Montazeri et al., arXiv 2401.12724).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes,
 * links or calls this code; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no header, helper, table
 * or constant with the HIP path.
 *
 * Every quantity is computed in double precision straight from the
 * paper's definitions, in the paper's order, with no blocking, fusion or
 * reordering.  Lengths are in yarn radii; angles in radians.  The local
 * yarn frame has tangent +z, reference normal +x.  Directions point away
 * from the hit (towards the camera / the light).
 */
#ifndef BYSDF_ORACLE_H
#define BYSDF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_PLIES 8
#define ORC_MAX_NODES 16
#define ORC_MAX_STRATA 16

/* Per-query flag bits (same numbering as the library's public flags). */
#define ORC_PASS_THROUGH      (1u << 0)  /* ray misses every implicit ply (Sec. 3.4) */
#define ORC_ILLCOND           (1u << 1)  /* oracle only: ply fixed point amplifies input error */
#define ORC_NEARTIE           (1u << 2)  /* oracle only: a decision at x within its margin */
#define ORC_NEARTANGENT       (1u << 3)  /* oracle only: a forward chord grazes a ply disc */
#define ORC_AXIAL             (1u << 4)  /* incident ray (almost) parallel to the yarn axis */
#define ORC_BACKFACING        (1u << 5)  /* wi below the fiber shading normal */
#define ORC_SAMPLE_FAIL       (1u << 6)  /* sampler produced no valid direction */
#define ORC_NEAR_LOBE_BOUNDARY (1u << 7) /* oracle only: xi0 within margin of a lobe/node edge */
#define ORC_NEAR_TIR          (1u << 8)  /* oracle only: refraction denominator / TIR margin */
#define ORC_BAD_INPUT         (1u << 9)  /* non-finite or non-unit direction, |h| > 1 */

/* Margin flags: the oracle's own statement that a query sits within the
 * rounding margin of one of the method's discrete decisions. */
#define ORC_MARGIN_MASK (ORC_ILLCOND | ORC_NEARTIE | ORC_NEARTANGENT | \
                         ORC_NEAR_LOBE_BOUNDARY | ORC_NEAR_TIR)

typedef struct {
    int32_t n_plies;         /* N_p */
    int32_t fibers_per_ply;  /* M */
    int32_t K;               /* forward quadrature nodes */
    int32_t n_iter;          /* ply fixed-point updates (3--5 in Sec. 3.4) */
    int32_t tex_size;        /* N_u texels of the fiber table */
    double ply_radius;       /* r_p, yarn radii */
    double ply_center_radius;/* R_pc, yarn radii */
    double fiber_radius;     /* r_f / r_p */
    double ply_twist;        /* alpha_p, helix angle to the yarn axis */
    double fiber_twist;      /* alpha_f, at the outermost fiber radius */
    double eta;              /* refractive index */
    double albedo[3];        /* k^B (RGB) */
    double beta;             /* GGX roughness along the fiber */
    double aniso;            /* roughness ratio across / along the fiber */
    double k_spec;           /* k^S */
    double B;                /* body energy fraction */
    double r;                /* reflected share of the body energy */
    double sigma_t;          /* extinction, per yarn radius */
    double ply_density;      /* rho_p, scales ply occlusion */
    double fiber_density;    /* rho_f, scales fiber occlusion */
    double shadow_halfwidth; /* Delta_p, angular box filter of G_p */
    /* fiber migration (Sec. 3.5.2): mig_tables > 1 switches between that
     * many fiber tables along the ply, one per period of mig_period yarn
     * radii of ply arc length, blending into the next period's table over
     * its last mig_blend share; table 0 is the regular layout, table m > 0
     * pulls each fiber inwards by a factor min(1, 1 + mig_spread (2 xi - 1));
     * the draws come from Philox4x32-10 keyed by mig_seed */
    int32_t mig_tables;
    double mig_period;
    double mig_blend;
    double mig_spread;
    uint32_t mig_seed;
} orc_params;

/* Fiber tables of one type: max(1, mig_tables) tables of N_u texels x 3
 * channels (dn, rho_hat, G_f), one after the other. */
int orc_table(const orc_params* p, double* tab);

/* Fiber migration, exposed for tests: the table index of ply k in period q,
 * and the fiber-table values at fiber phase uf and ply arc length vply. */
int orc_mig_table(const orc_params* p, int64_t q, int k);
void orc_fiber_lookup(const orc_params* p, const double* tab, double uf, double vply, int k,
                      double out[3]);

/* Query arrays: type[n], h[n], u[n], v[n], wi[3][n] (SoA x,y,z), wo[3][n],
 * shift[2][n] (nullable).  out_eval is n x 13 doubles:
 *   E_r E_g E_b  E_xS E_yS  E_xB_rgb  E_yB_rgb  pdf                    */
int orc_eval(const orc_params* types, const double* const* tables, int32_t n_types,
             int64_t n, const int32_t* type, const float* h, const float* u,
             const float* v, const float* wi, const float* wo, const float* shift,
             double* out_eval, uint32_t* flags, int nthreads);

/* Sampler: xi[3][n].  out is n x 12 doubles:
 *   wo_xyz  weight_rgb  pdf  exit_xyz  lobe  node                       */
int orc_sample(const orc_params* types, const double* const* tables, int32_t n_types,
               int64_t n, const int32_t* type, const float* h, const float* u,
               const float* v, const float* wi, const float* xi, const float* shift,
               double* out, uint32_t* flags, int nthreads);

/* White-furnace blocks: block b uses query b*block for (type, h, u, v, wi)
 * and the xi of queries b*block .. b*block+block-1.  mean/var: n_blocks x 3. */
int orc_furnace(const orc_params* types, const double* const* tables, int32_t n_types,
                int64_t n, int32_t block, const int32_t* type, const float* h,
                const float* u, const float* v, const float* wi, const float* xi,
                const float* shift, double* mean, double* var, int nthreads);

/* Far field: mean of E over N_h stratified h_j = -1 + 2(j + zeta)/N_h. */
int orc_eval_far(const orc_params* types, const double* const* tables, int32_t n_types,
                 int64_t n, int32_t n_h, double zeta, const int32_t* type,
                 const float* u, const float* v, const float* wi, const float* wo,
                 double* out_E, int nthreads);

/* Multi-scale BYSDF (Sec. 4.2, Eq. 8-11): per query the footprint
 * h1 <= h <= h2 in [-1, 1] and the strata offset zeta in [0, 1); up to
 * n_max (1..ORC_MAX_STRATA) strata with tent weights around h.  Eval: out
 * n x 13 as orc_eval.  Sampler: xi_s picks the stratum; out n x 13 =
 * orc_sample's 12 values and the stratum. */
int orc_eval_multi(const orc_params* types, const double* const* tables, int32_t n_types,
                   int64_t n, int32_t n_max, const int32_t* type, const float* h, const float* h1,
                   const float* h2, const float* zeta, const float* u, const float* v,
                   const float* wi, const float* wo, const float* shift, double* out,
                   uint32_t* flags, int nthreads);
int orc_sample_multi(const orc_params* types, const double* const* tables, int32_t n_types,
                     int64_t n, int32_t n_max, const int32_t* type, const float* h,
                     const float* h1, const float* h2, const float* zeta, const float* xi_s,
                     const float* u, const float* v, const float* wi, const float* xi,
                     const float* shift, double* out, uint32_t* flags, int nthreads);
uint32_t orc_eval_multi_query(const orc_params* p, const double* tab, double h0, double h1,
                              double h2, double zeta, int32_t n_max, double u, double v,
                              const double wi[3], const double wo[3], double out[13]);
uint32_t orc_sample_multi_query(const orc_params* p, const double* tab, double h0, double h1,
                                double h2, double zeta, double xi_s, int32_t n_max, double u,
                                double v, const double wi[3], const double xi[3], double out[13]);
/* The strata of one footprint: offsets hs[] and weights ws[] (n_max
 * entries), returns their number or -1 for an invalid footprint. */
int orc_footprint(double h0, double h1, double h2, double zeta, int32_t n_max, double* hs,
                  double* ws);

/* Implicit ply hit with the ply frame: out[11] = pass, ply, hit (x, y, v),
 * tangent (3), normal (3). */
uint32_t orc_ply_frame(const orc_params* p, double h, double u, double v, const double wi[3],
                       double out[11]);
/* Explicit helical plies around a circular-arc yarn of curvature kappa:
 * out[7] = ply (-1 none), hit point (3, query frame), ply tangent (3);
 * returns 0 when the ray meets the tube before the query's yarn hit. */
int orc_explicit_ply(const orc_params* p, double kappa, double h, double u, double v,
                     const double wi[3], double step, double out[7]);

/* Central finite differences of sum_q sum_c gE[q][c] E_c(q) with respect to
 * theta = (albedo r g b, beta, ply_twist, fiber_twist, ply_density,
 * fiber_density).  grad: n_types x 8.  per_query (nullable): n x 8. */
int orc_grad_fd(const orc_params* types, const double* const* tables, int32_t n_types,
                int64_t n, const int32_t* type, const float* h, const float* u,
                const float* v, const float* wi, const float* wo, const float* gE,
                double rel_step, double* grad, double* per_query, int nthreads);

/* Philox4x32-10 (Salmon et al., SC'11): counter[4], key[2] -> out[4]. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Internals exposed for the closed-form pins. */
double orc_fresnel(double cos_i, double eta_rel);
double orc_ggx_D(const double m[3], double ax, double ay);
double orc_smith_G1(const double w[3], const double m[3], double ax, double ay);
void orc_vndf(const double wi[3], double ax, double ay, double u1, double u2, double m[3]);
double orc_ls_albedo(double mu);
/* Ply shadowing (raw, before the density blend) at ply angle a for an
 * incident 2D angle phi relative to the ply normal. */
double orc_ply_shadow_raw(const orc_params* p, double a, double phi);
/* Geometry probe: ply hit of one query.  out[0..9] = pass, k*, s*, p2x, p2y,
 * n2x, n2y, v_hit, amplification, a; out[10 + k] = converged phase theta_k.
 * Returns flags. */
uint32_t orc_ply_hit(const orc_params* p, double h, double u, double v,
                     const double wi[3], double* out);

/* Forward-node probe: per node 16 doubles
 *   kind N ell att T wt(3) y(3) n_y(3) p2x p2y.  Returns flags. */
uint32_t orc_nodes(const orc_params* p, const double* tab, double h, double u, double v,
                   const double wi[3], const double* shift, double* out);
/* Shading-frame probe at x: t(3) b(3) n(3) Gp Gf mu_i w(4).  Returns flags. */
uint32_t orc_frame_x(const orc_params* p, const double* tab, double h, double u, double v,
                     const double wi[3], double* out);
void orc_set_margins(double geo, double shade, double amplify, double tir, double xi);

/* Single queries (one type and its table from orc_table). */
uint32_t orc_eval_query(const orc_params* p, const double* tab, double h, double u, double v,
                        const double wi[3], const double wo[3], double out[13]);
uint32_t orc_sample_query(const orc_params* p, const double* tab, double h, double u, double v,
                          const double wi[3], const double xi[3], double out[12]);

#ifdef __cplusplus
}
#endif
#endif
