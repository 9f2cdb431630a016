// bysdf_lib.hip -- gfx950 kernels and C ABI of libbysdf (see include/bysdf.h).
//
// Kernels
//   k_fiber_table   one workgroup per texel, FP64: first fiber hit along the
//                   radial ray (LDS argmin), occluder intervals per fiber,
//                   exact cosine measure of their union by endpoint coverage
//   k_eval          one query per lane, grid-stride; the fiber table of a
//                   single-table handle is staged in LDS once per workgroup
//   k_sample        the importance sampler, same layout
//   k_furnace       one workgroup per furnace block; weights reduced through
//                   LDS in a fixed tree order (bitwise reproducible)
//   k_set_theta     refresh the differentiable parameters on the device
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <new>
#include <vector>

#include "../../include/bysdf.h"
#include "bysdf_model.hpp"
#include "bysdf_multi.hpp"
#include "bysdf_opcount.hpp"
#include "bysdf_dual.hpp"
#include "lib_internal.hpp"

using namespace bysdf;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? BYSDF_ERR_OOM : BYSDF_ERR_LAUNCH,     \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                   \
    } while (0)

// shared with the other translation units of the library (scene, renderer)
__attribute__((visibility("hidden"))) int bysdf_set_error(int code, const char* msg)
{
    g_err = msg;
    return code;
}

extern "C" const char* bysdf_version(void) { return "bysdf-gfx950 0.1"; }
// Entry points that allocate host memory run through this: an exhausted
// heap becomes an error code instead of an exception through the C boundary.
template <class F>
static int host_guard(F&& body)
{
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail(BYSDF_ERR_OOM, "host memory exhausted");
    }
}

extern "C" const char* bysdf_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ handle
constexpr int kMaxLdsTexels = 2048;  // 32 KB of float4 texels

struct bysdf_types {
    int32_t n_types = 0;
    int32_t n_tables = 0;
    int32_t max_plies = 0, max_K = 0;
    int32_t single_table = 0;   // every type uses table 0
    int32_t any_mig = 0;        // some type has fiber migration
    int32_t table_texels = 0;   // texels of table 0 (LDS staging size)
    int device = 0;
    TypeRec* d_types = nullptr;
    float4* d_tables = nullptr;
    std::vector<TypeRec> h_types;
    std::vector<int32_t> h_table_size;
    std::vector<int32_t> h_table_off;
    std::vector<int32_t> h_type_table;
};


static int validate(const bysdf_type_params& p, int i)
{
    auto bad = [&](const char* what) {
        return fail(BYSDF_ERR_INVALID_PARAM, "type %d: %s", i, what);
    };
    if (p.n_plies < 1 || p.n_plies > kMaxPlies) return bad("n_plies must be in 1..8");
    if (p.fibers_per_ply < 1 || p.fibers_per_ply > 256) return bad("fibers_per_ply must be in 1..256");
    if (p.K < 1 || p.K > kMaxNodes) return bad("K must be in 1..16");
    if (p.n_iter < 0 || p.n_iter > 16) return bad("n_iter must be in 0..16");
    if (p.tex_size < 2 || p.tex_size > 4096) return bad("tex_size must be in 2..4096");
    if (!(p.ply_radius > 0.0f && p.ply_radius <= 1.0f)) return bad("ply_radius must be in (0, 1]");
    if (!(p.ply_center_radius >= 0.0f)) return bad("ply_center_radius must be >= 0");
    if (!(p.ply_center_radius + p.ply_radius <= 1.0f + 1e-6f))
        return bad("ply_center_radius + ply_radius must be <= 1");
    if (p.n_plies > 1 && !(p.ply_center_radius > 0.0f)) return bad("several plies need ply_center_radius > 0");
    if (!(p.fiber_radius > 0.0f && p.fiber_radius < 1.0f)) return bad("fiber_radius must be in (0, 1)");
    if (!(fabsf(p.ply_twist) < 1.5f)) return bad("|ply_twist| must be < 1.5 rad");
    if (!(fabsf(p.fiber_twist) < 1.5f)) return bad("|fiber_twist| must be < 1.5 rad");
    if (!(p.eta > 1.0f && p.eta < 10.0f)) return bad("eta must be in (1, 10)");
    for (int c = 0; c < 3; ++c)
        if (!(p.albedo[c] >= 0.0f && p.albedo[c] < 1e6f)) return bad("albedo must be >= 0");
    if (!(p.beta > 0.0f && p.beta < 10.0f)) return bad("beta must be in (0, 10)");
    if (!(p.aniso > 0.0f && p.aniso < 100.0f)) return bad("aniso must be in (0, 100)");
    if (!(p.k_spec >= 0.0f && p.k_spec < 1e6f)) return bad("k_spec must be >= 0");
    if (!(p.B >= 0.0f && p.B <= 1.0f)) return bad("B must be in [0, 1]");
    if (!(p.r >= 0.0f && p.r <= 1.0f)) return bad("r must be in [0, 1]");
    if (!(p.sigma_t >= 0.0f && p.sigma_t < 1e6f)) return bad("sigma_t must be >= 0");
    if (!(p.ply_density >= 0.0f && p.ply_density <= 1.0f)) return bad("ply_density must be in [0, 1]");
    if (!(p.fiber_density >= 0.0f && p.fiber_density <= 1.0f)) return bad("fiber_density must be in [0, 1]");
    if (!(p.shadow_halfwidth > 0.0f && p.shadow_halfwidth <= 1.5707964f))
        return bad("shadow_halfwidth must be in (0, pi/2]");
    if (p.mig_tables < 0 || p.mig_tables > kMaxMigTables) return bad("mig_tables must be in 0..8");
    if (p.mig_tables > 1) {
        if (!(p.mig_period > 0.0f && p.mig_period < 1e6f)) return bad("mig_period must be in (0, 1e6)");
        if (!(p.mig_blend >= 0.0f && p.mig_blend <= 1.0f)) return bad("mig_blend must be in [0, 1]");
        if (!(p.mig_spread >= 0.0f && p.mig_spread < 1.0f)) return bad("mig_spread must be in [0, 1)");
        if ((int64_t)p.mig_tables * p.tex_size > 16384) return bad("mig_tables x tex_size must be <= 16384");
    }
    return 0;
}


// ------------------------------------------------------------------ K1 tables
// One workgroup per texel (Sec. 3.5.1).  Fiber centres: Vogel spiral of M
// centres within radius 1 - rho (ply radii).  The texel looks radially
// inwards from the ply rim; lane j tests fiber j.
// Fiber migration (Sec. 3.5.2): table m > 0 pulls fiber j inwards by
// min(1, 1 + spread (2 xi - 1)), xi from Philox4x32-10 with counter
// (j, m, "MIGR", 0) and key (seed, "FIBR").
__device__ inline double mig_scale(int j, int m, double spread, uint32_t seed)
{
    if (m == 0) return 1.0;
    uint32_t o[4];
    rng::philox4x32_10((uint32_t)j, (uint32_t)m, 0x4d494752u, 0u, seed, 0x46494252u, o);
    const double xi = (double)(o[0] >> 8) * (1.0 / 16777216.0);
    const double f = 1.0 + spread * (2.0 * xi - 1.0);
    return f > 1.0 ? 1.0 : f;
}

__global__ __launch_bounds__(256) void k_fiber_table(int M, double rho, int Nu, float4* out, int m,
                                                      double spread, uint32_t seed)
{
    bysdf::stage_math_tables();
    __syncthreads();
    __shared__ double s_val[256];
    __shared__ int s_idx[256];
    __shared__ double s_lo[256], s_hi[256];
    __shared__ unsigned char s_ok[256];
    const int i = blockIdx.x, tid = threadIdx.x;
    const double gold = kPi * (3.0 - sqrt(5.0));
    double ze = kTwoPi * (i + 0.5) / Nu;
    double ex = cos(ze), ey = sin(ze);
    double ox = (1.0 + 1e-9) * ex, oy = (1.0 + 1e-9) * ey;
    double fx = 0.0, fy = 0.0, s = INFINITY;
    if (tid < M) {
        double rj = (1.0 - rho) * sqrt((tid + 0.5) / M);
        const double f = mig_scale(tid, m, spread, seed);
        fx = rj * cos(tid * gold) * f;
        fy = rj * sin(tid * gold) * f;
        double wx = ox - fx, wy = oy - fy;
        double b = -(wx * ex + wy * ey);
        double c = wx * wx + wy * wy - rho * rho;
        double disc = b * b - c;
        if (disc >= 0.0) {
            double sh = -b - sqrt(disc);
            if (sh >= 0.0) s = sh;
        }
    }
    s_val[tid] = s;
    s_idx[tid] = tid;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            double a = s_val[tid], b = s_val[tid + st];
            if (b < a || (b == a && s_idx[tid + st] < s_idx[tid])) {
                s_val[tid] = b;
                s_idx[tid] = s_idx[tid + st];
            }
        }
        __syncthreads();
    }
    const double sb = s_val[0];
    const int jb = s_idx[0];
    if (!(sb < INFINITY)) {
        if (tid == 0) out[i] = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
        return;
    }
    double rb = (1.0 - rho) * sqrt((jb + 0.5) / M);
    const double fb = mig_scale(jb, m, spread, seed);
    double bx = rb * cos(jb * gold) * fb, by = rb * sin(jb * gold) * fb;
    double qx = ox - sb * ex, qy = oy - sb * ey;
    double nx = (qx - bx) / rho, ny = (qy - by) / rho;
    bool ok = false;
    double lo = 0.0, hi = 0.0;
    if (tid < M && tid != jb) {
        double wx = fx - qx, wy = fy - qy;
        double dist = sqrt(wx * wx + wy * wy);
        double cen = atan2(nx * wy - ny * wx, nx * wx + ny * wy);
        double rt = rho / dist;
        double half = asin(rt < 1.0 ? rt : 1.0);
        lo = fmax(cen - half, -0.5 * kPi);
        hi = fmin(cen + half, 0.5 * kPi);
        ok = hi > lo;
    }
    s_lo[tid] = lo;
    s_hi[tid] = hi;
    s_ok[tid] = ok;
    __syncthreads();
    // Cosine measure of the union: every merged piece has exactly one lower
    // end and one upper end that no other interval covers (ties go to the
    // lower index); sum sin(upper) - sin(lower) over those ends.
    double contrib = 0.0;
    if (ok) {
        bool lo_cov = false, hi_cov = false;
        for (int j = 0; j < M; ++j) {
            if (j == tid || !s_ok[j]) continue;
            double lj = s_lo[j], hj = s_hi[j];
            if ((lj < lo && lo <= hj) || (lj == lo && j < tid)) lo_cov = true;
            if ((lj <= hi && hi < hj) || (hj == hi && lj <= hi && j < tid)) hi_cov = true;
        }
        if (!hi_cov) contrib += sin(hi);
        if (!lo_cov) contrib -= sin(lo);
    }
    s_val[tid] = contrib;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) s_val[tid] += s_val[tid + st];
        __syncthreads();
    }
    if (tid == 0) {
        double blocked = 0.5 * s_val[0];
        double gf = blocked < 1.0 ? 1.0 - blocked : 0.0;
        double dn = atan2(ex * ny - ey * nx, ex * nx + ey * ny);
        double rh = sqrt(bx * bx + by * by) / (1.0 - rho);
        out[i] = make_float4((float)dn, (float)rh, (float)gf, 0.0f);
    }
}

// ------------------------------------------------------------------ eval
struct QPtrs {
    const int32_t* type;
    const float *h, *u, *v, *wix, *wiy, *wiz, *wox, *woy, *woz, *s0, *s1;
};
struct OPtrs {
    float *Er, *Eg, *Eb, *ExS, *EyS, *ExBr, *ExBg, *ExBb, *EyBr, *EyBg, *EyBb, *pdf;
    uint32_t* flags;
};

constexpr int kBlock = 256;
constexpr int kWave = 64;  // wavefront width of gfx950
// Minimum wavefronts per SIMD (the register budget), chosen by measurement
// on 2^24 queries.  At one wavefront a kernel keeps 256 VGPRs plus
// accumulation registers and never spills, but a lone wavefront stalls on
// the latency of its FP64 dependency chains; at two the kernels spill
// 200-350 B per lane.  With the single-type path of the type waterfall, two
// wavefronts win for the eval (4.09 ms), the sampler (5.47 -> 4.88 ms), the
// fused eval + sample (4.43 ms) and the batched eval (20.2 -> 14.7 ms on
// 2^26 queries); one wins for the adjoint passes.
#ifndef BYSDF_EVAL_MIN_WAVES
#define BYSDF_EVAL_MIN_WAVES 2
#endif
#ifndef BYSDF_SAMPLE_MIN_WAVES
#define BYSDF_SAMPLE_MIN_WAVES 2
#endif
#ifndef BYSDF_EVAL_SAMPLE_MIN_WAVES
#define BYSDF_EVAL_SAMPLE_MIN_WAVES 2
#endif
#ifndef BYSDF_BATCHED_MIN_WAVES
#define BYSDF_BATCHED_MIN_WAVES 2
#endif
#ifndef BYSDF_BACKWARD_MIN_WAVES
#define BYSDF_BACKWARD_MIN_WAVES 1
#endif

template <bool kLds, int MP, bool MIG>
__global__ __launch_bounds__(kBlock, BYSDF_EVAL_MIN_WAVES) void k_eval(const TypeRec* __restrict__ types, int n_types,
                                                 const float4* __restrict__ tables, int lds_texels,
                                                 QPtrs q, OPtrs o, int64_t n)
{
    bysdf::stage_math_tables();
    __syncthreads();
    extern __shared__ float4 s_tab[];
    if (kLds) {
        for (int i = threadIdx.x; i < lds_texels; i += blockDim.x) s_tab[i] = tables[i];
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int t = q.type[i];
        V3<float> wi = mk3<float>(q.wix[i], q.wiy[i], q.wiz[i]);
        V3<float> wo = mk3<float>(q.wox[i], q.woy[i], q.woz[i]);
        float h = q.h[i], u = q.u[i], v = q.v[i];
        uint32_t fl = (t < 0 || t >= n_types) ? F_BAD_INPUT : 0u;
        fl |= check_inputs(h, u, v, wi) | check_dir(wo);
        EvalOut<float> e;
        for (int c = 0; c < 3; ++c) e.E[c] = e.ExB[c] = e.EyB[c] = 0.0f;
        e.ExS = e.EyS = e.pdf = 0.0f;
        const bool need = fl == 0u;
        for_each_wave_type(t, need, [&](int tu) {
            const Derived<double, float>& P = types[tu].d;
            TabPtrT<MIG> tab;
            tab.p = kLds ? s_tab : tables + types[tu].table_off;
            XState<double, float, MP> X;
            state_at_x(P, tab, h, u, v, wi, X);
            fl = X.ph.flags;
            if (!X.ph.pass) {
                if (!(X.mu_i > 0.0f)) fl |= F_BACKFACING;
                float s0 = q.s0 ? q.s0[i] : 0.0f, s1 = q.s1 ? q.s1[i] : 0.0f;
                V3<double> wo_g = mk3<double>(wo.x, wo.y, wo.z);
                lobes(P, tab, X, wo_g, s0, s1, q.s0 != nullptr, e, types[tu].node_disk);
            }
        });
        o.Er[i] = e.E[0]; o.Eg[i] = e.E[1]; o.Eb[i] = e.E[2];
        o.ExS[i] = e.ExS; o.EyS[i] = e.EyS;
        o.ExBr[i] = e.ExB[0]; o.ExBg[i] = e.ExB[1]; o.ExBb[i] = e.ExB[2];
        o.EyBr[i] = e.EyB[0]; o.EyBg[i] = e.EyB[1]; o.EyBb[i] = e.EyB[2];
        o.pdf[i] = e.pdf;
        o.flags[i] = fl;
    }
}

// ------------------------------------------------------------------ sample
struct SPtrs {
    const int32_t* type;
    const float *h, *u, *v, *wix, *wiy, *wiz, *xi0, *xi1, *xi2, *s0, *s1;
    uint64_t seed;  // the draws when xi0..xi2 are NULL
};

// The three uniforms of query i: the caller's arrays, or (arrays NULL)
// Philox4x32-10 with counter (i, i >> 32, 0, "SAMP") and key = seed, words
// 0-2 to [0, 1) by their top 24 bits.
constexpr uint32_t kXiStream = 0x53414d50u;
__device__ inline void query_xi(const SPtrs& q, int64_t i, float& x0, float& x1, float& x2)
{
    if (q.xi0) {
        x0 = q.xi0[i];
        x1 = q.xi1[i];
        x2 = q.xi2[i];
        return;
    }
    uint32_t o[4];
    rng::philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, kXiStream, (uint32_t)q.seed,
                       (uint32_t)(q.seed >> 32), o);
    x0 = rng::u01(o[0]);
    x1 = rng::u01(o[1]);
    x2 = rng::u01(o[2]);
}
struct SOPtrs {
    float *wox, *woy, *woz, *wr, *wg, *wb, *pdf, *exx, *exy, *exz;
    int32_t *lobe, *node;
    uint32_t* flags;
};

template <bool kLds, int MP, bool MIG>
__global__ __launch_bounds__(kBlock, BYSDF_SAMPLE_MIN_WAVES) void k_sample(const TypeRec* __restrict__ types, int n_types,
                                                   const float4* __restrict__ tables,
                                                   int lds_texels, SPtrs q, SOPtrs o, int64_t n)
{
    bysdf::stage_math_tables();
    __syncthreads();
    extern __shared__ float4 s_tab[];
    if (kLds) {
        for (int i = threadIdx.x; i < lds_texels; i += blockDim.x) s_tab[i] = tables[i];
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int t = q.type[i];
        SampleOut<float> so;
        for (int c = 0; c < 3; ++c) so.wo[c] = so.wgt[c] = so.ex[c] = 0.0f;
        so.pdf = 0.0f;
        so.lobe = -1;
        so.node = 0;
        uint32_t fl = (t < 0 || t >= n_types) ? F_BAD_INPUT : 0u;
        const bool need = fl == 0u;
        V3<float> wi = mk3<float>(q.wix[i], q.wiy[i], q.wiz[i]);
        float s0 = q.s0 ? q.s0[i] : 0.0f, s1 = q.s1 ? q.s1[i] : 0.0f;
        float h = q.h[i], u = q.u[i], v = q.v[i], x0, x1, x2;
        query_xi(q, i, x0, x1, x2);
        for_each_wave_type(t, need, [&](int tu) {
            const Derived<double, float>& P = types[tu].d;
            TabPtrT<MIG> tab;
            tab.p = kLds ? s_tab : tables + types[tu].table_off;
            fl = sample_query<double, float, MP>(P, tab, h, u, v, wi, x0, x1, x2, s0, s1,
                                                 q.s0 != nullptr, so, types[tu].node_disk);
        });
        o.wox[i] = so.wo[0]; o.woy[i] = so.wo[1]; o.woz[i] = so.wo[2];
        o.wr[i] = so.wgt[0]; o.wg[i] = so.wgt[1]; o.wb[i] = so.wgt[2];
        o.pdf[i] = so.pdf;
        o.exx[i] = so.ex[0]; o.exy[i] = so.ex[1]; o.exz[i] = so.ex[2];
        o.lobe[i] = so.lobe;
        o.node[i] = so.node;
        o.flags[i] = fl;
    }
}

// ------------------------------------------------------------------ eval + sample
// Both calls on one hit: the value and pdf at the query's wo, and one drawn
// direction.  The state at x and the K forward nodes are computed once and
// serve both directions, so a query costs about one evaluation plus the
// draw instead of an evaluation and a sample.
template <bool kLds, int MP, bool MIG>
__global__ __launch_bounds__(kBlock, BYSDF_EVAL_SAMPLE_MIN_WAVES) void k_eval_sample(
    const TypeRec* __restrict__ types, int n_types, const float4* __restrict__ tables, int lds_texels,
    QPtrs q, const float* __restrict__ xi0, const float* __restrict__ xi1,
    const float* __restrict__ xi2, OPtrs o, SOPtrs so_p, int64_t n)
{
    bysdf::stage_math_tables();
    __syncthreads();
    extern __shared__ float4 s_tab[];
    if (kLds) {
        for (int i = threadIdx.x; i < lds_texels; i += blockDim.x) s_tab[i] = tables[i];
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int t = q.type[i];
        V3<float> wi = mk3<float>(q.wix[i], q.wiy[i], q.wiz[i]);
        V3<float> wo = mk3<float>(q.wox[i], q.woy[i], q.woz[i]);
        float h = q.h[i], u = q.u[i], v = q.v[i], x0 = xi0[i], x1 = xi1[i], x2 = xi2[i];
        const uint32_t bad_t = (t < 0 || t >= n_types) ? F_BAD_INPUT : 0u;
        const uint32_t bad_hit = bad_t | check_inputs(h, u, v, wi);
        const uint32_t bad_wo = check_dir(wo);
        uint32_t fe = bad_hit | bad_wo, fs = bad_hit;
        EvalOut<float> e;
        for (int c = 0; c < 3; ++c) e.E[c] = e.ExB[c] = e.EyB[c] = 0.0f;
        e.ExS = e.EyS = e.pdf = 0.0f;
        SampleOut<float> so;
        for (int c = 0; c < 3; ++c) so.wo[c] = so.wgt[c] = so.ex[c] = 0.0f;
        so.pdf = 0.0f;
        so.lobe = -1;
        so.node = 0;
        for_each_wave_type(t, bad_hit == 0u, [&](int tu) {
            const Derived<double, float>& P = types[tu].d;
            TabPtrT<MIG> tab;
            tab.p = kLds ? s_tab : tables + types[tu].table_off;
            XState<double, float, MP> X;
            state_at_x(P, tab, h, u, v, wi, X);
            float s0 = q.s0 ? q.s0[i] : 0.0f, s1 = q.s1 ? q.s1[i] : 0.0f;
            NodesComputed<double, float, MP, TabPtrT<MIG>> nf{P, tab, X, s0, s1, q.s0 != nullptr,
                                                               types[tu].node_disk};
            V3<double> wo_g = mk3<double>(wo.x, wo.y, wo.z);
            fs = eval_sample_from_x(P, X, wi, wo_g, bad_wo == 0u, x0, x1, x2, nf, e, so);
            if (bad_wo == 0u) {
                fe = X.ph.flags;
                if (!X.ph.pass && !(X.mu_i > 0.0f)) fe |= F_BACKFACING;
            }
        });
        o.Er[i] = e.E[0]; o.Eg[i] = e.E[1]; o.Eb[i] = e.E[2];
        o.ExS[i] = e.ExS; o.EyS[i] = e.EyS;
        o.ExBr[i] = e.ExB[0]; o.ExBg[i] = e.ExB[1]; o.ExBb[i] = e.ExB[2];
        o.EyBr[i] = e.EyB[0]; o.EyBg[i] = e.EyB[1]; o.EyBb[i] = e.EyB[2];
        o.pdf[i] = e.pdf;
        o.flags[i] = fe;
        so_p.wox[i] = so.wo[0]; so_p.woy[i] = so.wo[1]; so_p.woz[i] = so.wo[2];
        so_p.wr[i] = so.wgt[0]; so_p.wg[i] = so.wgt[1]; so_p.wb[i] = so.wgt[2];
        so_p.pdf[i] = so.pdf;
        so_p.exx[i] = so.ex[0]; so_p.exy[i] = so.ex[1]; so_p.exz[i] = so.ex[2];
        so_p.lobe[i] = so.lobe;
        so_p.node[i] = so.node;
        so_p.flags[i] = fs;
    }
}

// ------------------------------------------------------------------ multi-scale
// The multi-scale model (Sec. 4.2, Eq. 8-11).  A footprint costs one
// near-field state per stratum for its aggregated geometry and one state
// plus the lobes per stratum for f_multi, and its strata count ranges over
// 1..n_max: one query per lane would let a wavefront run as long as its
// widest footprint.  Instead each wavefront takes 64 queries, numbers their
// (query, stratum) items (an exclusive scan of the strata counts) and deals
// the items to its lanes 64 at a time; each item's result returns to the
// lane of its query through cross-lane shuffles, summed in stratum order
// (the arithmetic and its order are those of the one-query-per-lane model
// functions, so results are bitwise reproducible).
struct FPtrs {
    const float *h1, *h2, *zeta, *xi_s;
};

#ifndef BYSDF_MULTI_MIN_WAVES
#define BYSDF_MULTI_MIN_WAVES 2
#endif

// Orders the LDS accesses of one wavefront's lanes to each other's slots
// (wavefront-scope fences around a wave barrier: the LDS serves a
// wavefront's operations in issue order, so this emits no wait and only
// keeps the compiler from moving accesses across it).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int wave_excl_scan(int x)
{
    const int lane = __lane_id();
    int s = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(s, d);
        if (lane >= d) s += y;
    }
    return s - x;
}

__device__ inline int wave_max(int x)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const int y = __shfl_xor(x, d);
        x = y > x ? y : x;
    }
    return x;
}

// The lane whose items include item k: the last lane whose first item is
// at most k (a lane without items shares its first item with the next).
__device__ inline int item_owner(int first, int k)
{
    int lo = 0;
#pragma unroll
    for (int step = kWave / 2; step >= 1; step >>= 1) {
        const int c = lo + step;
        if (__shfl(first, c) <= k) lo = c;
    }
    return lo;
}

__device__ inline V3<double> shfl3(const V3<double>& a, int src)
{
    return mk3<double>(__shfl(a.x, src), __shfl(a.y, src), __shfl(a.z, src));
}

// A multi-scale query read from the query arrays (eval or sampler layout).
struct MQuery {
    float h, u, v, h1, h2, zeta;
    V3<float> wi;
};
template <class QP>
__device__ inline MQuery load_mquery(const QP& q, const FPtrs& fp, int64_t i)
{
    MQuery m;
    m.h = q.h[i];
    m.u = q.u[i];
    m.v = q.v[i];
    m.h1 = fp.h1[i];
    m.h2 = fp.h2[i];
    m.zeta = fp.zeta[i];
    m.wi = mk3<float>(q.wix[i], q.wiy[i], q.wiz[i]);
    return m;
}

// Aggregated geometry (Eq. 9-11) of the wavefront's 64 footprints.  On
// return each lane holds its footprint's frame and shadowing, as
// footprint_geometry computes them; `any` is false when no stratum of
// positive weight hits a ply.
template <bool kLds, int MP, bool MIG, class QP>
__device__ inline void wave_footprint_geometry(const TypeRec* __restrict__ types,
                                               const float4* __restrict__ tables, const float4* s_tab,
                                               const QP& q, const FPtrs& fp, int n_max, int64_t b,
                                               int t, int first, int nq, int S, Frame<double>& F,
                                               float& Gm, bool& any, uint32_t& fl)
{
    V3<double> sn = mk3<double>(0.0, 0.0, 0.0), st = sn, n0 = sn, t0 = sn;
    double sg = 0.0, sw = 0.0, g0 = 0.0;
    int have = 0;
    for (int r0 = 0; r0 < S; r0 += kWave) {
        const int k = r0 + __lane_id();
        const bool item = k < S;
        const int own = item_owner(first, k);
        const int j = k - __shfl(first, own);
        const int to = __shfl(t, own);
        double w_it = 0.0, g_it = 0.0;
        V3<double> n_it = mk3<double>(0.0, 0.0, 0.0), t_it = n_it;
        uint32_t f_it = 0;
        for_each_wave_type<false>(to, item, [&](int tu) {
            const TypeRec& R = types[tu];
            TabPtrT<MIG> tab;
            tab.p = kLds ? s_tab : tables + R.table_off;
            const MQuery m = load_mquery(q, fp, b + own);
            Footprint fo;
            make_footprint(m.h, m.h1, m.h2, m.zeta, n_max, fo);
            const Derived<double, float> Pm = widened(R.d, R.beta, R.aniso, fo);
            const float hj = stratum_h(fo, j);
            const double w = stratum_w(fo, (double)hj);
            Frame<double> fx;
            double rawf;
            uint32_t sfl;
            const bool hit = stratum_frame<double, float, MP>(Pm, tab, hj, m.u, m.v, m.wi, fx, rawf, sfl);
            f_it = sfl & ~F_PASS_THROUGH;
            if (hit && w > 0.0) {
                w_it = w;
                n_it = fx.n;
                t_it = fx.t;
                g_it = 1.0 - (double)Pm.rho_f * (1.0 - rawf);
            }
        });
        // this lane's items of the round, in stratum order
        const int lo = first > r0 ? first : r0;
        const int hi = first + nq < r0 + kWave ? first + nq : r0 + kWave;
        const int cnt = hi > lo ? hi - lo : 0;
        const int cmax = wave_max(cnt);
        for (int jj = 0; jj < cmax; ++jj) {
            const int src = (lo + jj - r0) & (kWave - 1);
            const double ws = __shfl(w_it, src), gs = __shfl(g_it, src);
            const V3<double> ns = shfl3(n_it, src), ts = shfl3(t_it, src);
            const uint32_t fs = __shfl(f_it, src);
            if (jj < cnt) {
                fl |= fs;
                if (ws > 0.0) {
                    if (have == 0) {
                        n0 = ns;
                        t0 = ts;
                        g0 = gs;
                    }
                    sn = sn + ns * ws;
                    st = st + ts * ws;
                    sg = sg + gs * ws;
                    sw += ws;
                    ++have;
                }
            }
        }
    }
    any = have > 0;
    F.n = n0;
    F.t = t0;
    F.b = cross(n0, t0);
    Gm = (float)g0;
    if (have > 1) {
        Gm = (float)(sg / sw);
        const double ln2 = dot(sn, sn);
        if (ln2 > 1e-24 * sw * sw) {
            const V3<double> nn = sn * rsqrt_(ln2);
            const V3<double> tt = st - nn * dot(st, nn);
            const double lt2 = dot(tt, tt);
            if (lt2 > 1e-24 * sw * sw) {
                F.n = nn;
                F.t = tt * rsqrt_(lt2);
                F.b = cross(F.n, F.t);
            }
        }
    }
}

// Per-wavefront LDS of the multi-scale kernels: each lane's aggregated
// frame and shadowing (read by the lanes that take its footprint's strata)
// and its running sums.  Out of registers, they leave the per-stratum model
// (fixed point, nodes, lobes) its full register budget.
struct MultiLds {
    double fn[3][kWave], ft[3][kWave];
    float gm[kWave];
    int use[kWave];        // bit 0: single stratum, bit 1: aggregated frame
    float acc[12][kWave];  // E rgb, ExS, EyS, ExB rgb, EyB rgb, pdf
};

// The sampler's: the aggregated frame and shadowing, and each lane's draw
// (direction, exit point, lobe and node) while the strata evaluate it.
struct MultiSampleLds {
    double fn[3][kWave], ft[3][kWave], wo[3][kWave];
    float gm[kWave];
    int use[kWave];  // bit 0: single stratum
    float ex[3][kWave];
    int lobe[kWave], node[kWave];
};

template <bool kLds, int MP, bool MIG>
__global__ __launch_bounds__(kBlock, BYSDF_MULTI_MIN_WAVES) void k_eval_multi(
    const TypeRec* __restrict__ types, int n_types, const float4* __restrict__ tables, int lds_texels,
    QPtrs q, FPtrs fp, int n_max, OPtrs o, int64_t n)
{
    bysdf::stage_math_tables();
    __syncthreads();
    extern __shared__ float4 s_tab[];
    __shared__ MultiLds s_ml[kBlock / kWave];
    if (kLds) {
        for (int i = threadIdx.x; i < lds_texels; i += blockDim.x) s_tab[i] = tables[i];
        __syncthreads();
    }
    const int lane = __lane_id();
    MultiLds& L = s_ml[threadIdx.x / kWave];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // whole wavefronts iterate together (the cross-lane steps need every lane)
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); b < n; b += stride) {
        const int64_t i = b + lane;
        const bool in = i < n;
        const int t = in ? q.type[i] : 0;
        uint32_t fl = F_BAD_INPUT;
        double wsum = 1.0;
        int nq = 0;
        if (in) {
            const MQuery m = load_mquery(q, fp, i);
            const V3<float> wo = mk3<float>(q.wox[i], q.woy[i], q.woz[i]);
            fl = (t < 0 || t >= n_types) ? F_BAD_INPUT : 0u;
            fl |= check_inputs(m.h, m.u, m.v, m.wi) | check_dir(wo) | check_footprint(m.h, m.h1, m.h2, m.zeta);
            if (fl == 0u) {
                Footprint f;
                make_footprint(m.h, m.h1, m.h2, m.zeta, n_max, f);
                nq = f.n;
                wsum = f.wsum;
            }
        }
        // a single stratum is its own aggregate: only wider footprints take
        // part in the aggregation pass
        const bool single = nq == 1;
        const int nqa = nq > 1 ? nq : 0;
        const int firsta = wave_excl_scan(nqa);
        const int Sa = __shfl(firsta + nqa, kWave - 1);
        const int first = wave_excl_scan(nq);
        const int S = __shfl(first + nq, kWave - 1);
        {
            Frame<double> F;
            float Gm;
            bool any;
            wave_footprint_geometry<kLds, MP, MIG>(types, tables, s_tab, q, fp, n_max, b, t, firsta, nqa, Sa,
                                                   F, Gm, any, fl);
            if (nqa > 0 && !any) fl |= F_PASS_THROUGH;
            wave_lds_sync();
            L.fn[0][lane] = F.n.x; L.fn[1][lane] = F.n.y; L.fn[2][lane] = F.n.z;
            L.ft[0][lane] = F.t.x; L.ft[1][lane] = F.t.y; L.ft[2][lane] = F.t.z;
            L.gm[lane] = Gm;
            L.use[lane] = (single ? 1 : 0) | (any ? 2 : 0);
            for (int c = 0; c < 12; ++c) L.acc[c][lane] = 0.0f;
            wave_lds_sync();
        }
        int hit1 = 0;
        // f_multi: every stratum's lobes with the aggregated geometry
        for (int r0 = 0; r0 < S; r0 += kWave) {
            const int k = r0 + lane;
            const int own = item_owner(first, k);
            const int j = k - __shfl(first, own);
            const int to = __shfl(t, own);
            const int use_o = L.use[own];
            const bool item = k < S && use_o != 0;
            float ev[12];
            for (int c = 0; c < 12; ++c) ev[c] = 0.0f;
            float w_it = 0.0f;
            int back = 0, hit_it = 0;
            uint32_t f_it = 0;
            for_each_wave_type<false>(to, item, [&](int tu) {
                const TypeRec& R = types[tu];
                TabPtrT<MIG> tab;
                tab.p = kLds ? s_tab : tables + R.table_off;
                const int64_t io = b + own;
                const MQuery m = load_mquery(q, fp, io);
                Footprint fo;
                make_footprint(m.h, m.h1, m.h2, m.zeta, n_max, fo);
                const Derived<double, float> Pm = widened(R.d, R.beta, R.aniso, fo);
                const float hj = stratum_h(fo, j);
                XState<double, float, MP> X;
                state_at_x(Pm, tab, hj, m.u, m.v, m.wi, X);
                f_it = X.ph.flags & ~F_PASS_THROUGH;
                if (X.ph.pass) return;
                hit_it = 1;
                if (!(use_o & 1)) {
                    Frame<double> Fo;
                    Fo.n = mk3<double>(L.fn[0][own], L.fn[1][own], L.fn[2][own]);
                    Fo.t = mk3<double>(L.ft[0][own], L.ft[1][own], L.ft[2][own]);
                    Fo.b = cross(Fo.n, Fo.t);
                    apply_aggregate(Pm, X, Fo, L.gm[own]);
                }
                back = !(X.mu_i > 0.0f);
                const float s0 = q.s0 ? q.s0[io] : 0.0f, s1 = q.s1 ? q.s1[io] : 0.0f;
                const V3<double> wo_g = mk3<double>(q.wox[io], q.woy[io], q.woz[io]);
                EvalOut<float> e;
                lobes(Pm, tab, X, wo_g, s0, s1, q.s0 != nullptr, e);
                w_it = float(stratum_w(fo, (double)hj));
                ev[0] = e.E[0]; ev[1] = e.E[1]; ev[2] = e.E[2];
                ev[3] = e.ExS; ev[4] = e.EyS;
                ev[5] = e.ExB[0]; ev[6] = e.ExB[1]; ev[7] = e.ExB[2];
                ev[8] = e.EyB[0]; ev[9] = e.EyB[1]; ev[10] = e.EyB[2];
                ev[11] = e.pdf;
            });
            // this lane's strata of the round, in stratum order
            const int lo = first > r0 ? first : r0;
            const int hi = first + nq < r0 + kWave ? first + nq : r0 + kWave;
            const int cnt = hi > lo ? hi - lo : 0;
            const int cmax = wave_max(cnt);
            float a[12];
            for (int c = 0; c < 12; ++c) a[c] = L.acc[c][lane];
            for (int jj = 0; jj < cmax; ++jj) {
                const int src = (lo + jj - r0) & (kWave - 1);
                float es[12];
                for (int c = 0; c < 12; ++c) es[c] = __shfl(ev[c], src);
                const float ws = __shfl(w_it, src);
                const int bs = __shfl(back, src);
                const int hs = __shfl(hit_it, src);
                const uint32_t fs = __shfl(f_it, src);
                if (jj < cnt) {
                    if (bs) fl |= F_BACKFACING;
                    if (single) {
                        fl |= fs;
                        hit1 = hs != 0;
                    }
                    for (int c = 0; c < 12; ++c) a[c] = a[c] + ws * es[c];
                }
            }
            for (int c = 0; c < 12; ++c) L.acc[c][lane] = a[c];
            wave_lds_sync();
        }
        if (!in) continue;
        if (single && !hit1) fl |= F_PASS_THROUGH;
        const float iw = float(1.0 / wsum);
        o.Er[i] = L.acc[0][lane] * iw; o.Eg[i] = L.acc[1][lane] * iw; o.Eb[i] = L.acc[2][lane] * iw;
        o.ExS[i] = L.acc[3][lane] * iw; o.EyS[i] = L.acc[4][lane] * iw;
        o.ExBr[i] = L.acc[5][lane] * iw; o.ExBg[i] = L.acc[6][lane] * iw; o.ExBb[i] = L.acc[7][lane] * iw;
        o.EyBr[i] = L.acc[8][lane] * iw; o.EyBg[i] = L.acc[9][lane] * iw; o.EyBb[i] = L.acc[10][lane] * iw;
        o.pdf[i] = L.acc[11][lane] * iw;
        o.flags[i] = fl;
    }
}

// OWNXI: the uniforms come from the generator (xi arrays NULL).  Only the
// instance that needs it carries the generator: its code alone, never run,
// costs the multi-scale sampler a quarter of its speed in registers.
template <bool kLds, int MP, bool MIG, bool OWNXI>
__global__ __launch_bounds__(kBlock, BYSDF_MULTI_MIN_WAVES) void k_sample_multi(
    const TypeRec* __restrict__ types, int n_types, const float4* __restrict__ tables, int lds_texels,
    SPtrs q, FPtrs fp, int n_max, SOPtrs o, int64_t n)
{
    bysdf::stage_math_tables();
    __syncthreads();
    extern __shared__ float4 s_tab[];
    __shared__ MultiSampleLds s_ml[kBlock / kWave];
    if (kLds) {
        for (int i = threadIdx.x; i < lds_texels; i += blockDim.x) s_tab[i] = tables[i];
        __syncthreads();
    }
    const int lane = __lane_id();
    MultiSampleLds& L = s_ml[threadIdx.x / kWave];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); b < n; b += stride) {
        const int64_t i = b + lane;
        const bool in = i < n;
        int t = in ? q.type[i] : 0;
        uint32_t fl = F_BAD_INPUT;
        Footprint f;
        f.n = 0;
        f.wsum = 1.0;
        MQuery m{};
        float xs = 0.0f, x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
        if (in) {
            m = load_mquery(q, fp, i);
            xs = fp.xi_s[i];
            if (OWNXI) {
                query_xi(q, i, x0, x1, x2);
            } else {
                x0 = q.xi0[i];
                x1 = q.xi1[i];
                x2 = q.xi2[i];
            }
            fl = (t < 0 || t >= n_types) ? F_BAD_INPUT : 0u;
            fl |= check_inputs(m.h, m.u, m.v, m.wi) | check_footprint(m.h, m.h1, m.h2, m.zeta);
            if (!(xs >= 0.0f && xs < 1.0f)) fl |= F_BAD_INPUT;
            if (fl == 0u) make_footprint(m.h, m.h1, m.h2, m.zeta, n_max, f);
        }
        const bool good = fl == 0u;
        const int nq = good ? f.n : 0;
        const int first = wave_excl_scan(nq);
        const int S = __shfl(first + nq, kWave - 1);
        const bool single = nq == 1;
        const int nqa = nq > 1 ? nq : 0;
        const int firsta = wave_excl_scan(nqa);
        const int Sa = __shfl(firsta + nqa, kWave - 1);
        bool any;
        {
            Frame<double> F;
            float Gm;
            wave_footprint_geometry<kLds, MP, MIG>(types, tables, s_tab, q, fp, n_max, b, t, firsta, nqa, Sa,
                                                   F, Gm, any, fl);
            wave_lds_sync();
            L.fn[0][lane] = F.n.x; L.fn[1][lane] = F.n.y; L.fn[2][lane] = F.n.z;
            L.ft[0][lane] = F.t.x; L.ft[1][lane] = F.t.y; L.ft[2][lane] = F.t.z;
            L.gm[lane] = Gm;
            L.use[lane] = single ? 1 : 0;
            L.wo[0][lane] = L.wo[1][lane] = L.wo[2][lane] = 0.0;
            L.ex[0][lane] = L.ex[1][lane] = L.ex[2][lane] = 0.0f;
            L.lobe[lane] = -1;
            L.node[lane] = 0;
            wave_lds_sync();
        }
        // the stratum and the draw, per query
        int s = 0;
        if (good) {
            s = f.n - 1;
            const double xw = (double)xs * f.wsum;
            double cum = 0.0;
            for (int jj = 0; jj < f.n - 1; ++jj) {
                cum += stratum_w(f, (double)stratum_h(f, jj));
                if (xw < cum) {
                    s = jj;
                    break;
                }
            }
        }
        bool drawn = false, pass = good && !any && !single;
        const float s0 = in && q.s0 ? q.s0[i] : 0.0f, s1 = in && q.s1 ? q.s1[i] : 0.0f;
        for_each_wave_type<false>(t, good && (any || single), [&](int tu) {
            const TypeRec& R = types[tu];
            TabPtrT<MIG> tab;
            tab.p = kLds ? s_tab : tables + R.table_off;
            const Derived<double, float> Pm = widened(R.d, R.beta, R.aniso, f);
            XState<double, float, MP> X;
            state_at_x(Pm, tab, stratum_h(f, s), m.u, m.v, m.wi, X);
            if (single) fl |= X.ph.flags & ~F_PASS_THROUGH;
            pass = X.ph.pass;
            if (pass) return;
            if (!single) {
                Frame<double> Fo;
                Fo.n = mk3<double>(L.fn[0][lane], L.fn[1][lane], L.fn[2][lane]);
                Fo.t = mk3<double>(L.ft[0][lane], L.ft[1][lane], L.ft[2][lane]);
                Fo.b = cross(Fo.n, Fo.t);
                apply_aggregate(Pm, X, Fo, L.gm[lane]);
            }
            NodesComputed<double, float, MP, TabPtrT<MIG>> nf{Pm, tab, X, s0, s1, q.s0 != nullptr};
            SampleOut<float> so;
            V3<double> wo;
            fl |= sample_draw(Pm, X, m.wi, x0, x1, x2, nf, so, wo, drawn);
            L.wo[0][lane] = wo.x; L.wo[1][lane] = wo.y; L.wo[2][lane] = wo.z;
            L.ex[0][lane] = so.ex[0]; L.ex[1][lane] = so.ex[1]; L.ex[2][lane] = so.ex[2];
            L.lobe[lane] = so.lobe;
            L.node[lane] = so.node;
        });
        wave_lds_sync();
        // f_multi and its pdf at the drawn direction
        EvalOut<float> em;
        em.E[0] = em.E[1] = em.E[2] = 0.0f;
        em.pdf = 0.0f;
        for (int r0 = 0; r0 < S; r0 += kWave) {
            const int k = r0 + lane;
            const int own = item_owner(first, k);
            const int j = k - __shfl(first, own);
            const int to = __shfl(t, own);
            const int drawn_o = __shfl((int)drawn, own);
            const int single_o = L.use[own] & 1;
            const bool item = k < S && drawn_o != 0;
            float ev[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            float w_it = 0.0f;
            for_each_wave_type<false>(to, item, [&](int tu) {
                const TypeRec& R = types[tu];
                TabPtrT<MIG> tab;
                tab.p = kLds ? s_tab : tables + R.table_off;
                const int64_t io = b + own;
                const MQuery mo = load_mquery(q, fp, io);
                Footprint fo;
                make_footprint(mo.h, mo.h1, mo.h2, mo.zeta, n_max, fo);
                const Derived<double, float> Pm = widened(R.d, R.beta, R.aniso, fo);
                const float hj = stratum_h(fo, j);
                XState<double, float, MP> X;
                state_at_x(Pm, tab, hj, mo.u, mo.v, mo.wi, X);
                if (X.ph.pass) return;
                if (!single_o) {
                    Frame<double> Fo;
                    Fo.n = mk3<double>(L.fn[0][own], L.fn[1][own], L.fn[2][own]);
                    Fo.t = mk3<double>(L.ft[0][own], L.ft[1][own], L.ft[2][own]);
                    Fo.b = cross(Fo.n, Fo.t);
                    apply_aggregate(Pm, X, Fo, L.gm[own]);
                }
                const float t0 = q.s0 ? q.s0[io] : 0.0f, t1 = q.s1 ? q.s1[io] : 0.0f;
                const V3<double> wd = mk3<double>(L.wo[0][own], L.wo[1][own], L.wo[2][own]);
                EvalOut<float> e;
                lobes(Pm, tab, X, wd, t0, t1, q.s0 != nullptr, e);
                w_it = float(stratum_w(fo, (double)hj));
                ev[0] = e.E[0]; ev[1] = e.E[1]; ev[2] = e.E[2]; ev[3] = e.pdf;
            });
            const int lo = first > r0 ? first : r0;
            const int hi = first + nq < r0 + kWave ? first + nq : r0 + kWave;
            const int cnt = hi > lo ? hi - lo : 0;
            const int cmax = wave_max(cnt);
            for (int jj = 0; jj < cmax; ++jj) {
                const int src = (lo + jj - r0) & (kWave - 1);
                float es[4];
                for (int c = 0; c < 4; ++c) es[c] = __shfl(ev[c], src);
                const float ws = __shfl(w_it, src);
                if (jj < cnt) {
                    for (int c = 0; c < 3; ++c) em.E[c] = em.E[c] + ws * es[c];
                    em.pdf = em.pdf + ws * es[3];
                }
            }
        }
        if (!in) continue;
        SampleOut<float> so;
        for (int c = 0; c < 3; ++c) {
            so.wo[c] = so.wgt[c] = 0.0f;
            so.ex[c] = L.ex[c][lane];
        }
        so.pdf = 0.0f;
        so.lobe = L.lobe[lane];
        so.node = L.node[lane];
        if (pass) {
            so.wo[0] = -q.wix[i];
            so.wo[1] = -q.wiy[i];
            so.wo[2] = -q.wiz[i];
            so.wgt[0] = so.wgt[1] = so.wgt[2] = 1.0f;
            so.lobe = 4;
            fl |= F_PASS_THROUGH;
        }
        if (good) so.node += 16 * s;
        if (drawn) {
            const float iw = float(1.0 / f.wsum);
            for (int c = 0; c < 3; ++c) em.E[c] = em.E[c] * iw;
            em.pdf = em.pdf * iw;
            const V3<double> wo = mk3<double>(L.wo[0][lane], L.wo[1][lane], L.wo[2][lane]);
            fl = sample_finish(em, wo, fl, so);
        }
        o.wox[i] = so.wo[0]; o.woy[i] = so.wo[1]; o.woz[i] = so.wo[2];
        o.wr[i] = so.wgt[0]; o.wg[i] = so.wgt[1]; o.wb[i] = so.wgt[2];
        o.pdf[i] = so.pdf;
        o.exx[i] = so.ex[0]; o.exy[i] = so.ex[1]; o.exz[i] = so.ex[2];
        o.lobe[i] = so.lobe;
        o.node[i] = so.node;
        o.flags[i] = fl;
    }
}
// ------------------------------------------------------------------ ply geometry
// The implicit ply hit of Sec. 3.4 on its own (no fiber table, no lobes):
// the ply, the hit point and the ply's frame there, for studies of the
// cross-section construction.
struct PlyOPtrs {
    int32_t* ply;
    float *px, *py, *pz, *tx, *ty, *tz, *nx, *ny, *nz;
    uint32_t* flags;
};

template <int MP>
__global__ __launch_bounds__(kBlock) void k_ply_geometry(const TypeRec* __restrict__ types, int n_types,
                                                         QPtrs q, PlyOPtrs o, int64_t n)
{
    bysdf::stage_math_tables();
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int t = q.type[i];
        V3<float> wi = mk3<float>(q.wix[i], q.wiy[i], q.wiz[i]);
        float h = q.h[i], u = q.u[i], v = q.v[i];
        uint32_t fl = (t < 0 || t >= n_types) ? F_BAD_INPUT : 0u;
        fl |= check_inputs(h, u, v, wi);
        int ply = -1;
        V3<double> pt = mk3<double>(0.0, 0.0, 0.0), tp = pt, np = pt;
        for_each_wave_type(t, fl == 0u, [&](int tu) {
            const Derived<double, float>& P = types[tu].d;
            PlyHit<double, MP> ph;
            trace_plies(P, h, u, v, wi, ph);
            fl = ph.flags;
            if (ph.pass) return;
            double cth = 0.0, sth = 0.0;
#pragma unroll
            for (int k = 0; k < MP; ++k)
                if (k == ph.ks) {
                    cth = ph.cth[k];
                    sth = ph.sth[k];
                }
            // ply tangent: derivative of the centre helix; normal: the 2D
            // outward normal made orthogonal to it (as in the fiber frame)
            tp = mk3<double>(-P.slope * sth * P.tnorm_inv, P.slope * cth * P.tnorm_inv, P.tnorm_inv);
            const V3<double> n23 = mk3<double>(ph.n2x, ph.n2y, 0.0);
            np = normalize(n23 - tp * dot(n23, tp));
            pt = mk3<double>(ph.p2x, ph.p2y, ph.vhit);
            ply = ph.ks;
        });
        o.ply[i] = ply;
        o.px[i] = (float)pt.x; o.py[i] = (float)pt.y; o.pz[i] = (float)pt.z;
        o.tx[i] = (float)tp.x; o.ty[i] = (float)tp.y; o.tz[i] = (float)tp.z;
        o.nx[i] = (float)np.x; o.ny[i] = (float)np.y; o.nz[i] = (float)np.z;
        o.flags[i] = fl;
    }
}

// ------------------------------------------------------------------ furnace
// One workgroup per furnace block.  Every draw shares the block's hit, so
// the state at x is computed per lane (identical values) while the K
// forward nodes -- the costly part of each evaluation -- are computed once
// by lanes 0..K-1 into LDS and read by every draw.  Lane j draws with the xi
// of queries b*block + j, j + 256, ...; sums reduce through LDS in a fixed
// tree order (bitwise reproducible).
constexpr int kMaxDrawsPerLane = 4;  // block <= 1024 = 4 x 256

template <int MP, bool MIG>
__global__ __launch_bounds__(kBlock) void k_furnace(const TypeRec* __restrict__ types, int n_types,
                                                    const float4* __restrict__ tables, SPtrs q,
                                                    int block, float* mean, float* var)
{
    bysdf::stage_math_tables();
    __syncthreads();
    __shared__ Node<double, float> s_nodes[kMaxNodes];
    __shared__ XState<double, float, MP> s_X;
    __shared__ float s_red[3][kBlock];
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t q0 = b * (int64_t)block;
    const int t = __builtin_amdgcn_readfirstlane(q.type[q0]);
    const bool valid = t >= 0 && t < n_types;
    const TypeRec& rec = types[valid ? t : 0];
    const Derived<double, float>& P = rec.d;
    TabPtrT<MIG> tab;
    tab.p = tables + rec.table_off;
    V3<float> wi = mk3<float>(q.wix[q0], q.wiy[q0], q.wiz[q0]);
    const float h = q.h[q0], u = q.u[q0], v = q.v[q0];
    const float s0 = q.s0 ? q.s0[q0] : 0.0f, s1 = q.s1 ? q.s1[q0] : 0.0f;
    const bool bad = !valid || check_inputs(h, u, v, wi) != 0u;
    // the first wavefront computes the state at the shared hit (every lane
    // the same values) and the K nodes (lane k node k); all draws read both
    // from LDS
    if (!bad && tid < kWave) {
        XState<double, float, MP> X0;
        state_at_x(P, tab, h, u, v, wi, X0);
        if (tid == 0) s_X = X0;
        if (!X0.ph.pass && tid < P.K) {
            Node<double, float> nd;
            forward_node(P, tab, X0, tid, s0, s1, q.s0 != nullptr, nd);
            s_nodes[tid] = nd;
        }
    }
    __syncthreads();
    const XState<double, float, MP>& X = s_X;
    NodesStored<double, float> nodes{s_nodes};
    float w[kMaxDrawsPerLane][3];
    float sum[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 0; d < kMaxDrawsPerLane; ++d) {
        const int j = tid + d * kBlock;
        w[d][0] = w[d][1] = w[d][2] = 0.0f;
        if (j < block && !bad) {
            const int64_t qi = q0 + j;
            SampleOut<float> so;
            float x0, x1, x2;
            query_xi(q, qi, x0, x1, x2);
            sample_from_x(P, X, wi, x0, x1, x2, nodes, so);
            for (int c = 0; c < 3; ++c) w[d][c] = so.wgt[c];
        }
        for (int c = 0; c < 3; ++c) sum[c] += w[d][c];
    }
    for (int c = 0; c < 3; ++c) s_red[c][tid] = sum[c];
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int c = 0; c < 3; ++c) s_red[c][tid] += s_red[c][tid + st];
        __syncthreads();
    }
    float m[3];
    for (int c = 0; c < 3; ++c) m[c] = s_red[c][0] / (float)block;
    __syncthreads();
    float sq[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 0; d < kMaxDrawsPerLane; ++d) {
        const int j = tid + d * kBlock;
        if (j < block)
            for (int c = 0; c < 3; ++c) {
                float dv = w[d][c] - m[c];
                sq[c] += dv * dv;
            }
    }
    for (int c = 0; c < 3; ++c) s_red[c][tid] = sq[c];
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int c = 0; c < 3; ++c) s_red[c][tid] += s_red[c][tid + st];
        __syncthreads();
    }
    if (tid == 0) {
        for (int c = 0; c < 3; ++c) {
            mean[3 * b + c] = m[c];
            var[3 * b + c] = s_red[c][0] / (float)(block - 1);
        }
    }
}

// One wavefront per furnace block of at most 256 draws (4 per lane), four
// blocks per workgroup: each wavefront computes its own block's state at x
// and K nodes into its LDS slot, so no wavefront waits on another's setup;
// sums reduce across the wavefront's lanes in a fixed shuffle order.
#ifndef BYSDF_FURNACE_WAVE
#define BYSDF_FURNACE_WAVE 1
#endif
#ifndef BYSDF_FURNACE_MIN_WAVES
#define BYSDF_FURNACE_MIN_WAVES 1
#endif
constexpr int kFurnaceWaves = kBlock / kWave;


__device__ inline float wave_sum_f(float x)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d);
    return x;
}

// Each wavefront serves `group` consecutive blocks.  Their setups run side by
// side: lane g forms the state at block g's shared hit, then the lanes take
// the (block, node) items and form the forward nodes, all into the
// wavefront's LDS slots; a block's setup alone would keep the whole
// wavefront busy for one lane's work.  Then the blocks are drawn one after
// another, four draws per lane, reduced with shuffles in a fixed order.
#ifndef BYSDF_FURNACE_GROUP_MAX
#define BYSDF_FURNACE_GROUP_MAX 8
#endif
#ifndef BYSDF_FURNACE_NODE_ITEMS
#define BYSDF_FURNACE_NODE_ITEMS 32
#endif
constexpr int kFurnaceGroupMax = BYSDF_FURNACE_GROUP_MAX;

template <int MP, bool MIG>
__global__ __launch_bounds__(kBlock, BYSDF_FURNACE_MIN_WAVES) void k_furnace_w(const TypeRec* __restrict__ types, int n_types,
                                                      const float4* __restrict__ tables, SPtrs q,
                                                      int block, int64_t nb, int group, int kmax, float* mean,
                                                      float* var)
{
    bysdf::stage_math_tables();
    __syncthreads();
    __shared__ XState<double, float, MP> s_X[kFurnaceWaves][kFurnaceGroupMax];
    __shared__ int s_ord[kFurnaceWaves][kMaxDrawsPerLane * kWave];
    extern __shared__ Node<double, float> s_nd[];  // [kFurnaceWaves][group][kmax]
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    Node<double, float>* nodes_w = s_nd + wv * group * kmax;
    const int64_t b0 = ((int64_t)blockIdx.x * kFurnaceWaves + wv) * group;
    const bool has_shift = q.s0 != nullptr;
    // the hit of block b and whether it can be drawn
    auto block_hit = [&](int64_t b, int& t, V3<float>& wi, float& h, float& u, float& v, float& s0,
                         float& s1) -> bool {
        const int64_t q0 = b * (int64_t)block;
        t = q.type[q0];
        wi = mk3<float>(q.wix[q0], q.wiy[q0], q.wiz[q0]);
        h = q.h[q0];
        u = q.u[q0];
        v = q.v[q0];
        s0 = has_shift ? q.s0[q0] : 0.0f;
        s1 = has_shift ? q.s1[q0] : 0.0f;
        return t >= 0 && t < n_types && check_inputs(h, u, v, wi) == 0u;
    };
    // ---- states at the hits, lane g for block g
    if (lane < group && b0 + lane < nb) {
        int t;
        V3<float> wi;
        float h, u, v, s0, s1;
        if (block_hit(b0 + lane, t, wi, h, u, v, s0, s1)) {
            const TypeRec& rec = types[t];
            TabPtrT<MIG> tab;
            tab.p = tables + rec.table_off;
            XState<double, float, MP> X0;
            state_at_x(rec.d, tab, h, u, v, wi, X0);
            s_X[wv][lane] = X0;
        }
    }
    wave_lds_sync();
    // ---- forward nodes, one (block, node) item per lane
    for (int it = lane; it < group * kmax; it += kWave) {
        const int g = it / kmax, k = it - g * kmax;
        const int64_t b = b0 + g;
        if (b >= nb) continue;
        int t;
        V3<float> wi;
        float h, u, v, s0, s1;
        if (!block_hit(b, t, wi, h, u, v, s0, s1)) continue;
        const TypeRec& rec = types[t];
        const XState<double, float, MP>& Xg = s_X[wv][g];
        if (Xg.ph.pass || k >= rec.d.K) continue;
        TabPtrT<MIG> tab;
        tab.p = tables + rec.table_off;
        Node<double, float> nd;
        forward_node(rec.d, tab, Xg, k, s0, s1, has_shift, nd, rec.node_disk);
        nodes_w[g * kmax + k] = nd;
    }
    wave_lds_sync();
    // ---- the draws, block after block
    for (int g = 0; g < group; ++g) {
        const int64_t b = b0 + g;
        if (b >= nb) break;
        int t;
        V3<float> wi;
        float h, u, v, s0, s1;
        const bool bad = !block_hit(b, t, wi, h, u, v, s0, s1);
        t = __builtin_amdgcn_readfirstlane(bad ? 0 : t);
        const Derived<double, float>& P = types[t].d;
        const int64_t q0 = b * (int64_t)block;
        const XState<double, float, MP>& X = s_X[wv][g];
        NodesStored<double, float> nodes{nodes_w + g * kmax};
        // the draws in lobe order: a draw's lobe follows from its first
        // uniform and the block's lobe weights alone, so a stable counting
        // sort by lobe lets a wavefront's lanes take the same sampling and
        // evaluation branches (VNDF or cosine, at x or at a node)
        int key[kMaxDrawsPerLane];
#pragma unroll
        for (int d = 0; d < kMaxDrawsPerLane; ++d) {
            const int j = lane + d * kWave;
            key[d] = -1;
            if (j < block && !bad) {
                SampleOut<float> so;
                float x0, x1, x2;
                query_xi(q, q0 + j, x0, x1, x2);
                sample_pick(P, X, wi, x0, so);
                key[d] = so.lobe < 0 ? 0 : so.lobe;
            }
        }
        wave_lds_sync();
        {
            const unsigned long long below = (1ull << lane) - 1ull;
            int base = 0;
            for (int v = 0; v <= 4; ++v)
#pragma unroll
                for (int d = 0; d < kMaxDrawsPerLane; ++d) {
                    const unsigned long long m = __ballot(key[d] == v);
                    if (key[d] == v) s_ord[wv][base + __popcll(m & below)] = lane + d * kWave;
                    base += __popcll(m);
                }
        }
        wave_lds_sync();
        float w[kMaxDrawsPerLane][3];
        float sum[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int d = 0; d < kMaxDrawsPerLane; ++d) {
            const int p = lane + d * kWave;
            w[d][0] = w[d][1] = w[d][2] = 0.0f;
            if (p < block && !bad) {
                const int64_t qi = q0 + s_ord[wv][p];
                SampleOut<float> so;
                float x0, x1, x2;
                query_xi(q, qi, x0, x1, x2);
                sample_from_x(P, X, wi, x0, x1, x2, nodes, so);
                for (int c = 0; c < 3; ++c) w[d][c] = so.wgt[c];
            }
            for (int c = 0; c < 3; ++c) sum[c] += w[d][c];
        }
        float m[3];
        for (int c = 0; c < 3; ++c) m[c] = wave_sum_f(sum[c]) / (float)block;
        float sq[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int d = 0; d < kMaxDrawsPerLane; ++d) {
            const int j = lane + d * kWave;
            if (j < block)
                for (int c = 0; c < 3; ++c) {
                    const float dv = w[d][c] - m[c];
                    sq[c] += dv * dv;
                }
        }
        float vs[3];
        for (int c = 0; c < 3; ++c) vs[c] = wave_sum_f(sq[c]);
        if (lane == 0) {
            for (int c = 0; c < 3; ++c) {
                mean[3 * b + c] = m[c];
                var[3 * b + c] = vs[c] / (float)(block - 1);
            }
        }
    }
}

// ------------------------------------------------------------------ tiles
// Queries grouped by type (CSR offsets, device int64[n_types + 1]) are cut
// into tiles of at most kBlock queries that never straddle a type.
// tile_first[t] = index of the first tile of type t (exclusive scan of
// ceil(count_t / kBlock)); tile_first[n_types] = number of tiles.
__global__ __launch_bounds__(1024) void k_tile_scan(const int64_t* __restrict__ off, int n_types,
                                                    int32_t* __restrict__ tile_first, int tile_size)
{
    __shared__ int32_t s[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (n_types + nt - 1) / nt;
    const int lo = min(n_types, tid * chunk), hi = min(n_types, lo + chunk);
    int32_t sum = 0;
    for (int t = lo; t < hi; ++t) sum += (int32_t)((off[t + 1] - off[t] + tile_size - 1) / tile_size);
    s[tid] = sum;
    __syncthreads();
    for (int st = 1; st < nt; st <<= 1) {  // inclusive Hillis-Steele scan
        int32_t add = tid >= st ? s[tid - st] : 0;
        __syncthreads();
        s[tid] += add;
        __syncthreads();
    }
    int32_t run = s[tid] - sum;  // exclusive prefix of this chunk
    for (int t = lo; t < hi; ++t) {
        tile_first[t] = run;
        run += (int32_t)((off[t + 1] - off[t] + tile_size - 1) / tile_size);
    }
    if (tid == nt - 1) tile_first[n_types] = s[tid];
}

// tile -> (type, first query, count); false past the last tile
__device__ inline bool locate_tile(int tile, const int32_t* __restrict__ tile_first, int n_types,
                                   const int64_t* __restrict__ off, int* type, int64_t* start,
                                   int* count, int tile_size = kBlock)
{
    if (tile >= tile_first[n_types]) return false;
    int lo = 0, hi = n_types - 1;  // last t with tile_first[t] <= tile
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tile_first[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    *type = lo;
    *start = off[lo] + (int64_t)(tile - tile_first[lo]) * tile_size;
    int64_t left = off[lo + 1] - *start;
    *count = (int)(left < tile_size ? left : tile_size);
    return true;
}

// ------------------------------------------------------------------ adjoint
// One workgroup per tile.  Each lane recomputes its query three times with
// the tangent seeded on beta, ply twist and fiber twist (forward-mode dual
// scalars through the same model, shadowing included), contracts the
// tangents of E with grad_E, and adds the closed-form derivatives of the
// linear parameters (albedo, densities).  The tile's lanes reduce in a
// fixed tree order to one partial per tile.
// One pass of the adjoint per launch, so that each pass gets the register
// allocation of its own code: pass 0 differentiates beta (and writes the
// closed forms of the albedo and the densities), pass 1 the ply twist,
// pass 2 the fiber twist.  Parts of the model that do not depend on the
// seeded parameter run in plain arithmetic and are promoted to duals with
// zero tangents: everything at x for beta, the ply hit for the fiber twist.
template <int MP, int PASS>
__global__ __launch_bounds__(kBlock, BYSDF_BACKWARD_MIN_WAVES) void k_backward(const TypeRec* __restrict__ types,
                                                     const float4* __restrict__ tables, QPtrs q,
                                                     const int64_t* __restrict__ off, int n_types,
                                                     const int32_t* __restrict__ tile_first,
                                                     const float* __restrict__ gE,
                                                     float* __restrict__ partials,
                                                     float* __restrict__ per_query)
{
    bysdf::stage_math_tables();
    __syncthreads();
    constexpr int NS = PASS == 0 ? 6 : 1;
    // theta slots written by this pass
    constexpr int kSlot0[6] = {0, 1, 2, 3, 6, 7};
    __shared__ float s_red[NS][kBlock];
    int t = 0, count = 0;
    int64_t start = 0;
    if (!locate_tile(blockIdx.x, tile_first, n_types, off, &t, &start, &count)) return;
    t = __builtin_amdgcn_readfirstlane(t);
    const int tid = threadIdx.x;
    const TypeRec& rec = types[t];
    TabPtr tab;
    tab.p = tables + rec.table_off;
    float g[NS];
    for (int k = 0; k < NS; ++k) g[k] = 0.0f;
    if (tid < count) {
        const int64_t i = start + tid;
        V3<float> wi = mk3<float>(q.wix[i], q.wiy[i], q.wiz[i]);
        V3<float> wo = mk3<float>(q.wox[i], q.woy[i], q.woz[i]);
        const float h = q.h[i], u = q.u[i], v = q.v[i];
        const bool bad = (check_inputs(h, u, v, wi) | check_dir(wo)) != 0u;
        if (!bad) {
            const float ge[3] = {gE[3 * i], gE[3 * i + 1], gE[3 * i + 2]};
            const float s0 = q.s0 ? q.s0[i] : 0.0f, s1 = q.s1 ? q.s1[i] : 0.0f;
            V3<DD> wo_d = mk3<DD>(DD((double)wo.x), DD((double)wo.y), DD((double)wo.z));
            Derived<DD, DF> P = derive_dual(rec, PASS);
            XState<DD, DF, MP> X;
            if (PASS == 0) {
                XState<double, float, MP> Xp;
                state_at_x(rec.d, tab, h, u, v, wi, Xp);
                promote(Xp, X);
            } else if (PASS == 2) {
                PlyHit<double, MP> ph;
                trace_plies(rec.d, h, u, v, wi, ph);
                promote(ph, X.ph);
                state_after_plies(P, tab, wi, X);
            } else {
                state_at_x(P, tab, h, u, v, wi, X);
            }
            if (!X.ph.pass) {
                EvalOut<DF> e;
                lobes(P, tab, X, wo_d, s0, s1, q.s0 != nullptr, e, rec.node_disk);
                const float dE = ge[0] * e.E[0].d + ge[1] * e.E[1].d + ge[2] * e.E[2].d;
                if (PASS == 0) {
                    const float b0 = e.body0.v, Gp = X.Gp.v, Gf = X.Gf.v;
                    const float op = 1.0f - (float)X.rawp.v, of = 1.0f - (float)X.rawf.v;
                    float sa = 0.0f;
                    for (int c = 0; c < 3; ++c) {
                        g[c] = ge[c] * b0 * Gp * Gf;
                        sa += ge[c] * rec.d.alb[c];
                    }
                    g[3] = dE;
                    g[4] = -sa * b0 * Gf * op;
                    g[5] = -sa * b0 * Gp * of;
                } else {
                    g[0] = dE;
                }
            }
        }
        if (per_query)
            for (int k = 0; k < NS; ++k) per_query[8 * i + (PASS == 0 ? kSlot0[k] : 3 + PASS)] = g[k];
    }
    for (int k = 0; k < NS; ++k) s_red[k][tid] = g[k];
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int k = 0; k < NS; ++k) s_red[k][tid] += s_red[k][tid + st];
        __syncthreads();
    }
    if (tid < NS) partials[8 * (int64_t)blockIdx.x + (PASS == 0 ? kSlot0[tid] : 3 + PASS)] = s_red[tid][0];
}

// grad[t] = sum of the partials of type t's tiles, in tile order
__global__ void k_backward_sum(const int32_t* __restrict__ tile_first, int n_types,
                               const float* __restrict__ partials, float* __restrict__ grad)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_types) return;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int tl = tile_first[t]; tl < tile_first[t + 1]; ++tl)
        for (int k = 0; k < 8; ++k) acc[k] += partials[8 * (int64_t)tl + k];
    for (int k = 0; k < 8; ++k) grad[8 * (int64_t)t + k] = acc[k];
}

// ------------------------------------------------------------------ hetero
// Persistent evaluation of a batch grouped by type.  Workgroups take
// `chunk` consecutive tiles at a time from a device counter (reset by
// k_reset_counter on the same stream, so the pair can be captured in a
// graph); a tile holds at most kBlock queries of one type, whose scalars
// are read with scalar loads and whose fiber table is staged in LDS when
// the type changes.  Every workgroup loops until the counter passes the
// last tile, so the grid always drains.
__global__ void k_reset_counter(int* counter) { *counter = 0; }

template <int MP, bool kLds, int WAVES>
__global__ __launch_bounds__(kBlock, WAVES) void k_eval_batched(
    const TypeRec* __restrict__ types, const float4* __restrict__ tables,
    const int64_t* __restrict__ off, int n_types, const int32_t* __restrict__ tile_first,
    int* counter, QPtrs q, OPtrs o, int chunk)
{
    bysdf::stage_math_tables();
    __syncthreads();
    // a tile holds as many queries as the workgroup has lanes (128 or 256)
    __shared__ float4 s_tab[kLds ? kMaxLdsTexels : 1];
    __shared__ int s_next;
    const int tid = threadIdx.x;
    const int n_tiles = tile_first[n_types];
    int staged = -1;
    for (;;) {
        if (tid == 0) s_next = atomicAdd(counter, chunk);
        __syncthreads();
        const int t0 = s_next;
        __syncthreads();
        if (t0 >= n_tiles) break;
        for (int c = 0; c < chunk; ++c) {
            int type = 0, count = 0;
            int64_t start = 0;
            if (!locate_tile(t0 + c, tile_first, n_types, off, &type, &start, &count, (int)blockDim.x)) break;
            type = __builtin_amdgcn_readfirstlane(type);
            const TypeRec& rec = types[type];
            TabPtr tab;
            if (kLds) {
                if (type != staged) {
                    __syncthreads();
                    for (int k = tid; k < rec.table_texels; k += blockDim.x) s_tab[k] = tables[rec.table_off + k];
                    __syncthreads();
                    staged = type;
                }
                tab.p = s_tab;
            } else {
                tab.p = tables + rec.table_off;
            }
            if (tid >= count) continue;
            const int64_t i = start + tid;
            V3<float> wi = mk3<float>(q.wix[i], q.wiy[i], q.wiz[i]);
            V3<float> wo = mk3<float>(q.wox[i], q.woy[i], q.woz[i]);
            const float h = q.h[i], u = q.u[i], v = q.v[i];
            uint32_t fl = check_inputs(h, u, v, wi) | check_dir(wo);
            EvalOut<float> e;
            for (int k = 0; k < 3; ++k) e.E[k] = e.ExB[k] = e.EyB[k] = 0.0f;
            e.ExS = e.EyS = e.pdf = 0.0f;
            if (!fl) {
                const Derived<double, float>& P = rec.d;
                XState<double, float, MP> X;
                state_at_x(P, tab, h, u, v, wi, X);
                fl = X.ph.flags;
                if (!X.ph.pass) {
                    if (!(X.mu_i > 0.0f)) fl |= F_BACKFACING;
                    const float s0 = q.s0 ? q.s0[i] : 0.0f, s1 = q.s1 ? q.s1[i] : 0.0f;
                    V3<double> wo_g = mk3<double>(wo.x, wo.y, wo.z);
                    lobes(P, tab, X, wo_g, s0, s1, q.s0 != nullptr, e, rec.node_disk);
                }
            }
            o.Er[i] = e.E[0]; o.Eg[i] = e.E[1]; o.Eb[i] = e.E[2];
            o.ExS[i] = e.ExS; o.EyS[i] = e.EyS;
            o.ExBr[i] = e.ExB[0]; o.ExBg[i] = e.ExB[1]; o.ExBb[i] = e.ExB[2];
            o.EyBr[i] = e.EyB[0]; o.EyBg[i] = e.EyB[1]; o.EyBb[i] = e.EyB[2];
            o.pdf[i] = e.pdf;
            o.flags[i] = fl;
        }
    }
}

// ------------------------------------------------------------------ theta
__global__ void k_set_theta(TypeRec* types, const float* theta, int n)
{
    bysdf::stage_math_tables();
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    TypeRec t = types[i];
    const float* th = theta + 8 * i;
    for (int c = 0; c < 3; ++c) t.albedo[c] = fmaxf(th[c], 0.0f);
    t.beta = fmin(fmax((double)th[3], 1e-4), 10.0);
    t.ply_twist = fmin(fmax((double)th[4], -1.5), 1.5);
    t.fiber_twist = fmin(fmax((double)th[5], -1.5), 1.5);
    t.ply_density = fminf(fmaxf(th[6], 0.0f), 1.0f);
    t.fiber_density = fminf(fmaxf(th[7], 0.0f), 1.0f);
    fill_derived(t);
    types[i] = t;
}

// ------------------------------------------------------------------ host API
// the renderer (another translation unit) reads the handle's device data
__attribute__((visibility("hidden"))) BysdfTypesView bysdf_types_view(const bysdf_types_t* h)
{
    return BysdfTypesView{h->d_types, h->d_tables, h->n_types, h->max_plies, h->max_K};
}

static bool aligned4(const void* p) { return p && ((uintptr_t)p & 3u) == 0; }

static int types_create(const bysdf_type_params* p, int32_t n_types, bysdf_types_t** out, hipStream_t stream)
{
    if (!out) return fail(BYSDF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p || n_types < 1) return fail(BYSDF_ERR_INVALID_ARG, "need p != NULL and n_types >= 1");
    for (int i = 0; i < n_types; ++i) {
        int rc = validate(p[i], i);
        if (rc) return rc;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BYSDF_ERR_UNSUPPORTED_DEVICE, "device %d is %s, library is built for gfx950", dev,
                    prop.gcnArchName);
    bysdf_types* h = new bysdf_types();
    h->n_types = n_types;
    h->device = dev;
    // one table set per distinct (M, rho, N_u, migration tables, spread,
    // seed): its tables one after the other
    std::map<std::tuple<int, float, int, int, float, uint32_t>, int> uniq;
    int32_t texels = 0;
    struct Job {
        int M;
        double rho;
        int Nu, tables;
        double spread;
        uint32_t seed;
    };
    std::vector<Job> jobs;
    for (int i = 0; i < n_types; ++i) {
        const int nt = p[i].mig_tables > 1 ? p[i].mig_tables : 1;
        const float spread = nt > 1 ? p[i].mig_spread : 0.0f;
        const uint32_t seed = nt > 1 ? p[i].mig_seed : 0u;
        auto key = std::make_tuple(p[i].fibers_per_ply, p[i].fiber_radius, p[i].tex_size, nt, spread, seed);
        auto it = uniq.find(key);
        int ti;
        if (it == uniq.end()) {
            ti = (int)h->h_table_size.size();
            uniq[key] = ti;
            h->h_table_size.push_back(nt * p[i].tex_size);
            h->h_table_off.push_back(texels);
            texels += nt * p[i].tex_size;
            jobs.push_back(Job{p[i].fibers_per_ply, (double)p[i].fiber_radius, p[i].tex_size, nt,
                               (double)spread, seed});
        } else {
            ti = it->second;
        }
        TypeRec r = bysdf_make_rec(p[i]);
        r.table_off = h->h_table_off[ti];
        h->h_types.push_back(r);
        h->h_type_table.push_back(ti);
        h->max_plies = std::max(h->max_plies, p[i].n_plies);
        if (p[i].mig_tables > 1) h->any_mig = 1;
        h->max_K = std::max(h->max_K, p[i].K);
    }
    h->n_tables = (int32_t)h->h_table_size.size();
    // stage the table in LDS when one table serves every type and fits 32 KB
    h->single_table = h->n_tables == 1 && h->h_table_size[0] <= kMaxLdsTexels;
    h->table_texels = h->h_table_size[0];
    auto cleanup = [&](int rc) {
        if (h->d_types) (void)hipFree(h->d_types);
        if (h->d_tables) (void)hipFree(h->d_tables);
        delete h;
        return rc;
    };
    hipError_t e = hipMalloc(&h->d_types, sizeof(TypeRec) * n_types);
    if (e != hipSuccess) return cleanup(fail(BYSDF_ERR_OOM, "hipMalloc(types): %s", hipGetErrorString(e)));
    e = hipMalloc(&h->d_tables, sizeof(float4) * texels);
    if (e != hipSuccess) return cleanup(fail(BYSDF_ERR_OOM, "hipMalloc(tables): %s", hipGetErrorString(e)));
    e = hipMemcpyAsync(h->d_types, h->h_types.data(), sizeof(TypeRec) * n_types, hipMemcpyHostToDevice,
                       stream);
    if (e != hipSuccess) return cleanup(fail(BYSDF_ERR_LAUNCH, "upload: %s", hipGetErrorString(e)));
    for (size_t j = 0; j < jobs.size(); ++j) {
        const Job& jb = jobs[j];
        for (int m = 0; m < jb.tables; ++m) {
            hipLaunchKernelGGL(k_fiber_table, dim3(jb.Nu), dim3(256), 0, stream, jb.M, jb.rho, jb.Nu,
                               h->d_tables + h->h_table_off[j] + (int64_t)m * jb.Nu, m, jb.spread, jb.seed);
            e = hipGetLastError();
            if (e != hipSuccess)
                return cleanup(fail(BYSDF_ERR_LAUNCH, "k_fiber_table: %s", hipGetErrorString(e)));
        }
    }
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return cleanup(fail(BYSDF_ERR_LAUNCH, "table build: %s", hipGetErrorString(e)));
    *out = h;
    return BYSDF_OK;
}

extern "C" int bysdf_types_create(const bysdf_type_params* p, int32_t n_types, bysdf_types_t** out,
                                  hipStream_t stream)
{
    return host_guard([&] { return types_create(p, n_types, out, stream); });
}

extern "C" int bysdf_types_destroy(bysdf_types_t* h)
{
    if (!h) return BYSDF_OK;
    if (h->d_types) (void)hipFree(h->d_types);
    if (h->d_tables) (void)hipFree(h->d_tables);
    delete h;
    return BYSDF_OK;
}

extern "C" int32_t bysdf_types_count(const bysdf_types_t* h)
{
    if (!h) return fail(BYSDF_ERR_INVALID_ARG, "types is NULL");
    return h->n_types;
}

static int types_table(const bysdf_types_t* h, int32_t ti, float* host_out, int64_t cap)
{
    if (!h || !host_out) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (ti < 0 || ti >= h->n_types) return fail(BYSDF_ERR_INVALID_ARG, "type index out of range");
    int tb = h->h_type_table[ti];
    int Nu = h->h_table_size[tb];
    if (cap < 3LL * Nu) return fail(BYSDF_ERR_INVALID_ARG, "host_out needs %d floats", 3 * Nu);
    std::vector<float4> tmp(Nu);
    HIP_TRY(hipMemcpy(tmp.data(), h->d_tables + h->h_table_off[tb], sizeof(float4) * Nu,
                      hipMemcpyDeviceToHost));
    for (int i = 0; i < Nu; ++i) {
        host_out[3 * i] = tmp[i].x;
        host_out[3 * i + 1] = tmp[i].y;
        host_out[3 * i + 2] = tmp[i].z;
    }
    return BYSDF_OK;
}

extern "C" int bysdf_types_table(const bysdf_types_t* h, int32_t ti, float* host_out, int64_t cap)
{
    return host_guard([&] { return types_table(h, ti, host_out, cap); });
}

extern "C" int bysdf_types_set_theta(bysdf_types_t* h, const float* theta, hipStream_t stream)
{
    if (!h || !aligned4(theta)) return fail(BYSDF_ERR_INVALID_ARG, "NULL or misaligned argument");
    int nb = (h->n_types + 255) / 256;
    hipLaunchKernelGGL(k_set_theta, dim3(nb), dim3(256), 0, stream, h->d_types, theta, h->n_types);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

// kernel instance for a handle: ply bound, LDS-staged table, migration
#define BYSDF_PICK(K, h)                                                                               \
    ((h)->any_mig ? ((h)->max_plies <= 4 ? ((h)->single_table ? K<true, 4, true> : K<false, 4, true>)  \
                                         : ((h)->single_table ? K<true, 8, true> : K<false, 8, true>)) \
                  : ((h)->max_plies <= 4 ? ((h)->single_table ? K<true, 4, false> : K<false, 4, false>) \
                                         : ((h)->single_table ? K<true, 8, false> : K<false, 8, false>)))

static int grid_for(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    const int64_t cap = 256 * 16;  // 16 workgroups per CU keeps LDS staging amortised
    return (int)(g < cap ? g : cap);
}

extern "C" int bysdf_eval(const bysdf_types_t* h, const bysdf_query_soa* q, int64_t n,
                          const bysdf_eval_out_soa* o, hipStream_t stream)
{
    if (!h || !q || !o) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return BYSDF_OK;
    const void* need[] = {q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y,
                          q->wo_z, o->E_r, o->E_g, o->E_b, o->E_xS, o->E_yS, o->E_xB_r, o->E_xB_g,
                          o->E_xB_b, o->E_yB_r, o->E_yB_g, o->E_yB_b, o->pdf, o->flags};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "a query/output pointer is NULL or misaligned");
    if ((q->shift0 == nullptr) != (q->shift1 == nullptr) ||
        (q->shift0 && (!aligned4(q->shift0) || !aligned4(q->shift1))))
        return fail(BYSDF_ERR_INVALID_ARG, "shift0/shift1 must both be NULL or both valid");
    QPtrs qp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y, q->wo_z,
             q->shift0, q->shift1};
    OPtrs op{o->E_r, o->E_g, o->E_b, o->E_xS, o->E_yS, o->E_xB_r, o->E_xB_g, o->E_xB_b,
             o->E_yB_r, o->E_yB_g, o->E_yB_b, o->pdf, o->flags};
    int grid = grid_for(n);
    size_t lds = h->single_table ? sizeof(float4) * h->table_texels : 0;
    int tx = h->single_table ? h->table_texels : 0;
    auto kern = BYSDF_PICK(k_eval, h);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, stream, h->d_types, h->n_types,
                       h->d_tables, tx, qp, op, n);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

static int check_sample_args(const bysdf_sample_soa* q)
{
    const void* need[] = {q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "a query pointer is NULL or misaligned");
    const bool none = !q->xi0 && !q->xi1 && !q->xi2;
    if (!none && (!aligned4(q->xi0) || !aligned4(q->xi1) || !aligned4(q->xi2)))
        return fail(BYSDF_ERR_INVALID_ARG, "xi0..xi2 must all be NULL (Philox draws) or all valid");
    if ((q->shift0 == nullptr) != (q->shift1 == nullptr) ||
        (q->shift0 && (!aligned4(q->shift0) || !aligned4(q->shift1))))
        return fail(BYSDF_ERR_INVALID_ARG, "shift0/shift1 must both be NULL or both valid");
    return 0;
}

extern "C" int bysdf_sample_pdf(const bysdf_types_t* h, const bysdf_sample_soa* q, int64_t n,
                                const bysdf_sample_out_soa* o, hipStream_t stream)
{
    if (!h || !q || !o) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return BYSDF_OK;
    if (int rc = check_sample_args(q)) return rc;
    const void* need[] = {o->wo_x, o->wo_y, o->wo_z, o->w_r, o->w_g, o->w_b, o->pdf, o->exit_x,
                          o->exit_y, o->exit_z, o->lobe, o->node, o->flags};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "an output pointer is NULL or misaligned");
    SPtrs sp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->xi0, q->xi1, q->xi2,
             q->shift0, q->shift1, q->seed};
    SOPtrs op{o->wo_x, o->wo_y, o->wo_z, o->w_r, o->w_g, o->w_b, o->pdf, o->exit_x, o->exit_y,
              o->exit_z, o->lobe, o->node, o->flags};
    int grid = grid_for(n);
    size_t lds = h->single_table ? sizeof(float4) * h->table_texels : 0;
    int tx = h->single_table ? h->table_texels : 0;
    auto kern = BYSDF_PICK(k_sample, h);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, stream, h->d_types, h->n_types,
                       h->d_tables, tx, sp, op, n);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

extern "C" int bysdf_eval_sample(const bysdf_types_t* h, const bysdf_query_soa* q, const float* xi0,
                                 const float* xi1, const float* xi2, int64_t n,
                                 const bysdf_eval_out_soa* o, const bysdf_sample_out_soa* so,
                                 hipStream_t stream)
{
    if (!h || !q || !o || !so) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return BYSDF_OK;
    const void* need[] = {q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y,
                          q->wo_z, xi0, xi1, xi2, o->E_r, o->E_g, o->E_b, o->E_xS, o->E_yS,
                          o->E_xB_r, o->E_xB_g, o->E_xB_b, o->E_yB_r, o->E_yB_g, o->E_yB_b, o->pdf,
                          o->flags, so->wo_x, so->wo_y, so->wo_z, so->w_r, so->w_g, so->w_b, so->pdf,
                          so->exit_x, so->exit_y, so->exit_z, so->lobe, so->node, so->flags};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "a query/output pointer is NULL or misaligned");
    if ((q->shift0 == nullptr) != (q->shift1 == nullptr) ||
        (q->shift0 && (!aligned4(q->shift0) || !aligned4(q->shift1))))
        return fail(BYSDF_ERR_INVALID_ARG, "shift0/shift1 must both be NULL or both valid");
    QPtrs qp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y, q->wo_z,
             q->shift0, q->shift1};
    OPtrs op{o->E_r, o->E_g, o->E_b, o->E_xS, o->E_yS, o->E_xB_r, o->E_xB_g, o->E_xB_b,
             o->E_yB_r, o->E_yB_g, o->E_yB_b, o->pdf, o->flags};
    SOPtrs sop{so->wo_x, so->wo_y, so->wo_z, so->w_r, so->w_g, so->w_b, so->pdf, so->exit_x,
               so->exit_y, so->exit_z, so->lobe, so->node, so->flags};
    int grid = grid_for(n);
    size_t lds = h->single_table ? sizeof(float4) * h->table_texels : 0;
    int tx = h->single_table ? h->table_texels : 0;
    auto kern = BYSDF_PICK(k_eval_sample, h);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, stream, h->d_types, h->n_types,
                       h->d_tables, tx, qp, xi0, xi1, xi2, op, sop, n);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

static int check_footprint_args(const bysdf_footprint_soa* fp, bool sampler)
{
    if (!aligned4(fp->h1) || !aligned4(fp->h2) || !aligned4(fp->zeta) || (sampler && !aligned4(fp->xi_s)))
        return fail(BYSDF_ERR_INVALID_ARG, "a footprint pointer is NULL or misaligned");
    return 0;
}

extern "C" int bysdf_eval_multi(const bysdf_types_t* h, const bysdf_query_soa* q,
                                const bysdf_footprint_soa* fp, int64_t n, int32_t n_max,
                                const bysdf_eval_out_soa* o, hipStream_t stream)
{
    if (!h || !q || !o) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    if (!fp) return fail(BYSDF_ERR_INVALID_ARG, "NULL footprint");
    if (n_max < 1 || n_max > kMaxStrata) return fail(BYSDF_ERR_INVALID_ARG, "n_max must be in 1..16");
    if (n == 0) return BYSDF_OK;
    if (int rc = check_footprint_args(fp, false)) return rc;
    const void* need[] = {q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y,
                          q->wo_z, o->E_r, o->E_g, o->E_b, o->E_xS, o->E_yS, o->E_xB_r, o->E_xB_g,
                          o->E_xB_b, o->E_yB_r, o->E_yB_g, o->E_yB_b, o->pdf, o->flags};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "a query/output pointer is NULL or misaligned");
    if ((q->shift0 == nullptr) != (q->shift1 == nullptr) ||
        (q->shift0 && (!aligned4(q->shift0) || !aligned4(q->shift1))))
        return fail(BYSDF_ERR_INVALID_ARG, "shift0/shift1 must both be NULL or both valid");
    QPtrs qp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y, q->wo_z,
             q->shift0, q->shift1};
    FPtrs fpp{fp->h1, fp->h2, fp->zeta, nullptr};
    OPtrs op{o->E_r, o->E_g, o->E_b, o->E_xS, o->E_yS, o->E_xB_r, o->E_xB_g, o->E_xB_b,
             o->E_yB_r, o->E_yB_g, o->E_yB_b, o->pdf, o->flags};
    int grid = grid_for(n);
    size_t lds = h->single_table ? sizeof(float4) * h->table_texels : 0;
    int tx = h->single_table ? h->table_texels : 0;
    auto kern = BYSDF_PICK(k_eval_multi, h);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, stream, h->d_types, h->n_types,
                       h->d_tables, tx, qp, fpp, (int)n_max, op, n);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

extern "C" int bysdf_sample_multi(const bysdf_types_t* h, const bysdf_sample_soa* q,
                                  const bysdf_footprint_soa* fp, int64_t n, int32_t n_max,
                                  const bysdf_sample_out_soa* o, hipStream_t stream)
{
    if (!h || !q || !o) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    if (!fp) return fail(BYSDF_ERR_INVALID_ARG, "NULL footprint");
    if (n_max < 1 || n_max > kMaxStrata) return fail(BYSDF_ERR_INVALID_ARG, "n_max must be in 1..16");
    if (n == 0) return BYSDF_OK;
    if (int rc = check_footprint_args(fp, true)) return rc;
    if (int rc = check_sample_args(q)) return rc;
    const void* need[] = {o->wo_x, o->wo_y, o->wo_z, o->w_r, o->w_g, o->w_b, o->pdf, o->exit_x,
                          o->exit_y, o->exit_z, o->lobe, o->node, o->flags};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "an output pointer is NULL or misaligned");
    SPtrs sp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->xi0, q->xi1, q->xi2,
             q->shift0, q->shift1, q->seed};
    FPtrs fpp{fp->h1, fp->h2, fp->zeta, fp->xi_s};
    SOPtrs op{o->wo_x, o->wo_y, o->wo_z, o->w_r, o->w_g, o->w_b, o->pdf, o->exit_x, o->exit_y,
              o->exit_z, o->lobe, o->node, o->flags};
    int grid = grid_for(n);
    size_t lds = h->single_table ? sizeof(float4) * h->table_texels : 0;
    int tx = h->single_table ? h->table_texels : 0;
#define BYSDF_PICK_SM(X)                                                                                 \
    (h->any_mig ? (h->max_plies <= 4 ? (h->single_table ? k_sample_multi<true, 4, true, X>                  \
                                                        : k_sample_multi<false, 4, true, X>)               \
                                     : (h->single_table ? k_sample_multi<true, 8, true, X>                  \
                                                        : k_sample_multi<false, 8, true, X>))              \
                : (h->max_plies <= 4 ? (h->single_table ? k_sample_multi<true, 4, false, X>                 \
                                                        : k_sample_multi<false, 4, false, X>)              \
                                     : (h->single_table ? k_sample_multi<true, 8, false, X>                 \
                                                        : k_sample_multi<false, 8, false, X>)))
    auto kern = q->xi0 ? BYSDF_PICK_SM(false) : BYSDF_PICK_SM(true);
#undef BYSDF_PICK_SM
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, stream, h->d_types, h->n_types,
                       h->d_tables, tx, sp, fpp, (int)n_max, op, n);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

extern "C" int bysdf_ply_geometry(const bysdf_types_t* h, const bysdf_query_soa* q, int64_t n,
                                  const bysdf_ply_out_soa* o, hipStream_t stream)
{
    if (!h || !q || !o) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return BYSDF_OK;
    const void* need[] = {q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, o->ply, o->p_x, o->p_y,
                          o->p_z, o->t_x, o->t_y, o->t_z, o->n_x, o->n_y, o->n_z, o->flags};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "a query/output pointer is NULL or misaligned");
    QPtrs qp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, nullptr, nullptr, nullptr, nullptr, nullptr};
    PlyOPtrs op{o->ply, o->p_x, o->p_y, o->p_z, o->t_x, o->t_y, o->t_z, o->n_x, o->n_y, o->n_z, o->flags};
    auto kern = h->max_plies <= 4 ? k_ply_geometry<4> : k_ply_geometry<8>;
    hipLaunchKernelGGL(kern, dim3(grid_for(n)), dim3(kBlock), 0, stream, h->d_types, h->n_types, qp, op, n);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

extern "C" int bysdf_furnace_blocks(const bysdf_types_t* h, const bysdf_sample_soa* q, int64_t n,
                                    int32_t block, float* mean, float* var, hipStream_t stream)
{
    if (!h || !q) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    if (block < 64 || block > 1024 || block % 64)
        return fail(BYSDF_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
    int64_t nb = n / block;
    if (nb == 0) return BYSDF_OK;
    if (int rc = check_sample_args(q)) return rc;
    if (!aligned4(mean) || !aligned4(var)) return fail(BYSDF_ERR_INVALID_ARG, "mean/var NULL or misaligned");
    if (nb > 0x7fffffffLL) return fail(BYSDF_ERR_INVALID_ARG, "too many blocks");
    SPtrs sp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->xi0, q->xi1, q->xi2,
             q->shift0, q->shift1, q->seed};
    if (BYSDF_FURNACE_WAVE && block <= kWave * kMaxDrawsPerLane) {
        auto kw = h->any_mig ? (h->max_plies <= 4 ? k_furnace_w<4, true> : k_furnace_w<8, true>)
                             : (h->max_plies <= 4 ? k_furnace_w<4, false> : k_furnace_w<8, false>);
        // blocks per wavefront: up to 8, and at most 32 forward nodes to form
        const int kmax = h->max_K;
        int group = BYSDF_FURNACE_NODE_ITEMS / kmax;
        group = group < 1 ? 1 : (group > kFurnaceGroupMax ? kFurnaceGroupMax : group);
        const int64_t per_wg = (int64_t)kFurnaceWaves * group;
        const int64_t wgs = (nb + per_wg - 1) / per_wg;
        if (wgs > 0x7fffffffLL) return fail(BYSDF_ERR_INVALID_ARG, "too many blocks");
        const size_t lds = sizeof(Node<double, float>) * kFurnaceWaves * group * kmax;
        hipLaunchKernelGGL(kw, dim3((unsigned)wgs), dim3(kBlock), lds, stream, h->d_types, h->n_types,
                           h->d_tables, sp, block, nb, group, kmax, mean, var);
    } else {
        auto kern = h->any_mig ? (h->max_plies <= 4 ? k_furnace<4, true> : k_furnace<8, true>)
                               : (h->max_plies <= 4 ? k_furnace<4, false> : k_furnace<8, false>);
        hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kBlock), 0, stream, h->d_types, h->n_types,
                           h->d_tables, sp, block, mean, var);
    }
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

// ------------------------------------------------------------------ op count
namespace bysdf {
thread_local OpTally* g_tally = nullptr;
}

struct HostTab {
    static constexpr bool kMigration = true;
    const float4* p;
    float4 operator()(int i) const { return p[i]; }
};

static int count_ops(const bysdf_type_params* p, const float* table, int64_t n, const float* h, const float* u,
                     const float* v, const float* wi, const float* wo, const float* xi, int32_t mode,
                     double* counts)
{
    if (!p || !table || !h || !u || !v || !wi || !counts || n < 1 || mode < 0 || mode > 2)
        return fail(BYSDF_ERR_INVALID_ARG, "bad argument");
    if (mode != 1 && !wo) return fail(BYSDF_ERR_INVALID_ARG, "modes 0 and 2 need wo");
    if (mode != 0 && !xi) return fail(BYSDF_ERR_INVALID_ARG, "modes 1 and 2 need xi");
    if (int rc = validate(*p, 0)) return rc;
    TypeRec rec = bysdf_make_rec(*p);
    std::vector<float4> tb(rec.table_texels);
    for (int i = 0; i < rec.table_texels; ++i)
        tb[i] = make_float4(table[3 * i], table[3 * i + 1], table[3 * i + 2], 0.0f);
    HostTab tab{tb.data()};
    Derived<CD, CF> P = derive_counted(rec);
    OpTally tally;
    memset(&tally, 0, sizeof(tally));
    g_tally = &tally;
    for (int64_t i = 0; i < n; ++i) {
        V3<float> a = mk3<float>(wi[i], wi[n + i], wi[2 * n + i]);
        if (check_inputs(h[i], u[i], v[i], a)) continue;
        if (mode == 0) {
            XState<CD, CF, kMaxPlies> X;
            state_at_x(P, tab, h[i], u[i], v[i], a, X);
            if (X.ph.pass) continue;
            V3<CD> b = mk3<CD>(CD((double)wo[i]), CD((double)wo[n + i]), CD((double)wo[2 * n + i]));
            EvalOut<CF> e;
            lobes(P, tab, X, b, 0.0f, 0.0f, false, e, rec.node_disk);
        } else if (mode == 2) {
            XState<CD, CF, kMaxPlies> X;
            state_at_x(P, tab, h[i], u[i], v[i], a, X);
            V3<CD> b = mk3<CD>(CD((double)wo[i]), CD((double)wo[n + i]), CD((double)wo[2 * n + i]));
            NodesComputed<CD, CF, kMaxPlies, HostTab> nf{P, tab, X, 0.0f, 0.0f, false, rec.node_disk};
            EvalOut<CF> e;
            SampleOut<CF> so;
            eval_sample_from_x(P, X, a, b, true, xi[i], xi[n + i], xi[2 * n + i], nf, e, so);
        } else {
            SampleOut<CF> so;
            sample_query<CD, CF, kMaxPlies>(P, tab, h[i], u[i], v[i], a, xi[i], xi[n + i],
                                            xi[2 * n + i], 0.0f, 0.0f, false, so, rec.node_disk);
        }
    }
    g_tally = nullptr;
    for (int k = 0; k < 2; ++k) {
        counts[5 * k + 0] = tally.add[k] / n;
        counts[5 * k + 1] = tally.mul[k] / n;
        counts[5 * k + 2] = tally.div[k] / n;
        counts[5 * k + 3] = tally.sqrt[k] / n;
        counts[5 * k + 4] = tally.trans[k] / n;
    }
    return BYSDF_OK;
}

extern "C" int bysdf_count_ops(const bysdf_type_params* p, const float* table, int64_t n,
                               const float* h, const float* u, const float* v, const float* wi,
                               const float* wo, const float* xi, int32_t mode, double* counts)
{
    return host_guard([&] { return count_ops(p, table, n, h, u, v, wi, wo, xi, mode, counts); });
}

// ------------------------------------------------------------------ adjoint API
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int64_t max_tiles(int64_t n, int32_t n_types) { return (n + kBlock - 1) / kBlock + n_types; }

extern "C" size_t bysdf_backward_workspace_size(int64_t n, int32_t n_types)
{
    if (n < 0 || n_types < 1) return 0;
    return align256(sizeof(int32_t) * (size_t)(n_types + 1)) +
           sizeof(float) * 8 * (size_t)max_tiles(n, n_types);
}

extern "C" int bysdf_eval_backward(const bysdf_types_t* h, const bysdf_query_soa* q, int64_t n,
                                   const int64_t* type_offsets, const float* grad_E,
                                   float* grad_theta, float* per_query, void* workspace,
                                   size_t ws_bytes, hipStream_t stream)
{
    if (!h || !q || !type_offsets || !aligned4(grad_E) || !aligned4(grad_theta))
        return fail(BYSDF_ERR_INVALID_ARG, "NULL or misaligned argument");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    const void* need[] = {q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y, q->wo_z};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "a query pointer is NULL or misaligned");
    if (((uintptr_t)type_offsets & 7u) != 0) return fail(BYSDF_ERR_INVALID_ARG, "type_offsets misaligned");
    if (per_query && !aligned4(per_query)) return fail(BYSDF_ERR_INVALID_ARG, "per_query misaligned");
    if ((q->shift0 == nullptr) != (q->shift1 == nullptr))
        return fail(BYSDF_ERR_INVALID_ARG, "shift0/shift1 must both be NULL or both valid");
    size_t need_ws = bysdf_backward_workspace_size(n, h->n_types);
    if (!workspace || ws_bytes < need_ws || ((uintptr_t)workspace & 255u))
        return fail(BYSDF_ERR_INVALID_ARG, "workspace needs %zu bytes, 256-byte aligned", need_ws);
    int32_t* tile_first = (int32_t*)workspace;
    float* partials = (float*)((char*)workspace + align256(sizeof(int32_t) * (h->n_types + 1)));
    QPtrs qp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y, q->wo_z,
             q->shift0, q->shift1};
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, stream, type_offsets, h->n_types, tile_first,
                       kBlock);
    HIP_TRY(hipGetLastError());
    int64_t tiles = max_tiles(n, h->n_types);
    if (tiles > 0x7fffffffLL) return fail(BYSDF_ERR_INVALID_ARG, "too many tiles");
    const bool mp4 = h->max_plies <= 4;
    decltype(&k_backward<4, 0>) passes[3] = {mp4 ? k_backward<4, 0> : k_backward<8, 0>,
                                             mp4 ? k_backward<4, 1> : k_backward<8, 1>,
                                             mp4 ? k_backward<4, 2> : k_backward<8, 2>};
    for (auto kern : passes) {
        hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(kBlock), 0, stream, h->d_types, h->d_tables, qp,
                           type_offsets, h->n_types, tile_first, grad_E, partials, per_query);
        HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_backward_sum, dim3((h->n_types + 255) / 256), dim3(256), 0, stream, tile_first,
                       h->n_types, partials, grad_theta);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

// ------------------------------------------------------------------ hetero API
extern "C" size_t bysdf_batched_workspace_size(int32_t n_types)
{
    if (n_types < 1) return 0;
    return align256(sizeof(int32_t) * (size_t)(n_types + 1)) + 256;
}

template <int MP>
static void launch_batched(const bysdf_types_t* h, bool lds, int waves, int block, int grid,
                           hipStream_t stream, const int64_t* off, const int32_t* tile_first, int* counter,
                           QPtrs qp, OPtrs op, int chunk)
{
    auto kern = lds ? (waves == 1 ? k_eval_batched<MP, true, 1> : k_eval_batched<MP, true, 2>)
                    : (waves == 1 ? k_eval_batched<MP, false, 1> : k_eval_batched<MP, false, 2>);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, h->d_types, h->d_tables, off, h->n_types,
                       tile_first, counter, qp, op, chunk);
}

extern "C" int bysdf_eval_batched(const bysdf_types_t* h, const int64_t* type_offsets, int64_t n,
                                  const bysdf_query_soa* q, const bysdf_eval_out_soa* o,
                                  const bysdf_schedule* sched, void* workspace, size_t ws_bytes,
                                  hipStream_t stream)
{
    if (!h || !q || !o || !type_offsets) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (((uintptr_t)type_offsets & 7u) != 0) return fail(BYSDF_ERR_INVALID_ARG, "type_offsets misaligned");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    const void* need[] = {q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y, q->wo_z,
                          o->E_r, o->E_g, o->E_b, o->E_xS, o->E_yS, o->E_xB_r, o->E_xB_g, o->E_xB_b,
                          o->E_yB_r, o->E_yB_g, o->E_yB_b, o->pdf, o->flags};
    for (const void* ptr : need)
        if (!aligned4(ptr)) return fail(BYSDF_ERR_INVALID_ARG, "a query/output pointer is NULL or misaligned");
    if ((q->shift0 == nullptr) != (q->shift1 == nullptr))
        return fail(BYSDF_ERR_INVALID_ARG, "shift0/shift1 must both be NULL or both valid");
    size_t need_ws = bysdf_batched_workspace_size(h->n_types);
    if (!workspace || ws_bytes < need_ws || ((uintptr_t)workspace & 255u))
        return fail(BYSDF_ERR_INVALID_ARG, "workspace needs %zu bytes, 256-byte aligned", need_ws);
    int chunk = 4, grid = 0, use_lds = 1, block = kBlock, waves = BYSDF_BATCHED_MIN_WAVES;
    if (sched) {
        chunk = sched->chunk;
        grid = sched->grid;
        use_lds = sched->use_lds;
        if (sched->block) block = sched->block;
        if (sched->min_waves) waves = sched->min_waves;
    }
    if (chunk < 1 || chunk > 64) return fail(BYSDF_ERR_INVALID_ARG, "schedule chunk must be in 1..64");
    if (grid < 0 || grid > (1 << 20)) return fail(BYSDF_ERR_INVALID_ARG, "schedule grid out of range");
    if (block != 128 && block != 256) return fail(BYSDF_ERR_INVALID_ARG, "schedule block must be 128 or 256");
    if (waves != 1 && waves != 2) return fail(BYSDF_ERR_INVALID_ARG, "schedule min_waves must be 1 or 2");
    bool lds = use_lds != 0;
    for (int i = 0; lds && i < h->n_tables; ++i)
        if (h->h_table_size[i] > kMaxLdsTexels) lds = false;
    if (grid == 0) grid = 256 * 8;
    if (n == 0) return BYSDF_OK;
    int32_t* tile_first = (int32_t*)workspace;
    int* counter = (int*)((char*)workspace + align256(sizeof(int32_t) * (h->n_types + 1)));
    QPtrs qp{q->type_id, q->h, q->u, q->v, q->wi_x, q->wi_y, q->wi_z, q->wo_x, q->wo_y, q->wo_z,
             q->shift0, q->shift1};
    OPtrs op{o->E_r, o->E_g, o->E_b, o->E_xS, o->E_yS, o->E_xB_r, o->E_xB_g, o->E_xB_b,
             o->E_yB_r, o->E_yB_g, o->E_yB_b, o->pdf, o->flags};
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, stream, type_offsets, h->n_types, tile_first, block);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, stream, counter);
    if (h->max_plies <= 4)
        launch_batched<4>(h, lds, waves, block, grid, stream, type_offsets, tile_first, counter, qp, op, chunk);
    else if (h->max_plies <= 6)
        launch_batched<6>(h, lds, waves, block, grid, stream, type_offsets, tile_first, counter, qp, op, chunk);
    else
        launch_batched<8>(h, lds, waves, block, grid, stream, type_offsets, tile_first, counter, qp, op, chunk);
    HIP_TRY(hipGetLastError());
    return BYSDF_OK;
}

// ------------------------------------------------------------------ no-alloc hetero API
// Workspace of bysdf_eval_batched_noalloc in static device memory: the
// per-type tile offsets of up to kNoAllocMaxTypes types and the queue
// counter, laid out as bysdf_eval_batched lays out a caller's workspace.
// Each GPU the library runs on holds its own copy until the process ends.
constexpr int kNoAllocMaxTypes = BYSDF_NOALLOC_MAX_TYPES;
constexpr size_t kNoAllocScratchBytes =
    ((sizeof(int32_t) * (size_t)(kNoAllocMaxTypes + 1) + 255) / 256) * 256 + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of this GPU's copy of the scratch array, looked up once per
// device with that device current.  In host code `scratch` only names the
// symbol; kernels receive the address found here.
static int scratch_address(void** out)
{
    static std::mutex mu;
    static std::map<int, void*> addr;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & 255u)) return fail(BYSDF_ERR_LAUNCH, "scratch address of device %d unusable", dev);
        it = addr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return BYSDF_OK;
}

extern "C" int bysdf_eval_batched_noalloc(const bysdf_types_t* h, const int64_t* type_offsets, int64_t n,
                                          const bysdf_query_soa* q, const bysdf_eval_out_soa* o,
                                          const bysdf_schedule* sched, hipStream_t stream)
{
    if (!h) return fail(BYSDF_ERR_INVALID_ARG, "NULL argument");
    if (h->n_types > kNoAllocMaxTypes)
        return fail(BYSDF_ERR_INVALID_ARG, "bysdf_eval_batched_noalloc serves at most %d types (handle has %d)",
                    kNoAllocMaxTypes, h->n_types);
    void* ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc != BYSDF_OK) return rc;
    return bysdf_eval_batched(h, type_offsets, n, q, o, sched, ws, kNoAllocScratchBytes, stream);
}
