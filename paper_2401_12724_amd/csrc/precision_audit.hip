// precision_audit.hip -- libbysdf_audit: the kernels' per-query model
// (bysdf_model.hpp, the same templates the kernels instantiate) run on the
// host with the geometry scalar Emu, so that chosen stages of the geometry
// chain compute in single precision and the rest in double.  It measures
// how far each stage's precision moves the outputs; it is a measurement
// tool, not a compute path, and libbysdf does not link it.
//
// Entry points take the queries of ONE type, host arrays of n elements
// (direction arrays: 3 x n, component-major), and write host arrays.
// stage_mask: bit s (GeomStage numbering, bysdf_model.hpp) puts stage s in
// single precision; 0 reproduces the kernels' double-precision geometry
// (with the host's libm square roots and quotients in place of the
// device's sequences).  Returns 0, or -1 on a bad argument.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/bysdf.h"
#include "bysdf_model.hpp"
#include "bysdf_precision.hpp"
#include "lib_internal.hpp"

namespace bysdf {
thread_local unsigned g_audit_mask = 0u;
thread_local int g_audit_stage = kStageRest;
}  // namespace bysdf

using namespace bysdf;

namespace {

struct HostTab4 {
    static constexpr bool kMigration = true;
    const float4* p;
    float4 operator()(int i) const { return p[i]; }
};

bool usable(const bysdf_type_params* p)
{
    return p && p->n_plies >= 1 && p->n_plies <= kMaxPlies && p->K >= 1 && p->K <= kMaxNodes &&
           p->n_iter >= 0 && p->n_iter <= 16 && p->tex_size >= 2 && p->tex_size <= 4096 &&
           p->mig_tables >= 0 && p->mig_tables <= kMaxMigTables;
}

// table: texels x 3 floats (delta n, rho hat, G_f), as bysdf_types_table
std::vector<float4> texels(const TypeRec& rec, const float* table)
{
    std::vector<float4> tb(rec.table_texels);
    for (int i = 0; i < rec.table_texels; ++i)
        tb[i] = make_float4(table[3 * i], table[3 * i + 1], table[3 * i + 2], 0.0f);
    return tb;
}

struct MaskScope {
    explicit MaskScope(uint32_t m) { g_audit_mask = m; g_audit_stage = kStageRest; }
    ~MaskScope() { g_audit_mask = 0u; g_audit_stage = kStageRest; }
};

}  // namespace

// Evaluation (as bysdf_eval): out is 12 x n, rows E_r, E_g, E_b, E_xS, E_yS,
// E_xB (3), E_yB (3), pdf; flags as the kernel's.  s0, s1: lattice shifts
// (both NULL for none).
extern "C" int bysdf_audit_eval(const bysdf_type_params* p, const float* table, int64_t n, const float* h,
                                const float* u, const float* v, const float* wi, const float* wo,
                                const float* s0, const float* s1, uint32_t stage_mask, float* out,
                                uint32_t* flags)
{
    if (!usable(p) || !table || n < 0 || !h || !u || !v || !wi || !wo || !out || !flags) return -1;
    if ((s0 == nullptr) != (s1 == nullptr)) return -1;
    const TypeRec rec = bysdf_make_rec(*p);
    const std::vector<float4> tb = texels(rec, table);
    const HostTab4 tab{tb.data()};
    const Derived<Emu, float> P = rebind<Emu, float>(derive(rec));
    MaskScope scope(stage_mask);
    for (int64_t i = 0; i < n; ++i) {
        const V3<float> a = mk3<float>(wi[i], wi[n + i], wi[2 * n + i]);
        const V3<float> b = mk3<float>(wo[i], wo[n + i], wo[2 * n + i]);
        uint32_t fl = check_inputs(h[i], u[i], v[i], a) | check_dir(b);
        EvalOut<float> e;
        for (int c = 0; c < 3; ++c) e.E[c] = e.ExB[c] = e.EyB[c] = 0.0f;
        e.ExS = e.EyS = e.pdf = 0.0f;
        if (fl == 0u) {
            XState<Emu, float, kMaxPlies> X;
            state_at_x(P, tab, h[i], u[i], v[i], a, X);
            fl = X.ph.flags;
            if (!X.ph.pass) {
                if (!(X.mu_i > 0.0f)) fl |= F_BACKFACING;
                const V3<Emu> bg = mk3<Emu>(Emu((double)b.x), Emu((double)b.y), Emu((double)b.z));
                lobes(P, tab, X, bg, s0 ? s0[i] : 0.0f, s1 ? s1[i] : 0.0f, s0 != nullptr, e);
            }
        }
        const float row[12] = {e.E[0], e.E[1], e.E[2], e.ExS, e.EyS, e.ExB[0], e.ExB[1], e.ExB[2],
                               e.EyB[0], e.EyB[1], e.EyB[2], e.pdf};
        for (int c = 0; c < 12; ++c) out[c * n + i] = row[c];
        flags[i] = fl;
    }
    return 0;
}

// Sampling (as bysdf_sample_pdf): xi is 3 x n; out is 7 x n, rows wo (3),
// weight (3), pdf; flags as the kernel's.
extern "C" int bysdf_audit_sample(const bysdf_type_params* p, const float* table, int64_t n, const float* h,
                                  const float* u, const float* v, const float* wi, const float* xi,
                                  const float* s0, const float* s1, uint32_t stage_mask, float* out,
                                  uint32_t* flags)
{
    if (!usable(p) || !table || n < 0 || !h || !u || !v || !wi || !xi || !out || !flags) return -1;
    if ((s0 == nullptr) != (s1 == nullptr)) return -1;
    const TypeRec rec = bysdf_make_rec(*p);
    const std::vector<float4> tb = texels(rec, table);
    const HostTab4 tab{tb.data()};
    const Derived<Emu, float> P = rebind<Emu, float>(derive(rec));
    MaskScope scope(stage_mask);
    for (int64_t i = 0; i < n; ++i) {
        const V3<float> a = mk3<float>(wi[i], wi[n + i], wi[2 * n + i]);
        SampleOut<float> so;
        const uint32_t fl = sample_query<Emu, float, kMaxPlies>(P, tab, h[i], u[i], v[i], a, xi[i], xi[n + i],
                                                               xi[2 * n + i], s0 ? s0[i] : 0.0f,
                                                               s1 ? s1[i] : 0.0f, s0 != nullptr, so);
        const float row[7] = {so.wo[0], so.wo[1], so.wo[2], so.wgt[0], so.wgt[1], so.wgt[2], so.pdf};
        for (int c = 0; c < 7; ++c) out[c * n + i] = row[c];
        flags[i] = fl;
    }
    return 0;
}
