// lib_internal.hpp -- declarations shared by the translation units of
// libbysdf (hidden from the C ABI).
#pragma once

#include <cstring>

#include "../../include/bysdf.h"
#include "bysdf_model.hpp"
#include "yarn_tube.hpp"

// Fiber tables in device memory (or LDS).  MIG: the kernel may serve types
// with fiber migration (several tables per type); kernels instantiated
// without it skip that code, which keeps their register allocation.
template <bool MIG> struct TabPtrT {
    static constexpr bool kMigration = MIG;
    const float4* p;
    __host__ __device__ float4 operator()(int i) const { return p[i]; }
};
using TabPtr = TabPtrT<true>;

// The device record of one type: its parameters and the derived scalars.
inline bysdf::TypeRec bysdf_make_rec(const bysdf_type_params& p)
{
    bysdf::TypeRec t;
    memset(&t, 0, sizeof(t));
    t.n_plies = p.n_plies;
    t.K = p.K;
    t.n_iter = p.n_iter;
    t.tex_size = p.tex_size;
    t.rp = p.ply_radius;
    t.Rpc = p.ply_center_radius;
    t.ply_twist = p.ply_twist;
    t.fiber_twist = p.fiber_twist;
    t.rho_f_geom = p.fiber_radius;
    t.beta = p.beta;
    t.aniso = p.aniso;
    t.eta = p.eta;
    for (int c = 0; c < 3; ++c) t.albedo[c] = p.albedo[c];
    t.k_spec = p.k_spec;
    t.B = p.B;
    t.r = p.r;
    t.sigma_t = p.sigma_t;
    t.ply_density = p.ply_density;
    t.fiber_density = p.fiber_density;
    t.shadow_hw = p.shadow_halfwidth;
    t.mig_tables = p.mig_tables > 1 ? p.mig_tables : 1;
    t.mig_seed = p.mig_seed;
    t.mig_period = p.mig_tables > 1 ? p.mig_period : 1.0;
    t.mig_blend = p.mig_blend;
    t.mig_spread = p.mig_spread;
    t.table_texels = t.mig_tables * p.tex_size;
    bysdf::fill_derived(t);
    bysdf::fill_node_disk(t);
    return t;
}

// record a thread-local error message and return `code`
int bysdf_set_error(int code, const char* msg);

// device data behind a types handle
struct BysdfTypesView {
    const bysdf::TypeRec* types;
    const float4* tables;
    int n_types, max_plies, max_K;
};
BysdfTypesView bysdf_types_view(const bysdf_types_t* h);

// device data behind a scene handle, and its largest yarn type index
yarn::SceneView yarn_scene_view(const yarn_scene_t* s);
int yarn_scene_max_type(const yarn_scene_t* s);

// Lanes of a wavefront are served one distinct type at a time (a wavefront
// of one type -- sorted or per-block input -- takes a single pass): the
// type index is made wavefront-uniform, so its record is read with scalar
// loads and its scalars stay out of the vector registers.  The index handed
// to the body goes through readfirstlane: inside the body the optimiser
// knows it equals the lane's own index and would otherwise address the
// record with that per-lane value, turning every parameter read into a
// vector load.  kScalar = false hands over the index unchanged: the
// multi-scale kernels copy the record into a per-footprint variant, and
// there the vector loads measured faster.  The body is inlined at both of
// its call sites: a body left as a call keeps everything it captures, and
// its own structures, on the private stack.
template <bool kScalar = true, class F>
__device__ inline void for_each_wave_type(int t, bool need, F&& body)
{
    unsigned long long pending = __ballot(need);
    if (!pending) return;
    {
        // the common case, a wavefront of one type, runs the body on a
        // straight-line path: no value has to stay live around a loop
        const int t0 = __builtin_amdgcn_readlane(t, __ffsll((long long)pending) - 1);
        if (__ballot(need && t != t0) == 0ull) {
            if (need) [[clang::always_inline]] body(kScalar ? __builtin_amdgcn_readfirstlane(t0) : t0);
            return;
        }
    }
    while (pending) {
        const int lead = __ffsll((long long)pending) - 1;
        const int tu = __builtin_amdgcn_readlane(t, lead);
        const bool mine = need && t == tu;
        if (mine) [[clang::always_inline]] body(kScalar ? __builtin_amdgcn_readfirstlane(tu) : tu);
        pending &= ~__ballot(mine);
    }
}
