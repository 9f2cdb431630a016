// lib_internal.hpp -- declarations shared by the translation units of
// libbysdf (hidden from the C ABI).
#pragma once

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
// loads and its scalars stay out of the vector registers.
template <class F>
__device__ inline void for_each_wave_type(int t, bool need, F&& body)
{
    unsigned long long pending = __ballot(need);
    if (!pending) return;
    {
        // the common case, a wavefront of one type, runs the body on a
        // straight-line path: no value has to stay live around a loop
        const int t0 = __builtin_amdgcn_readlane(t, __ffsll((long long)pending) - 1);
        if (__ballot(need && t != t0) == 0ull) {
            if (need) body(t0);
            return;
        }
    }
    while (pending) {
        const int lead = __ffsll((long long)pending) - 1;
        const int tu = __builtin_amdgcn_readlane(t, lead);
        const bool mine = need && t == tu;
        if (mine) body(tu);
        pending &= ~__ballot(mine);
    }
}
