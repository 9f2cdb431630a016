// yarn_scene.hip -- yarn scenes (B-spline centrelines, frames, BVH) and the
// ray / yarn-tube intersection kernel of libbysdf (see include/bysdf.h).
//
// Scene build (host threads, once per scene, yarn_build.hpp): per span the rotation-minimising
// frame at its start (double reflection, 16 steps per span) and the arc
// length from the yarn start (5-point Gauss-Legendre per span); a binned
// SAH BVH over the span boxes (control-point hull grown by R), with object
// median splits below depth 40, collapsed to four children per node.
// Spans are stored in leaf order next to their records.
//
// Kernel k_intersect: one ray per lane, 128-lane workgroups, an LDS stack
// per lane ([entry][lane], no bank conflicts) of 3 (depth + 1) entries.  A point query
// first collects the yarns whose tube holds the origin, then the closest
// entering hit is searched; hit frame, h and v are formed for the winner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bysdf.h"
#include "lib_internal.hpp"
#include "yarn_build.hpp"
#include "yarn_tube.hpp"

using namespace yarn;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return bysdf_set_error(code, buf);
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? BYSDF_ERR_OOM : BYSDF_ERR_LAUNCH,     \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                   \
    } while (0)

struct yarn_scene {
    int device = 0;
    int32_t n_yarns = 0;
    int64_t n_cp = 0, n_spans = 0, n_nodes = 0;
    int depth = 0;
    int max_type = 0;  // largest yarn type index (checked against a types handle)
    float4* d_cp = nullptr;
    SpanRec* d_span = nullptr;
    float4* d_frame = nullptr;
    WNode* d_node = nullptr;
    float* d_phase = nullptr;
    int* d_type = nullptr;
    size_t bytes = 0;
    SceneView view() const
    {
        SceneView v;
        v.cp = d_cp;
        v.span = d_span;
        v.frame = d_frame;
        v.node = d_node;
        v.yarn_phase = d_phase;
        v.yarn_type = d_type;
        v.n_nodes = (int)n_nodes;
        return v;
    }
};

// ------------------------------------------------------------ kernel
constexpr int kIsectBlock = 128;

#ifndef YARN_ISECT_MIN_WAVES
#define YARN_ISECT_MIN_WAVES 3
#endif
__global__ __launch_bounds__(kIsectBlock, YARN_ISECT_MIN_WAVES) void k_intersect(SceneView S, yarn_ray_soa R,
                                                                                 int64_t n, double t_min,
                                                                                 yarn_hit_soa H)
{
    extern __shared__ int stk[];  // stack_entries(depth) x kIsectBlock
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        intersect_ray(S, i, R, t_min, H, stk + threadIdx.x, kIsectBlock);
}

// ------------------------------------------------------------ C ABI
static int check_gfx950(int* dev)
{
    HIP_TRY(hipGetDevice(dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, *dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BYSDF_ERR_UNSUPPORTED_DEVICE, "device %d is %s, library is built for gfx950", *dev,
                    prop.gcnArchName);
    return 0;
}

static void free_scene(yarn_scene* s)
{
    if (!s) return;
    (void)hipFree(s->d_cp);
    (void)hipFree(s->d_span);
    (void)hipFree(s->d_frame);
    (void)hipFree(s->d_node);
    (void)hipFree(s->d_phase);
    (void)hipFree(s->d_type);
    delete s;
}

extern "C" int yarn_scene_build_threads(int32_t n)
{
    if (n < 0 || n > 256) return fail(BYSDF_ERR_INVALID_ARG, "build threads must be in 0..256");
    build_threads_setting().store(n);
    return 0;
}

extern "C" int yarn_scene_create(const float* ctrl, const int64_t* off, int32_t n_yarns,
                                 const int32_t* yarn_type, const float* yarn_phase, yarn_scene_t** out,
                                 hipStream_t stream)
{
    if (!out) return fail(BYSDF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    HostScene hs;
    std::string err;
    int rc;
    try {
        rc = yarn_scene_build_host(ctrl, off, n_yarns, yarn_type, yarn_phase, &hs, &err);
    } catch (const std::bad_alloc&) {
        return fail(BYSDF_ERR_OOM, "host memory exhausted while building the scene");
    }
    if (rc) return fail(rc, "%s", err.c_str());
    int dev = 0;
    rc = check_gfx950(&dev);
    if (rc) return rc;
    int64_t n_cp = (int64_t)hs.cp.size(), n_spans = (int64_t)hs.span.size();
    std::vector<SpanRec>& rec_o = hs.span;
    std::vector<float4>& frame_o = hs.frame;
    std::vector<float4>& cp = hs.cp;
    std::vector<float>& phase = hs.phase;
    std::vector<int>& type = hs.type;
    struct {
        std::vector<WNode>& nodes;
        int max_depth;
    } B{hs.node, hs.depth};
    yarn_scene* s = new yarn_scene();
    s->device = dev;
    s->n_yarns = n_yarns;
    s->n_cp = n_cp;
    s->n_spans = n_spans;
    s->n_nodes = (int64_t)B.nodes.size();
    s->depth = B.max_depth;
    for (int y = 0; y < n_yarns; ++y) s->max_type = std::max(s->max_type, type[y]);
    auto up = [&](void** dst, const void* src, size_t bytes) -> int {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return fail(BYSDF_ERR_OOM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        s->bytes += bytes;
        e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return fail(BYSDF_ERR_LAUNCH, "upload: %s", hipGetErrorString(e));
        return 0;
    };
    if ((rc = up((void**)&s->d_cp, cp.data(), sizeof(float4) * n_cp)) ||
        (rc = up((void**)&s->d_span, rec_o.data(), sizeof(SpanRec) * n_spans)) ||
        (rc = up((void**)&s->d_frame, frame_o.data(), sizeof(float4) * n_spans)) ||
        (rc = up((void**)&s->d_node, B.nodes.data(), sizeof(WNode) * B.nodes.size())) ||
        (rc = up((void**)&s->d_phase, phase.data(), sizeof(float) * n_yarns)) ||
        (rc = up((void**)&s->d_type, type.data(), sizeof(int) * n_yarns))) {
        (void)hipStreamSynchronize(stream);
        free_scene(s);
        return rc;
    }
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        free_scene(s);
        return fail(BYSDF_ERR_LAUNCH, "scene upload: %s", hipGetErrorString(e));
    }
    *out = s;
    return 0;
}

extern "C" int yarn_scene_destroy(yarn_scene_t* s)
{
    free_scene(s);
    return 0;
}

extern "C" int yarn_scene_info(const yarn_scene_t* s, int64_t* info)
{
    if (!s || !info) return fail(BYSDF_ERR_INVALID_ARG, "scene and info must be non-NULL");
    info[0] = s->n_yarns;
    info[1] = s->n_cp;
    info[2] = s->n_spans;
    info[3] = s->n_nodes;
    info[4] = s->depth;
    info[5] = (int64_t)s->bytes;
    return 0;
}

// scene view for the renderer (same library)
__attribute__((visibility("hidden"))) SceneView yarn_scene_view(const yarn_scene_t* s) { return s->view(); }
__attribute__((visibility("hidden"))) int yarn_scene_max_type(const yarn_scene_t* s) { return s->max_type; }

extern "C" int yarn_tube_intersect(const yarn_scene_t* s, const yarn_ray_soa* rays, int64_t n, float t_min,
                                   const yarn_hit_soa* hits, hipStream_t stream)
{
    if (!s || !rays || !hits) return fail(BYSDF_ERR_INVALID_ARG, "scene, rays and hits must be non-NULL");
    if (n < 0) return fail(BYSDF_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return 0;
    const void* in[] = {rays->o_x, rays->o_y, rays->o_z, rays->d_x, rays->d_y, rays->d_z, rays->t_max};
    for (const void* p : in)
        if (!p || ((uintptr_t)p & 3u)) return fail(BYSDF_ERR_INVALID_ARG, "ray arrays must be non-NULL and 4-byte aligned");
    const void* o[] = {hits->t, hits->yarn, hits->seg, hits->s, hits->h, hits->u, hits->v, hits->tan_x,
                       hits->tan_y, hits->tan_z, hits->nrm_x, hits->nrm_y, hits->nrm_z, hits->flags};
    for (const void* p : o)
        if (!p || ((uintptr_t)p & 3u)) return fail(BYSDF_ERR_INVALID_ARG, "hit arrays must be non-NULL and 4-byte aligned");
    if (!std::isfinite(t_min)) return fail(BYSDF_ERR_INVALID_ARG, "t_min must be finite");
    int64_t blocks = (n + kIsectBlock - 1) / kIsectBlock;
    if (blocks > 65536 * 8) blocks = 65536 * 8;
    hipLaunchKernelGGL(k_intersect, dim3((unsigned)blocks), dim3(kIsectBlock),
                       sizeof(int) * stack_entries(s->depth) * kIsectBlock, stream, s->view(), *rays, n,
                       (double)t_min, *hits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BYSDF_ERR_LAUNCH, "k_intersect: %s", hipGetErrorString(e));
    return 0;
}
