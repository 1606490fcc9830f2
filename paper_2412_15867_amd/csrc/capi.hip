// C ABI of the 2D Gaussian ray tracer: argument checks, device buffers of a
// scene, per-call scratch, and dispatch to the kernels.  Declared in
// include/irgs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/irgs.h"
#include "irgs_internal.hpp"

using namespace irgs;

struct irgs_scene_s {
    int64_t n = 0;
    int32_t F = 0;
    irgs_surfels p{};
    bool built = false;
    float alpha_min = 0.0f;
    float sigma = 0.0f;
    int32_t max_depth = 0;
    SurfelRec* rec = nullptr;
    BvhNode* nodes = nullptr;
    int* leaf_parent = nullptr;
    uint32_t* order = nullptr;
    float* leafbox = nullptr;
    uint32_t* counters = nullptr;
    int* depth = nullptr;
    int2* brange = nullptr;
    WideNode* wnodes = nullptr;
    int4* wsrc = nullptr;
    int* wscratch = nullptr;
    int n_wide = 0;
    int wide_depth = 0;
    int leaf_size = kLeafDefault;
    bool ploc = true;
    std::vector<int> levels;  // level offsets of the refit (host)
};

namespace {

thread_local std::string g_err;

irgs_status fail(irgs_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
irgs_status fail(irgs_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

irgs_status hip_fail(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory) return fail(IRGS_E_OOM, "%s: out of device memory", what);
    return fail(IRGS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int64_t n_internal(int64_t n) { return n > 1 ? n - 1 : 1; }

template <typename T>
hipError_t dalloc(T** p, size_t count)
{
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count > 0 ? count : 1));
}

void free_scene_buffers(irgs_scene s)
{
    hipFree(s->rec);
    hipFree(s->nodes);
    hipFree(s->leaf_parent);
    hipFree(s->order);
    hipFree(s->leafbox);
    hipFree(s->counters);
    hipFree(s->depth);
    hipFree(s->brange);
    hipFree(s->wnodes);
    hipFree(s->wsrc);
    hipFree(s->wscratch);
    s->brange = nullptr;
    s->wnodes = nullptr;
    s->wsrc = nullptr;
    s->wscratch = nullptr;
    s->rec = nullptr;
    s->nodes = nullptr;
    s->leaf_parent = nullptr;
    s->order = nullptr;
    s->leafbox = nullptr;
    s->counters = nullptr;
    s->depth = nullptr;
    s->built = false;
}

// SH degree whose RGB coefficients make F features, or -1.
int sh_degree(int32_t F)
{
    for (int d = 0; d <= 3; ++d)
        if (F == 3 * (d + 1) * (d + 1)) return d;
    return -1;
}

irgs_status check_params(const irgs_params* p, int32_t F)
{
    if (!p) return fail(IRGS_E_INVALID, "params is NULL");
    const int k = p->k;
    if (!(k == 1 || k == 2 || k == 4 || k == 8 || k == 16 || k == 32 || k == 64))
        return fail(IRGS_E_INVALID, "k = %d: must be one of 1, 2, 4, 8, 16, 32, 64", k);
    if (p->feature_dim != F) return fail(IRGS_E_INVALID, "feature_dim %d != scene F %d", p->feature_dim, F);
    if (!(p->alpha_min >= 0.0f) || !(p->T_min >= 0.0f) || std::isnan(p->t_min) || std::isnan(p->t_max) ||
        !(p->support_sigma > 0.0f))
        return fail(IRGS_E_INVALID, "alpha_min, T_min >= 0, support_sigma > 0 and finite-or-inf t window required");
    if (p->flags & IRGS_FLAG_SH) {
        if (sh_degree(F) < 0)
            return fail(IRGS_E_INVALID, "IRGS_FLAG_SH needs 3 (deg + 1)^2 features, deg <= 3 (3, 12, 27, 48); F = %d", F);
        if (k != 16 && k != 32 && k != 64) return fail(IRGS_E_INVALID, "IRGS_FLAG_SH supports k = 16, 32 or 64");
    }
    if (p->flags & IRGS_FLAG_NORMAL) {
        if (p->flags & IRGS_FLAG_SH) return fail(IRGS_E_INVALID, "IRGS_FLAG_NORMAL and IRGS_FLAG_SH are exclusive");
        if (F > 5) return fail(IRGS_E_INVALID, "IRGS_FLAG_NORMAL supports F <= 5 (got %d)", F);
        if (k != 16 && k != 32 && k != 64) return fail(IRGS_E_INVALID, "IRGS_FLAG_NORMAL supports k = 16, 32 or 64");
    }
    return IRGS_OK;
}

BuildArgs build_args(irgs_scene s)
{
    BuildArgs a{};
    a.n = static_cast<int>(s->n);
    a.mu = s->p.mu;
    a.quat = s->p.quat;
    a.scale = s->p.scale;
    a.opac = s->p.opacity;
    a.alpha_min = s->alpha_min;
    a.sigma = s->sigma;
    a.order = s->order;
    a.sorted_keys = nullptr;
    a.rec = s->rec;
    a.leafbox = s->leafbox;
    a.nodes = s->nodes;
    a.leaf_parent = s->leaf_parent;
    a.counters = s->counters;
    a.level_nodes = reinterpret_cast<int*>(s->counters);
    a.levels = &s->levels;
    a.depth = s->depth;
    a.brange = s->brange;
    a.wnodes = s->wnodes;
    a.wsrc = s->wsrc;
    a.wscratch = s->wscratch;
    a.n_wide = s->n_wide;
    a.wide_depth = s->wide_depth;
    a.leaf_size = s->leaf_size;
    a.ploc = s->ploc;
    return a;
}

SceneView view_of(irgs_scene s)
{
    SceneView v{};
    v.rec = s->rec;
    v.wnodes = s->wnodes;
    v.feat = s->p.feat;
    v.n = static_cast<int32_t>(s->n);
    v.F = s->F;
    return v;
}

// Entries a traversal stack can hold at most: every wide level above the
// current node pushes at most 3 siblings.
int stack_need(irgs_scene s) { return 3 * s->wide_depth + 1; }

int ovf_slots_of(irgs_scene s)
{
    const int extra = stack_need(s) - kStackLds;
    return extra > 0 ? extra : 0;
}

// Forward scratch: the ray-claim counter heads the deferred-list buffer.
constexpr size_t kClaimBytes = 256;
// Backward without stored hit lists: list capacity of the retrace and the
// size its batches of lists (ids, T, O, D, n_hits, features) stay within.
constexpr int kRetraceCap = 256;
constexpr size_t kRetraceBytes = size_t(4) << 30;
FlatScratch flat_scratch(void* ovf, int slots, void* dq)
{
    FlatScratch f{};
    f.ovf = static_cast<int*>(ovf);
    f.ovf_slots = slots;
    f.next_ray = static_cast<unsigned long long*>(dq);
    f.dbuf = dq ? reinterpret_cast<int*>(static_cast<char*>(dq) + kClaimBytes) : nullptr;
    f.defer_cap = kDeferCap;
    f.fixed_words = 0;
    return f;
}

OutPtrs out_ptrs(const irgs_out* o)
{
    OutPtrs r{};
    r.O = o->opacity;
    r.feat = o->feat;
    r.D = o->depth;
    r.T = o->T;
    r.n_hits = o->n_hits;
    r.hit_ids = o->hit_ids;
    r.hit_T = o->hit_ids ? o->hit_T : nullptr;
    r.H_cap = o->hit_ids ? o->H_cap : 0;
    r.counters = o->counters;
    return r;
}

irgs_status check_trace_common(irgs_scene s, const irgs_params* p, int64_t R, const float* ro, const float* rd)
{
    if (!s) return fail(IRGS_E_INVALID, "scene is NULL");
    irgs_status st = check_params(p, s->F);
    if (st != IRGS_OK) return st;
    if (R < 0) return fail(IRGS_E_INVALID, "R = %lld < 0", static_cast<long long>(R));
    if (R > 0 && (!ro || !rd)) return fail(IRGS_E_INVALID, "ro/rd is NULL");
    if (!s->built) return fail(IRGS_E_STATE, "scene is not built");
    if (p->alpha_min != s->alpha_min || p->support_sigma != s->sigma)
        return fail(IRGS_E_STATE, "scene was built with alpha_min %g, support_sigma %g (got %g, %g)",
                    static_cast<double>(s->alpha_min), static_cast<double>(s->sigma),
                    static_cast<double>(p->alpha_min), static_cast<double>(p->support_sigma));
    if (s->n > 0 && !s->p.feat) return fail(IRGS_E_INVALID, "scene features are NULL");
    return IRGS_OK;
}

TraceParams trace_params(const irgs_params* p, int32_t F)
{
    TraceParams t{};
    t.t_min = p->t_min;
    t.t_max = p->t_max;
    t.T_min = p->T_min;
    t.F = F;
    t.sh_deg = (p->flags & IRGS_FLAG_SH) ? sh_degree(F) : -1;
    t.normals = (p->flags & IRGS_FLAG_NORMAL) ? 1 : 0;
    return t;
}

// Scratch of irgs_trace_noalloc: the ray-claim counter, then every
// thread's stack overflow and deferred lists.  One copy per device, held by
// the library's code object until the process ends; host code uses only the
// device address looked up per device (the array's name is a host-side
// stand-in that no kernel may be handed).
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

namespace {

// Device address of the no-alloc scratch on the current device, looked up
// once per device with that device current.
irgs_status noalloc_scratch_ptr(char** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(IRGS_E_INVALID, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "no-alloc scratch lookup");
        g_noalloc_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_noalloc_ptr[dev];
    return IRGS_OK;
}

struct AsyncBuf {
    void* p = nullptr;
    hipStream_t st = nullptr;
    ~AsyncBuf()
    {
        if (p) hipFreeAsync(p, st);
    }
    hipError_t alloc(size_t bytes, hipStream_t s)
    {
        st = s;
        if (bytes == 0) return hipSuccess;
        return hipMallocAsync(&p, bytes, s);
    }
};

}  // namespace

extern "C" {

const char* irgs_version(void) { return "irgs-gfx950 0.1"; }

irgs_status irgs_mc_rays(int64_t P, int32_t S_t, int32_t S_p, const float* x, const float* n, const float* u,
                         float offset, float* ro, float* rd, void* stream)
{
    if (P < 0 || S_t < 1 || S_p < 1) return fail(IRGS_E_INVALID, "P >= 0, S_t >= 1 and S_p >= 1 required");
    if (P > 0 && (!x || !n || !u || !ro || !rd)) return fail(IRGS_E_INVALID, "NULL pointer");
    if (!std::isfinite(offset)) return fail(IRGS_E_INVALID, "offset must be finite");
    const hipError_t e = launch_mc_rays(P, S_t, S_p, x, n, u, offset, ro, rd, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IRGS_OK : hip_fail(e, "mc rays launch");
}

static irgs_status check_shade(const irgs_shade_in* in, ShadeArgs* a)
{
    if (!in) return fail(IRGS_E_INVALID, "shade inputs are NULL");
    if (in->P < 0 || in->N < 1 || in->E < 1) return fail(IRGS_E_INVALID, "P >= 0, N >= 1 and E >= 1 required");
    if (in->P > 0 && (!in->n || !in->wo || !in->albedo || !in->rough || !in->wi || !in->O || !in->Lind || !in->env))
        return fail(IRGS_E_INVALID, "NULL shade input");
    *a = ShadeArgs{in->P, in->N, in->E, in->n, in->wo, in->albedo, in->rough, in->wi, in->O, in->Lind, in->env,
                   in->wgt};
    return IRGS_OK;
}

irgs_status irgs_mc_shade(const irgs_shade_in* in, float* c, void* stream)
{
    ShadeArgs a;
    const irgs_status st = check_shade(in, &a);
    if (st != IRGS_OK) return st;
    if (a.P > 0 && !c) return fail(IRGS_E_INVALID, "c is NULL");
    const hipError_t e = launch_mc_shade(a, c, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IRGS_OK : hip_fail(e, "shade launch");
}

irgs_status irgs_env_prefilter(int32_t E, const float* env, int32_t M, float* irr, float* pref, void* stream)
{
    if (E < 1 || E > 256 || M < 0 || M > 32) return fail(IRGS_E_INVALID, "1 <= E <= 256 and 0 <= M <= 32 required");
    if (!env || (!irr && !pref) || (M > 0 && !pref)) return fail(IRGS_E_INVALID, "NULL pointer");
    const hipError_t e = launch_env_prefilter(E, env, M, irr, pref, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IRGS_OK : hip_fail(e, "prefilter launch");
}

irgs_status irgs_brdf_table(int32_t S, float* table, void* stream)
{
    if (S < 1 || S > 1024 || !table) return fail(IRGS_E_INVALID, "1 <= S <= 1024 and a table are required");
    const hipError_t e = launch_brdf_table(S, table, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IRGS_OK : hip_fail(e, "table launch");
}

irgs_status irgs_relight_lind(int64_t R, const float* O, const float* Fo, const float* rd, int32_t E, const float* irr,
                              int32_t M, const float* pref, int32_t S, const float* table, float* lind, void* stream)
{
    if (R < 0 || E < 1 || M < 1 || S < 1) return fail(IRGS_E_INVALID, "R >= 0, E, M, S >= 1 required");
    if (R > 0 && (!O || !Fo || !rd || !irr || !pref || !table || !lind)) return fail(IRGS_E_INVALID, "NULL pointer");
    const RelightArgs a{R, O, Fo, rd, E, M, S, irr, pref, table};
    const hipError_t e = launch_relight_lind(a, lind, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IRGS_OK : hip_fail(e, "relight launch");
}

irgs_status irgs_env_cdf(int32_t E, const float* env, float* cdf, void* stream)
{
    if (E < 1 || E > 256) return fail(IRGS_E_INVALID, "1 <= E <= 256 required");
    if (!env || !cdf) return fail(IRGS_E_INVALID, "NULL pointer");
    const hipError_t e = launch_env_cdf(E, env, cdf, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IRGS_OK : hip_fail(e, "env cdf launch");
}

irgs_status irgs_env_rays(int64_t P, int32_t N, const float* x, const float* n, const float* u, int32_t E,
                          const float* cdf, float offset, float* ro, float* rd, float* wgt, void* stream)
{
    if (P < 0 || N < 1 || E < 1 || E > 256) return fail(IRGS_E_INVALID, "P >= 0, N >= 1 and 1 <= E <= 256 required");
    if (P > (int64_t(1) << 40) / N) return fail(IRGS_E_INVALID, "P N too large");
    if (P > 0 && (!x || !n || !u || !cdf || !ro || !rd || !wgt)) return fail(IRGS_E_INVALID, "NULL pointer");
    if (!std::isfinite(offset)) return fail(IRGS_E_INVALID, "offset must be finite");
    const EnvRayArgs a{P, N, E, x, n, u, cdf, offset, ro, rd, wgt};
    const hipError_t e = launch_env_rays(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IRGS_OK : hip_fail(e, "env rays launch");
}

irgs_status irgs_mc_shade_backward(const irgs_shade_in* in, const float* g_c, irgs_shade_grads* grads,
                                   void* stream)
{
    ShadeArgs a;
    const irgs_status st = check_shade(in, &a);
    if (st != IRGS_OK) return st;
    if (!grads) return fail(IRGS_E_INVALID, "grads is NULL");
    if (a.P > 0 && !g_c) return fail(IRGS_E_INVALID, "g_c is NULL");
    const ShadeGrads g{grads->albedo, grads->rough, grads->env, grads->O, grads->Lind};
    const hipError_t e = launch_mc_shade_backward(a, g_c, g, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? IRGS_OK : hip_fail(e, "shade backward launch");
}

const char* irgs_last_error(void) { return g_err.c_str(); }

const char* irgs_status_str(irgs_status s)
{
    switch (s) {
        case IRGS_OK: return "ok";
        case IRGS_E_INVALID: return "invalid argument";
        case IRGS_E_OOM: return "out of device memory";
        case IRGS_E_HIP: return "HIP error";
        case IRGS_E_STATE: return "invalid scene state";
        case IRGS_E_BUSY: return "busy";
    }
    return "unknown status";
}

size_t irgs_scene_bytes(int64_t n, int32_t F)
{
    (void)F;
    if (n < 0) return 0;
    size_t sort = 0;
    lbvh_sort_scratch_bytes(static_cast<int>(n), &sort);
    const size_t ni = static_cast<size_t>(n_internal(n));
    return static_cast<size_t>(n) * (sizeof(SurfelRec) + sizeof(int) + sizeof(uint32_t) + 6 * sizeof(float)) +
           ni * (sizeof(BvhNode) + sizeof(uint32_t) + sizeof(int2) + sizeof(WideNode) + sizeof(int4) +
                 3 * sizeof(int)) +
           sizeof(int) * 5 + sort;
}

size_t irgs_trace_bytes(int64_t R, int32_t F, uint32_t flags)
{
    if (R <= 0) return 0;
    const size_t thr = static_cast<size_t>(trace_threads(R));
    size_t b = thr * (64 + 2 * kDeferCap) * sizeof(int) + kClaimBytes;  // stack overflow, deferred lists
    if (flags & IRGS_FLAG_SORT_RAYS) b += ray_sort_words(R) * sizeof(float);
    if (flags & IRGS_FLAG_RECOMPUTE) {  // the backward's retrace: one batch of lists, its checkpoints
        const int fo = (flags & IRGS_FLAG_SH) ? 3 : F;
        const size_t per_ray = static_cast<size_t>(kRetraceCap) * 8 + (3 + fo) * sizeof(float);
        const int64_t bmax = std::max<int64_t>(1, static_cast<int64_t>(kRetraceBytes / per_ray));
        const int64_t nb = (R + bmax - 1) / bmax;
        b += static_cast<size_t>((R + nb - 1) / nb) * per_ray + remarch_words(R) * sizeof(float);
    }
    return b;  // plus, for a backward, 4 * (ceil32(10 + F) + ceil32(12 + F)) bytes per surfel
}

irgs_status irgs_scene_create(int64_t n, int32_t F, const irgs_surfels* params, irgs_scene* out)
{
    if (!out) return fail(IRGS_E_INVALID, "out is NULL");
    *out = nullptr;
    // leaf references pack a position in 27 bits (cluster_ref: first << 4)
    if (n < 0 || n > (int64_t(1) << 27)) return fail(IRGS_E_INVALID, "n = %lld out of range [0, 2^27]", (long long)n);
    if (F < 1 || F > kMaxF) return fail(IRGS_E_INVALID, "F = %d out of range [1, %d]", F, kMaxF);
    if (!params) return fail(IRGS_E_INVALID, "params is NULL");
    if (n > 0 && (!params->mu || !params->quat || !params->scale || !params->opacity || !params->feat))
        return fail(IRGS_E_INVALID, "a surfel parameter pointer is NULL");
    irgs_scene s = new (std::nothrow) irgs_scene_s();
    if (!s) return fail(IRGS_E_OOM, "host allocation failed");
    s->n = n;
    s->F = F;
    s->p = *params;
    *out = s;
    return IRGS_OK;
}

irgs_status irgs_scene_set_params(irgs_scene s, const irgs_surfels* params)
{
    if (!s || !params) return fail(IRGS_E_INVALID, "scene or params is NULL");
    if (s->n > 0 && (!params->mu || !params->quat || !params->scale || !params->opacity || !params->feat))
        return fail(IRGS_E_INVALID, "a surfel parameter pointer is NULL");
    s->p = *params;
    return IRGS_OK;
}

irgs_status irgs_scene_build(irgs_scene s, const irgs_params* p, void* stream)
{
    if (!s) return fail(IRGS_E_INVALID, "scene is NULL");
    if (!p) return fail(IRGS_E_INVALID, "params is NULL");
    if (!(p->alpha_min >= 0.0f) || !(p->support_sigma > 0.0f))
        return fail(IRGS_E_INVALID, "alpha_min >= 0 and support_sigma > 0 required");
    if (p->leaf_size < 0 || p->leaf_size > 16) return fail(IRGS_E_INVALID, "leaf_size %d out of [0, 16]", p->leaf_size);
    s->leaf_size = p->leaf_size == 0 ? kLeafDefault : p->leaf_size;
    s->ploc = (p->flags & IRGS_FLAG_RADIX_TREE) == 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = s->n;
    hipError_t e = hipSuccess;
    if (!s->rec) {
        if ((e = dalloc(&s->rec, n)) != hipSuccess || (e = dalloc(&s->nodes, n_internal(n))) != hipSuccess ||
            (e = dalloc(&s->leaf_parent, n)) != hipSuccess || (e = dalloc(&s->order, n)) != hipSuccess ||
            (e = dalloc(&s->leafbox, 6 * n)) != hipSuccess || (e = dalloc(&s->counters, n_internal(n))) != hipSuccess ||
            (e = dalloc(&s->depth, 1)) != hipSuccess || (e = dalloc(&s->brange, n_internal(n))) != hipSuccess ||
            (e = dalloc(&s->wnodes, n_internal(n))) != hipSuccess ||
            (e = dalloc(&s->wsrc, n_internal(n))) != hipSuccess ||
            (e = dalloc(&s->wscratch, 3 * n_internal(n) + 4)) != hipSuccess) {
            free_scene_buffers(s);
            return hip_fail(e, "scene allocation");
        }
    }
    s->alpha_min = p->alpha_min;
    s->sigma = p->support_sigma;
    s->built = false;
    if (n == 0) {
        s->max_depth = 0;
        s->built = true;
        return IRGS_OK;
    }
    size_t sort_bytes = 0;
    lbvh_sort_scratch_bytes(static_cast<int>(n), &sort_bytes);
    void* scratch = nullptr;
    if ((e = hipMalloc(&scratch, sort_bytes)) != hipSuccess) return hip_fail(e, "build scratch");
    BuildArgs ba = build_args(s);
    e = lbvh_build(ba, scratch, st);
    s->n_wide = ba.n_wide;
    s->wide_depth = ba.wide_depth;
    int depth = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&depth, s->depth, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(scratch);
    if (e != hipSuccess) return hip_fail(e, "build");
    s->max_depth = depth;
    s->built = true;
    return IRGS_OK;
}

irgs_status irgs_scene_refit(irgs_scene s, void* stream)
{
    if (!s) return fail(IRGS_E_INVALID, "scene is NULL");
    if (!s->built) return fail(IRGS_E_STATE, "scene is not built");
    hipError_t e = lbvh_refit(build_args(s), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "refit");
    return IRGS_OK;
}

irgs_status irgs_trace(irgs_scene s, const irgs_params* p, int64_t R, const float* ro, const float* rd,
                       const irgs_out* out, void* stream)
{
    irgs_status st = check_trace_common(s, p, R, ro, rd);
    if (st != IRGS_OK) return st;
    if (!out) return fail(IRGS_E_INVALID, "out is NULL");
    if (R > 0 && (!out->opacity || !out->feat || !out->depth))
        return fail(IRGS_E_INVALID, "out->opacity, feat and depth are required");
    if (out->hit_ids && out->H_cap < 0) return fail(IRGS_E_INVALID, "H_cap < 0");
    if (R == 0) return IRGS_OK;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const bool bvh = !(p->flags & IRGS_FLAG_BRUTE_FORCE);
    const int slots = bvh ? ovf_slots_of(s) : 0;
    const bool sorted = bvh && (p->flags & IRGS_FLAG_SORT_RAYS) && ray_sort_words(R) > 0;
    AsyncBuf ovf, dq, srt;
    const size_t thr = static_cast<size_t>(trace_threads(R));
    hipError_t e = ovf.alloc(thr * slots * sizeof(int), hs);
    if (e == hipSuccess && bvh) e = dq.alloc(kClaimBytes + thr * 2 * kDeferCap * sizeof(int), hs);
    if (e == hipSuccess && sorted) e = srt.alloc(ray_sort_words(R) * sizeof(float), hs);
    if (e != hipSuccess) return hip_fail(e, "trace scratch");
    const SceneView sv = view_of(s);
    FlatScratch fs = flat_scratch(ovf.p, slots, dq.p);
    if (sorted) {
        e = ray_order_by_origin(sv, R, ro, srt.p, &fs.order, hs);
        if (e != hipSuccess) return hip_fail(e, "ray order");
    }
    e = launch_trace(sv, trace_params(p, s->F), p->k, bvh, R, ro, rd, out_ptrs(out), fs, hs);
    if (e != hipSuccess) return hip_fail(e, "trace launch");
    return IRGS_OK;
}

irgs_status irgs_trace_noalloc(irgs_scene s, const irgs_params* p, int64_t R, const float* ro, const float* rd,
                               const irgs_out* out, void* stream)
{
    irgs_status st = check_trace_common(s, p, R, ro, rd);
    if (st != IRGS_OK) return st;
    if (!out) return fail(IRGS_E_INVALID, "out is NULL");
    if (R > 0 && (!out->opacity || !out->feat || !out->depth))
        return fail(IRGS_E_INVALID, "out->opacity, feat and depth are required");
    if (out->hit_ids && out->H_cap < 0) return fail(IRGS_E_INVALID, "H_cap < 0");
    if (p->flags & IRGS_FLAG_SORT_RAYS)
        return fail(IRGS_E_INVALID, "IRGS_FLAG_SORT_RAYS needs a per-ray workspace: use irgs_trace");
    const bool bvh = !(p->flags & IRGS_FLAG_BRUTE_FORCE);
    const int slots = bvh ? ovf_slots_of(s) : 0;
    const size_t words = (kNoAllocBytes - kClaimBytes) / sizeof(int);
    if (bvh && !fixed_scratch_fits(words, slots, kBlock))
        return fail(IRGS_E_INVALID, "scene tree too deep for the %zu-byte no-alloc scratch (%d overflow slots per thread)",
                    kNoAllocBytes, slots);
    if (R == 0) return IRGS_OK;
    char* base = nullptr;
    st = noalloc_scratch_ptr(&base);
    if (st != IRGS_OK) return st;
    FlatScratch fs = flat_scratch(base + kClaimBytes, slots, base);
    fs.dbuf = nullptr;  // placed by the launch after every thread's overflow slots
    fs.fixed_words = words;
    const hipError_t e = launch_trace(view_of(s), trace_params(p, s->F), p->k, bvh, R, ro, rd, out_ptrs(out), fs,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "trace launch");
    return IRGS_OK;
}

irgs_status irgs_trace_backward(irgs_scene s, const irgs_params* p, int64_t R, const float* ro, const float* rd,
                                const irgs_out* saved, const irgs_grad_in* gin, irgs_grads* grads, void* stream)
{
    irgs_status st = check_trace_common(s, p, R, ro, rd);
    if (st != IRGS_OK) return st;
    if (!saved || !gin || !grads) return fail(IRGS_E_INVALID, "saved, grad_in and grads are required");
    if (R > 0 && !saved->n_hits) return fail(IRGS_E_INVALID, "saved->n_hits is required");
    if (R == 0 || s->n == 0) return IRGS_OK;
    const bool use_saved = !(p->flags & IRGS_FLAG_RECOMPUTE) && saved->hit_ids && saved->hit_T && saved->H_cap > 0;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const TraceParams tp = trace_params(p, s->F);
    RawSurfels raw{s->p.mu, s->p.quat, s->p.scale, s->p.opacity, s->p.feat, nullptr, pack_stride(s->F)};
    GradIn g{gin->g_opacity, gin->g_feat, gin->g_depth};
    GradOut go{grads->mu, grads->quat, grads->scale, grads->opacity, grads->feat};
    const int slots = stack_need(s);  // the backward keeps its whole re-march stack in global memory
    // the parameters packed one row per surfel, read by every hit's gradient
    AsyncBuf pk;
    hipError_t pe = pk.alloc(static_cast<size_t>(s->n) * raw.ps * sizeof(float), hs);
    if (pe == hipSuccess) pe = pack_surfels(raw, s->n, s->F, static_cast<float*>(pk.p), hs);
    if (pe != hipSuccess) return hip_fail(pe, "backward parameter pack");
    raw.pk = static_cast<const float*>(pk.p);
    if (use_saved) {
        const size_t thr = static_cast<size_t>(trace_threads(R));
        AsyncBuf ovf, ck;
        hipError_t e = ovf.alloc(thr * slots * sizeof(int), hs);
        if (e == hipSuccess) e = ck.alloc(backward_scratch_words(R, s->n, s->F) * sizeof(float), hs);
        if (e != hipSuccess) return hip_fail(e, "backward scratch");
        e = launch_backward(view_of(s), raw, tp, p->k, R, ro, rd, out_ptrs(saved), true, g, go,
                            static_cast<int*>(ovf.p), slots, static_cast<float*>(ck.p), hs);
        if (e != hipSuccess) return hip_fail(e, "backward launch");
        return IRGS_OK;
    }
    // Without stored lists the rays are traced again, a batch at a time, into
    // a transient list workspace, and the batch then takes the stored-list
    // walk (the retrace composites exactly as the forward did, so its lists
    // and T are the forward's); rays with more than kRetraceCap hits
    // re-march.  The accumulated gradients add into `grads` per batch.
    const int fo = tp.sh_deg >= 0 ? 3 : (tp.normals ? s->F + 3 : s->F);  // composited (and upstream) channels
    const size_t per_ray = static_cast<size_t>(kRetraceCap) * 8 + (3 + fo) * sizeof(float);
    const int64_t bmax = std::max<int64_t>(1, static_cast<int64_t>(kRetraceBytes / per_ray));
    const int64_t nbatch = (R + bmax - 1) / bmax;
    const int64_t B = (R + nbatch - 1) / nbatch;  // equal batches: no short last launch
    const bool bvh = !(p->flags & IRGS_FLAG_BRUTE_FORCE);
    const size_t thr = static_cast<size_t>(trace_threads(B));
    const bool sorted = bvh && (p->flags & IRGS_FLAG_SORT_RAYS) && ray_sort_words(B) > 0;
    AsyncBuf ovf, dq, ck, lists, srt;
    hipError_t e = ovf.alloc(thr * slots * sizeof(int), hs);
    if (e == hipSuccess && bvh) e = dq.alloc(kClaimBytes + thr * 2 * kDeferCap * sizeof(int), hs);
    if (e == hipSuccess && sorted) e = srt.alloc(ray_sort_words(B) * sizeof(float), hs);
    if (e == hipSuccess) e = ck.alloc(backward_scratch_words(B, s->n, s->F) * sizeof(float), hs);
    if (e == hipSuccess) e = lists.alloc(static_cast<size_t>(B) * per_ray, hs);
    if (e != hipSuccess) return hip_fail(e, "backward scratch");
    OutPtrs tmp{};
    tmp.hit_ids = static_cast<int32_t*>(lists.p);
    tmp.hit_T = reinterpret_cast<float*>(tmp.hit_ids + static_cast<size_t>(B) * kRetraceCap);
    tmp.O = tmp.hit_T + static_cast<size_t>(B) * kRetraceCap;
    tmp.D = tmp.O + B;
    tmp.n_hits = reinterpret_cast<int32_t*>(tmp.D + B);
    tmp.feat = reinterpret_cast<float*>(tmp.n_hits + B);
    tmp.H_cap = kRetraceCap;
    const SceneView sv = view_of(s);
    FlatScratch fs = flat_scratch(ovf.p, bvh ? ovf_slots_of(s) : 0, dq.p);
    for (int64_t b0 = 0; b0 < R; b0 += B) {
        const int64_t nb = std::min(B, R - b0);
        const float* bro = ro + 3 * b0;
        const float* brd = rd + 3 * b0;
        if (sorted) {
            e = ray_order_by_origin(sv, nb, bro, srt.p, &fs.order, hs);
            if (e != hipSuccess) return hip_fail(e, "ray order");
        }
        e = launch_trace(sv, tp, p->k, bvh, nb, bro, brd, tmp, fs, hs);
        if (e != hipSuccess) return hip_fail(e, "backward retrace");
        const GradIn gb{g.gO ? g.gO + b0 : nullptr, g.gF ? g.gF + b0 * fo : nullptr, g.gD ? g.gD + b0 : nullptr};
        e = launch_backward(sv, raw, tp, p->k, nb, bro, brd, tmp, true, gb, go, static_cast<int*>(ovf.p), slots,
                            static_cast<float*>(ck.p), hs);
        if (e != hipSuccess) return hip_fail(e, "backward launch");
    }
    return IRGS_OK;
}

irgs_status irgs_trace_packed(const irgs_scene* scenes, int32_t n_scenes, const irgs_params* p,
                              const irgs_work* items, int32_t n_items, void* stream)
{
    if (!scenes || n_scenes <= 0) return fail(IRGS_E_INVALID, "no scenes");
    if (!p) return fail(IRGS_E_INVALID, "params is NULL");
    if (n_items < 0 || (n_items > 0 && !items)) return fail(IRGS_E_INVALID, "bad items");
    if (p->k != 16 && p->k != 32) return fail(IRGS_E_INVALID, "packed launch supports k = 16 or 32");
    if (p->flags & (IRGS_FLAG_SH | IRGS_FLAG_NORMAL))
        return fail(IRGS_E_INVALID, "IRGS_FLAG_SH / IRGS_FLAG_NORMAL are not supported by the packed launch");
    int32_t Fmax = 0;
    int slots = 0;
    std::vector<SceneView> views(n_scenes);
    for (int i = 0; i < n_scenes; ++i) {
        irgs_scene s = scenes[i];
        if (!s) return fail(IRGS_E_INVALID, "scene %d is NULL", i);
        if (!s->built) return fail(IRGS_E_STATE, "scene %d is not built", i);
        if (p->alpha_min != s->alpha_min || p->support_sigma != s->sigma)
            return fail(IRGS_E_STATE, "scene %d was built with other alpha_min/support_sigma", i);
        if (s->n > 0 && !s->p.feat) return fail(IRGS_E_INVALID, "scene %d features are NULL", i);
        Fmax = s->F > Fmax ? s->F : Fmax;
        slots = ovf_slots_of(s) > slots ? ovf_slots_of(s) : slots;
        views[i] = view_of(s);
    }
    if (p->feature_dim < Fmax) return fail(IRGS_E_INVALID, "feature_dim %d < largest scene F %d", p->feature_dim, Fmax);
    std::vector<WorkItem> w(n_items);
    int64_t chunks = 0;
    bool counters = false;
    for (int i = 0; i < n_items; ++i) {
        const irgs_work& it = items[i];
        if (it.scene < 0 || it.scene >= n_scenes) return fail(IRGS_E_INVALID, "item %d: bad scene %d", i, it.scene);
        if (it.ray_begin < 0 || it.ray_count < 0) return fail(IRGS_E_INVALID, "item %d: negative range", i);
        if (it.ray_count > 0 && (!it.ro || !it.rd || !it.out.opacity || !it.out.feat || !it.out.depth))
            return fail(IRGS_E_INVALID, "item %d: NULL ray or output pointer", i);
        if (it.out.hit_ids && it.out.H_cap < 0) return fail(IRGS_E_INVALID, "item %d: H_cap < 0", i);
        w[i].scene = it.scene;
        w[i].ray_begin = it.ray_begin;
        w[i].ray_count = it.ray_count;
        w[i].chunk_begin = chunks;  // first slot of the item in the concatenation of all rays
        w[i].ro = it.ro;
        w[i].rd = it.rd;
        w[i].out = out_ptrs(&it.out);
        counters = counters || it.out.counters != nullptr;
        chunks += it.ray_count;
    }
    if (chunks == 0) return IRGS_OK;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int grid = static_cast<int>(trace_threads(chunks) / kBlock);
    const size_t thr = static_cast<size_t>(grid) * kBlock;
    const size_t vb = sizeof(SceneView) * n_scenes, wb = sizeof(WorkItem) * n_items;
    const size_t items_off = (vb + 63) / 64 * 64;
    AsyncBuf meta, ovf, dq;
    hipError_t e = meta.alloc(items_off + wb, hs);
    if (e == hipSuccess) e = ovf.alloc(thr * slots * sizeof(int), hs);
    if (e == hipSuccess) e = dq.alloc(kClaimBytes + thr * 2 * kDeferCap * sizeof(int), hs);
    if (e != hipSuccess) return hip_fail(e, "packed scratch");
    char* base = static_cast<char*>(meta.p);
    SceneView* dviews = reinterpret_cast<SceneView*>(base);
    WorkItem* ditems = reinterpret_cast<WorkItem*>(base + items_off);
    // Pageable host sources: the copies are staged before hipMemcpyAsync
    // returns, so the vectors may go out of scope afterwards.
    e = hipMemcpyAsync(dviews, views.data(), vb, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(ditems, w.data(), wb, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) {
        TraceParams tp = trace_params(p, Fmax);
        e = launch_packed(dviews, ditems, n_items, chunks, tp, p->k, flat_scratch(ovf.p, slots, dq.p), grid, counters,
                          hs);
    }
    if (e != hipSuccess) return hip_fail(e, "packed launch");
    return IRGS_OK;
}

irgs_status irgs_scene_info(irgs_scene s, int64_t* n_int, int32_t* max_depth)
{
    if (!s) return fail(IRGS_E_INVALID, "scene is NULL");
    if (!s->built) return fail(IRGS_E_STATE, "scene is not built");
    if (n_int) *n_int = s->n > 1 ? s->n - 1 : (s->n == 1 ? 1 : 0);
    if (max_depth) *max_depth = s->max_depth;
    return IRGS_OK;
}

irgs_status irgs_scene_export(irgs_scene s, int32_t* order, int32_t* nodes, int32_t* leaf_parent, void* stream)
{
    if (!s) return fail(IRGS_E_INVALID, "scene is NULL");
    if (!s->built) return fail(IRGS_E_STATE, "scene is not built");
    if (s->n == 0) return IRGS_OK;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (order) e = hipMemcpyAsync(order, s->order, sizeof(int32_t) * s->n, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess && nodes)
        e = hipMemcpyAsync(nodes, s->nodes, sizeof(BvhNode) * n_internal(s->n), hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess && leaf_parent)
        e = hipMemcpyAsync(leaf_parent, s->leaf_parent, sizeof(int32_t) * s->n, hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "export");
    return IRGS_OK;
}

irgs_status irgs_scene_destroy(irgs_scene s)
{
    if (!s) return IRGS_OK;
    free_scene_buffers(s);  // hipFree waits for work still using the buffers
    delete s;
    return IRGS_OK;
}

}  // extern "C"
