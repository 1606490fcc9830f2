// Host-side interfaces between the translation units of the HIP library.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "irgs_device.hpp"

namespace irgs {

struct BuildArgs {
    int n;
    const float* mu;
    const float* quat;
    const float* scale;
    const float* opac;
    float alpha_min;
    float sigma;
    uint32_t* order;        // leaf position -> surfel id
    uint64_t* sorted_keys;  // optional copy of the sorted Morton codes
    SurfelRec* rec;
    float* leafbox;         // 6 floats per leaf position
    BvhNode* nodes;
    int* leaf_parent;
    uint32_t* counters;     // unused by the level refit (kept for the buffer layout)
    int* level_nodes;       // internal node ids grouped by depth
    std::vector<int>* levels;  // host: level offsets into level_nodes (depth + 2 entries)
    int* depth;             // device int: max number of internal ancestors of a leaf
    int2* brange;           // per binary node: first leaf, leaf count
    WideNode* wnodes;       // up to max(N - 1, 1) wide nodes
    int4* wsrc;             // per wide node and slot: (binary parent << 1 | side), -1 = empty
    int* wscratch;          // 2 * max(N - 1, 1) + 4 ints: frontiers and counters
    int leaf_size;          // surfels per cluster leaf (1..16)
    bool ploc;              // binary tree by PLOC (else the Morton radix tree)
    int n_wide;             // out (host): wide nodes built; also the refit input
    int wide_depth;         // out (host): levels of the wide tree
};

hipError_t lbvh_sort_scratch_bytes(int n, size_t* bytes);
// Build: synchronises `st` (the wide collapse reads each level's size back).
hipError_t lbvh_build(BuildArgs& a, void* scratch, hipStream_t st);
hipError_t lbvh_refit(const BuildArgs& a, hipStream_t st);

struct OutPtrs {
    float* O;
    float* feat;
    float* D;
    float* T;
    int32_t* n_hits;
    int32_t* hit_ids;
    float* hit_T;
    int32_t H_cap;
    int32_t* counters;  // optional R x 4 work counters
};

struct GradIn {
    const float* gO;
    const float* gF;
    const float* gD;
};

struct GradOut {
    float* mu;
    float* quat;
    float* scale;
    float* opac;
    float* feat;
};

struct RawSurfels {
    const float* mu;
    const float* quat;
    const float* scale;
    const float* opac;
    const float* feat;
    // The backward's copy of the same parameters, one row of `ps` floats per
    // surfel id: (mu, o), q, (s_u, s_v, -, -), then the F features.  A hit
    // then reads one 128-byte line (F <= 20) instead of five scattered ones.
    const float* pk;
    int ps;
};

// Floats per packed row: 12 + F rounded up to a multiple of 32.
inline int pack_stride(int F) { return ((12 + F + 31) / 32) * 32; }
// Fill pk (n rows of pack_stride(F) floats) from the raw arrays.
hipError_t pack_surfels(const RawSurfels& raw, int64_t n, int F, float* pk, hipStream_t st);

// Largest k-buffer / feature count the kernels are instantiated for.
constexpr int kMaxK = 64;
constexpr int kMaxF = 64;

// Upper bound on the persistent trace threads of a launch over R rays;
// scratch is sized per thread of this bound.
int64_t trace_threads(int64_t R);

// Blocks of `kern` (block_size threads each) that the whole device keeps
// resident at once, or 0 if the runtime cannot say.  Persistent launches use
// at most this many, so no block waits for another to finish.
template <class Kern>
int64_t resident_blocks(Kern kern, int block_size)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block_size, 0) != hipSuccess) return 0;
    return per_cu > 0 && cus > 0 ? static_cast<int64_t>(per_cu) * cus : 0;
}

inline unsigned persistent_grid(int64_t max_blocks, int64_t resident)
{
    return static_cast<unsigned>(resident > 0 && resident < max_blocks ? resident : max_blocks);
}

// Device scratch of a persistent forward launch, sized for trace_threads(R)
// threads (the launch may use fewer).
constexpr int kDeferCap = 192;
// Deferred-list entries a lane stages in LDS before writing them as one
// group (kDeferCap and every fitted list size are multiples of it).
constexpr int kDeferStage = 8;
// Smallest deferred-list half a launch into a fixed scratch area takes
// before it gives up resident blocks instead.
constexpr int kDeferCapMin = 32;
struct FlatScratch {
    int* ovf;                      // stack overflow: ovf_slots ints per thread, or null when ovf_slots == 0
    int ovf_slots;
    int* dbuf;                     // deferred-work lists: 2 * defer_cap ints per thread (BVH launches)
    unsigned long long* next_ray;  // ray-claim counter (BVH launches); the launch zeroes it
    const uint32_t* order;         // optional claim order (slot -> ray), BVH launches over one scene
    int defer_cap;                 // entries per half of a thread's deferred list
    // 0: ovf and dbuf are sized for trace_threads(R) threads at defer_cap.
    // Otherwise they share one area of this many ints (ovf first, dbuf
    // right after it, placed by the launch): the launch picks its grid and
    // the deferred-list size so that both fit (fewer resident blocks only
    // when even kDeferCapMin entries per half do not fit every one).
    size_t fixed_words;
};

// True when a launch into a fixed area of `words` ints can run at least one
// block (its threads' stack overflow and deferred-list halves of
// kDeferCapMin entries).
inline size_t fixed_scratch_block_words(int ovf_slots, int block)
{
    return static_cast<size_t>(block) * (ovf_slots + 2 * kDeferCapMin) + kDeferStage;  // + alignment of dbuf
}
inline bool fixed_scratch_fits(size_t words, int ovf_slots, int block)
{
    return words >= fixed_scratch_block_words(ovf_slots, block);
}

// Claim order of a forward trace: rays sorted by the Morton code of their
// origin in the scene's root box.  `buf` holds ray_sort_words(R) floats;
// *order points into it afterwards.  Needs R <= 2^31 - 1 and a built scene.
hipError_t ray_order_by_origin(const SceneView& sc, int64_t R, const float* ro, void* buf, const uint32_t** order,
                               hipStream_t st);

// Forward trace.  use_bvh = false tests every record (the plain tracer).
hipError_t launch_trace(const SceneView& sc, const TraceParams& P, int k, bool use_bvh, int64_t R,
                        const float* ro, const float* rd, const OutPtrs& out, const FlatScratch& fs,
                        hipStream_t st);

// Backward.  Store mode reads saved ids and T (rays with n_hits > H_cap are
// re-marched); recompute mode re-marches every ray.  `ck` is scratch of
// backward_scratch_words(R, N, F) floats: the re-march lanes' checkpoints and
// private hit lists, the interleaved per-surfel gradient accumulator, then a
// chunk-claim counter.
constexpr int kBwdCheckpoints = 16;
constexpr int kBwdClaimWords = 64;
// Re-march lanes keep each ray's first kRemarchList hits (id and
// transmittance) in a private list and walk it back to front; the re-march
// launch uses at most kRemarchThreads lanes, which sizes those lists.
constexpr int kRemarchList = 512;
constexpr int64_t kRemarchThreads = 131072;
inline int64_t remarch_threads(int64_t R)
{
    const int64_t t = trace_threads(R);
    return t < kRemarchThreads ? t : kRemarchThreads;
}
// floats of the re-march area: checkpoints (4 per entry), then ids and T
inline size_t remarch_words(int64_t R)
{
    return static_cast<size_t>(remarch_threads(R)) * (kBwdCheckpoints * 4 + 2 * kRemarchList);
}
inline int grad_stride(int F) { return ((10 + F + 31) / 32) * 32; }
size_t sort_pairs_count_bytes(int n);
hipError_t sort_pairs(int n, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint32_t* counts, int passes,
                      hipStream_t st);
// Ray order of the backward for gradients wider than its LDS table (rays
// sorted by where they land): two key and two value buffers plus the sort's
// tile counters, in words; none for launches too large for 32-bit indices.
inline size_t ray_sort_words(int64_t R)
{
    if (R <= 0 || R > 0x7fffffffLL) return 0;
    return (static_cast<size_t>(R) * (2 * sizeof(uint64_t) + 2 * sizeof(uint32_t)) +
            sort_pairs_count_bytes(static_cast<int>(R))) / sizeof(float) + 64;
}
inline size_t backward_scratch_words(int64_t R, int64_t N, int F)
{
    // the ray order is used only for gradients wider than the LDS table (the
    // backward sorts exactly when F > 8: keep the two conditions the same)
    // (then the list of rays to re-march, R ints, and alignment slack)
    return remarch_words(R) + static_cast<size_t>(N) * grad_stride(F) + kBwdClaimWords + static_cast<size_t>(R) +
           128 + (F > 8 ? ray_sort_words(R) : 0);
}
hipError_t launch_backward(const SceneView& sc, const RawSurfels& raw, const TraceParams& P, int k, int64_t R,
                           const float* ro, const float* rd, const OutPtrs& saved, bool use_saved,
                           const GradIn& gin, const GradOut& gout, int* ovf, int ovf_slots, float* ck,
                           hipStream_t st);

// Packed launch over work items of several scenes (serving).  Item i owns
// the slots [chunk_begin, chunk_begin + ray_count) of the concatenation of
// every item's rays.
struct WorkItem {
    int32_t scene;
    int32_t pad;
    int64_t ray_begin;
    int64_t ray_count;
    int64_t chunk_begin;
    const float* ro;
    const float* rd;
    OutPtrs out;
};

// counters: some item asks for work counters.
hipError_t launch_packed(const SceneView* scenes_dev, const WorkItem* items_dev, int n_items, int64_t n_rays,
                         const TraceParams& P, int k, const FlatScratch& fs, int grid_blocks, bool counters,
                         hipStream_t st);

// Monte Carlo rendering-equation consumer (shade.hip).
struct ShadeArgs {
    int64_t P;            // pixels
    int32_t N;            // samples per pixel
    int32_t E;            // cubemap face resolution
    const float* n;       // P x 3
    const float* wo;      // P x 3
    const float* albedo;  // P x 3
    const float* rough;   // P
    const float* wi;      // P x N x 3
    const float* O;       // P x N
    const float* Lind;    // P x N x 3
    const float* env;     // 6 x E x E x 3
    const float* wgt;     // P x N per-sample weights, or null: 2 pi / N each
};

struct ShadeGrads {
    float* albedo;  // P x 3, accumulated
    float* rough;   // P, accumulated
    float* env;     // 6 x E x E x 3, accumulated
    float* O;       // P x N, written
    float* Lind;    // P x N x 3, written
};

hipError_t launch_mc_rays(int64_t P, int St, int Sp, const float* x, const float* n, const float* u, float offset,
                          float* ro, float* rd, hipStream_t st);
hipError_t launch_mc_shade(const ShadeArgs& a, float* c, hipStream_t st);
hipError_t launch_mc_shade_backward(const ShadeArgs& a, const float* g_c, const ShadeGrads& g, hipStream_t st);

// Relighting variant (relight.hip).
struct RelightArgs {
    int64_t R;
    const float* O;      // R
    const float* Fo;     // R x 7: blended albedo (3), roughness, normal (3), all times O
    const float* rd;     // R x 3
    int32_t E, M, S;     // cube resolution, prefilter levels, table size
    const float* irr;    // 6 x E x E x 3
    const float* pref;   // M x 6 x E x E x 3
    const float* table;  // S x S x 2
};

hipError_t launch_env_prefilter(int E, const float* env, int M, float* irr, float* pref, hipStream_t st);
hipError_t launch_brdf_table(int S, float* table, hipStream_t st);
hipError_t launch_relight_lind(const RelightArgs& a, float* lind, hipStream_t st);

// Importance sampling of the sky by intensity (relight.hip).
struct EnvRayArgs {
    int64_t P;          // pixels
    int32_t N;          // samples per pixel
    int32_t E;          // cube resolution
    const float* x;     // P x 3 surface points
    const float* n;     // P x 3 unit normals
    const float* u;     // P x N x 3 uniforms in [0, 1)
    const float* cdf;   // 6 E^2 inclusive CDF of the texel weights
    float offset;       // origin offset along n
    float* ro;          // P N x 3
    float* rd;          // P N x 3
    float* wgt;         // P N estimator weights
};
hipError_t launch_env_cdf(int E, const float* env, float* cdf, hipStream_t st);
hipError_t launch_env_rays(const EnvRayArgs& a, hipStream_t st);

// Fill n 32-bit words with v (a kernel, so it can be captured in a graph).
hipError_t fill_u32(void* p, int64_t n, uint32_t v, hipStream_t st);

}  // namespace irgs
