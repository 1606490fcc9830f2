// Forward 2D Gaussian ray tracing (Sec. 3.2, Eq. 2, 6-8) on gfx950.
//
// One lane traces one ray at a time: with the BVH, through the flat state
// machine of trace_flat.hpp (rays claimed per wave from a counter); the
// plain tracer strides a persistent grid over the rays.  Each k-buffer
// round collects the K nearest hits after the resume key (by BVH traversal,
// or by testing every record in the plain tracer), then composites them
// front to back in registers:
//     w = T alpha;  O += w;  F += w f;  D += w tau;  T *= (1 - alpha)
// and stops once T < T_min (the hit that crosses the cutoff is included).
// A round with fewer than K hits is the last one.
#include <hip/hip_runtime.h>

#include "irgs_internal.hpp"
#include "march.hpp"
#include "trace_flat.hpp"

namespace irgs {

int64_t trace_threads(int64_t R)
{
    constexpr int64_t kMaxBlocks = 256 * 8;  // 256 CUs x 8 resident blocks
    int64_t blocks = (R + kBlock - 1) / kBlock;
    if (blocks > kMaxBlocks) blocks = kMaxBlocks;
    if (blocks < 1) blocks = 1;
    return blocks * kBlock;
}

namespace {

template <int K, int FM, bool BVH, int CM>
__device__ __forceinline__ void trace_one(const SceneView& sc, const TraceParams& P, const Ray& ray, int64_t r,
                                          const OutPtrs& out, Stack& st)
{
    float T = 1.0f, O = 0.0f, D = 0.0f;
    float acc[FM];
#pragma unroll
    for (int c = 0; c < FM; ++c) acc[c] = 0.0f;
    int nh = 0;
    Counters ct;
    if (sc.n > 0 && ray_valid(ray)) {
        const SlabRay q = slab_ray(ray);
        uint64_t after = 0;  // resume key: hits strictly above it (0 = from the start)
        bool done = false;
        while (!done) {
            KBuf<K> kb;
            kb.clear();
            if (BVH)
                collect_bvh<K>(kb, sc, ray, q, P.t_min, P.t_max, after, st, ct);
            else
                collect_all<K>(kb, sc, ray, P.t_min, P.t_max, after, ct);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (j < kb.cnt && !done) {
                    const SurfelRec s = load_rec(sc.rec, kb.pos(j));
                    float tau, rho2;
                    plane_hit(s, ray, &tau, &rho2);
                    const float a = alpha_of(s, rho2);
                    const int id = __float_as_int(s.c.w);
                    const float w = T * a;
                    O += w;
                    D = fmaf(w, tau, D);
                    add_features<FM, CM>(sc, P, ray, id, s.b, w, acc);
                    if (out.hit_ids && nh < out.H_cap) {
                        out.hit_ids[r * out.H_cap + nh] = id;
                        if (out.hit_T) out.hit_T[r * out.H_cap + nh] = T;
                    }
                    T = T * (1.0f - a);
                    ++nh;
                    if (T < P.T_min) done = true;
                }
            }
            if (kb.cnt < K)
                done = true;
            else
                after = kb.last();
        }
    }
    out.O[r] = O;
    out.D[r] = D;
    const int FO = CM == kColSH ? 3 : (CM == kColNormal ? P.F + 3 : P.F);  // composited channels
#pragma unroll
    for (int c = 0; c < FM; ++c)
        if (c < FO) out.feat[r * FO + c] = acc[c];
    if (out.T) out.T[r] = T;
    if (out.n_hits) out.n_hits[r] = nh;
    if (out.counters)
        reinterpret_cast<int4*>(out.counters)[r] = make_int4(ct.nodes, ct.tests, ct.inserts, ct.rounds);
}

template <int K, int FM, bool BVH, int CM, bool CT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(K <= 16 && FM <= 8 ? 4 : 1))) void k_trace(SceneView sc, TraceParams P, int64_t R,
                                                  const float* __restrict__ ro, const float* __restrict__ rd,
                                                  OutPtrs out, FlatScratch fs)
{
    __shared__ int lds_stack[BVH ? kStackLds * kBlock : 1];
    __shared__ int lds_stage[BVH && K <= 16 ? kDeferRing * kBlock : 1];
    const int64_t gtid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t nthr = static_cast<int64_t>(gridDim.x) * kBlock;
    Stack st{as_lds(lds_stack), as_glb(fs.ovf_slots > 0 ? fs.ovf + gtid : nullptr), static_cast<int>(nthr),
             static_cast<int>(threadIdx.x), 0, kStackLds};
    if (BVH) {
        const PlainSource src{sc, out, ro, rd, R, fs.order};
        Deferred<(K <= 16)> dq{as_glb(fs.dbuf + gtid * 2 * fs.defer_cap), as_lds(lds_stage) + threadIdx.x, fs.defer_cap, 0, 0, 0, 0, 0};
        trace_flat<K, FM, CM, CT>(src, fs.next_ray, P, st, dq);
    } else {
        for (int64_t r = gtid; r < R; r += nthr) {
            const Ray ray = load_ray(ro, rd, r);
            trace_one<K, FM, false, CM>(sc, P, ray, r, out, st);
        }
    }
}

template <int K, int FM, bool BVH, int CM, bool CT>
hipError_t launch_kct(const SceneView& sc, const TraceParams& P, int64_t R, const float* ro, const float* rd,
                      const OutPtrs& out, const FlatScratch& fs, hipStream_t st)
{
    if (BVH) {
        const hipError_t e = fill_u32(fs.next_ray, 2, 0u, st);
        if (e != hipSuccess) return e;
    }
    unsigned grid = persistent_grid(trace_threads(R) / kBlock, resident_blocks(k_trace<K, FM, BVH, CM, CT>, kBlock));
    FlatScratch f = fs;
    if (BVH && fs.fixed_words > 0) {
        // One fixed area: the stack overflow of every thread, then the
        // deferred lists.  Keep every resident block while a half of at
        // least kDeferCapMin entries fits, else drop blocks.
        // (the lists start 32-byte aligned and hold whole staged groups)
        const size_t per_block_min = fixed_scratch_block_words(fs.ovf_slots, kBlock);
        if (fs.fixed_words < per_block_min) return hipErrorInvalidValue;
        const size_t fit_blocks = fs.fixed_words / per_block_min;
        if (grid > fit_blocks) grid = static_cast<unsigned>(fit_blocks);
        const size_t thr = static_cast<size_t>(grid) * kBlock;
        const size_t ovf_words = (thr * fs.ovf_slots + kDeferStage - 1) / kDeferStage * kDeferStage;
        size_t cap = (fs.fixed_words - ovf_words) / thr / 2;
        cap = cap / kDeferStage * kDeferStage;
        f.defer_cap = static_cast<int>(cap < static_cast<size_t>(kDeferCap) ? cap : kDeferCap);
        f.dbuf = f.ovf + ovf_words;
        if (fs.ovf_slots == 0) f.ovf = nullptr;
    }
    k_trace<K, FM, BVH, CM, CT><<<grid, kBlock, 0, st>>>(sc, P, R, ro, rd, out, f);
    return hipGetLastError();
}

// BVH launches that do not ask for work counters run an instance without
// them (their four registers free; the plain tracer keeps its own).
template <int K, int FM, bool BVH, int CM>
hipError_t launch_kf(const SceneView& sc, const TraceParams& P, int64_t R, const float* ro, const float* rd,
                     const OutPtrs& out, const FlatScratch& fs, hipStream_t st)
{
    if constexpr (BVH) {
        if (!out.counters) return launch_kct<K, FM, BVH, CM, false>(sc, P, R, ro, rd, out, fs, st);
    }
    return launch_kct<K, FM, BVH, CM, true>(sc, P, R, ro, rd, out, fs, st);
}

template <int K, bool BVH>
hipError_t launch_k(const SceneView& sc, const TraceParams& P, int64_t R, const float* ro, const float* rd,
                    const OutPtrs& out, const FlatScratch& fs, hipStream_t st)
{
    if constexpr (K == 16 || K == 32 || K == 64) {
        if (P.sh_deg >= 0) return launch_kf<K, 4, BVH, kColSH>(sc, P, R, ro, rd, out, fs, st);  // 3 colour channels
        if (P.normals) {
            if (P.F <= 5) return launch_kf<K, 8, BVH, kColNormal>(sc, P, R, ro, rd, out, fs, st);  // F + 3 channels
            return hipErrorInvalidValue;
        }
    }
    if (P.sh_deg >= 0 || P.normals) return hipErrorInvalidValue;
    if (P.F <= 4) return launch_kf<K, 4, BVH, kColPlain>(sc, P, R, ro, rd, out, fs, st);
    if (P.F <= 8) return launch_kf<K, 8, BVH, kColPlain>(sc, P, R, ro, rd, out, fs, st);
    if constexpr (K == 16 || K == 32) {
        if (P.F <= 16) return launch_kf<K, 16, BVH, kColPlain>(sc, P, R, ro, rd, out, fs, st);
        if (P.F <= 64) return launch_kf<K, 64, BVH, kColPlain>(sc, P, R, ro, rd, out, fs, st);
    }
    return hipErrorInvalidValue;
}

template <bool BVH>
hipError_t launch_b(const SceneView& sc, const TraceParams& P, int k, int64_t R, const float* ro, const float* rd,
                    const OutPtrs& out, const FlatScratch& fs, hipStream_t st)
{
    switch (k) {
        case 1: return launch_k<1, BVH>(sc, P, R, ro, rd, out, fs, st);
        case 2: return launch_k<2, BVH>(sc, P, R, ro, rd, out, fs, st);
        case 4: return launch_k<4, BVH>(sc, P, R, ro, rd, out, fs, st);
        case 8: return launch_k<8, BVH>(sc, P, R, ro, rd, out, fs, st);
        case 16: return launch_k<16, BVH>(sc, P, R, ro, rd, out, fs, st);
        case 32: return launch_k<32, BVH>(sc, P, R, ro, rd, out, fs, st);
        case 64: return launch_k<64, BVH>(sc, P, R, ro, rd, out, fs, st);
        default: return hipErrorInvalidValue;
    }
}

// Packed persistent launch: lanes claim slots of the concatenation of every
// work item's rays (an item is one request on one scene), so different
// requests and scenes share one launch.
template <int K, int FM, bool CT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(K == 32 && FM <= 8 ? 3 : 1))) void k_packed(const SceneView* __restrict__ scenes,
                                                   const WorkItem* __restrict__ items, int n_items,
                                                   int64_t n_rays, TraceParams P, FlatScratch fs)
{
    __shared__ int lds_stack[kStackLds * kBlock];
    __shared__ int lds_stage[K <= 16 ? kDeferRing * kBlock : 1];
    const int64_t gtid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t nthr = static_cast<int64_t>(gridDim.x) * kBlock;
    Stack st{as_lds(lds_stack), as_glb(fs.ovf_slots > 0 ? fs.ovf + gtid : nullptr), static_cast<int>(nthr),
             static_cast<int>(threadIdx.x), 0, kStackLds};
    const PackedSource src{scenes, items, n_items, n_rays};
    Deferred<(K <= 16)> dq{as_glb(fs.dbuf + gtid * 2 * fs.defer_cap), as_lds(lds_stage) + threadIdx.x, fs.defer_cap, 0, 0, 0, 0, 0};
    trace_flat<K, FM, kColPlain, CT>(src, fs.next_ray, P, st, dq);
}

template <int K, int FM, bool CT>
hipError_t launch_packed_kct(const SceneView* scenes, const WorkItem* items, int n_items, int64_t n_rays,
                             const TraceParams& P, const FlatScratch& fs, int grid_blocks, hipStream_t st)
{
    const hipError_t e = fill_u32(fs.next_ray, 2, 0u, st);
    if (e != hipSuccess) return e;
    const unsigned grid = persistent_grid(grid_blocks, resident_blocks(k_packed<K, FM, CT>, kBlock));
    k_packed<K, FM, CT><<<grid, kBlock, 0, st>>>(scenes, items, n_items, n_rays, P, fs);
    return hipGetLastError();
}

template <int K, int FM>
hipError_t launch_packed_kf(const SceneView* scenes, const WorkItem* items, int n_items, int64_t n_rays,
                            const TraceParams& P, const FlatScratch& fs, int grid_blocks, bool counters,
                            hipStream_t st)
{
    return counters ? launch_packed_kct<K, FM, true>(scenes, items, n_items, n_rays, P, fs, grid_blocks, st)
                    : launch_packed_kct<K, FM, false>(scenes, items, n_items, n_rays, P, fs, grid_blocks, st);
}

}  // namespace

hipError_t launch_packed(const SceneView* scenes_dev, const WorkItem* items_dev, int n_items, int64_t n_rays,
                         const TraceParams& P, int k, const FlatScratch& fs, int grid_blocks, bool counters,
                         hipStream_t st)
{
    if (n_rays <= 0 || n_items <= 0) return hipSuccess;
    const SceneView* sv = scenes_dev;
    const WorkItem* it = items_dev;
    if (k == 16 && P.F <= 8) return launch_packed_kf<16, 8>(sv, it, n_items, n_rays, P, fs, grid_blocks, counters, st);
    if (k == 16 && P.F <= 64) return launch_packed_kf<16, 64>(sv, it, n_items, n_rays, P, fs, grid_blocks, counters, st);
    if (k == 32 && P.F <= 8) return launch_packed_kf<32, 8>(sv, it, n_items, n_rays, P, fs, grid_blocks, counters, st);
    if (k == 32 && P.F <= 64) return launch_packed_kf<32, 64>(sv, it, n_items, n_rays, P, fs, grid_blocks, counters, st);
    return hipErrorInvalidValue;
}

namespace {

// Sort key of a ray for the forward's claim order: the Morton code of its
// origin in the root's box (origins outside it clamp to its faces).
__global__ void k_origin_keys(int64_t R, const float* __restrict__ ro, const WideNode* __restrict__ root,
                              uint64_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (r >= R) return;
    float lo[3], hi[3];
    root_box(root, lo, hi);
    const float x[3] = {ro[3 * r], ro[3 * r + 1], ro[3 * r + 2]};
    keys[r] = lo[0] <= hi[0] ? morton30(x, lo, hi) : 0u;  // NaN coordinates clamp to a face
    vals[r] = static_cast<uint32_t>(r);
}

}  // namespace

hipError_t ray_order_by_origin(const SceneView& sc, int64_t R, const float* ro, void* buf, const uint32_t** order,
                               hipStream_t st)
{
    *order = nullptr;
    if (R <= 1 || R > 0x7fffffffLL || sc.n <= 0) return hipSuccess;
    uint64_t* k0 = static_cast<uint64_t*>(buf);
    uint64_t* k1 = k0 + R;
    uint32_t* v0 = reinterpret_cast<uint32_t*>(k1 + R);
    uint32_t* v1 = v0 + R;
    uint32_t* counts = v1 + R;
    k_origin_keys<<<static_cast<unsigned>((R + 255) / 256), 256, 0, st>>>(R, ro, sc.wnodes, k0, v0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = sort_pairs(static_cast<int>(R), k0, v0, k1, v1, counts, 4, st);
    if (e == hipSuccess) *order = v0;
    return e;
}

hipError_t launch_trace(const SceneView& sc, const TraceParams& P, int k, bool use_bvh, int64_t R,
                        const float* ro, const float* rd, const OutPtrs& out, const FlatScratch& fs,
                        hipStream_t st)
{
    if (R <= 0) return hipSuccess;
    return use_bvh ? launch_b<true>(sc, P, k, R, ro, rd, out, fs, st) : launch_b<false>(sc, P, k, R, ro, rd, out, fs, st);
}

}  // namespace irgs
