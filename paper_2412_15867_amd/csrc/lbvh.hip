// Software LBVH over surfel bounding boxes (gfx950).
//
// The paper bounds each 2D Gaussian by an icosahedron proxy sized to enclose
// the region where its alpha reaches alpha_min (Eq. 5) and hands the 20N
// triangles to a hardware BVH builder, updated every training iteration
// (Sec. 3.2, implementation details: about 3 ms per update).  CDNA4 has no
// ray-tracing units, so the same role is played here by a linear BVH built in
// software:
//   1. per surfel: record (frame, scaled tangents, support) and the exact box
//      of its support ellipse  rho <= min(sigma, sqrt(2 ln(o / alpha_min)))
//      -- the radius of Eq. 5's proxy, capped at sigma;
//   2. scene bounds of the centres, 63-bit Morton codes (21 bits per axis);
//   3. stable LSD radix sort of (code, id) -- 8 passes of 8-bit digits,
//      per-tile histograms, one scan, stable wave-ballot ranking;
//   4. Karras' hierarchy (longest common prefix of adjacent codes, index
//      tie-break for equal codes);
//   5. node boxes level by level from the deepest (nodes grouped by depth
//      once per build; one launch per level, no atomics).
// Refit repeats 1 (in the existing leaf order) and 5 with the topology kept.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "irgs_device.hpp"
#include "irgs_internal.hpp"

namespace irgs {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per tile
constexpr int kRadixBins = 256;

__device__ __forceinline__ bool surfel_valid(float3 m, float4 q, float2 s, float o)
{
    const bool fin = isfinite(m.x) && isfinite(m.y) && isfinite(m.z) && isfinite(q.x) && isfinite(q.y) &&
                     isfinite(q.z) && isfinite(q.w) && isfinite(s.x) && isfinite(s.y) && isfinite(o);
    const float qq = q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w;
    return fin && qq > 0.0f && isfinite(qq) && s.x > 0.0f && s.y > 0.0f;
}

__device__ __forceinline__ float3 ld3(const float* p, int64_t i)
{
    return make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}
__device__ __forceinline__ float4 ld4(const float* p, int64_t i)
{
    return make_float4(p[4 * i], p[4 * i + 1], p[4 * i + 2], p[4 * i + 3]);
}
__device__ __forceinline__ float2 ld2(const float* p, int64_t i) { return make_float2(p[2 * i], p[2 * i + 1]); }

// ---------------------------------------------------------------- bounds
__global__ void k_bounds_partial(int n, const float* __restrict__ mu, const float* __restrict__ quat,
                                 const float* __restrict__ scale, const float* __restrict__ opac,
                                 float* __restrict__ partial)
{
    __shared__ float red[6][kSortThreads];
    float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float3 m = ld3(mu, i);
        if (!surfel_valid(m, ld4(quat, i), ld2(scale, i), opac[i])) continue;
        lo[0] = fminf(lo[0], m.x), lo[1] = fminf(lo[1], m.y), lo[2] = fminf(lo[2], m.z);
        hi[0] = fmaxf(hi[0], m.x), hi[1] = fmaxf(hi[1], m.y), hi[2] = fmaxf(hi[2], m.z);
    }
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = lo[k];
        red[k + 3][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int off = kSortThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            for (int k = 0; k < 3; ++k) {
                red[k][threadIdx.x] = fminf(red[k][threadIdx.x], red[k][threadIdx.x + off]);
                red[k + 3][threadIdx.x] = fmaxf(red[k + 3][threadIdx.x], red[k + 3][threadIdx.x + off]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_bounds_final(int nparts, const float* __restrict__ partial, float* __restrict__ bounds)
{
    if (threadIdx.x >= 6) return;
    const int k = threadIdx.x;
    float v = k < 3 ? 3.0e38f : -3.0e38f;
    for (int b = 0; b < nparts; ++b) v = k < 3 ? fminf(v, partial[b * 6 + k]) : fmaxf(v, partial[b * 6 + k]);
    bounds[k] = v;
}

// ---------------------------------------------------------------- morton
__device__ __forceinline__ uint64_t spread21(uint32_t x)
{
    uint64_t v = x & 0x1fffffu;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ uint32_t quantize21(float x, float lo, float hi)
{
    const float ext = hi - lo;
    if (!(ext > 0.0f)) return 0u;
    float f = (x - lo) / ext * 2097152.0f;
    f = fminf(fmaxf(f, 0.0f), 2097151.0f);
    return static_cast<uint32_t>(f);
}

__global__ void k_morton(int n, const float* __restrict__ mu, const float* __restrict__ quat,
                         const float* __restrict__ scale, const float* __restrict__ opac,
                         const float* __restrict__ bounds, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float3 m = ld3(mu, i);
    uint64_t key = ~0ull >> 1;  // invalid surfels sort last
    if (surfel_valid(m, ld4(quat, i), ld2(scale, i), opac[i])) {
        key = (spread21(quantize21(m.x, bounds[0], bounds[3])) << 2) |
              (spread21(quantize21(m.y, bounds[1], bounds[4])) << 1) |
              spread21(quantize21(m.z, bounds[2], bounds[5]));
    }
    keys[i] = key;
    vals[i] = static_cast<uint32_t>(i);
}

// ---------------------------------------------------------------- radix sort
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(int n, int shift, const uint64_t* __restrict__ keys,
                                                              uint32_t* __restrict__ counts, int ntiles)
{
    __shared__ uint32_t h[kRadixBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * kSortTile;
    for (int s = 0; s < kSortItems; ++s) {
        const int i = base + s * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xff], 1u);
    }
    __syncthreads();
    counts[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `len` counters in one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_exclusive(uint32_t* __restrict__ data, int len)
{
    __shared__ uint32_t part[1024];
    const int per = (len + 1023) / 1024;
    const int b = threadIdx.x * per;
    const int e = min(len, b + per);
    uint32_t s = 0;
    for (int i = b; i < e; ++i) s += data[i];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int i = b; i < e; ++i) {
        const uint32_t c = data[i];
        data[i] = run;
        run += c;
    }
}

// Stable scatter of one tile: keys are ranked in input order, 256 at a time;
// inside a wave the rank among equal digits comes from 8 ballots.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(int n, int shift, int ntiles,
                                                                 const uint64_t* __restrict__ kin,
                                                                 const uint32_t* __restrict__ vin,
                                                                 uint64_t* __restrict__ kout,
                                                                 uint32_t* __restrict__ vout,
                                                                 const uint32_t* __restrict__ offsets)
{
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t base[kRadixBins];
    __shared__ uint32_t wcnt[kWaves][kRadixBins];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    base[threadIdx.x] = offsets[threadIdx.x * ntiles + blockIdx.x];
    const int tile0 = blockIdx.x * kSortTile;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int s = 0; s < kSortItems; ++s) {
        for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        const int i = tile0 + s * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        uint64_t key = 0;
        uint32_t val = 0;
        uint32_t dg = 0;
        if (valid) {
            key = kin[i];
            val = vin[i];
            dg = static_cast<uint32_t>((key >> shift) & 0xff);
        }
        uint64_t m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = __popcll(m & lt_mask);
        if (valid && rank == 0) wcnt[wave][dg] = __popcll(m);
        __syncthreads();
        // per digit: exclusive prefix over the waves, then advance the base
        {
            const int d = threadIdx.x;
            uint32_t run = base[d];
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wcnt[w][d];
                wcnt[w][d] = run;
                run += c;
            }
            base[d] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcnt[wave][dg] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- records
// Record + leaf box of the surfel at leaf position p.
__global__ void k_records(int n, const uint32_t* __restrict__ order, const float* __restrict__ mu,
                          const float* __restrict__ quat, const float* __restrict__ scale,
                          const float* __restrict__ opac, float alpha_min, float sigma,
                          SurfelRec* __restrict__ rec, float* __restrict__ leafbox)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = static_cast<int>(order[p]);
    const float3 m = ld3(mu, i);
    const float4 q = ld4(quat, i);
    const float2 s = ld2(scale, i);
    const float o = opac[i];
    float tu[3] = {0, 0, 0}, tv[3] = {0, 0, 0}, nn[3] = {0, 0, 1};
    float rho2max = -1.0f;
    const bool ok = surfel_valid(m, q, s, o);
    if (ok) {
        quat_frame(q, tu, tv, nn);
        if (o >= alpha_min) {
            const float lim = 2.0f * logf(o / alpha_min);
            rho2max = fminf(sigma * sigma, fmaxf(lim, 0.0f));
        }
    }
    SurfelRec r;
    r.a = make_float4(m.x, m.y, m.z, o);
    r.b = make_float4(nn[0], nn[1], nn[2], rho2max);
    r.c = make_float4(tu[0] / s.x, tu[1] / s.x, tu[2] / s.x, __int_as_float(i));
    const float inf_slab = __uint_as_float(0x7c007c00u);  // cluster bound (+inf, +inf), set by k_cluster_slabs
    r.d = make_float4(tv[0] / s.y, tv[1] / s.y, tv[2] / s.y, inf_slab);
    if (!ok) {
        r.c = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(i));
        r.d = make_float4(0.0f, 0.0f, 0.0f, inf_slab);
    }
    rec[p] = r;
    float* bx = leafbox + 6 * static_cast<int64_t>(p);
    if (rho2max < 0.0f) {
        const float inf = __int_as_float(0x7f800000);
        for (int k = 0; k < 6; ++k) bx[k] = inf;
        return;
    }
    // Box of the ellipse mu + a s_u t_u + b s_v t_v, a^2 + b^2 <= rho^2,
    // padded so that FP32 rounding in the hit and slab tests can never put a
    // hit outside it.
    const float rho = sqrtf(rho2max);
    const float amax = fmaxf(fmaxf(fabsf(m.x), fabsf(m.y)), fabsf(m.z));
    const float pad_abs = 1e-5f * (1.0f + amax);
    for (int k = 0; k < 3; ++k) {
        const float eu = s.x * tu[k], ev = s.y * tv[k];
        const float h = rho * sqrtf(eu * eu + ev * ev);
        const float pad = pad_abs + 1e-4f * rho * fmaxf(s.x, s.y);
        const float c = k == 0 ? m.x : (k == 1 ? m.y : m.z);
        bx[k] = c - h - pad;
        bx[k + 3] = c + h + pad;
    }
}

// ---------------------------------------------------------------- Karras
__device__ __forceinline__ int lcp(const uint64_t* __restrict__ keys, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint64_t a = keys[i], b = keys[j];
    if (a != b) return __clzll(static_cast<long long>(a ^ b));
    return 64 + __clz(static_cast<int>(static_cast<uint32_t>(i) ^ static_cast<uint32_t>(j)));
}

__global__ void k_karras(int n, const uint64_t* __restrict__ keys, BvhNode* __restrict__ nodes,
                         int* __restrict__ leaf_parent, int2* __restrict__ brange)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (lcp(keys, n, i, i + 1) - lcp(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = lcp(keys, n, i, i - d);
    int lmax = 2;
    while (lcp(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (lcp(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = lcp(keys, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (lcp(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int g = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    brange[i] = make_int2(lo, hi - lo + 1);
    const int left = (lo == g) ? (g | kLeafBit) : g;
    const int right = (hi == g + 1) ? ((g + 1) | kLeafBit) : (g + 1);
    nodes[i].ch.x = left;
    nodes[i].ch.y = right;
    if (left & kLeafBit)
        leaf_parent[g] = i;
    else
        nodes[g].ch.z = i;
    if (right & kLeafBit)
        leaf_parent[g + 1] = i;
    else
        nodes[g + 1].ch.z = i;
    if (i == 0) nodes[0].ch.z = -1;
}

__global__ void k_single_root(BvhNode* nodes, int* leaf_parent, int2* brange)
{
    const float inf = __int_as_float(0x7f800000);
    brange[0] = make_int2(0, 1);
    nodes[0].ch = make_int4(0 | kLeafBit, kNoChild, -1, 0);
    nodes[0].p1.z = inf, nodes[0].p1.w = inf;
    nodes[0].p2 = make_float4(inf, inf, inf, inf);
    leaf_parent[0] = 0;
}

// ---------------------------------------------------------------- boxes
__device__ __forceinline__ void child_box(const BvhNode& nd, int which, float* b)
{
    if (which == 0) {
        b[0] = nd.p0.x, b[1] = nd.p0.y, b[2] = nd.p0.z, b[3] = nd.p0.w, b[4] = nd.p1.x, b[5] = nd.p1.y;
    } else {
        b[0] = nd.p1.z, b[1] = nd.p1.w, b[2] = nd.p2.x, b[3] = nd.p2.y, b[4] = nd.p2.z, b[5] = nd.p2.w;
    }
}

__device__ __forceinline__ bool box_empty(const float* b) { return isinf(b[0]) && b[0] > 0.0f; }

// Union of the two child boxes stored in `nd` (empty boxes are skipped).
__device__ __forceinline__ void node_union(const BvhNode& nd, float* out)
{
    float a[6], b[6];
    child_box(nd, 0, a);
    child_box(nd, 1, b);
    const bool ea = nd.ch.x == kNoChild || box_empty(a);
    const bool eb = nd.ch.y == kNoChild || box_empty(b);
    for (int k = 0; k < 6; ++k) {
        if (ea && eb)
            out[k] = __int_as_float(0x7f800000);
        else if (ea)
            out[k] = b[k];
        else if (eb)
            out[k] = a[k];
        else
            out[k] = k < 3 ? fminf(a[k], b[k]) : fmaxf(a[k], b[k]);
    }
}

// ---------------------------------------------------------------- levels
// The refit goes up the tree one depth level per launch (deepest first):
// the kernel boundary orders a level's writes before the next level's
// reads, so no atomics or cross-XCD cache maintenance are needed.  The
// nodes are grouped by depth once per build.
__global__ void k_node_depth(int nint, const BvhNode* __restrict__ nodes, int* __restrict__ ndepth,
                             int* __restrict__ maxd)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nint) return;
    int d = 0;
    for (int p = nodes[x].ch.z; p >= 0; p = nodes[p].ch.z) ++d;
    ndepth[x] = d;
    atomicMax(maxd, d);
}

// Nodes per depth.  Trees of at most kLevelBins levels count in LDS first
// (one global add per block and level instead of one per node: all nodes
// fall into a few dozen bins, whose global atomics would serialise).
constexpr int kLevelBins = 1024;

__global__ void k_level_hist(int nint, int nbins, const int* __restrict__ ndepth, int* __restrict__ hist)
{
    __shared__ int h[kLevelBins];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (nbins > kLevelBins) {
        if (x < nint) atomicAdd(&hist[ndepth[x]], 1);
        return;
    }
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    if (x < nint) atomicAdd(&h[ndepth[x]], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += blockDim.x)
        if (h[i] > 0) atomicAdd(&hist[i], h[i]);
}

// Node ids grouped by depth: `cursor` starts at each level's offset.  Within
// a level the order is arbitrary (the refit of a level is order-free).
__global__ void k_level_scatter(int nint, int nbins, const int* __restrict__ ndepth, int* __restrict__ cursor,
                                int* __restrict__ level_nodes)
{
    __shared__ int h[kLevelBins];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (nbins > kLevelBins) {
        if (x < nint) level_nodes[atomicAdd(&cursor[ndepth[x]], 1)] = x;
        return;
    }
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int d = x < nint ? ndepth[x] : 0;
    const int rank = x < nint ? atomicAdd(&h[d], 1) : 0;
    __syncthreads();
    // each level's block count becomes the block's base slot in that level
    for (int i = threadIdx.x; i < nbins; i += blockDim.x)
        if (h[i] > 0) h[i] = atomicAdd(&cursor[i], h[i]);
    __syncthreads();
    if (x < nint) level_nodes[h[d] + rank] = x;
}

// Box b into slot `which` of node nd: six scalar stores, so that the two
// children of a node (whose slots share a 16-byte word) never overwrite
// each other's half.
__device__ __forceinline__ void put_child_box(BvhNode* nd, int which, const float* b)
{
    float* f = reinterpret_cast<float*>(nd) + (which == 0 ? 0 : 6);
    for (int k = 0; k < 6; ++k) f[k] = b[k];
}

__global__ void k_leaf_up(int n, const float* __restrict__ leafbox, BvhNode* __restrict__ nodes,
                          const int* __restrict__ leaf_parent)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float b[6];
    for (int k = 0; k < 6; ++k) b[k] = leafbox[6 * static_cast<int64_t>(p) + k];
    const int node = leaf_parent[p];
    put_child_box(&nodes[node], nodes[node].ch.x == (p | kLeafBit) ? 0 : 1, b);
}

// Every node of one level: the union of its two slots into its parent's.
__global__ void k_level_up(int cnt, const int* __restrict__ ids, BvhNode* __restrict__ nodes)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const int x = ids[t];
    const BvhNode nd = nodes[x];
    float b[6];
    node_union(nd, b);
    const int parent = nd.ch.z;
    put_child_box(&nodes[parent], nodes[parent].ch.x == x ? 0 : 1, b);
}

// An FP16 no smaller than x >= 0 (+inf past the FP16 range), as its bits.
__device__ __forceinline__ uint32_t half_up(float x)
{
    if (!(x < 65504.0f)) return 0x7c00u;
    const _Float16 h = static_cast<_Float16>(x);
    uint32_t b = __builtin_bit_cast(uint16_t, h);
    if (static_cast<float>(h) < x) ++b;
    return b;
}

// Cluster bounds: record i of a leaf cluster stores in its last word, as two
// FP16 rounded up, the half-thickness h of a slab about its own plane,
// |n_i.(x - mu_i)| <= h (low half), and the radius c of a cylinder about the
// normal through its centre, |P_i (x - mu_i)| <= c with P_i the projection
// onto the plane (high half), that hold the support ellipse of every record
// from i to the end of the cluster.  An ellipse mu_j + a s_u t_u + b s_v t_v,
// a^2 + b^2 <= rho_j^2, reaches rho_j sqrt((s_u n_i.t_u)^2 + (s_v n_i.t_v)^2)
// off its centre along n_i (the record rows are t/s, so s n.t = n.row /
// |row|^2) and at most rho_j max(s_u, s_v) across it.  A ray that does not
// pass through both inside its depth window cannot hit any of those records.
// Records that never hit are skipped; a record without a plane of its own
// keeps (+inf, +inf) (never culls).
__global__ void k_cluster_slabs(int nw, const WideNode* __restrict__ wn, SurfelRec* __restrict__ rec)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * nw) return;
    const int ref = reinterpret_cast<const int*>(&wn[t >> 2].child)[t & 3];
    if (ref == kNoChild || (ref & kLeafBit) == 0) return;
    const int first = (ref & ~kLeafBit) >> 4, cnt = (ref & 15) + 1;
    const float inf = __int_as_float(0x7f800000);
    for (int i = 0; i < cnt; ++i) {
        const SurfelRec si = rec[first + i];
        float h = inf, c = inf;
        if (si.b.w >= 0.0f) {
            const float nx = si.b.x, ny = si.b.y, nz = si.b.z;
            h = 0.0f;
            c = 0.0f;
            for (int j = i; j < cnt; ++j) {
                const SurfelRec sj = j == i ? si : rec[first + j];
                if (sj.b.w < 0.0f) continue;  // never hits
                const float ex = sj.a.x - si.a.x, ey = sj.a.y - si.a.y, ez = sj.a.z - si.a.z;
                const float dn = dot3(nx, ny, nz, ex, ey, ez);
                const float uu = dot3(sj.c.x, sj.c.y, sj.c.z, sj.c.x, sj.c.y, sj.c.z);
                const float vv = dot3(sj.d.x, sj.d.y, sj.d.z, sj.d.x, sj.d.y, sj.d.z);
                const float cu = dot3(nx, ny, nz, sj.c.x, sj.c.y, sj.c.z) / uu;
                const float cv = dot3(nx, ny, nz, sj.d.x, sj.d.y, sj.d.z) / vv;
                const float rho = sqrtf(sj.b.w);
                h = fmaxf(h, fabsf(dn) + rho * sqrtf(fmaf(cu, cu, cv * cv)));
                const float px = ex - dn * nx, py = ey - dn * ny, pz = ez - dn * nz;
                c = fmaxf(c, sqrtf(dot3(px, py, pz, px, py, pz)) + rho * fmaxf(rsqrtf(uu), rsqrtf(vv)));
            }
            const float m = fmaxf(fmaxf(fabsf(si.a.x), fabsf(si.a.y)), fabsf(si.a.z));
            h = fmaf(h, 1.001f, 1e-6f * (1.0f + m));  // rounding of the sums above
            c = fmaf(c, 1.001f, 1e-6f * (1.0f + m));
        }
        // non-finite geometry packs as +inf: never culls
        reinterpret_cast<uint32_t*>(rec + first + i)[15] = half_up(h) | (half_up(c) << 16);
    }
}

__global__ void k_depth(int n, const int* __restrict__ leaf_parent, const BvhNode* __restrict__ nodes,
                        int* __restrict__ depth_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int d = 0;
    int node = leaf_parent[p];
    while (node >= 0) {
        ++d;
        node = nodes[node].ch.z;
    }
    atomicMax(depth_out, d);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------- wide tree
__device__ __forceinline__ float box_area(const float* b)
{
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
}

__device__ __forceinline__ void set_wide_box(WideNode* w, int slot, const float* b)
{
    float* f = reinterpret_cast<float*>(w);
    for (int k = 0; k < 6; ++k) f[k * 4 + slot] = b[k];
}

// One level of the top-down collapse: wide node w stands for binary node b;
// its up-to-four children are found by repeatedly opening the candidate with
// the largest box area, as long as that candidate holds more than leaf_max
// surfels.  Candidates with at most leaf_max surfels become cluster leaves
// (their surfels are contiguous in leaf order); larger ones become new wide
// nodes of the next level.
__global__ void k_collapse(int nfront, const int* __restrict__ front_in, int* __restrict__ front_out,
                           int* __restrict__ counts, int* __restrict__ wide_src, const BvhNode* __restrict__ bn,
                           const int2* __restrict__ brange, WideNode* __restrict__ wn, int4* __restrict__ wsrc,
                           int leaf_max)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nfront) return;
    const int w = front_in[t];
    const int b = wide_src[w];
    int ref[4], par[4], side[4];
    float area[4];
    int m = 0;
    auto add = [&](int p, int sd) {
        const int r = sd == 0 ? bn[p].ch.x : bn[p].ch.y;
        if (r == kNoChild) return;
        float bx[6];
        child_box(bn[p], sd, bx);
        ref[m] = r, par[m] = p, side[m] = sd, area[m] = box_area(bx);
        ++m;
    };
    add(b, 0);
    add(b, 1);
    while (m < 4) {
        int best = -1;
        float ba = -1.0f;
        for (int c = 0; c < m; ++c) {
            const bool internal = (ref[c] & kLeafBit) == 0;
            if (internal && brange[ref[c]].y > leaf_max && area[c] > ba) {
                best = c;
                ba = area[c];
            }
        }
        if (best < 0) break;
        const int open = ref[best];
        // replace `best` by its first child, append the second
        const int r0 = bn[open].ch.x, r1 = bn[open].ch.y;
        float bx[6];
        child_box(bn[open], 0, bx);
        ref[best] = r0, par[best] = open, side[best] = 0, area[best] = box_area(bx);
        child_box(bn[open], 1, bx);
        ref[m] = r1, par[m] = open, side[m] = 1, area[m] = box_area(bx);
        ++m;
    }
    WideNode node;
    int4 src = make_int4(-1, -1, -1, -1);
    int* srcp = reinterpret_cast<int*>(&src);
    int* chp = reinterpret_cast<int*>(&node.child);
    const float inf = __int_as_float(0x7f800000);
    const float empty[6] = {inf, inf, inf, inf, inf, inf};
    for (int c = 0; c < 4; ++c) {
        if (c >= m) {
            set_wide_box(&node, c, empty);
            chp[c] = kNoChild;
            continue;
        }
        float bx[6];
        child_box(bn[par[c]], side[c], bx);
        set_wide_box(&node, c, bx);
        srcp[c] = (par[c] << 1) | side[c];
        const int r = ref[c];
        if (r & kLeafBit) {
            chp[c] = cluster_ref(r & ~kLeafBit, 1);
        } else if (brange[r].y <= leaf_max) {
            chp[c] = cluster_ref(brange[r].x, brange[r].y);
        } else {
            const int nw = atomicAdd(&counts[0], 1);
            wide_src[nw] = r;
            front_out[atomicAdd(&counts[1], 1)] = nw;
            chp[c] = nw;
        }
    }
    node.meta = make_int4(0, 0, 0, 0);
    wn[w] = node;
    wsrc[w] = src;
}

// Wide boxes from the (refit) binary boxes they were taken from.
__global__ void k_wide_refit(int nw, const int4* __restrict__ wsrc, const BvhNode* __restrict__ bn,
                             WideNode* __restrict__ wn)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    const int4 s4 = wsrc[w];
    const int sv[4] = {s4.x, s4.y, s4.z, s4.w};
    for (int c = 0; c < 4; ++c) {
        if (sv[c] < 0) continue;
        float bx[6];
        child_box(bn[sv[c] >> 1], sv[c] & 1, bx);
        set_wide_box(&wn[w], c, bx);
    }
}

inline int blocks_for(int64_t n, int t) { return static_cast<int>((n + t - 1) / t); }

// ---------------------------------------------------------------- PLOC
// Parallel locally-ordered clustering (Meister and Bittner 2018): clusters
// start as the leaves in Morton order; per iteration every cluster finds,
// within kPlocRadius positions on either side, the cluster whose union with
// it has the smallest surface area; mutually nearest pairs merge into a new
// internal node (kept at the lower position), and the survivors are
// compacted in order.  Ties go to the smaller position, so the pair with the
// globally smallest (area, positions) is always mutual and every iteration
// merges.  Node ids count down from n - 2: the last merge is the root, 0.
constexpr int kPlocRadius = 8;
constexpr int kPlocBlock = 256;

__device__ __forceinline__ void box_union(const float* a, const float* b, float* u)
{
    const bool ea = box_empty(a), eb = box_empty(b);
    for (int k = 0; k < 3; ++k) {
        u[k] = ea ? b[k] : (eb ? a[k] : fminf(a[k], b[k]));
        u[k + 3] = ea ? b[k + 3] : (eb ? a[k + 3] : fmaxf(a[k + 3], b[k + 3]));
    }
}

// Merge cost: half the surface area of the union (0 for two empty boxes,
// +inf for a non-finite area).  Symmetric bit for bit in its arguments.
__device__ __forceinline__ float union_cost(const float* a, const float* b)
{
    if (box_empty(a) && box_empty(b)) return 0.0f;
    float u[6];
    box_union(a, b, u);
    const float c = box_area(u);
    return c == c ? c : __int_as_float(0x7f800000);
}

__global__ void k_ploc_init(int n, const float* __restrict__ leafbox, int* __restrict__ ref,
                            float* __restrict__ box)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ref[i] = i | kLeafBit;
    for (int k = 0; k < 6; ++k) box[6 * static_cast<int64_t>(i) + k] = leafbox[6 * static_cast<int64_t>(i) + k];
}

__global__ __launch_bounds__(kPlocBlock) void k_ploc_nn(int m, const float* __restrict__ box, int* __restrict__ nn)
{
    constexpr int kSpan = kPlocBlock + 2 * kPlocRadius;
    __shared__ float sb[kSpan * 6];
    const int base = blockIdx.x * kPlocBlock - kPlocRadius;
    for (int t = threadIdx.x; t < kSpan * 6; t += kPlocBlock) {
        const int g = base + t / 6;
        sb[t] = (g >= 0 && g < m) ? box[6 * static_cast<int64_t>(base) + t] : 0.0f;
    }
    __syncthreads();
    const int i = blockIdx.x * kPlocBlock + threadIdx.x;
    if (i >= m) return;
    const float* bi = sb + (threadIdx.x + kPlocRadius) * 6;
    float best = 0.0f;
    int bj = -1;
    for (int d = -kPlocRadius; d <= kPlocRadius; ++d) {  // increasing positions: ties keep the smaller
        const int j = i + d;
        if (d == 0 || j < 0 || j >= m) continue;
        const float c = union_cost(bi, bi + 6 * d);
        if (bj < 0 || c < best) {
            best = c;
            bj = j;
        }
    }
    nn[i] = bj;
}

// Mutual pairs merge (the lower position leads and keeps the new cluster in
// place; pairs are disjoint, so no slot is read and written by two threads);
// keep[i] flags the survivors and each block adds its count to *total.
__global__ __launch_bounds__(kPlocBlock) void k_ploc_merge(int m, int* __restrict__ ref, float* __restrict__ box,
                                                            const int* __restrict__ nn, BvhNode* __restrict__ nodes,
                                                            uint32_t* __restrict__ keep,
                                                            uint32_t* __restrict__ block_counts,
                                                            int* __restrict__ node_counter, int top,
                                                            uint32_t* __restrict__ total)
{
    __shared__ uint32_t wave_cnt[kPlocBlock / 64];
    const int i = blockIdx.x * kPlocBlock + threadIdx.x;
    bool kept = false;
    if (i < m) {
        const int j = nn[i];
        const bool mutual = j >= 0 && nn[j] == i;
        kept = !(mutual && j < i);
        if (mutual && i < j) {
            const int id = top - atomicAdd(node_counter, 1);
            const int a = ref[i], b = ref[j];
            const int ca = (a & kLeafBit) ? 1 : nodes[a].ch.w;
            const int cb = (b & kLeafBit) ? 1 : nodes[b].ch.w;
            nodes[id].ch = make_int4(a, b, -1, ca + cb);
            if (!(a & kLeafBit)) nodes[a].ch.z = id;
            if (!(b & kLeafBit)) nodes[b].ch.z = id;
            float bi[6], bj[6], u[6];
            for (int k = 0; k < 6; ++k) {
                bi[k] = box[6 * static_cast<int64_t>(i) + k];
                bj[k] = box[6 * static_cast<int64_t>(j) + k];
            }
            box_union(bi, bj, u);
            for (int k = 0; k < 6; ++k) box[6 * static_cast<int64_t>(i) + k] = u[k];
            ref[i] = id;
        }
        keep[i] = kept ? 1u : 0u;
    }
    const uint64_t bal = __ballot(kept);
    if ((threadIdx.x & 63) == 0) wave_cnt[threadIdx.x >> 6] = static_cast<uint32_t>(__popcll(bal));
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0;
        for (int w = 0; w < kPlocBlock / 64; ++w) c += wave_cnt[w];
        block_counts[blockIdx.x] = c;
        atomicAdd(total, c);
    }
}

// Survivors to their compacted positions, in order (block offsets from the
// exclusive scan of the block counts, ranks inside the block by ballots).
__global__ __launch_bounds__(kPlocBlock) void k_ploc_scatter(int m, const uint32_t* __restrict__ keep,
                                                              const uint32_t* __restrict__ offsets,
                                                              const int* __restrict__ ref_in,
                                                              const float* __restrict__ box_in,
                                                              int* __restrict__ ref_out, float* __restrict__ box_out)
{
    __shared__ uint32_t wave_cnt[kPlocBlock / 64];
    const int i = blockIdx.x * kPlocBlock + threadIdx.x;
    const bool kept = i < m && keep[i] != 0;
    const uint64_t bal = __ballot(kept);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wave_cnt[wave] = static_cast<uint32_t>(__popcll(bal));
    __syncthreads();
    if (!kept) return;
    uint32_t pos = offsets[blockIdx.x];
    for (int w = 0; w < wave; ++w) pos += wave_cnt[w];
    pos += static_cast<uint32_t>(__popcll(bal & ((1ull << lane) - 1ull)));
    ref_out[pos] = ref_in[i];
    for (int k = 0; k < 6; ++k) box_out[6 * static_cast<int64_t>(pos) + k] = box_in[6 * static_cast<int64_t>(i) + k];
}

__device__ __forceinline__ int ref_count(const BvhNode* nodes, int r)
{
    return (r & kLeafBit) ? 1 : nodes[r].ch.w;
}

// First depth-first leaf of every internal node: the leaves of the left
// siblings of its ancestors (and of itself, when it is a right child).
__global__ void k_tree_offsets(int nint, const BvhNode* __restrict__ nodes, int* __restrict__ first)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nint) return;
    int off = 0, c = x, p = nodes[x].ch.z;
    while (p >= 0) {
        const int4 ch = nodes[p].ch;
        if (ch.y == c) off += ref_count(nodes, ch.x);
        c = p;
        p = ch.z;
    }
    first[x] = off;
}

// Leaves renumbered in depth-first order: new order, leaf parents, leaf
// references and the leaf range of every internal node.
__global__ void k_tree_renumber(int nint, BvhNode* __restrict__ nodes, const int* __restrict__ first,
                                const uint32_t* __restrict__ order_in, uint32_t* __restrict__ order_out,
                                int* __restrict__ leaf_parent, int2* __restrict__ brange)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nint) return;
    const int4 ch = nodes[x].ch;
    const int f = first[x];
    brange[x] = make_int2(f, ch.w);
    if (ch.x & kLeafBit) {
        order_out[f] = order_in[ch.x & ~kLeafBit];
        leaf_parent[f] = x;
        nodes[x].ch.x = f | kLeafBit;
    }
    if (ch.y & kLeafBit) {
        const int pos = f + ref_count(nodes, ch.x);
        order_out[pos] = order_in[ch.y & ~kLeafBit];
        leaf_parent[pos] = x;
        nodes[x].ch.y = pos | kLeafBit;
    }
}



}  // namespace

// ---------------------------------------------------------------- host side
hipError_t fill_u32(void* p, int64_t n, uint32_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int nb = static_cast<int>(n < 256 * 1024 ? (n + 255) / 256 : 1024);
    k_fill_u32<<<nb, 256, 0, st>>>(static_cast<uint32_t*>(p), n, v);
    return hipGetLastError();
}

size_t sort_pairs_count_bytes(int n)
{
    return static_cast<size_t>(blocks_for(n, kSortTile)) * kRadixBins * sizeof(uint32_t);
}

// Stable LSD sort of (key, value) pairs on the low 8 * passes key bits; an
// even number of passes leaves the result in k0 / v0.
hipError_t sort_pairs(int n, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint32_t* counts, int passes,
                      hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int ntiles = blocks_for(n, kSortTile);
    for (int pass = 0; pass < passes; ++pass) {
        k_radix_hist<<<ntiles, kSortThreads, 0, st>>>(n, pass * 8, k0, counts, ntiles);
        k_scan_exclusive<<<1, 1024, 0, st>>>(counts, ntiles * kRadixBins);
        k_radix_scatter<<<ntiles, kSortThreads, 0, st>>>(n, pass * 8, ntiles, k0, v0, k1, v1, counts);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* tk = k0;
        k0 = k1;
        k1 = tk;
        uint32_t* tv = v0;
        v0 = v1;
        v1 = tv;
    }
    return hipSuccess;
}

// PLOC scratch: two cluster buffers (reference + box), neighbours, survivor
// flags, first leaves, the renumbered order, block counts and two counters.
static size_t ploc_scratch_bytes(int n)
{
    const size_t nb = static_cast<size_t>(blocks_for(n, kPlocBlock));
    return static_cast<size_t>(n) * (2 * (sizeof(int) + 6 * sizeof(float)) + 4 * sizeof(int)) +
           nb * sizeof(uint32_t) + 256;
}

hipError_t lbvh_sort_scratch_bytes(int n, size_t* bytes)
{
    const int ntiles = blocks_for(n, kSortTile);
    const size_t sort = static_cast<size_t>(n) * (2 * sizeof(uint64_t) + 2 * sizeof(uint32_t)) +
                        static_cast<size_t>(ntiles) * kRadixBins * sizeof(uint32_t) + 64 * 6 * sizeof(float) + 256;
    const size_t ploc = ploc_scratch_bytes(n);
    *bytes = sort > ploc ? sort : ploc;
    return hipSuccess;
}

// Binary tree by PLOC over the leaf boxes of the Morton order in a.leafbox;
// afterwards the leaves are renumbered depth first (a.order rewritten) and
// nodes, leaf_parent and brange describe the tree in that order.  The whole
// scratch is reused (the sort is over).
static hipError_t ploc_tree(BuildArgs& a, void* scratch, hipStream_t st)
{
    const int n = a.n;
    const int nint = n - 1;
    char* p = static_cast<char*>(scratch);
    auto take = [&](size_t bytes) {
        char* r = p;
        p += (bytes + 255) & ~static_cast<size_t>(255);
        return r;
    };
    int* refA = reinterpret_cast<int*>(take(sizeof(int) * n));
    int* refB = reinterpret_cast<int*>(take(sizeof(int) * n));
    float* boxA = reinterpret_cast<float*>(take(sizeof(float) * 6 * n));
    float* boxB = reinterpret_cast<float*>(take(sizeof(float) * 6 * n));
    int* nn = reinterpret_cast<int*>(take(sizeof(int) * n));
    uint32_t* keep = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * n));
    uint32_t* counts = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * blocks_for(n, kPlocBlock)));
    int* ctr = reinterpret_cast<int*>(take(2 * sizeof(int)));  // node counter, survivors

    k_ploc_init<<<blocks_for(n, 256), 256, 0, st>>>(n, a.leafbox, refA, boxA);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = fill_u32(ctr, 2, 0u, st);
    int m = n;
    for (int iter = 0; e == hipSuccess && m > 1; ++iter) {
        const int nb = blocks_for(m, kPlocBlock);
        k_ploc_nn<<<nb, kPlocBlock, 0, st>>>(m, boxA, nn);
        e = hipGetLastError();
        if (e == hipSuccess) e = fill_u32(ctr + 1, 1, 0u, st);
        if (e != hipSuccess) break;
        k_ploc_merge<<<nb, kPlocBlock, 0, st>>>(m, refA, boxA, nn, a.nodes, keep, counts, ctr, n - 2,
                                                reinterpret_cast<uint32_t*>(ctr + 1));
        k_scan_exclusive<<<1, 1024, 0, st>>>(counts, nb);
        k_ploc_scatter<<<nb, kPlocBlock, 0, st>>>(m, keep, counts, refA, boxA, refB, boxB);
        e = hipGetLastError();
        int survivors = m;
        if (e == hipSuccess) e = hipMemcpyAsync(&survivors, ctr + 1, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        if (survivors >= m || iter > 4 * n) return hipErrorUnknown;  // no merge: cannot happen
        m = survivors;
        int* tr = refA;
        refA = refB;
        refB = tr;
        float* tb = boxA;
        boxA = boxB;
        boxB = tb;
    }
    if (e != hipSuccess) return e;
    // the cluster buffers are free again
    int* first = refA;
    uint32_t* order_new = reinterpret_cast<uint32_t*>(refB);
    k_tree_offsets<<<blocks_for(nint, 256), 256, 0, st>>>(nint, a.nodes, first);
    k_tree_renumber<<<blocks_for(nint, 256), 256, 0, st>>>(nint, a.nodes, first, a.order, order_new, a.leaf_parent,
                                                           a.brange);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(a.order, order_new, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st);
    return e;
}

__global__ void k_collapse_init(int* wide_src, int* front, int* counts)
{
    wide_src[0] = 0;
    front[0] = 0;
    counts[0] = 1;
    counts[1] = 0;
}

// Records + leaf boxes in the current leaf order, then the node boxes level
// by level from the deepest (the levels are grouped at build time).
static hipError_t refit_boxes(const BuildArgs& a, hipStream_t st)
{
    const int n = a.n;
    k_records<<<blocks_for(n, 256), 256, 0, st>>>(n, a.order, a.mu, a.quat, a.scale, a.opac, a.alpha_min,
                                                    a.sigma, a.rec, a.leafbox);
    k_leaf_up<<<blocks_for(n, 256), 256, 0, st>>>(n, a.leafbox, a.nodes, a.leaf_parent);
    hipError_t e = hipGetLastError();
    const std::vector<int>& off = *a.levels;
    for (int d = static_cast<int>(off.size()) - 2; e == hipSuccess && d >= 1; --d) {
        const int cnt = off[d + 1] - off[d];
        if (cnt <= 0) continue;
        k_level_up<<<blocks_for(cnt, 256), 256, 0, st>>>(cnt, a.level_nodes + off[d], a.nodes);
        e = hipGetLastError();
    }
    return e;
}

// Internal nodes grouped by depth (root = depth 0): a.level_nodes holds their
// ids level after level and *a.levels the level offsets (depth + 2 entries).
// Uses the build scratch and reads the level sizes back (synchronises st).
static hipError_t group_levels(BuildArgs& a, void* scratch, hipStream_t st)
{
    const int nint = a.n > 1 ? a.n - 1 : 1;
    int* ndepth = static_cast<int*>(scratch);
    int* maxd = ndepth + nint;
    hipError_t e = fill_u32(maxd, 1, 0u, st);
    if (e != hipSuccess) return e;
    k_node_depth<<<blocks_for(nint, 256), 256, 0, st>>>(nint, a.nodes, ndepth, maxd);
    int D = 0;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&D, maxd, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    int* hist = maxd + 1;
    e = fill_u32(hist, D + 1, 0u, st);
    if (e != hipSuccess) return e;
    k_level_hist<<<blocks_for(nint, 256), 256, 0, st>>>(nint, D + 1, ndepth, hist);
    std::vector<int> h(D + 1);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), hist, sizeof(int) * (D + 1), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    std::vector<int>& off = *a.levels;
    off.assign(D + 2, 0);
    for (int d = 0; d <= D; ++d) off[d + 1] = off[d] + h[d];
    e = hipMemcpyAsync(hist, off.data(), sizeof(int) * (D + 1), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    k_level_scatter<<<blocks_for(nint, 256), 256, 0, st>>>(nint, D + 1, ndepth, hist, a.level_nodes);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host offsets outlive this call
    return e;
}

hipError_t lbvh_build(BuildArgs& a, void* scratch, hipStream_t st)
{
    const int n = a.n;
    if (n <= 0) return hipSuccess;
    const int ntiles = blocks_for(n, kSortTile);
    char* p = static_cast<char*>(scratch);
    uint64_t* k0 = reinterpret_cast<uint64_t*>(p);
    p += sizeof(uint64_t) * n;
    uint64_t* k1 = reinterpret_cast<uint64_t*>(p);
    p += sizeof(uint64_t) * n;
    uint32_t* v0 = reinterpret_cast<uint32_t*>(p);
    p += sizeof(uint32_t) * n;
    uint32_t* v1 = reinterpret_cast<uint32_t*>(p);
    p += sizeof(uint32_t) * n;
    uint32_t* counts = reinterpret_cast<uint32_t*>(p);
    p += sizeof(uint32_t) * ntiles * kRadixBins;
    float* partial = reinterpret_cast<float*>(p);
    p += sizeof(float) * 6 * 64;
    float* bounds = reinterpret_cast<float*>(p);

    k_bounds_partial<<<64, kSortThreads, 0, st>>>(n, a.mu, a.quat, a.scale, a.opac, partial);
    k_bounds_final<<<1, 64, 0, st>>>(64, partial, bounds);
    k_morton<<<blocks_for(n, 256), 256, 0, st>>>(n, a.mu, a.quat, a.scale, a.opac, bounds, k0, v0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = pass * 8;
        k_radix_hist<<<ntiles, kSortThreads, 0, st>>>(n, shift, k0, counts, ntiles);
        k_scan_exclusive<<<1, 1024, 0, st>>>(counts, ntiles * kRadixBins);
        k_radix_scatter<<<ntiles, kSortThreads, 0, st>>>(n, shift, ntiles, k0, v0, k1, v1, counts);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* tk = k0;
        k0 = k1;
        k1 = tk;
        uint32_t* tv = v0;
        v0 = v1;
        v1 = tv;
    }
    // after an even number of passes the sorted data is back in k0/v0
    e = hipMemcpyAsync(a.order, v0, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    if (a.sorted_keys) {
        e = hipMemcpyAsync(a.sorted_keys, k0, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    const int nint = n > 1 ? n - 1 : 1;
    e = fill_u32(a.nodes, static_cast<int64_t>(nint) * (sizeof(BvhNode) / 4), 0u, st);
    if (e != hipSuccess) return e;
    if (n == 1) {
        k_single_root<<<1, 1, 0, st>>>(a.nodes, a.leaf_parent, a.brange);
    } else if (a.ploc) {
        // leaf boxes in Morton order, then the clustering rewrites the order
        k_records<<<blocks_for(n, 256), 256, 0, st>>>(n, a.order, a.mu, a.quat, a.scale, a.opac, a.alpha_min,
                                                        a.sigma, a.rec, a.leafbox);
        e = hipGetLastError();
        if (e == hipSuccess) e = ploc_tree(a, scratch, st);
        if (e != hipSuccess) return e;
    } else {
        k_karras<<<blocks_for(n - 1, 256), 256, 0, st>>>(n, k0, a.nodes, a.leaf_parent, a.brange);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = group_levels(a, scratch, st);
    if (e != hipSuccess) return e;
    e = refit_boxes(a, st);
    if (e != hipSuccess) return e;
    // top-down collapse into the 4-wide tree, one level per launch
    {
        const int nmax = nint;
        int* wide_src = a.wscratch;
        int* fa = a.wscratch + nmax;
        int* fb = a.wscratch + 2 * nmax;
        int* counts = a.wscratch + 3 * nmax;
        k_collapse_init<<<1, 1, 0, st>>>(wide_src, fa, counts);
        int nfront = 1, levels = 0;
        while (nfront > 0) {
            e = fill_u32(counts + 1, 1, 0u, st);
            if (e != hipSuccess) return e;
            k_collapse<<<blocks_for(nfront, 128), 128, 0, st>>>(nfront, fa, fb, counts, wide_src, a.nodes,
                                                                  a.brange, a.wnodes, a.wsrc, a.leaf_size);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(&nfront, counts + 1, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return e;
            int* t = fa;
            fa = fb;
            fb = t;
            ++levels;
        }
        int nw = 0;
        e = hipMemcpyAsync(&nw, counts, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        a.n_wide = nw;
        a.wide_depth = levels;
    }
    if (a.n_wide > 0) {
        k_cluster_slabs<<<blocks_for(4 * static_cast<int64_t>(a.n_wide), 256), 256, 0, st>>>(a.n_wide, a.wnodes,
                                                                                            a.rec);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    e = fill_u32(a.depth, 1, 0u, st);
    if (e != hipSuccess) return e;
    k_depth<<<blocks_for(n, 256), 256, 0, st>>>(n, a.leaf_parent, a.nodes, a.depth);
    return hipGetLastError();
}

hipError_t lbvh_refit(const BuildArgs& a, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    hipError_t e = refit_boxes(a, st);
    if (e != hipSuccess) return e;
    if (a.n_wide <= 0) return hipGetLastError();
    k_wide_refit<<<blocks_for(a.n_wide, 256), 256, 0, st>>>(a.n_wide, a.wsrc, a.nodes, a.wnodes);
    k_cluster_slabs<<<blocks_for(4 * static_cast<int64_t>(a.n_wide), 256), 256, 0, st>>>(a.n_wide, a.wnodes, a.rec);
    return hipGetLastError();
}

}  // namespace irgs
