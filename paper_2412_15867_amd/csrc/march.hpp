// Per-ray k-buffer hit marching (Sec. 3.2: the k-buffer per-ray sorting the
// paper takes from 3DGRT gives the exact depth order of the intersected
// Gaussians).
//
// One round collects, into a register-resident buffer of K entries sorted by
// (tau, id), the K smallest hit keys strictly after the last key composited;
// the caller composites them and resumes after the K-th.  The buffer content
// after a round is a pure function of the hit set (the K smallest keys above
// the resume key), so it does not depend on the order in which candidates
// are visited: the brute-force collector and the BVH collector give
// bit-identical rounds whenever the BVH reaches every hit.
#pragma once

#include "irgs_device.hpp"

namespace irgs {

// Work counters of one ray (kept in registers, written only on request).
struct Counters {
    int nodes = 0, tests = 0, inserts = 0, rounds = 0;
};

// The k-buffer holds hit keys (tau, leaf position), ascending.  Equal
// depths are ordered by leaf position, which every kernel shares.  alpha
// and the surfel id are re-read from the record when an entry is composited.
template <int K>
struct KBuf {
    uint64_t k[K];
    int cnt;

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int j = 0; j < K; ++j) k[j] = kKeyNone;
        cnt = 0;
    }

    __device__ __forceinline__ bool full() const { return cnt >= K; }
    __device__ __forceinline__ uint64_t last() const { return k[K - 1]; }
    __device__ __forceinline__ int pos(int j) const { return key_pos(k[j]); }

    // Insert `key` when `ins` holds (then key is below the last entry; keys
    // are unique); the last entry falls off the end and is returned
    // (kKeyNone when nothing fell off).  Read as doubles the keys are in
    // reverse order and kKeyNone is -inf, so entry j of the merged sequence
    // is FP64 min(entry j-1, max(key, entry j)) of the old one: two
    // full-rate instructions per entry, all independent (a 64-bit compare
    // and four selects per entry as integers).  With ins false the key is
    // kKeyNone and nothing moves (the entries are sorted).
    __device__ __forceinline__ uint64_t insert_if(bool ins, uint64_t key)
    {
        const uint64_t out = ins ? k[K - 1] : kKeyNone;
        const double x = as_f64(ins ? key : kKeyNone);
#pragma unroll
        for (int j = K - 1; j > 0; --j) k[j] = bits_of(f64_min(as_f64(k[j - 1]), f64_max(x, as_f64(k[j]))));
        k[0] = bits_of(f64_max(x, as_f64(k[0])));
        cnt += (ins && cnt < K) ? 1 : 0;
        return out;
    }

  private:
    static __device__ __forceinline__ double as_f64(uint64_t b) { return __longlong_as_double(static_cast<long long>(b)); }
    static __device__ __forceinline__ uint64_t bits_of(double d) { return static_cast<uint64_t>(__double_as_longlong(d)); }
    // The instructions themselves: through the fmin/fmax builtins the
    // compiler first quiets every loop-carried entry (a third instruction per
    // entry), which keys, never NaN, do not need.
    static __device__ __forceinline__ double f64_min(double a, double b)
    {
        double r;
        asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
        return r;
    }
    static __device__ __forceinline__ double f64_max(double a, double b)
    {
        double r;
        asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
        return r;
    }
};

// Offer the record at leaf position `pos` to the buffer: Eq. 6-7 test,
// above the resume key, below the K-th key once full.
template <int K>
__device__ __forceinline__ void offer(KBuf<K>& kb, const SurfelRec& s, int pos, const Ray& ray, float t_min,
                                      float t_max, uint64_t after, Counters& ct)
{
    ++ct.tests;
    float tau, rho2;
    if (!hit_test(s, ray, t_min, t_max, &tau, &rho2)) return;
    const uint64_t key = hit_key(tau, pos);
    if (key <= after || key >= kb.last()) return;
    ++ct.inserts;
    kb.insert_if(true, key);
}

// Per-lane traversal stack: the first `lds_slots` entries live in LDS
// (slot-major, so a wave's pushes hit distinct banks), deeper entries in a
// global overflow area sized from the tree depth at build time.  The two
// areas are typed by address space so that the LDS arm compiles to ds_*
// instructions instead of a merged generic (flat) access.
typedef __attribute__((address_space(3))) int lds_int;
typedef __attribute__((address_space(1))) int glb_int;

struct Stack {
    lds_int* lds;   // this block's LDS stack base: [lds_slots][kBlock]
    glb_int* ovf;   // global overflow base for slot 0 of this thread
    int ovf_stride; // distance between overflow slots
    int tid;        // thread index within the block
    int sp;
    int lds_slots;

    __device__ __forceinline__ void push(int v)
    {
        if (sp < lds_slots)
            lds[sp * kBlock + tid] = v;
        else
            __builtin_nontemporal_store(v, ovf + (sp - lds_slots) * ovf_stride);
        ++sp;
    }
    __device__ __forceinline__ int pop()
    {
        --sp;
        if (sp < lds_slots) return lds[sp * kBlock + tid];
        return __builtin_nontemporal_load(ovf + (sp - lds_slots) * ovf_stride);
    }
};

__device__ __forceinline__ lds_int* as_lds(int* p) { return (lds_int*)p; }
__device__ __forceinline__ glb_int* as_glb(int* p) { return (glb_int*)p; }

// One round of collection by traversal of the 4-wide tree.  Child boxes
// are culled against the window [max(t_min, resume depth), min(t_max, K-th key)];
// cluster leaves are tested on the spot, inner children are visited nearest
// first (the others are pushed farthest first).
template <int K>
__device__ __forceinline__ void collect_bvh(KBuf<K>& kb, const SceneView& sc, const Ray& ray, const SlabRay& q,
                                            float t_min, float t_max, uint64_t after, Stack& st,
                                            Counters& ct)
{
    ++ct.rounds;
    const float lo = after == 0 ? t_min : fmaxf(t_min, key_tau(after));
    const float tmax_c = fminf(t_max, 3.0e38f);
    const float inf = __int_as_float(0x7f800000);
    st.sp = 0;
    int node = 0;
    while (true) {
        ++ct.nodes;
        const float4* np = reinterpret_cast<const float4*>(sc.wnodes + node);
        const float4 lx = np[0], ly = np[1], lz = np[2], hx = np[3], hy = np[4], hz = np[5];
        const int4 ch = reinterpret_cast<const int4*>(np)[6];
        const float hi = kb.full() ? fminf(key_tau(kb.last()), tmax_c) : tmax_c;
        float te[4];
        bool h[4];
        h[0] = box_hit(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, q, lo, hi, &te[0]);
        h[1] = box_hit(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, q, lo, hi, &te[1]);
        h[2] = box_hit(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, q, lo, hi, &te[2]);
        h[3] = box_hit(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, q, lo, hi, &te[3]);
        const int c4[4] = {ch.x, ch.y, ch.z, ch.w};
        float key[4];
        int ref[4];
        int leaves = 0;  // bit c: cluster child c was hit
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bool leaf = c4[c] < 0;  // cluster (kNoChild never passes the box test)
            leaves |= (h[c] && leaf) ? (1 << c) : 0;
            key[c] = (h[c] && !leaf) ? te[c] : inf;
            ref[c] = c4[c];
        }
        while (leaves) {
            const int c = __ffs(leaves) - 1;
            leaves &= leaves - 1;
            const int r = c == 0 ? ch.x : (c == 1 ? ch.y : (c == 2 ? ch.z : ch.w));
            const int first = (r & ~kLeafBit) >> 4;
            const int cnt = (r & 15) + 1;
            for (int q = first; q < first + cnt; ++q)
                offer<K>(kb, load_rec(sc.rec, q), q, ray, t_min, t_max, after, ct);
        }
        // sort the four (entry distance, child) pairs ascending
#define IRGS_CSWAP(a, b)                                      \
    if (key[b] < key[a]) {                                    \
        const float tk = key[a];                              \
        key[a] = key[b];                                      \
        key[b] = tk;                                          \
        const int tr = ref[a];                                \
        ref[a] = ref[b];                                      \
        ref[b] = tr;                                          \
    }
        IRGS_CSWAP(0, 1)
        IRGS_CSWAP(2, 3)
        IRGS_CSWAP(0, 2)
        IRGS_CSWAP(1, 3)
        IRGS_CSWAP(1, 2)
#undef IRGS_CSWAP
        if (key[3] < inf) st.push(ref[3]);
        if (key[2] < inf) st.push(ref[2]);
        if (key[1] < inf) st.push(ref[1]);
        if (key[0] < inf) {
            node = ref[0];
        } else {
            if (st.sp == 0) break;
            node = st.pop();
        }
    }
}

// One round of collection by testing every record (the plain GPU tracer).
// The record index is uniform across the wave, so loads are broadcast.
template <int K>
__device__ __forceinline__ void collect_all(KBuf<K>& kb, const SceneView& sc, const Ray& ray, float t_min,
                                            float t_max, uint64_t after, Counters& ct)
{
    ++ct.rounds;
    for (int i = 0; i < sc.n; ++i) offer<K>(kb, load_rec(sc.rec, i), i, ray, t_min, t_max, after, ct);
}

__device__ __forceinline__ bool ray_valid(const Ray& r)
{
    const bool fin = isfinite(r.ox) && isfinite(r.oy) && isfinite(r.oz) && isfinite(r.dx) && isfinite(r.dy) &&
                     isfinite(r.dz);
    return fin && (r.dx != 0.0f || r.dy != 0.0f || r.dz != 0.0f);
}

__device__ __forceinline__ Ray load_ray(const float* __restrict__ ro, const float* __restrict__ rd, int64_t r)
{
    Ray ray;
    ray.ox = ro[3 * r + 0];
    ray.oy = ro[3 * r + 1];
    ray.oz = ro[3 * r + 2];
    ray.dx = rd[3 * r + 0];
    ray.dy = rd[3 * r + 1];
    ray.dz = rd[3 * r + 2];
    return ray;
}

}  // namespace irgs
