// Forward trace as a flat per-lane state machine (BVH path).
//
// The k-buffer marching of Sec. 3.2 nests three loops per ray -- rounds,
// traversal steps inside a round, and the composite of a round's buffer.
// Written as nested loops, a wave of 64 rays runs every level in lockstep:
// lanes that finished a round (or their ray) idle until the slowest lane of
// the wave catches up.  Here each loop iteration advances every lane by one
// unit of its own work:
//   TRAV  visit one wide node (4 box tests; children pushed far to near, the
//         nearest becomes the current item) or test up to two surfels of a
//         cluster (both records in one round trip), skipping the rest of the
//         cluster when the records' bounds show that the ray cannot hit it
//         inside its depth window; a hit for the buffer enters it at the top
//         of the next iteration; an empty stack ends the round;
//   COMP  composite the nearest buffered hit (Eq. 2: w = T alpha, T *= 1 - a)
//         or, with the buffer drained, start the next round or finish the ray;
//   FETCH claim the lane's next ray from a global counter (rays go to lanes
//         as lanes free up, so the launch drains evenly).
// Per ray the arithmetic and its order are exactly those of the nested form,
// so results are bit-identical; only the interleaving across lanes changes.
#pragma once

#include "irgs_internal.hpp"
#include "march.hpp"

namespace irgs {

constexpr int kItemEmpty = 0x7fffffff;  // no current item (stack drained)

// Where a lane's rays come from and where their results go.
struct LaneRay {
    int64_t r;     // ray index within its output arrays
    int item;      // work item (packed launches), 0 otherwise
    SceneView sc;  // the item's scene (packed launches only)
};

// One scene, rays [0, R), claimed in `order` when given.
struct PlainSource {
    SceneView sc;
    OutPtrs o;
    const float* ro;
    const float* rd;
    int64_t R;
    const uint32_t* order;

    __device__ __forceinline__ bool load(int64_t slot, LaneRay& lr, Ray& ray) const
    {
        if (slot >= R) return false;
        if (order) slot = order[slot];
        lr.r = slot;
        lr.item = 0;
        ray = load_ray(ro, rd, slot);
        return true;
    }
    __device__ __forceinline__ const OutPtrs& out(const LaneRay&) const { return o; }
    // the one scene of the launch (uniform: kept out of per-lane registers)
    __device__ __forceinline__ const SceneView& view(const LaneRay&) const { return sc; }
};

// Several requests over several scenes: a slot indexes the concatenation of
// the items' rays; the owning item is found by bisection.
struct PackedSource {
    const SceneView* scenes;
    const WorkItem* items;
    int n_items;
    int64_t total;

    __device__ __forceinline__ bool load(int64_t slot, LaneRay& lr, Ray& ray) const
    {
        if (slot >= total) return false;
        int lo = 0, hi = n_items - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].chunk_begin <= slot)  // chunk_begin holds the item's first slot here
                lo = mid;
            else
                hi = mid - 1;
        }
        const WorkItem& it = items[lo];
        const int64_t local = slot - it.chunk_begin;
        lr.r = it.ray_begin + local;
        lr.item = lo;
        lr.sc = scenes[it.scene];
        ray = load_ray(it.ro, it.rd, lr.r);
        return true;
    }
    __device__ __forceinline__ const OutPtrs& out(const LaneRay& lr) const { return items[lr.item].out; }
    __device__ __forceinline__ const SceneView& view(const LaneRay& lr) const { return lr.sc; }
};

// Claim one slot per calling lane from a global counter: one atomic per
// wave, slots in lane order (consecutive lanes get consecutive rays).  Call
// with exactly the lanes that need a slot active.
__device__ __forceinline__ int64_t claim_slot(unsigned long long* next)
{
    const uint64_t need = __ballot(1);
    const int rank = __popcll(need & __lanemask_lt());
    const int leader = __ffsll(static_cast<unsigned long long>(need)) - 1;
    unsigned long long base = 0;
    if (rank == 0) base = atomicAdd(next, static_cast<unsigned long long>(__popcll(need)));
    base = __shfl(base, leader);
    return static_cast<int64_t>(base) + rank;
}

// True when the ray cannot hit the disc of record s nor any later disc of
// its leaf cluster inside the depth window (lo, t_max).  The record's last
// word holds two FP16 bounds of those discs: the half-thickness h of a slab
// about its plane and the radius c of a cylinder about its normal.  The ray
// crosses the slab for t in (num -+ h) / den; at the middle depth
// t_c = num / den it lies on the plane at t_c d - w from the centre and
// within the slab it moves across the plane by at most |d| h / |den|.  Both
// bounds take a pad for the rounding of these FP32 depths; a NaN or an
// infinity from a ray parallel to the plane never culls.
__device__ __forceinline__ bool cluster_miss(const SurfelRec& s, const Ray& ray, float lo, float t_max)
{
    const float wx = s.a.x - ray.ox, wy = s.a.y - ray.oy, wz = s.a.z - ray.oz;
    const float num = dot3(s.b.x, s.b.y, s.b.z, wx, wy, wz);
    const float rden = __builtin_amdgcn_rcpf(dot3(s.b.x, s.b.y, s.b.z, ray.dx, ray.dy, ray.dz));
    const uint32_t hc = __float_as_uint(s.d.w);
    const float pad = 1e-5f * (1.0f + fabsf(wx) + fabsf(wy) + fabsf(wz));
    const float h = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(hc))) + pad;
    const float cr = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(hc >> 16))) + pad;
    const float ta = (num - h) * rden, tb = (num + h) * rden;
    const float tc = num * rden;
    const float ex = fmaf(tc, ray.dx, -wx), ey = fmaf(tc, ray.dy, -wy), ez = fmaf(tc, ray.dz, -wz);
    // |d| by the hardware square root (within an ulp; the bound's 1e-4 margin
    // below covers it, and the cull only ever skips discs that cannot hit)
    const float dn = __builtin_amdgcn_sqrtf(dot3(ray.dx, ray.dy, ray.dz, ray.dx, ray.dy, ray.dz));
    const float reach = fmaf(dn, h * fabsf(rden), cr);
    const bool wide = dot3(ex, ey, ez, ex, ey, ez) > reach * reach * 1.0001f;
    return (ta < lo && tb < lo) || (ta > t_max && tb > t_max) || wide;
}

// Stored hit lists are written four entries at a time (one 16-byte
// streaming store for the ids, one for the transmittances: the lists are read
// by the backward, not by this launch, so they need no room in L2) when rows
// start 16-byte aligned.
__device__ __forceinline__ bool pair_stores(const OutPtrs& out)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(out.hit_ids) | reinterpret_cast<uintptr_t>(out.hit_T);
    return (out.H_cap & 3) == 0 && (a & 15) == 0;
}

template <int FM, int CM, bool CT, class Source>
__device__ __forceinline__ void write_result(const Source& src, const LaneRay& lr, float O, float D, float T,
                                             const float* acc, int nh, const Counters& ct)
{
    const OutPtrs& out = src.out(lr);
    const int64_t r = lr.r;
    const int F = src.view(lr).F;
    const int FO = CM == kColSH ? 3 : (CM == kColNormal ? F + 3 : F);  // composited channels
    out.O[r] = O;
    out.D[r] = D;
#pragma unroll
    for (int c = 0; c < FM; ++c)
        if (c < FO) out.feat[r * FO + c] = acc[c];
    if (out.T) out.T[r] = T;
    if (out.n_hits) out.n_hits[r] = nh;
    if (CT && out.counters)
        reinterpret_cast<int4*>(out.counters)[r] = make_int4(ct.nodes, ct.tests, ct.inserts, ct.rounds);
}

// Add w times the features (with SH: the view-dependent colour; with the
// normal mode: the features, then the record's unit normal `nr` turned to
// face the ray) of surfel `id` to the accumulators.
template <int FM, int CM>
__device__ __forceinline__ void add_features(const SceneView& sc, const TraceParams& P, const Ray& ray, int id,
                                             const float4& nr, float w, float* acc)
{
    const float* f = sc.feat + static_cast<int64_t>(id) * sc.F;
    if constexpr (CM == kColSH) {
        float Y[16], raw[3];
        sh_basis(ray.dx, ray.dy, ray.dz, P.sh_deg, Y);
        sh_raw(f, P.sh_deg, Y, raw);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = fmaf(w, fmaxf(raw[c], 0.0f), acc[c]);
    } else {
#pragma unroll
        for (int c = 0; c < FM; ++c)
            if (c < sc.F) acc[c] = fmaf(w, f[c], acc[c]);
        if constexpr (CM == kColNormal) {
            const float s = dot3(nr.x, nr.y, nr.z, ray.dx, ray.dy, ray.dz) > 0.0f ? -w : w;
            const float nv[3] = {nr.x, nr.y, nr.z};
#pragma unroll
            for (int c = 0; c < FM; ++c)
                if (c >= sc.F && c < sc.F + 3) acc[c] = fmaf(s, nv[c - sc.F], acc[c]);
        }
    }
}

// Per-lane deferred work carried from one k-buffer round to the next: the
// children culled only because they start beyond the round's K-th key, the
// hits found beyond it, and the keys pushed out of the buffer.  Every hit
// after the round's last key lies in exactly one of them, so the next round
// starts from this list instead of the root.  Two halves (this round's input,
// next round's output); an overflowing output falls back to a root restart.
//
// A lane's puts are spread over many iterations, long enough for L2 to evict
// a line between two of them, so single 4-byte stores would each write a
// partial line back.  Puts are therefore staged in an LDS ring of
// 2 kDeferStage entries per lane (slot-major, so a wave's writes fall in
// distinct banks) and written back kDeferStage at a time (32 bytes, one
// after the other, so L2 holds the whole group in one line) by one flush
// step at the top of each iteration; the round's end writes the rest.  An
// iteration puts at most 5 entries (4 children, or 2 hits, plus 1 pushed out
// of the buffer) and each flush step retires a full group, so at most 12
// entries are ever staged and the ring never overwrites one that is waiting.
// With kStaged false (the k = 32 and 64 instances, whose rounds defer half
// as much or less and which measured slower with the staging) each put is
// a direct store.
constexpr int kDeferRing = 2 * kDeferStage;

template <bool kStaged>
struct Deferred {
    glb_int* base;   // 2 * cap entries of this lane (cap a multiple of kDeferStage)
    lds_int* stage;  // this lane's ring slots: stage[g * kBlock], g < kDeferRing (staged lists)
    int cap;
    int half;        // half holding this round's input
    int n_in, i_in, n_out;
    int flushed;     // output entries written back (a multiple of kDeferStage; staged lists)

    __device__ __forceinline__ void reset()
    {
        half = 0;
        n_in = i_in = n_out = flushed = 0;
    }
    __device__ __forceinline__ void put(int item)
    {
        if (n_out < cap) {
            if constexpr (kStaged)
                stage[(n_out & (kDeferRing - 1)) * kBlock] = item;
            else
                base[(half ^ 1) * cap + n_out] = item;
        }
        ++n_out;
    }
    // A full group waits (an overflowing list is dropped whole: nothing to write).
    __device__ __forceinline__ bool group_ready() const
    {
        return kStaged && n_out <= cap && n_out - flushed >= kDeferStage;
    }
    __device__ __forceinline__ void flush_group()
    {
        glb_int* dst = base + (half ^ 1) * cap + flushed;
        const int s0 = flushed & (kDeferRing - 1);
#pragma unroll
        for (int g = 0; g < kDeferStage; ++g) dst[g] = stage[(s0 + g) * kBlock];
        flushed += kDeferStage;
    }
    __device__ __forceinline__ int take() { return base[half * cap + i_in++]; }
    __device__ __forceinline__ bool has() const { return i_in < n_in; }
    // Next round: consume what this one deferred; false = it overflowed.  The
    // staged rest is written first, a partly filled last group whole
    // (entries past n_out are never read; flushed + kDeferStage <= cap).
    __device__ __forceinline__ bool flip()
    {
        const bool ok = n_out <= cap;
        if (kStaged && ok)
            while (flushed < n_out) flush_group();
        half ^= 1;
        n_in = ok ? n_out : 0;
        i_in = 0;
        n_out = 0;
        flushed = 0;
        return ok;
    }
};

// CT: keep the per-ray work counters (launches that ask for them); without,
// their registers stay free.
template <int K, int FM, int CM, bool CT, class Source>
__device__ __forceinline__ void trace_flat(const Source& src, unsigned long long* next_ray, const TraceParams& P,
                                           Stack& st, Deferred<(K <= 16)> dq)
{
    enum { kTrav = 0, kComp = 1, kFetch = 2, kDead = 3, kIns = 4 };
    const float inf = __int_as_float(0x7f800000);
    LaneRay lr;
    Ray ray;
    SlabRay q{};
    float T = 1.0f, O = 0.0f, D = 0.0f;
    float acc[FM];
#pragma unroll
    for (int c = 0; c < FM; ++c) acc[c] = 0.0f;
    int nh = 0;
    uint64_t after = 0;          // resume key; while compositing, the key just composited
    uint64_t pend = kKeyNone;    // hit key entering the buffer at the next iteration (mode kIns)
    int pend_id = 0, pend_id1 = 0, pend_id2 = 0;  // stored hit list: entries waiting for their quad
    float pend_T = 0.0f, pend_T1 = 0.0f, pend_T2 = 0.0f;
    bool round_full = false, term = false;
    int cur = kItemEmpty;
    int mode = kFetch;
    KBuf<K> kb;
    kb.clear();
    Counters ct;
    auto next_item = [&]() -> int {
        if (st.sp > 0) return st.pop();
        if (dq.has()) return dq.take();
        return kItemEmpty;
    };
    while (true) {
        // Hits found by the previous leaf step enter the buffer first,
        // predicated over the wave (the buffer is modified outside any
        // divergent region, so it needs no per-branch copy); the branch on
        // the ballot is wave-uniform and costs no memory round trip.
        const bool want_ins = mode == kIns;
        if (__ballot(want_ins)) {
            const uint64_t ev = kb.insert_if(want_ins, pend);
            if (want_ins) {
                if constexpr (CT) ++ct.inserts;
                if (ev != kKeyNone) dq.put(cluster_ref(key_pos(ev), 1));  // pushed out of the buffer
                pend = kKeyNone;
                mode = kTrav;
            }
        }
        // Staged deferred entries: write a full group back (wave-uniform
        // branch, at the point of the loop with the fewest live registers).
        if constexpr (K <= 16) {
            const bool want_flush = dq.group_ready();
            if (__ballot(want_flush)) {
                if (want_flush) dq.flush_group();
            }
        }
        // Phase vote: the wave runs, per iteration, only the kind of step the
        // most lanes are waiting for (wave-uniform branch); the rest wait.
        // Node and leaf steps stay apart: each memory instruction of a step
        // then fetches one kind of data.
        const bool want_node = mode == kTrav && cur != kItemEmpty && cur >= 0;
        const bool want_leaf = mode == kTrav && cur < 0;
        const bool want_other = mode != kDead && !want_node && !want_leaf;
        const uint64_t bn = __ballot(want_node), bl = __ballot(want_leaf), bo = __ballot(want_other);
        if ((bn | bl | bo) == 0) break;
        const int cn = __popcll(bn), cl = __popcll(bl), co = __popcll(bo);
        // node steps count double against leaf steps: a node step hands its
        // lanes new items, and a leaf step that waits loses nothing;
        // compositing and fetch steps count double against both with the
        // normal channels, and with plain features for K >= 32 (measured:
        // at K = 16 on a 200K-surfel scene with 24 hits per ray the double
        // weight costs 14%; the SH compositing step, with the basis and 48
        // coefficients, is the costliest step and never takes it)
        constexpr int kOtherW = (CM == kColNormal || (CM == kColPlain && K >= 32)) ? 2 : 1;
        if (cn > 0 && 2 * cn >= cl && cn >= kOtherW * co) {
            if (want_node) {
                if constexpr (CT) ++ct.nodes;
                const float4* np = reinterpret_cast<const float4*>(src.view(lr).wnodes + cur);
                const float4 lx = np[0], ly = np[1], lz = np[2], hx = np[3], hy = np[4], hz = np[5];
                const int4 ch = reinterpret_cast<const int4*>(np)[6];
                const float lo = after == 0 ? P.t_min : fmaxf(P.t_min, key_tau(after));
                const float tmax_c = fminf(P.t_max, 3.0e38f);
                const float hi = kb.full() ? fminf(key_tau(kb.last()), tmax_c) : tmax_c;
                float key[4], tn[4], tf[4];
                int ref[4] = {ch.x, ch.y, ch.z, ch.w};
                box_span(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, q, lo, tmax_c, &tn[0], &tf[0]);
                box_span(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, q, lo, tmax_c, &tn[1], &tf[1]);
                box_span(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, q, lo, tmax_c, &tn[2], &tf[2]);
                box_span(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, q, lo, tmax_c, &tn[3], &tf[3]);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    // an empty slot has an all +inf box, which is never crossed
                    const bool crossed = tn[c] <= tf[c];
                    const bool inside = crossed && tn[c] <= hi;
                    if (crossed && !inside) dq.put(ref[c]);  // beyond this round's K-th key
                    key[c] = inside ? tn[c] : inf;
                }
#define IRGS_CSWAP(a, b)                    \
    if (key[b] < key[a]) {                  \
        const float tk = key[a];            \
        key[a] = key[b];                    \
        key[b] = tk;                        \
        const int tr = ref[a];              \
        ref[a] = ref[b];                    \
        ref[b] = tr;                        \
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
                cur = key[0] < inf ? ref[0] : next_item();
            }
        } else if (cl >= kOtherW * co) {
            // Test the next surfels of the current cluster: both records of
            // a pair are fetched together (one memory round trip), the
            // second is tested only if the first does not enter the buffer.
            // A hit for the buffer waits in `pend` and is inserted at the top
            // of the next iteration.
            if (want_leaf) {
                const int first = (cur & ~kLeafBit) >> 4;
                const int cnt = (cur & 15) + 1;
                const SurfelRec* recs = src.view(lr).rec;
                const SurfelRec s0 = load_rec(recs, first);
                const SurfelRec s1 = load_rec(recs, cnt > 1 ? first + 1 : first);
                // Each record's bounds hold its own disc and every later disc of
                // its cluster: outside the first record's, none of the cluster's
                // remaining discs can be a hit; outside the second's, none after
                // the first.
                const float lo = after == 0 ? P.t_min : fmaxf(P.t_min, key_tau(after));
                const bool past = cluster_miss(s0, ray, lo, P.t_max);
                const bool past1 = !past && cnt > 1 && cluster_miss(s1, ray, lo, P.t_max);
                int used = past || past1 ? cnt : 1;
                if constexpr (CT) ct.tests += past ? 0 : 1;
                float tau = 0.0f, rho2 = 0.0f;
                bool hit = !past && hit_test(s0, ray, P.t_min, P.t_max, &tau, &rho2);
                uint64_t key = hit_key(tau, first);
                bool above = hit && key > after;
                bool ins = above && key < kb.last();
                if (above && !ins) dq.put(cluster_ref(first, 1));  // beyond this round's K-th key
                if (!past && !past1 && !ins && cnt > 1) {
                    used = 2;
                    if constexpr (CT) ++ct.tests;
                    hit = hit_test(s1, ray, P.t_min, P.t_max, &tau, &rho2);
                    key = hit_key(tau, first + 1);
                    above = hit && key > after;
                    ins = above && key < kb.last();
                    if (above && !ins) dq.put(cluster_ref(first + 1, 1));
                }
                cur = cnt > used ? cluster_ref(first + used, cnt - used) : next_item();
                if (ins) {
                    pend = key;
                    mode = kIns;
                }
            }
        } else if (want_other) {
            if (mode == kFetch) {
                if (!src.load(claim_slot(next_ray), lr, ray)) {
                    mode = kDead;
                } else {
                    T = 1.0f, O = 0.0f, D = 0.0f, nh = 0;
#pragma unroll
                    for (int c = 0; c < FM; ++c) acc[c] = 0.0f;
                    ct = Counters();
                    after = 0;
                    term = false;
                    kb.clear();
                    dq.reset();
                    if (src.view(lr).n <= 0 || !ray_valid(ray)) {
                        write_result<FM, CM, CT>(src, lr, O, D, T, acc, nh, ct);
                    } else {
                        q = slab_ray(ray);
                        cur = 0;
                        st.sp = 0;
                        if constexpr (CT) ++ct.rounds;
                        mode = kTrav;
                    }
                }
            } else if (mode == kTrav) {  // stack and deferred input drained: the buffer is final
                round_full = kb.full();
                mode = kComp;
            } else if (kb.cnt > 0 && !term) {
                const int pos = kb.pos(0);
                after = kb.k[0];
#pragma unroll
                for (int j = 0; j < K - 1; ++j) kb.k[j] = kb.k[j + 1];
                kb.k[K - 1] = kKeyNone;
                --kb.cnt;
                const SurfelRec s = load_rec(src.view(lr).rec, pos);
                float tau, rho2;
                plane_hit(s, ray, &tau, &rho2);
                const float a = alpha_of(s, rho2);
                const int id = __float_as_int(s.c.w);
                const float w = T * a;
                O += w;
                D = fmaf(w, tau, D);
                add_features<FM, CM>(src.view(lr), P, ray, id, s.b, w, acc);
                const OutPtrs& out = src.out(lr);
                if (out.hit_ids && nh < out.H_cap) {
                    const int64_t at = lr.r * out.H_cap + nh;
                    if (!pair_stores(out)) {
                        out.hit_ids[at] = id;
                        if (out.hit_T) out.hit_T[at] = T;
                    } else if ((nh & 3) == 3) {  // the fourth of a quad: all four in one store each
                        typedef int v4i __attribute__((ext_vector_type(4)));
                        typedef float v4f __attribute__((ext_vector_type(4)));
                        v4i vi; vi.x = pend_id; vi.y = pend_id1; vi.z = pend_id2; vi.w = id;
                        __builtin_nontemporal_store(vi, reinterpret_cast<v4i*>(out.hit_ids + at - 3));
                        if (out.hit_T) {
                            v4f vt; vt.x = pend_T; vt.y = pend_T1; vt.z = pend_T2; vt.w = T;
                            __builtin_nontemporal_store(vt, reinterpret_cast<v4f*>(out.hit_T + at - 3));
                        }
                    } else {
                        const int c = nh & 3;
                        pend_id = c == 0 ? id : pend_id;
                        pend_T = c == 0 ? T : pend_T;
                        pend_id1 = c == 1 ? id : pend_id1;
                        pend_T1 = c == 1 ? T : pend_T1;
                        pend_id2 = c == 2 ? id : pend_id2;
                        pend_T2 = c == 2 ? T : pend_T2;
                    }
                }
                T = T * (1.0f - a);
                ++nh;
                if (T < P.T_min) term = true;
            } else if (term || !round_full) {
                const OutPtrs& out = src.out(lr);
                const int c = nh & 3;
                if (out.hit_ids && pair_stores(out) && c != 0 && nh - 1 < out.H_cap) {  // the last entries
                    const int64_t b = lr.r * out.H_cap + (nh - c);
                    out.hit_ids[b] = pend_id;
                    if (out.hit_T) out.hit_T[b] = pend_T;
                    if (c > 1) {
                        out.hit_ids[b + 1] = pend_id1;
                        if (out.hit_T) out.hit_T[b + 1] = pend_T1;
                    }
                    if (c > 2) {
                        out.hit_ids[b + 2] = pend_id2;
                        if (out.hit_T) out.hit_T[b + 2] = pend_T2;
                    }
                }
                write_result<FM, CM, CT>(src, lr, O, D, T, acc, nh, ct);
                mode = kFetch;
            } else {
                kb.clear();  // `after` is the round's last (K-th) key
                st.sp = 0;
                if constexpr (CT) ++ct.rounds;
                cur = dq.flip() ? next_item() : 0;  // deferred list, or the root after an overflow
                mode = kTrav;
            }
        }
    }
}

}  // namespace irgs
