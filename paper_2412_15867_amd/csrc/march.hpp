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

template <int K>
struct KBuf {
    float t[K];
    int id[K];
    float a[K];
    int cnt;

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            t[j] = __int_as_float(0x7f800000);  // +inf
            id[j] = 0x7fffffff;
            a[j] = 0.0f;
        }
        cnt = 0;
    }

    // Far bound of the current round: the K-th key once the buffer is full.
    __device__ __forceinline__ bool full() const { return cnt >= K; }

    // Insert (tt, ii, aa); the largest key falls off the end when full.
    __device__ __forceinline__ void insert(float tt, int ii, float aa)
    {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const bool lt = key_less(tt, ii, t[j], id[j]);
            const float t2 = lt ? t[j] : tt;
            const int i2 = lt ? id[j] : ii;
            const float a2 = lt ? a[j] : aa;
            t[j] = lt ? tt : t[j];
            id[j] = lt ? ii : id[j];
            a[j] = lt ? aa : a[j];
            tt = t2;
            ii = i2;
            aa = a2;
        }
        cnt = cnt < K ? cnt + 1 : K;
    }
};

// Offer one record to the buffer: Eq. 6-7 test, resume-key window, and the
// K-th-key cut once full.
template <int K>
__device__ __forceinline__ void offer(KBuf<K>& kb, const SurfelRec& s, const Ray& ray, float t_min, float t_max,
                                      float last_t, int last_i, Counters& ct)
{
    ++ct.tests;
    float tau, rho2;
    if (!hit_test(s, ray, t_min, t_max, &tau, &rho2)) return;
    const int id = __float_as_int(s.c.w);
    if (!key_less(last_t, last_i, tau, id)) return;
    if (!key_less(tau, id, kb.t[K - 1], kb.id[K - 1])) return;
    const float alpha = s.a.w * __expf(-0.5f * rho2);
    ++ct.inserts;
    kb.insert(tau, id, alpha);
}

// Per-lane traversal stack: the first kStackLds entries live in LDS
// (slot-major, so a wave's pushes hit distinct banks), deeper entries in a
// global overflow area sized from the tree depth at build time.
struct Stack {
    int* lds;       // this block's LDS stack base: [kStackLds][kBlock]
    int* ovf;       // global overflow base for slot 0 of this thread
    int ovf_stride; // distance between overflow slots
    int tid;        // thread index within the block
    int sp;

    __device__ __forceinline__ void push(int v)
    {
        if (sp < kStackLds)
            lds[sp * kBlock + tid] = v;
        else
            ovf[(sp - kStackLds) * ovf_stride] = v;
        ++sp;
    }
    __device__ __forceinline__ int pop()
    {
        --sp;
        return sp < kStackLds ? lds[sp * kBlock + tid] : ovf[(sp - kStackLds) * ovf_stride];
    }
};

// One round of collection by BVH traversal.  Boxes are culled against the
// window [max(t_min, last_t), min(t_max, K-th key)], nearer child first.
template <int K>
__device__ __forceinline__ void collect_bvh(KBuf<K>& kb, const SceneView& sc, const Ray& ray, float ix, float iy,
                                            float iz, float t_min, float t_max, float last_t, int last_i, Stack& st,
                                            Counters& ct)
{
    ++ct.rounds;
    const float lo = fmaxf(t_min, last_t);
    const float tmax_c = fminf(t_max, 3.0e38f);
    st.sp = 0;
    int node = 0;
    while (true) {
        ++ct.nodes;
        const float4* np = reinterpret_cast<const float4*>(sc.nodes + node);
        const float4 p0 = np[0], p1 = np[1], p2 = np[2];
        const int4 ch = reinterpret_cast<const int4*>(np)[3];
        const float hi = kb.full() ? fminf(kb.t[K - 1], tmax_c) : tmax_c;
        float te0, te1;
        bool h0 = ch.x != kNoChild &&
                  box_hit(p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, ray.ox, ray.oy, ray.oz, ix, iy, iz, lo, hi, &te0);
        bool h1 = ch.y != kNoChild &&
                  box_hit(p1.z, p1.w, p2.x, p2.y, p2.z, p2.w, ray.ox, ray.oy, ray.oz, ix, iy, iz, lo, hi, &te1);
        if (h0 && (ch.x & kLeafBit)) {
            offer<K>(kb, load_rec(sc.rec, ch.x & ~kLeafBit), ray, t_min, t_max, last_t, last_i, ct);
            h0 = false;
        }
        if (h1 && (ch.y & kLeafBit)) {
            offer<K>(kb, load_rec(sc.rec, ch.y & ~kLeafBit), ray, t_min, t_max, last_t, last_i, ct);
            h1 = false;
        }
        if (h0 && h1) {
            const bool first0 = te0 <= te1;
            st.push(first0 ? ch.y : ch.x);
            node = first0 ? ch.x : ch.y;
        } else if (h0) {
            node = ch.x;
        } else if (h1) {
            node = ch.y;
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
                                            float t_max, float last_t, int last_i, Counters& ct)
{
    ++ct.rounds;
    for (int i = 0; i < sc.n; ++i) offer<K>(kb, load_rec(sc.rec, i), ray, t_min, t_max, last_t, last_i, ct);
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
