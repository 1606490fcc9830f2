// Adjoint of the 2D Gaussian ray trace (the paper's trace is differentiable so
// that gradients of the indirect radiance reach the surfels, Sec. 3.3).
//
// With c_i = g_O + g_F . f_i + g_D tau_i the loss seen by one ray is
// L = sum_i T_i alpha_i c_i, T_i = prod_{j<i} (1 - alpha_j) (Eq. 2).  Walking
// the ray's hits back to front with the suffix composite
//     S_i = alpha_i c_i + (1 - alpha_i) S_{i+1},   S_end = 0,
// gives, without ever dividing by (1 - alpha),
//     dL/dalpha_i = T_i (c_i - S_{i+1}),   dL/df_i = T_i alpha_i g_F,
//     dL/dtau_i (through D) = T_i alpha_i g_D.
// alpha = o exp(-(u^2+v^2)/2) with u, v, tau from Eq. 6-7 chains these to
// the centre, the raw quaternion (through its normalisation), the scales and
// the opacity; per-surfel sums use FP32 global atomics.
//
// The hit list of a ray is either read back from the forward pass (ids and
// the transmittance before each hit) or re-marched: a first pass records the
// state at the start of each k-buffer round, a second pass re-collects the
// rounds last to first and walks each one back to front.
#include <hip/hip_runtime.h>

#include "irgs_internal.hpp"
#include "march.hpp"

namespace irgs {

namespace {

template <int FM>
__device__ __forceinline__ void grad_hit(const RawSurfels& raw, int F, int id, const Ray& ray, float Ti, float& S,
                                         float gO, const float* gF, float gD, const GradOut& go)
{
    const int64_t i = id;
    const float mx = raw.mu[3 * i], my = raw.mu[3 * i + 1], mz = raw.mu[3 * i + 2];
    const float4 q = make_float4(raw.quat[4 * i], raw.quat[4 * i + 1], raw.quat[4 * i + 2], raw.quat[4 * i + 3]);
    const float su = raw.scale[2 * i], sv = raw.scale[2 * i + 1];
    const float o = raw.opac[i];
    float tu[3], tv[3], nn[3];
    const float qn = quat_frame(q, tu, tv, nn);

    const float wx = mx - ray.ox, wy = my - ray.oy, wz = mz - ray.oz;
    const float den = dot3(nn[0], nn[1], nn[2], ray.dx, ray.dy, ray.dz);
    const float num = dot3(nn[0], nn[1], nn[2], wx, wy, wz);
    const float tau = num / den;
    const float px = fmaf(tau, ray.dx, -wx), py = fmaf(tau, ray.dy, -wy), pz = fmaf(tau, ray.dz, -wz);
    const float u = dot3(px, py, pz, tu[0], tu[1], tu[2]) / su;
    const float v = dot3(px, py, pz, tv[0], tv[1], tv[2]) / sv;
    const float G = __expf(-0.5f * fmaf(u, u, v * v));
    const float alpha = o * G;

    float c = fmaf(gD, tau, gO);
    const float* f = raw.feat + i * F;
    float fv[FM];
#pragma unroll
    for (int k = 0; k < FM; ++k) {
        fv[k] = k < F ? f[k] : 0.0f;
        c = fmaf(gF[k], fv[k], c);
    }
    const float wgt = Ti * alpha;
    const float dA = Ti * (c - S);
    S = fmaf(alpha, c, (1.0f - alpha) * S);

    if (go.feat) {
#pragma unroll
        for (int k = 0; k < FM; ++k)
            if (k < F) atomicAdd(go.feat + i * F + k, wgt * gF[k]);
    }
    if (go.opac) atomicAdd(go.opac + i, dA * G);

    const float gu = -dA * alpha * u;
    const float gv = -dA * alpha * v;
    if (go.scale) {
        atomicAdd(go.scale + 2 * i, -gu * u / su);
        atomicAdd(go.scale + 2 * i + 1, -gv * v / sv);
    }
    // p - mu = tau d - w;  du/d(p-mu) = t_u / s_u
    const float gpx = gu * tu[0] / su + gv * tv[0] / sv;
    const float gpy = gu * tu[1] / su + gv * tv[1] / sv;
    const float gpz = gu * tu[2] / su + gv * tv[2] / sv;
    const float gtau = fmaf(wgt, gD, dot3(gpx, gpy, gpz, ray.dx, ray.dy, ray.dz));
    const float gt_den = gtau / den;
    if (go.mu) {
        atomicAdd(go.mu + 3 * i, fmaf(gt_den, nn[0], -gpx));
        atomicAdd(go.mu + 3 * i + 1, fmaf(gt_den, nn[1], -gpy));
        atomicAdd(go.mu + 3 * i + 2, fmaf(gt_den, nn[2], -gpz));
    }
    if (go.quat) {
        // dtau/dn = -(p - mu) / den;  du/dt_u = (p - mu) / s_u
        const float gn0 = -gt_den * px, gn1 = -gt_den * py, gn2 = -gt_den * pz;
        const float au = gu / su, av = gv / sv;
        const float gu0 = au * px, gu1 = au * py, gu2 = au * pz;
        const float gv0 = av * px, gv1 = av * py, gv2 = av * pz;
        const float inv = 1.0f / qn;
        const float w = q.x * inv, x = q.y * inv, y = q.z * inv, z = q.w * inv;
        // derivatives of the rotation columns with respect to (w, x, y, z)
        const float dw = 2.0f * (z * gu1 - y * gu2 - z * gv0 + x * gv2 + y * gn0 - x * gn1);
        const float dx = 2.0f * (y * gu1 + z * gu2 + y * gv0 - 2.0f * x * gv1 + w * gv2 + z * gn0 - w * gn1 -
                                 2.0f * x * gn2);
        const float dy = 2.0f * (-2.0f * y * gu0 + x * gu1 - w * gu2 + x * gv0 + z * gv2 + w * gn0 + z * gn1 -
                                 2.0f * y * gn2);
        const float dz = 2.0f * (-2.0f * z * gu0 + w * gu1 + x * gu2 - w * gv0 - 2.0f * z * gv1 + y * gv2 +
                                 x * gn0 + y * gn1);
        const float proj = w * dw + x * dx + y * dy + z * dz;
        atomicAdd(go.quat + 4 * i, (dw - w * proj) * inv);
        atomicAdd(go.quat + 4 * i + 1, (dx - x * proj) * inv);
        atomicAdd(go.quat + 4 * i + 2, (dy - y * proj) * inv);
        atomicAdd(go.quat + 4 * i + 3, (dz - z * proj) * inv);
    }
}

template <int K>
__device__ __forceinline__ void entry(const KBuf<K>& kb, const float* Tj, int j, int* id, float* T)
{
    int ri = 0;
    float rt = 0.0f;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        ri = q == j ? kb.id[q] : ri;
        rt = q == j ? Tj[q] : rt;
    }
    *id = ri;
    *T = rt;
}

struct Checkpoint {
    float last_t;
    int last_i;
    float T;
    int nb;  // hits composited before this round
};

template <int K, int FM>
__device__ __forceinline__ void bwd_one(const SceneView& sc, const RawSurfels& raw, const TraceParams& P,
                                        const Ray& ray, int64_t r, const OutPtrs& saved, bool use_saved,
                                        const GradIn& gin, const GradOut& go, Stack& st, float4* ck,
                                        int64_t ck_stride)
{
    const float gO = gin.gO ? gin.gO[r] : 0.0f;
    const float gD = gin.gD ? gin.gD[r] : 0.0f;
    float gF[FM];
    bool any = gO != 0.0f || gD != 0.0f;
#pragma unroll
    for (int k = 0; k < FM; ++k) {
        gF[k] = (gin.gF && k < P.F) ? gin.gF[r * P.F + k] : 0.0f;
        any = any || gF[k] != 0.0f;
    }
    if (!any || sc.n <= 0 || !ray_valid(ray)) return;
    const int nh_saved = saved.n_hits ? saved.n_hits[r] : -1;
    if (nh_saved == 0) return;
    float S = 0.0f;
    if (use_saved && nh_saved > 0 && nh_saved <= saved.H_cap) {
        for (int h = nh_saved - 1; h >= 0; --h) {
            const int id = saved.hit_ids[r * saved.H_cap + h];
            const float Ti = saved.hit_T[r * saved.H_cap + h];
            grad_hit<FM>(raw, P.F, id, ray, Ti, S, gO, gF, gD, go);
        }
        return;
    }
    // ---- re-march: pass 1 records the state at the start of each round
    Counters ct;
    const float ix = safe_inv(ray.dx), iy = safe_inv(ray.dy), iz = safe_inv(ray.dz);
    float last_t = -__int_as_float(0x7f800000);
    int last_i = -1;
    float T = 1.0f;
    int nh = 0;
    int rounds = 0;
    bool done = false;
    while (!done) {
        if (rounds < kBwdCheckpoints)
            ck[rounds * ck_stride] = make_float4(last_t, __int_as_float(last_i), T, __int_as_float(nh));
        KBuf<K> kb;
        kb.clear();
        collect_bvh<K>(kb, sc, ray, ix, iy, iz, P.t_min, P.t_max, last_t, last_i, st, ct);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j < kb.cnt && !done) {
                T = T * (1.0f - kb.a[j]);
                ++nh;
                if (T < P.T_min) done = true;
            }
        }
        if (kb.cnt < K) {
            done = true;
        } else {
            last_t = kb.t[K - 1];
            last_i = kb.id[K - 1];
        }
        ++rounds;
    }
    const int total = nh;
    // ---- pass 2: rounds last to first, each walked back to front
    for (int rr = rounds - 1; rr >= 0; --rr) {
        const int base = rr < kBwdCheckpoints ? rr : kBwdCheckpoints - 1;
        float4 c4 = ck[base * ck_stride];
        last_t = c4.x;
        last_i = __float_as_int(c4.y);
        T = c4.z;
        int nb = __float_as_int(c4.w);
        KBuf<K> kb;
        for (int adv = base; adv < rr; ++adv) {  // rounds past the last checkpoint
            kb.clear();
            collect_bvh<K>(kb, sc, ray, ix, iy, iz, P.t_min, P.t_max, last_t, last_i, st, ct);
#pragma unroll
            for (int j = 0; j < K; ++j) T = j < kb.cnt ? T * (1.0f - kb.a[j]) : T;
            nb += kb.cnt;
            last_t = kb.t[K - 1];
            last_i = kb.id[K - 1];
        }
        kb.clear();
        collect_bvh<K>(kb, sc, ray, ix, iy, iz, P.t_min, P.t_max, last_t, last_i, st, ct);
        const int m = min(kb.cnt, total - nb);
        float Tj[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            Tj[j] = T;
            T = j < m ? T * (1.0f - kb.a[j]) : T;
        }
        for (int j = m - 1; j >= 0; --j) {
            int id;
            float Ti;
            entry<K>(kb, Tj, j, &id, &Ti);
            grad_hit<FM>(raw, P.F, id, ray, Ti, S, gO, gF, gD, go);
        }
    }
}

template <int K, int FM>
__global__ __launch_bounds__(kBlock) void k_backward(SceneView sc, RawSurfels raw, TraceParams P, int64_t R,
                                                     const float* __restrict__ ro, const float* __restrict__ rd,
                                                     OutPtrs saved, bool use_saved, GradIn gin, GradOut go, int* ovf,
                                                     int ovf_slots, float4* ck)
{
    __shared__ int lds_stack[kStackLds * kBlock];
    const int64_t gtid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t nthr = static_cast<int64_t>(gridDim.x) * kBlock;
    Stack st{lds_stack, ovf_slots > 0 ? ovf + gtid : nullptr, static_cast<int>(nthr), static_cast<int>(threadIdx.x),
             0};
    float4* myck = ck ? ck + gtid : nullptr;
    for (int64_t r = gtid; r < R; r += nthr) {
        const Ray ray = load_ray(ro, rd, r);
        bwd_one<K, FM>(sc, raw, P, ray, r, saved, use_saved, gin, go, st, myck, nthr);
    }
}

template <int K, int FM>
hipError_t launch_kf(const SceneView& sc, const RawSurfels& raw, const TraceParams& P, int64_t R, const float* ro,
                     const float* rd, const OutPtrs& saved, bool use_saved, const GradIn& gin, const GradOut& go,
                     int* ovf, int ovf_slots, float* ck, hipStream_t st)
{
    const int64_t nthr = trace_threads(R);
    k_backward<K, FM><<<static_cast<unsigned>(nthr / kBlock), kBlock, 0, st>>>(
        sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, reinterpret_cast<float4*>(ck));
    return hipGetLastError();
}

template <int K>
hipError_t launch_k(const SceneView& sc, const RawSurfels& raw, const TraceParams& P, int64_t R, const float* ro,
                    const float* rd, const OutPtrs& saved, bool use_saved, const GradIn& gin, const GradOut& go,
                    int* ovf, int ovf_slots, float* ck, hipStream_t st)
{
    if (P.F <= 4) return launch_kf<K, 4>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
    if (P.F <= 8) return launch_kf<K, 8>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
    if constexpr (K == 16 || K == 32) {
        if (P.F <= 16)
            return launch_kf<K, 16>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        if (P.F <= 64)
            return launch_kf<K, 64>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_backward(const SceneView& sc, const RawSurfels& raw, const TraceParams& P, int k, int64_t R,
                           const float* ro, const float* rd, const OutPtrs& saved, bool use_saved,
                           const GradIn& gin, const GradOut& go, int* ovf, int ovf_slots, float* ck,
                           hipStream_t st)
{
    if (R <= 0) return hipSuccess;
    switch (k) {
        case 1: return launch_k<1>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        case 2: return launch_k<2>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        case 4: return launch_k<4>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        case 8: return launch_k<8>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        case 16: return launch_k<16>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        case 32: return launch_k<32>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        case 64: return launch_k<64>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace irgs
