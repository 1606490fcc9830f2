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

constexpr int kBwdBlock = 64;    // one wave per block: one table per 64 consecutive rays
constexpr int kHashProbes = 8;
constexpr int kLdsFeat = 8;      // feature gradients pre-reduced in LDS (the rest go straight to global)
constexpr int kLdsComp = 10 + kLdsFeat;
// The LDS table's slots and the hits of a ray that use it (only its first
// hits, shared by neighbouring rays).  The table is sized so that LDS allows
// the walk's 3 waves per SIMD: 96 slots with at most 8 features staged
// (12.3 KB per one-wave block), 64 with more (at 1M surfels, F = 8: 64 slots
// and 24 near hits 19.2 ms, 96 and 32 18.2 ms, 96 and 40 18.4 ms, 104 and
// 32 18.7 ms).
template <int FM>
struct TableShape {
    static constexpr int slots = FM <= 8 ? 96 : 64;
    static constexpr int near_hits = FM <= 8 ? 32 : 24;
    static constexpr int val_row = slots + 1;
};

// Per-surfel gradient components of one hit: mu (3), raw quaternion (4),
// scales (2), opacity (1), features (F).
template <int FM>
struct HitGrad {
    float g[10 + FM];
};

// Block-local pre-reduction: rays of one surface point share most of their
// near hits, so their per-surfel gradients are summed in an LDS hash table
// (LDS float atomics) and written to global memory once per chunk of rays.
// A surfel that finds no slot within kHashProbes probes goes straight to the
// global atomics.
template <int kSlots>
struct GradAcc {
    static constexpr int kFill = kSlots * 3 / 4;  // no new keys once this many slots are taken
    static constexpr int kValRow = kSlots + 1;    // value rows padded by a word: lanes reading one slot hit different banks
    int* keys;     // kSlots, -1 = empty
    float* vals;   // [kLdsComp][kValRow]
    int* filled;   // slots taken in this chunk
    float* gbuf;   // per-surfel interleaved accumulator: gbuf[id * gs + c]
    int gs;        // stride of gbuf in floats (a multiple of 32: one 128 B line per surfel at F <= 22)
    int F;

    __device__ __forceinline__ int ncomp() const { return 10 + F; }

    // Direct accumulation of one hit (used by the re-march path).
    template <int FM>
    __device__ __forceinline__ void direct(int id, const HitGrad<FM>& h) const
    {
        float* g = gbuf + static_cast<int64_t>(id) * gs;
#pragma unroll
        for (int c = 0; c < 10 + FM; ++c)
            if (c < 10 + F && h.g[c] != 0.0f) atomicAdd(g + c, h.g[c]);
    }

    // Try the LDS table; on success the components below kLdsComp are
    // accumulated there and zeroed in h (the rest stay for the caller).
    template <int FM>
    __device__ __forceinline__ bool table(int id, HitGrad<FM>& h) const
    {
        uint32_t slot = __umulhi(static_cast<uint32_t>(id) * 2654435761u, static_cast<uint32_t>(kSlots));
        const bool may_insert = *filled < kFill;
        int found = -1;
        for (int p = 0; p < kHashProbes; ++p) {
            const int k = keys[slot];
            if (k == id) {
                found = static_cast<int>(slot);
                break;
            }
            if (k == -1) {
                if (!may_insert) break;
                const int prev = atomicCAS(&keys[slot], -1, id);
                if (prev == -1) atomicAdd(filled, 1);
                if (prev == -1 || prev == id) {
                    found = static_cast<int>(slot);
                    break;
                }
            }
            slot = slot + 1 == kSlots ? 0 : slot + 1;
        }
        if (found < 0) return false;
#pragma unroll
        for (int c = 0; c < kLdsComp && c < 10 + FM; ++c) {
            if (c < 10 + F) atomicAdd(vals + c * kValRow + found, h.g[c]);
            h.g[c] = 0.0f;
        }
        return true;
    }

    // Table to gbuf: consecutive lanes take consecutive components of one
    // entry, so each atomic instruction touches few cache lines.
    __device__ __forceinline__ void flush(int tid) const
    {
        const int nc = 10 + (F < kLdsFeat ? F : kLdsFeat);
        for (int flat = tid; flat < kSlots * nc; flat += kBwdBlock) {
            const int slot = flat / nc, c = flat - slot * nc;
            const int id = keys[slot];
            if (id < 0) continue;
            const float v = vals[c * kValRow + slot];
            if (v != 0.0f) atomicAdd(gbuf + static_cast<int64_t>(id) * gs + c, v);
        }
    }

    __device__ __forceinline__ void clear(int tid) const
    {
        if (tid == 0) *filled = 0;
        for (int i = tid; i < kSlots; i += kBwdBlock) keys[i] = -1;
        for (int i = tid; i < kLdsComp * kValRow; i += kBwdBlock) vals[i] = 0.0f;
    }
};

// Gradient of one hit.  The geometry and the chain rule are evaluated in
// FP64 from the FP32 parameters: for a grazing ray (small n.r_d) FP32
// rounding of the depth is amplified into u, v and into dtau/dmu; FP64 keeps
// every surfel's gradient at FP32 accuracy.  Only the per-surfel
// contributions are rounded to FP32 for accumulation.  The transmittance
// before the hit (Ti) is the forward pass's own.
// With SH the features are RGB coefficients: the hit's colour is recomputed
// exactly as in the forward (FP32), and the coefficient gradients are
// T alpha g_F,c Y_j(d) wherever the channel is not clamped.
// With NRM (the relighting blend) the upstream holds F feature channels and
// then 3 for the hit's normal turned to face the ray, s n with s = -1 where
// n . d > 0; the turn is decided exactly as in the forward (the FP32 frame
// of the record, the same dot product), and s T alpha g_N adds to the
// gradient of n, which the rotation chain below carries to the quaternion.
template <int FM, int FU, bool SH, bool NRM = false>
__device__ __forceinline__ void grad_hit(const RawSurfels& raw, const TraceParams& P, int id, const Ray& ray,
                                         float Ti_f, float& S_f, float gO, const float* gF, float gD,
                                         HitGrad<FM>& h)
{
    const int F = P.F;
    const int64_t i = id;
    const float* row = raw.pk + i * raw.ps;  // the packed copy of surfel i's parameters
    const float4 mo = *reinterpret_cast<const float4*>(row);
    const float4 qf = *reinterpret_cast<const float4*>(row + 4);
    const float2 sc = *reinterpret_cast<const float2*>(row + 8);
    const double mx = mo.x, my = mo.y, mz = mo.z;
    const double su = sc.x, sv = sc.y;
    const double o = mo.w;
    const double qn = sqrt(double(qf.x) * qf.x + double(qf.y) * qf.y + double(qf.z) * qf.z + double(qf.w) * qf.w);
    const double inv = 1.0 / qn;
    const double w = qf.x * inv, x = qf.y * inv, y = qf.z * inv, z = qf.w * inv;
    const double tu0 = 1.0 - 2.0 * (y * y + z * z), tu1 = 2.0 * (x * y + w * z), tu2 = 2.0 * (x * z - w * y);
    const double tv0 = 2.0 * (x * y - w * z), tv1 = 1.0 - 2.0 * (x * x + z * z), tv2 = 2.0 * (y * z + w * x);
    const double n0 = 2.0 * (x * z + w * y), n1 = 2.0 * (y * z - w * x), n2 = 1.0 - 2.0 * (x * x + y * y);
    const double dx_ = ray.dx, dy_ = ray.dy, dz_ = ray.dz;
    const double wx = mx - ray.ox, wy = my - ray.oy, wz = mz - ray.oz;
    const double den = n0 * dx_ + n1 * dy_ + n2 * dz_;
    const double tau = (n0 * wx + n1 * wy + n2 * wz) / den;
    const double px = tau * dx_ - wx, py = tau * dy_ - wy, pz = tau * dz_ - wz;
    const double u = (px * tu0 + py * tu1 + pz * tu2) / su;
    const double v = (px * tv0 + py * tv1 + pz * tv2) / sv;
    const double G = exp(-0.5 * (u * u + v * v));
    const double alpha = o * G;
    const double Ti = Ti_f;
    const double S = S_f;

    double c = gO + gD * tau;
    const float* f = row + 12;
    const double wgt = Ti * alpha;
    if constexpr (SH) {
        float Y[16], col[3];
        sh_basis(ray.dx, ray.dy, ray.dz, P.sh_deg, Y);
        sh_raw(f, P.sh_deg, Y, col);
        const int nb = (P.sh_deg + 1) * (P.sh_deg + 1);
        double gc[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            c += double(gF[ch]) * fmaxf(col[ch], 0.0f);
            gc[ch] = col[ch] > 0.0f ? wgt * gF[ch] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                if (3 * j + ch < FM) h.g[10 + 3 * j + ch] = j < nb ? static_cast<float>(gc[ch] * Y[j]) : 0.0f;
#pragma unroll
        for (int k = 48; k < FM; ++k) h.g[10 + k] = 0.0f;
    } else {
        static_assert(SH || FU == FM, "plain features: one upstream channel per feature");
#pragma unroll
        for (int k = 0; k < FM; ++k) {
            const float fv = k < F ? f[k] : 0.0f;
            c += double(gF[k]) * fv;
        }
#pragma unroll
        for (int k = 0; k < FM; ++k) h.g[10 + k] = (!NRM || k < F) ? static_cast<float>(wgt * gF[k]) : 0.0f;
    }
    double sN = 0.0, gN0 = 0.0, gN1 = 0.0, gN2 = 0.0;  // normal channels: turn and upstream
    if constexpr (NRM) {
        float tf[3], vf[3], nf[3];
        quat_frame(qf, tf, vf, nf);
        sN = dot3(nf[0], nf[1], nf[2], ray.dx, ray.dy, ray.dz) > 0.0f ? -1.0 : 1.0;
#pragma unroll
        for (int k = 0; k < FM; ++k) {
            gN0 += k == F ? double(gF[k]) : 0.0;
            gN1 += k == F + 1 ? double(gF[k]) : 0.0;
            gN2 += k == F + 2 ? double(gF[k]) : 0.0;
        }
        c += sN * (gN0 * n0 + gN1 * n1 + gN2 * n2);
    }
    const double dA = Ti * (c - S);
    S_f = static_cast<float>(alpha * c + (1.0 - alpha) * S);

    h.g[9] = static_cast<float>(dA * G);

    const double gu = -dA * alpha * u;
    const double gv = -dA * alpha * v;
    h.g[7] = static_cast<float>(-gu * u / su);
    h.g[8] = static_cast<float>(-gv * v / sv);
    // p - mu = tau d - w;  du/d(p-mu) = t_u / s_u
    const double au = gu / su, av = gv / sv;
    const double gpx = au * tu0 + av * tv0, gpy = au * tu1 + av * tv1, gpz = au * tu2 + av * tv2;
    const double gtau = wgt * gD + gpx * dx_ + gpy * dy_ + gpz * dz_;
    const double gt_den = gtau / den;
    h.g[0] = static_cast<float>(gt_den * n0 - gpx);
    h.g[1] = static_cast<float>(gt_den * n1 - gpy);
    h.g[2] = static_cast<float>(gt_den * n2 - gpz);
    // dtau/dn = -(p - mu) / den;  du/dt_u = (p - mu) / s_u; the normal
    // channels add s T alpha g_N
    const double wn = wgt * sN;
    const double gn0 = -gt_den * px + wn * gN0, gn1 = -gt_den * py + wn * gN1, gn2 = -gt_den * pz + wn * gN2;
    const double gu0 = au * px, gu1 = au * py, gu2 = au * pz;
    const double gv0 = av * px, gv1 = av * py, gv2 = av * pz;
    // derivatives of the rotation columns with respect to (w, x, y, z)
    const double dw = 2.0 * (z * gu1 - y * gu2 - z * gv0 + x * gv2 + y * gn0 - x * gn1);
    const double dx = 2.0 * (y * gu1 + z * gu2 + y * gv0 - 2.0 * x * gv1 + w * gv2 + z * gn0 - w * gn1 - 2.0 * x * gn2);
    const double dy = 2.0 * (-2.0 * y * gu0 + x * gu1 - w * gu2 + x * gv0 + z * gv2 + w * gn0 + z * gn1 - 2.0 * y * gn2);
    const double dz = 2.0 * (-2.0 * z * gu0 + w * gu1 + x * gu2 - w * gv0 - 2.0 * z * gv1 + y * gv2 + x * gn0 + y * gn1);
    const double proj = w * dw + x * dx + y * dy + z * dz;
    h.g[3] = static_cast<float>((dw - w * proj) * inv);
    h.g[4] = static_cast<float>((dx - x * proj) * inv);
    h.g[5] = static_cast<float>((dy - y * proj) * inv);
    h.g[6] = static_cast<float>((dz - z * proj) * inv);
}

// alpha of the k-buffer entry at leaf position pos (the same arithmetic as
// the forward composite, so T is reproduced bit for bit).
__device__ __forceinline__ float entry_alpha(const SceneView& sc, const Ray& ray, int pos)
{
    const SurfelRec s = load_rec(sc.rec, pos);
    float tau, rho2;
    plane_hit(s, ray, &tau, &rho2);
    return alpha_of(s, rho2);
}

template <int K>
__device__ __forceinline__ void entry(const KBuf<K>& kb, const float* Tj, int j, int* pos, float* T)
{
    int ri = 0;
    float rt = 0.0f;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        ri = q == j ? kb.pos(q) : ri;
        rt = q == j ? Tj[q] : rt;
    }
    *pos = ri;
    *T = rt;
}

template <int FU>
struct LaneUp {
    float gO, gD, gF[FU];
    bool any;
};

// Upstream gradients of ray r; FO = composited channels (the g_feat stride).
template <int FU>
__device__ __forceinline__ LaneUp<FU> load_upstream(const GradIn& gin, int64_t r, int FO)
{
    const int F = FO;
    LaneUp<FU> u;
    u.gO = gin.gO ? gin.gO[r] : 0.0f;
    u.gD = gin.gD ? gin.gD[r] : 0.0f;
    u.any = u.gO != 0.0f || u.gD != 0.0f;
#pragma unroll
    for (int k = 0; k < FU; ++k) {
        u.gF[k] = (gin.gF && k < F) ? gin.gF[r * F + k] : 0.0f;
        u.any = u.any || u.gF[k] != 0.0f;
    }
    return u;
}

// Re-march one ray (no saved list, or more hits than were saved).  Pass 1
// marches the k-buffer rounds again (the forward's arithmetic, so T is
// reproduced bit for bit), recording each composited hit (id and the
// transmittance before it) in the lane's private list while it fits, and
// the state at the start of rounds as checkpoints.  Pass 2 walks the
// private list back to front or, for a ray longer than the list,
// re-collects the rounds last to first from the nearest checkpoint.
// Checkpoints are kept for every stride-th round: once all kBwdCheckpoints
// are taken every other one is dropped and the stride doubles, so pass 2
// re-collects at most stride - 1 extra rounds per round (instead of
// re-marching from the last checkpoint for every round past them).
template <int K, int FM, int FU, bool SH, bool NRM, class Acc>
__device__ __forceinline__ void bwd_remarch(const SceneView& sc, const RawSurfels& raw, const TraceParams& P,
                                            const Ray& ray, const LaneUp<FU>& up, const Acc& acc, Stack& st,
                                            float4* ck, int64_t ck_stride, int* pid, float* pT)
{
    float S = 0.0f;
    Counters ct;
    const SlabRay q = slab_ray(ray);
    uint64_t after = 0;
    float T = 1.0f;
    int nh = 0;
    int rounds = 0;
    int stride = 1;  // a power of two: checkpoint i holds the start of round i * stride
    int nck = 0;
    bool done = false;
    while (!done) {
        if ((rounds & (stride - 1)) == 0) {
            if (nck == kBwdCheckpoints) {
                for (int i = 1; i < kBwdCheckpoints / 2; ++i) ck[i * ck_stride] = ck[2 * i * ck_stride];
                nck = kBwdCheckpoints / 2;
                stride *= 2;
            }
            if ((rounds & (stride - 1)) == 0)
                ck[(nck++) * ck_stride] = make_float4(__uint_as_float(static_cast<uint32_t>(after >> 32)),
                                                      __uint_as_float(static_cast<uint32_t>(after)), T,
                                                      __int_as_float(nh));
        }
        KBuf<K> kb;
        kb.clear();
        collect_bvh<K>(kb, sc, ray, q, P.t_min, P.t_max, after, st, ct);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j < kb.cnt && !done) {
                const int pos = kb.pos(j);
                if (nh < kRemarchList) {
                    pid[nh] = __float_as_int(sc.rec[pos].c.w);
                    pT[nh] = T;
                }
                T = T * (1.0f - entry_alpha(sc, ray, pos));
                ++nh;
                if (T < P.T_min) done = true;
            }
        }
        if (kb.cnt < K)
            done = true;
        else
            after = kb.last();
        ++rounds;
    }
    const int total = nh;
    if (total <= kRemarchList) {
        for (int h = total - 1; h >= 0; --h) {
            const int id = pid[h];
            HitGrad<FM> hg;
            grad_hit<FM, FU, SH, NRM>(raw, P, id, ray, pT[h], S, up.gO, up.gF, up.gD, hg);
            acc.template direct<FM>(id, hg);
        }
        return;
    }
    for (int rr = rounds - 1; rr >= 0; --rr) {
        const int base = rr / stride;
        float4 c4 = ck[base * ck_stride];
        after = (static_cast<uint64_t>(__float_as_uint(c4.x)) << 32) | __float_as_uint(c4.y);
        T = c4.z;
        int nb = __float_as_int(c4.w);
        KBuf<K> kb;
        for (int adv = base * stride; adv < rr; ++adv) {  // rounds between the checkpoint and rr
            kb.clear();
            collect_bvh<K>(kb, sc, ray, q, P.t_min, P.t_max, after, st, ct);
#pragma unroll
            for (int j = 0; j < K; ++j) T = j < kb.cnt ? T * (1.0f - entry_alpha(sc, ray, kb.pos(j))) : T;
            nb += kb.cnt;
            after = kb.last();
        }
        kb.clear();
        collect_bvh<K>(kb, sc, ray, q, P.t_min, P.t_max, after, st, ct);
        const int m = min(kb.cnt, total - nb);
        float Tj[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            Tj[j] = T;
            T = j < m ? T * (1.0f - entry_alpha(sc, ray, kb.pos(j))) : T;
        }
        for (int j = m - 1; j >= 0; --j) {
            int pos;
            float Ti;
            entry<K>(kb, Tj, j, &pos, &Ti);
            const int id = __float_as_int(sc.rec[pos].c.w);
            HitGrad<FM> h;
            grad_hit<FM, FU, SH, NRM>(raw, P, id, ray, Ti, S, up.gO, up.gF, up.gD, h);
            acc.template direct<FM>(id, h);
        }
    }
}

// RM = false: rays whose stored hit list is complete, walked back to front
// (the re-march code is compiled out, which keeps the register count low);
// RM = true: the other rays (no stored lists, or a list cut at H_cap),
// re-marched.  A backward runs the first over every ray when lists are
// stored, then the second.
// The walk over stored lists is latency-bound: it is held to the registers
// of 3 waves per SIMD (no spills for F <= 16), and the LDS table is sized so
// that LDS allows as many (measured at 1M surfels, F = 8: 256 slots and 2
// waves 33.3 ms; 64 slots and 3 waves 24.5 ms; no table 28.0 ms).
template <int K, int FM, int FU, bool SH, bool NRM, bool RM>
__global__ __launch_bounds__(kBwdBlock) __attribute__((amdgpu_waves_per_eu(!RM && FM <= 16 ? 3 : 1)))
void k_backward(SceneView sc, RawSurfels raw, TraceParams P, int64_t R,
                                                        const float* __restrict__ ro, const float* __restrict__ rd,
                                                        OutPtrs saved, bool use_saved, GradIn gin, float* gbuf,
                                                        int gs, int* ovf, int ovf_slots, float4* ck, int* plist,
                                                        unsigned long long* next_chunk,
                                                        const uint32_t* __restrict__ order, int* rm_list,
                                                        unsigned long long* rm_count)
{
    using Shape = TableShape<FM>;
    __shared__ int hkeys[Shape::slots];
    __shared__ float hvals[kLdsComp * Shape::val_row];
    __shared__ int hfilled;
    __shared__ long long claimed;
    __shared__ int stage_id[kBwdBlock];
    // staged gradients, one row per component; rows padded by one word so
    // that the scatter's reads (consecutive lanes: consecutive components
    // of one hit) fall in different banks
    constexpr int kRow = kBwdBlock + 1;
    __shared__ float stage[(10 + FM) * kRow];
    const int tid = threadIdx.x;
    const int64_t gtid = static_cast<int64_t>(blockIdx.x) * kBwdBlock + tid;
    const int64_t nthr = static_cast<int64_t>(gridDim.x) * kBwdBlock;
    // the re-march stack lives entirely in the global area (0 LDS slots)
    Stack st{nullptr, as_glb(ovf_slots > 0 ? ovf + gtid : nullptr), static_cast<int>(nthr), tid, 0, 0};
    // re-march lanes (gtid < kRemarchThreads): checkpoints slot-major, the
    // private list contiguous per lane (ids, then T)
    float4* myck = RM ? ck + gtid : nullptr;
    int* my_ids = RM ? plist + gtid * (2 * kRemarchList) : nullptr;
    float* my_T = RM ? reinterpret_cast<float*>(my_ids + kRemarchList) : nullptr;
    const GradAcc<Shape::slots> acc{hkeys, hvals, &hfilled, gbuf, gs, P.F};
    const int nc = 10 + P.F;
    // The scatter below hands lane l the elements l, l + 64, ... of a
    // block's hits x components: its first (hit, component) pair and the step
    // between pairs, so that no element needs an integer division.
    const int sc_h0 = tid / nc, sc_c0 = tid - sc_h0 * nc;
    const int sc_dh = kBwdBlock / nc, sc_dc = kBwdBlock - sc_dh * nc;
    // With stored lists the walk instance collects the rays it leaves (lists
    // cut at H_cap) in rm_list; the re-march instance then claims chunks of
    // that list only, instead of scanning every ray.
    const bool listed = RM && use_saved && rm_list;
    const int64_t Rw = listed ? static_cast<int64_t>(*rm_count) : R;
    const int64_t chunks = (Rw + kBwdBlock - 1) / kBwdBlock;
    // chunks of kBwdBlock rays are claimed from a global counter as blocks
    // free up, so the launch drains evenly
    while (true) {
        if (tid == 0) claimed = static_cast<long long>(atomicAdd(next_chunk, 1ull));
        // the re-march accumulates with direct atomics only: its instance
        // neither clears nor flushes the table (most of its chunks hold no
        // ray to re-march, and the table pass would be its whole cost)
        if constexpr (!RM) acc.clear(tid);
        __syncthreads();
        const int64_t c = claimed;
        if (c >= chunks) break;
        // a chunk takes the next 64 rays of `order` or of the launch
        const int64_t slot = c * kBwdBlock + tid;
        const int64_t r = listed ? (slot < Rw ? static_cast<int64_t>(rm_list[slot]) : R)
                                 : (slot < R && order ? static_cast<int64_t>(order[slot]) : slot);
        Ray ray{};
        LaneUp<FU> up{};
        int nh = 0;
        bool stored = false;
        bool cut = false;  // walk instance: a ray left to the re-march
        if (r < R) {
            // each instance loads only the rays it owns
            const int nh_saved = saved.n_hits ? saved.n_hits[r] : -1;
            const bool complete = use_saved && nh_saved > 0 && nh_saved <= saved.H_cap;
            cut = !RM && !complete && nh_saved != 0;
            if (RM ? (!complete && nh_saved != 0) : complete) {
                ray = load_ray(ro, rd, r);
                up = load_upstream<FU>(gin, r, SH ? 3 : (NRM ? P.F + 3 : P.F));
                if (up.any && sc.n > 0 && ray_valid(ray)) {
                    if constexpr (!RM) {
                        stored = true;
                        nh = nh_saved;
                    } else {
                        bwd_remarch<K, FM, FU, SH, NRM>(sc, raw, P, ray, up, acc, st, myck, nthr, my_ids, my_T);
                    }
                }
            }
        }
        if constexpr (!RM) {
            if (rm_list) {  // one atomic per wave for the rays it leaves
                const uint64_t m = __ballot(cut);
                if (m) {
                    const int rank = __popcll(m & __lanemask_lt());
                    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
                    unsigned long long base = 0;
                    if (cut && rank == 0) base = atomicAdd(rm_count, static_cast<unsigned long long>(__popcll(m)));
                    base = __shfl(base, leader);
                    if (cut) rm_list[base + rank] = static_cast<int>(r);
                }
            }
        }
        // Saved lists: all lanes step together, back to front, so that the
        // wave can hand every hit's gradient to the scatter below.
        int hmax = nh;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) hmax = max(hmax, __shfl_xor(hmax, off));
        const int* ids = saved.hit_ids + (stored ? r * saved.H_cap : 0);
        const float* Ts = saved.hit_T + (stored ? r * saved.H_cap : 0);
        float S = 0.0f;
        for (int step = 0; step < hmax; ++step) {
            const int h = nh - 1 - step;
            const bool valid = stored && h >= 0;
            HitGrad<FM> hg;
            int id = -1;
            if (valid) {
                id = ids[h];
                grad_hit<FM, FU, SH, NRM>(raw, P, id, ray, Ts[h], S, up.gO, up.gF, up.gD, hg);
                if (h < Shape::near_hits) acc.template table<FM>(id, hg);
            } else {
#pragma unroll
                for (int k = 0; k < 10 + FM; ++k) hg.g[k] = 0.0f;
            }
            // What the table did not take goes to global memory; a step whose
            // hits the table took whole (a block is one wave: the branch is
            // uniform) skips the staging.
            bool left = false;
#pragma unroll
            for (int k = 0; k < 10 + FM; ++k) left = left || hg.g[k] != 0.0f;
            const uint64_t lm = __ballot(left);
            if (lm) {
                // only the hits with something left are staged, packed into
                // the first rows
                const int n_left = __popcll(lm);
                if (left) {
                    const int row = __popcll(lm & __lanemask_lt());
                    stage_id[row] = id;
#pragma unroll
                    for (int k = 0; k < 10 + FM; ++k) stage[k * kRow + row] = hg.g[k];
                }
                __syncthreads();
                // Transposed scatter: lane l takes component (q*64 + l) % nc
                // of staged hit (q*64 + l) / nc, so consecutive lanes add
                // consecutive components of one surfel -- a few cache lines per
                // instruction.
                for (int hit = sc_h0, comp = sc_c0; hit < n_left;) {
                    const int sid = stage_id[hit];
                    const float v = stage[comp * kRow + hit];
                    if (sid >= 0 && v != 0.0f) atomicAdd(gbuf + static_cast<int64_t>(sid) * gs + comp, v);
                    hit += sc_dh;
                    comp += sc_dc;
                    if (comp >= nc) {
                        comp -= nc;
                        ++hit;
                    }
                }
                __syncthreads();
            }
        }
        if constexpr (!RM) {
            __syncthreads();
            acc.flush(tid);
        }
        __syncthreads();
    }
}

// Sort key of a ray for the backward's chunks: the Morton code (10 bits per
// axis) of its mean hit point ro + (D / O) rd inside the root's box; a ray
// without a hit sorts last.
__global__ void k_ray_keys(int64_t R, const float* __restrict__ ro, const float* __restrict__ rd,
                           const float* __restrict__ O, const float* __restrict__ D, const WideNode* __restrict__ root,
                           uint64_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (r >= R) return;
    float lo[3], hi[3];
    root_box(root, lo, hi);
    uint64_t key = 0xffffffffull;
    const float o = O[r];
    if (o > 0.0f && lo[0] <= hi[0]) {
        const float t = D[r] / o;
        const float x[3] = {fmaf(t, rd[3 * r], ro[3 * r]), fmaf(t, rd[3 * r + 1], ro[3 * r + 1]),
                            fmaf(t, rd[3 * r + 2], ro[3 * r + 2])};
        key = morton30(x, lo, hi);
    }
    keys[r] = key;
    vals[r] = static_cast<uint32_t>(r);
}

// One packed row per surfel (see RawSurfels): consecutive threads take
// consecutive surfels and write their rows whole.
__global__ void k_pack(int64_t n, int F, int ps, const float* __restrict__ mu, const float* __restrict__ quat,
                       const float* __restrict__ scale, const float* __restrict__ opac,
                       const float* __restrict__ feat, float* __restrict__ pk)
{
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    float4* row = reinterpret_cast<float4*>(pk + i * ps);
    row[0] = make_float4(mu[3 * i], mu[3 * i + 1], mu[3 * i + 2], opac[i]);
    row[1] = *reinterpret_cast<const float4*>(quat + 4 * i);
    const float2 s = *reinterpret_cast<const float2*>(scale + 2 * i);
    row[2] = make_float4(s.x, s.y, 0.0f, 0.0f);
    float* f = pk + i * ps + 12;
    for (int c = 0; c < F; ++c) f[c] = feat[i * F + c];
}

// gbuf (interleaved per surfel) added into the caller's gradient arrays.
__global__ void k_grad_out(int64_t n, int F, int gs, const float* __restrict__ gbuf, GradOut go)
{
    const int nc = 10 + F;
    for (int64_t flat = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; flat < n * nc;
         flat += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = flat / nc;
        const int c = static_cast<int>(flat - i * nc);
        const float v = gbuf[i * gs + c];
        if (v == 0.0f) continue;
        if (c < 3) {
            if (go.mu) go.mu[3 * i + c] += v;
        } else if (c < 7) {
            if (go.quat) go.quat[4 * i + c - 3] += v;
        } else if (c < 9) {
            if (go.scale) go.scale[2 * i + c - 7] += v;
        } else if (c == 9) {
            if (go.opac) go.opac[i] += v;
        } else {
            if (go.feat) go.feat[i * F + c - 10] += v;
        }
    }
}

template <int K, int FM, int FU, bool SH, bool NRM = false>
hipError_t launch_kf(const SceneView& sc, const RawSurfels& raw, const TraceParams& P, int64_t R, const float* ro,
                     const float* rd, const OutPtrs& saved, bool use_saved, const GradIn& gin, const GradOut& go,
                     int* ovf, int ovf_slots, float* ck, hipStream_t st)
{
    const int64_t nthr = trace_threads(R);
    const int64_t rm_thr = remarch_threads(R);
    const int gs = grad_stride(P.F);
    int* plist = reinterpret_cast<int*>(ck + static_cast<size_t>(rm_thr) * kBwdCheckpoints * 4);
    float* gbuf = ck + remarch_words(R);
    unsigned long long* next_chunk =
        reinterpret_cast<unsigned long long*>(gbuf + static_cast<size_t>(sc.n) * gs);
    unsigned long long* rm_count = next_chunk + 2;  // zeroed with the claim counters
    char* after_claims = reinterpret_cast<char*>(next_chunk) + kBwdClaimWords * sizeof(float);
    int* rm_list = reinterpret_cast<int*>((reinterpret_cast<uintptr_t>(after_claims) + 255) & ~static_cast<uintptr_t>(255));
    // zero the accumulator and the claim counter behind it
    hipError_t e = fill_u32(gbuf, static_cast<int64_t>(sc.n) * gs + kBwdClaimWords, 0u, st);
    if (e != hipSuccess) return e;
    // Gradients wider than the LDS table (SH coefficients, F > 8) send most
    // components straight to global atomics; their chunks then take rays in
    // the order of where they land (stored lists with O and D), so that the
    // surfels a block updates stay in L2 (at 1M surfels, SH degree 3: 95.6
    // -> 81.6 ms; for F <= 8 the sort costs more than it saves).
    const uint32_t* order = nullptr;
    // (the condition on P.F is the one the scratch is sized by)
    if (P.F > kLdsFeat && use_saved && saved.O && saved.D && ray_sort_words(R) > 0 && sc.n > 0) {
        char* p = reinterpret_cast<char*>(rm_list + R);
        p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 255) & ~static_cast<uintptr_t>(255));
        uint64_t* k0 = reinterpret_cast<uint64_t*>(p);
        uint64_t* k1 = k0 + R;
        uint32_t* v0 = reinterpret_cast<uint32_t*>(k1 + R);
        uint32_t* v1 = v0 + R;
        uint32_t* counts = v1 + R;
        k_ray_keys<<<static_cast<unsigned>((R + 255) / 256), 256, 0, st>>>(R, ro, rd, saved.O, saved.D, sc.wnodes, k0,
                                                                             v0);
        e = hipGetLastError();
        if (e == hipSuccess) e = sort_pairs(static_cast<int>(R), k0, v0, k1, v1, counts, 4, st);
        if (e != hipSuccess) return e;
        order = v0;
    }
    if (use_saved) {
        const unsigned grid =
            persistent_grid(nthr / kBwdBlock, resident_blocks(k_backward<K, FM, FU, SH, NRM, false>, kBwdBlock));
        k_backward<K, FM, FU, SH, NRM, false><<<grid, kBwdBlock, 0, st>>>(sc, raw, P, R, ro, rd, saved, use_saved, gin,
                                                                     gbuf, gs, ovf, ovf_slots,
                                                                     reinterpret_cast<float4*>(ck), plist, next_chunk,
                                                                     order, rm_list, rm_count);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // rays without a complete stored list (all of them without stored lists)
    // (at most rm_thr lanes: the checkpoints and private lists are sized for them)
    const unsigned grid =
        persistent_grid(rm_thr / kBwdBlock, resident_blocks(k_backward<K, FM, FU, SH, NRM, true>, kBwdBlock));
    k_backward<K, FM, FU, SH, NRM, true><<<grid, kBwdBlock, 0, st>>>(sc, raw, P, R, ro, rd, saved, use_saved, gin, gbuf,
                                                                gs, ovf, ovf_slots, reinterpret_cast<float4*>(ck),
                                                                plist, next_chunk + 1, nullptr, rm_list, rm_count);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t work = static_cast<int64_t>(sc.n) * (10 + P.F);
    const int blocks = static_cast<int>(work < 2048 * 256 ? (work + 255) / 256 : 2048);
    k_grad_out<<<blocks > 0 ? blocks : 1, 256, 0, st>>>(sc.n, P.F, gs, gbuf, go);
    return hipGetLastError();
}

template <int K>
hipError_t launch_k(const SceneView& sc, const RawSurfels& raw, const TraceParams& P, int64_t R, const float* ro,
                    const float* rd, const OutPtrs& saved, bool use_saved, const GradIn& gin, const GradOut& go,
                    int* ovf, int ovf_slots, float* ck, hipStream_t st)
{
    if constexpr (K == 16 || K == 32 || K == 64) {  // SH: 48 coefficient gradients, 3 upstream channels
        if (P.sh_deg >= 0)
            return launch_kf<K, 48, 4, true>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        // relighting blend: F <= 5 features and 3 normal channels upstream
        if (P.normals && P.F <= 5)
            return launch_kf<K, 8, 8, false, true>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots,
                                                   ck, st);
    }
    if (P.sh_deg >= 0 || P.normals) return hipErrorInvalidValue;
    if (P.F <= 4)
        return launch_kf<K, 4, 4, false>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
    if (P.F <= 8)
        return launch_kf<K, 8, 8, false>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
    if constexpr (K == 16 || K == 32) {
        if (P.F <= 16)
            return launch_kf<K, 16, 16, false>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
        if (P.F <= 64)
            return launch_kf<K, 64, 64, false>(sc, raw, P, R, ro, rd, saved, use_saved, gin, go, ovf, ovf_slots, ck, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t pack_surfels(const RawSurfels& raw, int64_t n, int F, float* pk, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_pack<<<static_cast<unsigned>((n + 255) / 256), 256, 0, st>>>(n, F, pack_stride(F), raw.mu, raw.quat, raw.scale,
                                                                   raw.opac, raw.feat, pk);
    return hipGetLastError();
}

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
