// Monte Carlo rendering-equation consumer of the trace (Sec. 3.3,
// "Rendering").  Per pixel (surface point x, normal n, view direction w_o,
// albedo a, roughness r) N = S_t * S_p incident directions are sampled by
// stratified uniform hemisphere sampling, traced, and combined as Eq. 15:
//
//     c = 2 pi / N  sum_i (f_d + f_s(w_i)) L_i (w_i . n)
//     L_i = V_i L_dir(w_i) + L_ind,i,   V_i = 1 - O_i        (Eq. 13-14)
//     f_d = a / pi,  f_s = D F G / (4 (w_i . n)(w_o . n))    (Eq. 4)
//
// where O_i and L_ind,i are the opacity and the composited colour of the
// trace.  Readings of the terms the paper only names: D is GGX with
// alpha = r^2, F is Schlick with F0 = 0.04 (dielectric), G is Smith with the
// Schlick-GGX G1 and k = (r + 1)^2 / 8; the two cosines enter G and the
// denominator clamped below at 1e-4; L_dir is the nearest texel of an RGB
// cubemap (faces +x, -x, +y, -y, +z, -z, OpenGL face coordinates); the
// sampling frame is the branchless orthonormal basis of Duff et al. (2017).
// With another sampling density (the relighting variant draws directions by
// the sky's intensity) each sample carries its own weight 1 / (N pdf) in
// place of 2 pi / N.
#include <hip/hip_runtime.h>

#include "irgs_internal.hpp"

namespace irgs {

namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kF0 = 0.04f;
constexpr float kEpsCos = 1e-4f;
constexpr int kShadeBlock = 256;  // 4 pixels per block, one wave each

// Orthonormal basis (t1, t2) completing the unit normal n (Duff et al. 2017).
__device__ __forceinline__ void onb(float nx, float ny, float nz, float* t1, float* t2)
{
    const float sign = nz >= 0.0f ? 1.0f : -1.0f;
    const float a = -1.0f / (sign + nz);
    const float b = nx * ny * a;
    t1[0] = 1.0f + sign * nx * nx * a;
    t1[1] = sign * b;
    t1[2] = -sign * nx;
    t2[0] = b;
    t2[1] = sign + ny * ny * a;
    t2[2] = -ny;
}

__global__ void k_mc_rays(int64_t P, int St, int Sp, const float* __restrict__ x, const float* __restrict__ n,
                          const float* __restrict__ u, float offset, float* __restrict__ ro, float* __restrict__ rd)
{
    const int N = St * Sp;
    const int64_t total = P * N;
    for (int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; r < total;
         r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t p = r / N;
        const int i = static_cast<int>(r - p * N);
        const int s = i / Sp, t = i - s * Sp;
        const float nx = n[3 * p], ny = n[3 * p + 1], nz = n[3 * p + 2];
        const float ct = (static_cast<float>(s) + u[2 * r]) / static_cast<float>(St);
        const float phi = 2.0f * kPi * (static_cast<float>(t) + u[2 * r + 1]) / static_cast<float>(Sp);
        const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
        float sp, cp;
        sincosf(phi, &sp, &cp);
        float t1[3], t2[3];
        onb(nx, ny, nz, t1, t2);
        const float lx = st * cp, ly = st * sp;
        rd[3 * r] = lx * t1[0] + ly * t2[0] + ct * nx;
        rd[3 * r + 1] = lx * t1[1] + ly * t2[1] + ct * ny;
        rd[3 * r + 2] = lx * t1[2] + ly * t2[2] + ct * nz;
        ro[3 * r] = fmaf(offset, nx, x[3 * p]);
        ro[3 * r + 1] = fmaf(offset, ny, x[3 * p + 1]);
        ro[3 * r + 2] = fmaf(offset, nz, x[3 * p + 2]);
    }
}

// Flat index of the nearest cubemap texel of direction d (E x E faces).
__device__ __forceinline__ int cube_texel(float x, float y, float z, int E)
{
    const float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    int face;
    float s, t, m;
    if (ax >= ay && ax >= az) {
        m = ax;
        face = x >= 0.0f ? 0 : 1;
        s = x >= 0.0f ? -z : z;
        t = -y;
    } else if (ay >= az) {
        m = ay;
        face = y >= 0.0f ? 2 : 3;
        s = x;
        t = y >= 0.0f ? z : -z;
    } else {
        m = az;
        face = z >= 0.0f ? 4 : 5;
        s = z >= 0.0f ? x : -x;
        t = -y;
    }
    s /= m;
    t /= m;
    const int col = min(max(static_cast<int>(floorf((s + 1.0f) * E * 0.5f)), 0), E - 1);
    const int row = min(max(static_cast<int>(floorf((t + 1.0f) * E * 0.5f)), 0), E - 1);
    return (face * E + row) * E + col;
}

// Specular lobe of one sample and, optionally, its derivative in r.
struct Spec {
    float fs, ndl, dfs_dr;
};

template <bool DERIV>
__device__ __forceinline__ Spec spec(const float* n, const float* wo, float ndv, const float* wi, float r)
{
    float h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    const float hn = 1.0f / sqrtf(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    h[0] *= hn, h[1] *= hn, h[2] *= hn;
    Spec o;
    o.ndl = wi[0] * n[0] + wi[1] * n[1] + wi[2] * n[2];
    const float ndh = h[0] * n[0] + h[1] * n[1] + h[2] * n[2];
    const float vdh = h[0] * wo[0] + h[1] * wo[1] + h[2] * wo[2];
    const float l = fmaxf(o.ndl, kEpsCos), v = fmaxf(ndv, kEpsCos);
    const float a2 = (r * r) * (r * r);
    // q = (n.h)^2 (alpha^2 - 1) + 1 written as |n x h|^2 + (n.h)^2 alpha^2: the
    // same value without the cancellation of 1 - (n.h)^2 near the mirror
    // direction, where a small roughness makes D peak at 1 / (pi alpha^2)
    const float cx = n[1] * h[2] - n[2] * h[1], cy = n[2] * h[0] - n[0] * h[2], cz = n[0] * h[1] - n[1] * h[0];
    const float s2 = cx * cx + cy * cy + cz * cz;
    const float q = fmaf(ndh * ndh, a2, s2);
    const float D = a2 / (kPi * q * q);
    const float om = 1.0f - vdh;
    const float om2 = om * om;
    const float F = kF0 + (1.0f - kF0) * (om2 * om2 * om);
    const float k = (r + 1.0f) * (r + 1.0f) * 0.125f;
    const float dl = l * (1.0f - k) + k, dv = v * (1.0f - k) + k;
    const float G1l = l / dl, G1v = v / dv;
    const float G = G1l * G1v;
    const float inv4 = 1.0f / (4.0f * l * v);
    o.fs = D * F * G * inv4;
    o.dfs_dr = 0.0f;
    if (DERIV) {
        const float dD_da2 = (s2 - a2 * ndh * ndh) / (kPi * q * q * q);  // (q - 2 a2 (n.h)^2) / (pi q^3)
        const float dD = dD_da2 * 4.0f * r * r * r;
        const float dG1l = -l * (1.0f - l) / (dl * dl), dG1v = -v * (1.0f - v) / (dv * dv);
        const float dG = (dG1l * G1v + G1l * dG1v) * (r + 1.0f) * 0.25f;
        o.dfs_dr = (dD * G + D * dG) * F * inv4;
    }
    return o;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ __launch_bounds__(kShadeBlock) void k_mc_shade(ShadeArgs a, float* __restrict__ c)
{
    const int lane = threadIdx.x & 63;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * (kShadeBlock / 64) + (threadIdx.x >> 6);
    if (p >= a.P) return;  // whole waves leave together
    const float n[3] = {a.n[3 * p], a.n[3 * p + 1], a.n[3 * p + 2]};
    const float wo[3] = {a.wo[3 * p], a.wo[3 * p + 1], a.wo[3 * p + 2]};
    const float ndv = n[0] * wo[0] + n[1] * wo[1] + n[2] * wo[2];
    const float r = a.rough[p];
    float s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0};  // sum L_i cos, sum f_s L_i cos
    for (int i = lane; i < a.N; i += 64) {
        const int64_t ri = p * a.N + i;
        const float wi[3] = {a.wi[3 * ri], a.wi[3 * ri + 1], a.wi[3 * ri + 2]};
        const Spec sp = spec<false>(n, wo, ndv, wi, r);
        const float* L = a.env + 3 * static_cast<int64_t>(cube_texel(wi[0], wi[1], wi[2], a.E));
        const float V = 1.0f - a.O[ri];
        const float cw = a.wgt ? sp.ndl * a.wgt[ri] : sp.ndl;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float Li = fmaf(V, L[ch], a.Lind[3 * ri + ch]);
            s1[ch] = fmaf(Li, cw, s1[ch]);
            s2[ch] = fmaf(sp.fs * Li, cw, s2[ch]);
        }
    }
    const float scale = a.wgt ? 1.0f : 2.0f * kPi / static_cast<float>(a.N);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float t1 = wave_sum(s1[ch]), t2 = wave_sum(s2[ch]);
        if (lane == 0) c[3 * p + ch] = scale * (a.albedo[3 * p + ch] / kPi * t1 + t2);
    }
}

__global__ __launch_bounds__(kShadeBlock) void k_mc_shade_bwd(ShadeArgs a, const float* __restrict__ g_c,
                                                              ShadeGrads g)
{
    const int lane = threadIdx.x & 63;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * (kShadeBlock / 64) + (threadIdx.x >> 6);
    if (p >= a.P) return;
    const float n[3] = {a.n[3 * p], a.n[3 * p + 1], a.n[3 * p + 2]};
    const float wo[3] = {a.wo[3 * p], a.wo[3 * p + 1], a.wo[3 * p + 2]};
    const float ndv = n[0] * wo[0] + n[1] * wo[1] + n[2] * wo[2];
    const float r = a.rough[p];
    const float scale = a.wgt ? 1.0f : 2.0f * kPi / static_cast<float>(a.N);
    const float gc[3] = {scale * g_c[3 * p], scale * g_c[3 * p + 1], scale * g_c[3 * p + 2]};
    const float fd[3] = {a.albedo[3 * p] / kPi, a.albedo[3 * p + 1] / kPi, a.albedo[3 * p + 2] / kPi};
    float ga[3] = {0, 0, 0}, gr = 0.0f;
    for (int i = lane; i < a.N; i += 64) {
        const int64_t ri = p * a.N + i;
        const float wi[3] = {a.wi[3 * ri], a.wi[3 * ri + 1], a.wi[3 * ri + 2]};
        const Spec sp = spec<true>(n, wo, ndv, wi, r);
        const int64_t texel = cube_texel(wi[0], wi[1], wi[2], a.E);
        const float* L = a.env + 3 * texel;
        const float V = 1.0f - a.O[ri];
        const float cw = a.wgt ? sp.ndl * a.wgt[ri] : sp.ndl;
        float gO = 0.0f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float Li = fmaf(V, L[ch], a.Lind[3 * ri + ch]);
            const float w = gc[ch] * cw;             // d c_ch / d (brdf_ch L_i)
            const float brdf = fd[ch] + sp.fs;
            ga[ch] = fmaf(w / kPi, Li, ga[ch]);
            gr = fmaf(w * Li, sp.dfs_dr, gr);
            if (g.Lind) g.Lind[3 * ri + ch] = w * brdf;
            gO = fmaf(-w * brdf, L[ch], gO);
            if (g.env) atomicAdd(g.env + 3 * texel + ch, w * brdf * V);
        }
        if (g.O) g.O[ri] = gO;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float t = wave_sum(ga[ch]);
        if (lane == 0 && g.albedo) g.albedo[3 * p + ch] += t;
    }
    const float t = wave_sum(gr);
    if (lane == 0 && g.rough) g.rough[p] += t;
}

unsigned blocks_for(int64_t n, int per_block)
{
    const int64_t b = (n + per_block - 1) / per_block;
    return static_cast<unsigned>(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_mc_rays(int64_t P, int St, int Sp, const float* x, const float* n, const float* u, float offset,
                          float* ro, float* rd, hipStream_t st)
{
    const int64_t total = P * St * Sp;
    if (total <= 0) return hipSuccess;
    const int64_t b = (total + 255) / 256;
    k_mc_rays<<<static_cast<unsigned>(b < 65536 ? b : 65536), 256, 0, st>>>(P, St, Sp, x, n, u, offset, ro, rd);
    return hipGetLastError();
}

hipError_t launch_mc_shade(const ShadeArgs& a, float* c, hipStream_t st)
{
    if (a.P <= 0) return hipSuccess;
    k_mc_shade<<<blocks_for(a.P, kShadeBlock / 64), kShadeBlock, 0, st>>>(a, c);
    return hipGetLastError();
}

hipError_t launch_mc_shade_backward(const ShadeArgs& a, const float* g_c, const ShadeGrads& g, hipStream_t st)
{
    if (a.P <= 0) return hipSuccess;
    k_mc_shade_bwd<<<blocks_for(a.P, kShadeBlock / 64), kShadeBlock, 0, st>>>(a, g_c, g);
    return hipGetLastError();
}

}  // namespace irgs
