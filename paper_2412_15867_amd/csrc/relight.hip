// Relighting variant of the trace's consumer.  To relight, the trace
// alpha-blends albedo, roughness and the normal along each incident ray
// (normalised weights T_i alpha_i / sum T_i alpha_i), and the ray's indirect
// radiance is shaded in one query with the split-sum approximation:
// L_ind = L_d + L_s, L_d = A / pi * E(N), L_s = P_R(refl) (F0 S_A + S_B),
// where E is the irradiance of the sky, P_R the sky prefiltered with the GGX
// lobe of roughness R, and (S_A, S_B) a pre-integrated BRDF table.
//
// Readings (the construction is cited, no numbers are given): the sky is a
// cubemap of 6 E x E texels, each integral a sum over texel centres with
// their exact solid angle 4 / (E^2 (1 + s^2 + t^2)^{3/2}); P_R assumes
// normal = view = reflection direction; roughness levels r_l = (l + 1) / M,
// nearest level; the table at cell centres ((i + 1/2)/S, (j + 1/2)/S) is the
// GGX-importance-sampled estimate over 256 Hammersley points; F0 = 0.04 and
// the Smith G of the shading BRDF; lookups take the nearest texel / cell;
// the surface is viewed from -d; a ray with no hit carries no indirect light.
#include <hip/hip_runtime.h>

#include "irgs_internal.hpp"

namespace irgs {

namespace {

constexpr float kPiR = 3.14159265358979323846f;
constexpr float kF0R = 0.04f;
constexpr int kHammersley = 256;

// Unnormalised direction of face coordinates (s, t) in [-1, 1]^2 on a face:
// the inverse of the nearest-texel addressing below.
__device__ __forceinline__ void face_point(int face, float s, float t, float* d)
{
    switch (face) {
        case 0: d[0] = 1.0f, d[1] = -t, d[2] = -s; break;
        case 1: d[0] = -1.0f, d[1] = -t, d[2] = s; break;
        case 2: d[0] = s, d[1] = 1.0f, d[2] = t; break;
        case 3: d[0] = s, d[1] = -1.0f, d[2] = -t; break;
        case 4: d[0] = s, d[1] = -t, d[2] = 1.0f; break;
        default: d[0] = -s, d[1] = -t, d[2] = -1.0f; break;
    }
}

// Centre direction (unit) and solid angle of texel `idx` of an E x E cube.
__device__ __forceinline__ void texel_dir(int idx, int E, float* d, float* dw)
{
    const int face = idx / (E * E);
    const int rc = idx - face * E * E;
    const int row = rc / E, col = rc - row * E;
    const float s = 2.0f * (col + 0.5f) / E - 1.0f;
    const float t = 2.0f * (row + 0.5f) / E - 1.0f;
    face_point(face, s, t, d);
    const float q = 1.0f + s * s + t * t;
    const float inv = 1.0f / sqrtf(q);
    d[0] *= inv, d[1] *= inv, d[2] *= inv;
    *dw = 4.0f / (E * E * q * sqrtf(q));
}

// Nearest texel of direction (x, y, z): the same addressing as the shading.
__device__ __forceinline__ int texel_of(float x, float y, float z, int E)
{
    const float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    int face;
    float s, t, m;
    if (ax >= ay && ax >= az) {
        m = ax, face = x >= 0.0f ? 0 : 1, s = x >= 0.0f ? -z : z, t = -y;
    } else if (ay >= az) {
        m = ay, face = y >= 0.0f ? 2 : 3, s = x, t = y >= 0.0f ? z : -z;
    } else {
        m = az, face = z >= 0.0f ? 4 : 5, s = z >= 0.0f ? x : -x, t = -y;
    }
    s /= m;
    t /= m;
    const int col = min(max(static_cast<int>(floorf((s + 1.0f) * E * 0.5f)), 0), E - 1);
    const int row = min(max(static_cast<int>(floorf((t + 1.0f) * E * 0.5f)), 0), E - 1);
    return (face * E + row) * E + col;
}

// GGX D of the unit vectors c, h (alpha = r^2), with q = (c.h)^2 (alpha^2 - 1) + 1
// evaluated as |c x h|^2 + (c.h)^2 alpha^2 (no cancellation near the peak).
__device__ __forceinline__ float ggx(const float* c, const float* h, float r)
{
    const float a2 = (r * r) * (r * r);
    const float ch = c[0] * h[0] + c[1] * h[1] + c[2] * h[2];
    const float x = c[1] * h[2] - c[2] * h[1], y = c[2] * h[0] - c[0] * h[2], z = c[0] * h[1] - c[1] * h[0];
    const float q = fmaf(ch * ch, a2, x * x + y * y + z * z);
    return a2 / (kPiR * q * q);
}

__device__ __forceinline__ float smith(float l, float v, float r)
{
    const float k = (r + 1.0f) * (r + 1.0f) * 0.125f;
    return l / (l * (1.0f - k) + k) * (v / (v * (1.0f - k) + k));
}

// One output texel per thread, every input texel summed (FP32 accumulate of
// at most 6 E^2 terms).
__global__ void k_irradiance(int E, const float* __restrict__ env, float* __restrict__ irr)
{
    const int n = 6 * E * E;
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    float c[3], dwo;
    texel_dir(o, E, c, &dwo);
    float acc[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        float w[3], dw;
        texel_dir(i, E, w, &dw);
        const float cs = w[0] * c[0] + w[1] * c[1] + w[2] * c[2];
        if (cs <= 0.0f) continue;
        const float f = cs * dw;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc[ch] = fmaf(f, env[3 * i + ch], acc[ch]);
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) irr[3 * o + ch] = acc[ch];
}

__global__ void k_prefilter(int E, int M, const float* __restrict__ env, float* __restrict__ pref)
{
    const int n = 6 * E * E;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= static_cast<int64_t>(n) * M) return;
    const int l = static_cast<int>(g / n), o = static_cast<int>(g - static_cast<int64_t>(l) * n);
    const float r = static_cast<float>(l + 1) / M;
    float c[3], dwo;
    texel_dir(o, E, c, &dwo);
    float acc[3] = {0, 0, 0}, wsum = 0.0f;
    for (int i = 0; i < n; ++i) {
        float w[3], dw;
        texel_dir(i, E, w, &dw);
        const float cs = w[0] * c[0] + w[1] * c[1] + w[2] * c[2];
        if (cs <= 0.0f) continue;
        float h[3] = {w[0] + c[0], w[1] + c[1], w[2] + c[2]};
        const float hn = 1.0f / sqrtf(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
        h[0] *= hn, h[1] *= hn, h[2] *= hn;
        const float wt = ggx(c, h, r) * cs * dw;
        wsum += wt;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] = fmaf(wt, env[3 * i + k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) pref[3 * g + k] = acc[k] / wsum;
}

__global__ void k_brdf_table(int S, float* __restrict__ table)
{
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= S * S) return;
    const int i = cell / S, j = cell - i * S;
    const float nv = (i + 0.5f) / S, r = (j + 0.5f) / S;
    const float vx = sqrtf(1.0f - nv * nv), vz = nv;  // view in the xz plane, normal +z
    const float a2 = (r * r) * (r * r);
    float A = 0.0f, B = 0.0f;
    for (int k = 0; k < kHammersley; ++k) {
        const float x = (k + 0.5f) / kHammersley;
        const float y = static_cast<float>(__brev(static_cast<unsigned>(k))) * 2.3283064365386963e-10f;  // 2^-32
        // cos^2 and sin^2 of the sampled half vector over one exact
        // denominator (1 - y is exact), so neither cancels at small roughness
        const float den = fmaf(a2, y, 1.0f - y);
        const float ct = sqrtf((1.0f - y) / den), st = sqrtf(a2 * y / den);
        float sp, cp;
        sincosf(2.0f * kPiR * x, &sp, &cp);
        const float hx = st * cp, hz = ct;
        const float vh = hx * vx + hz * vz;
        const float lz = 2.0f * vh * hz - vz;
        if (lz <= 0.0f) continue;
        const float g = smith(lz, nv, r) * vh / (hz * nv);
        const float om = 1.0f - vh, om2 = om * om;
        const float fc = om2 * om2 * om;
        A = fmaf(1.0f - fc, g, A);
        B = fmaf(fc, g, B);
    }
    table[2 * cell] = A / kHammersley;
    table[2 * cell + 1] = B / kHammersley;
}

__global__ void k_relight_lind(RelightArgs a, float* __restrict__ lind)
{
    for (int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; r < a.R;
         r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float O = a.O[r];
        float out[3] = {0, 0, 0};
        if (O > 0.0f) {
            const float* f = a.Fo + 7 * r;
            const float inv = 1.0f / O;
            const float A[3] = {f[0] * inv, f[1] * inv, f[2] * inv};
            const float Rg = fminf(fmaxf(f[3] * inv, 0.0f), 1.0f);
            float N[3] = {f[4] * inv, f[5] * inv, f[6] * inv};
            const float nn = sqrtf(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
            if (nn > 0.0f) N[0] /= nn, N[1] /= nn, N[2] /= nn;
            float d[3] = {a.rd[3 * r], a.rd[3 * r + 1], a.rd[3 * r + 2]};
            const float dn = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            d[0] /= dn, d[1] /= dn, d[2] /= dn;
            const float* E = a.irr + 3 * static_cast<int64_t>(texel_of(N[0], N[1], N[2], a.E));
            const float nv = fminf(fmaxf(-(N[0] * d[0] + N[1] * d[1] + N[2] * d[2]), 0.0f), 1.0f);
            const float dd = d[0] * N[0] + d[1] * N[1] + d[2] * N[2];
            const float refl[3] = {d[0] - 2.0f * dd * N[0], d[1] - 2.0f * dd * N[1], d[2] - 2.0f * dd * N[2]};
            const int lev = min(max(static_cast<int>(floorf(Rg * a.M + 0.5f)) - 1, 0), a.M - 1);
            const float* Pr = a.pref + 3 * (static_cast<int64_t>(lev) * 6 * a.E * a.E +
                                              texel_of(refl[0], refl[1], refl[2], a.E));
            const int ti = min(max(static_cast<int>(floorf(nv * a.S)), 0), a.S - 1);
            const int tj = min(max(static_cast<int>(floorf(Rg * a.S)), 0), a.S - 1);
            const float spec = kF0R * a.table[2 * (ti * a.S + tj)] + a.table[2 * (ti * a.S + tj) + 1];
#pragma unroll
            for (int c = 0; c < 3; ++c) out[c] = A[c] / kPiR * E[c] + Pr[c] * spec;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) lind[3 * r + c] = out[c];
    }
}

// Sampling weight of texel i: max(mean RGB, 0) times its solid angle at the
// centre, in FP64 (a NaN texel weighs 0).
__device__ __forceinline__ double texel_weight(int i, int E, const float* __restrict__ env)
{
    const int rc = i % (E * E);
    const int row = rc / E, col = rc - row * E;
    const double s = 2.0 * (col + 0.5) / E - 1.0, t = 2.0 * (row + 0.5) / E - 1.0;
    const double q = 1.0 + s * s + t * t;
    const double inten = fmax((static_cast<double>(env[3 * i]) + env[3 * i + 1] + env[3 * i + 2]) / 3.0, 0.0);
    return inten * 4.0 / (static_cast<double>(E) * E * q * sqrt(q));
}

constexpr int kCdfBlock = 1024;

// Inclusive CDF of the texel weights in texel order, one block: each thread
// sums a run of consecutive texels in FP64, a block scan offsets the runs,
// and each run is rewritten as running sums rounded once to FP32 (so the
// table never decreases).
__global__ __launch_bounds__(kCdfBlock) void k_env_cdf(int E, const float* __restrict__ env, float* __restrict__ cdf)
{
    __shared__ double part[kCdfBlock];
    const int n = 6 * E * E;
    const int per = (n + kCdfBlock - 1) / kCdfBlock;
    const int b = min(static_cast<int>(threadIdx.x) * per, n), e = min(b + per, n);
    double run = 0.0;
    for (int i = b; i < e; ++i) run += texel_weight(i, E, env);
    part[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < kCdfBlock; off <<= 1) {
        const double v = threadIdx.x >= static_cast<unsigned>(off) ? part[threadIdx.x - off] : 0.0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0.0;
    for (int i = b; i < e; ++i) {
        run += texel_weight(i, E, env);
        cdf[i] = static_cast<float>(run);
    }
}

// One ray per sample drawn from the sky's intensity: the first texel whose
// CDF exceeds u0 * total (FP32), a point uniform in that texel's face
// coordinates, density p_j E^2 / 4 (1 + s^2 + t^2)^{3/2}, estimator weight
// 1 / (N pdf) above the horizon of n and 0 below it or for an empty sky.
__global__ void k_env_rays(EnvRayArgs a)
{
    const int nt = 6 * a.E * a.E;
    const float total = a.cdf[nt - 1];
    const float step = 2.0f / a.E;
    for (int64_t r = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; r < a.P * a.N;
         r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t p = r / a.N;
        const float* u = a.u + 3 * r;
        float target = u[0] * total;
        if (!(target < total)) target = nextafterf(total, 0.0f);
        int lo = 0, hi = nt - 1;  // first index with cdf > target (the last one if none)
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a.cdf[mid] > target) hi = mid;
            else lo = mid + 1;
        }
        const int face = lo / (a.E * a.E);
        const int rc = lo - face * a.E * a.E;
        const int row = rc / a.E, col = rc - row * a.E;
        const float s = (static_cast<float>(col) + u[1]) * step - 1.0f;
        const float t = (static_cast<float>(row) + u[2]) * step - 1.0f;
        float d[3];
        face_point(face, s, t, d);
        const float q = 1.0f + s * s + t * t;
        const float inv = 1.0f / sqrtf(q);
        d[0] *= inv, d[1] *= inv, d[2] *= inv;
        const float n[3] = {a.n[3 * p], a.n[3 * p + 1], a.n[3 * p + 2]};
        const float pj = (a.cdf[lo] - (lo > 0 ? a.cdf[lo - 1] : 0.0f)) / total;
        const float pdf = pj * (0.25f * a.E * a.E) * (q * sqrtf(q));
        const bool ok = d[0] * n[0] + d[1] * n[1] + d[2] * n[2] > 0.0f && pdf > 0.0f && total > 0.0f;
        a.wgt[r] = ok ? 1.0f / (static_cast<float>(a.N) * pdf) : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.ro[3 * r + c] = fmaf(a.offset, n[c], a.x[3 * p + c]);
            a.rd[3 * r + c] = d[c];
        }
    }
}

unsigned grid_for(int64_t n, int block)
{
    const int64_t b = (n + block - 1) / block;
    return static_cast<unsigned>(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

hipError_t launch_env_prefilter(int E, const float* env, int M, float* irr, float* pref, hipStream_t st)
{
    const int n = 6 * E * E;
    if (irr) k_irradiance<<<grid_for(n, 128), 128, 0, st>>>(E, env, irr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !pref || M <= 0) return e;
    const int64_t total = static_cast<int64_t>(n) * M;
    k_prefilter<<<static_cast<unsigned>((total + 127) / 128), 128, 0, st>>>(E, M, env, pref);
    return hipGetLastError();
}

hipError_t launch_brdf_table(int S, float* table, hipStream_t st)
{
    k_brdf_table<<<grid_for(static_cast<int64_t>(S) * S, 128), 128, 0, st>>>(S, table);
    return hipGetLastError();
}

hipError_t launch_relight_lind(const RelightArgs& a, float* lind, hipStream_t st)
{
    if (a.R <= 0) return hipSuccess;
    k_relight_lind<<<grid_for(a.R, 256), 256, 0, st>>>(a, lind);
    return hipGetLastError();
}

hipError_t launch_env_cdf(int E, const float* env, float* cdf, hipStream_t st)
{
    k_env_cdf<<<1, kCdfBlock, 0, st>>>(E, env, cdf);
    return hipGetLastError();
}

hipError_t launch_env_rays(const EnvRayArgs& a, hipStream_t st)
{
    if (a.P * a.N <= 0) return hipSuccess;
    k_env_rays<<<grid_for(a.P * a.N, 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace irgs
