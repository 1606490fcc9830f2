// Device-side building blocks of the 2D Gaussian ray tracer (gfx950).
//
// Geometry follows Sec. 3.2 of the paper:
//   * a surfel has centre mu, opacity o, a rotation quaternion q = (w,x,y,z)
//     whose rotation matrix has columns (t_u, t_v, n), and scales (s_u, s_v);
//   * Eq. 6: the ray meets the surfel plane at tau = n.(mu - r_o) / n.r_d;
//   * Eq. 7: at p = r_o + tau r_d the local coordinates are
//     u = (p - mu).t_u / s_u and v = (p - mu).t_v / s_v and the influence is
//     G = exp(-(u^2 + v^2) / 2); alpha = o G;
//   * Eq. 2 / Eq. 8: hits are alpha-blended front to back.
// Readings fixed here (the paper gives no value): a hit needs
// t_min < tau < t_max, u^2 + v^2 <= min(sigma^2, 2 ln(o / alpha_min)) (the
// support cap and the alpha_min test of Eq. 5's proxy, both inclusive);
// hits are ordered by (tau, surfel id); compositing includes a hit and then
// stops once T < T_min.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace irgs {

constexpr int kBlock = 256;          // threads per block of the trace kernels
constexpr int kStackLds = 24;        // per-lane traversal stack entries kept in LDS
constexpr int kLeafBit = 0x80000000; // child reference: leaf flag
constexpr int kNoChild = -1;         // child reference: empty slot (N == 1 root)

// 64-byte surfel record, stored in BVH leaf order.
//   a = (mu.xyz, o)            b = (n.xyz, rho2_max)
//   c = (t_u / s_u, id bits)   d = (t_v / s_v, 0)
// rho2_max = min(sigma^2, 2 ln(o / alpha_min)), or -1 for a surfel that can
// never be hit (o < alpha_min or an invalid parameter).
struct __align__(16) SurfelRec {
    float4 a, b, c, d;
};

// Internal BVH node: the boxes of both children plus their references.
// A reference r >= 0 is an internal node, r with kLeafBit set is the leaf at
// leaf position (r & ~kLeafBit), kNoChild is an empty slot.
struct __align__(16) BvhNode {
    float4 p0;  // lo0.xyz, hi0.x
    float4 p1;  // hi0.yz, lo1.xy
    float4 p2;  // lo1.z, hi1.xyz
    int4 ch;    // child0, child1, parent, unused
};

// 4-wide node used by the traversal (collapsed from the binary tree), child
// boxes stored per axis so the four slab tests share instructions.  A child
// reference r >= 0 is a wide node; r with kLeafBit set is a cluster of
// ((r & 15) + 1) surfels starting at leaf position ((r & ~kLeafBit) >> 4);
// kNoChild is an empty slot (its box is all +inf).
struct __align__(16) WideNode {
    float4 lo_x, lo_y, lo_z;
    float4 hi_x, hi_y, hi_z;
    int4 child;
    int4 meta;  // unused
};

constexpr int kLeafDefault = 12;  // surfels per cluster leaf (at most 16)

__host__ __device__ __forceinline__ int cluster_ref(int first, int count)
{
    return kLeafBit | (first << 4) | (count - 1);
}

// What a trace kernel needs of one scene (passed by value).
struct SceneView {
    const SurfelRec* rec;   // N records, leaf order
    const WideNode* wnodes; // 4-wide nodes, root = 0
    const float* feat;      // N x F, caller layout (original ids)
    int32_t n;
    int32_t F;
};

// How the composited channels are formed from a hit (template argument of
// the forward kernels).
enum ColourMode : int {
    kColPlain = 0,   // the surfel's F features
    kColSH = 1,      // view-dependent colour from RGB SH coefficients (3 channels)
    kColNormal = 2,  // the F features, then the unit normal turned to face the ray (F + 3)
};

struct TraceParams {
    float t_min, t_max, T_min;
    int32_t F;       // features per surfel
    int32_t sh_deg;  // -1: features composited as they are; 0..3: RGB SH coefficients (3 output channels)
    int32_t normals; // 1: the features, then the ray-facing unit normal (F + 3 output channels)
};

struct Ray {
    float ox, oy, oz, dx, dy, dz;
};

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz)
{
    return fmaf(ax, bx, fmaf(ay, by, az * bz));
}

// Columns (t_u, t_v, n) of the rotation of q = (w,x,y,z), normalised here.
// Returns the norm of q.
__device__ __forceinline__ float quat_frame(float4 q, float* tu, float* tv, float* nn)
{
    float qn = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
    float inv = 1.0f / qn;
    float w = q.x * inv, x = q.y * inv, y = q.z * inv, z = q.w * inv;
    tu[0] = 1.0f - 2.0f * (y * y + z * z);
    tu[1] = 2.0f * (x * y + w * z);
    tu[2] = 2.0f * (x * z - w * y);
    tv[0] = 2.0f * (x * y - w * z);
    tv[1] = 1.0f - 2.0f * (x * x + z * z);
    tv[2] = 2.0f * (y * z + w * x);
    nn[0] = 2.0f * (x * z + w * y);
    nn[1] = 2.0f * (y * z - w * x);
    nn[2] = 1.0f - 2.0f * (x * x + y * y);
    return qn;
}

// Eq. 6-7 against one record: depth tau and rho2 = u^2 + v^2 of the ray's
// crossing of the surfel plane.  Every kernel (brute force, BVH, packed,
// composite, backward re-march) evaluates a (ray, surfel) pair through this
// one function, so the pair is decided and ordered identically everywhere.
__device__ __forceinline__ void plane_hit(const SurfelRec& s, const Ray& r, float* tau_out, float* rho2_out)
{
    const float wx = s.a.x - r.ox, wy = s.a.y - r.oy, wz = s.a.z - r.oz;
    const float den = dot3(s.b.x, s.b.y, s.b.z, r.dx, r.dy, r.dz);
    const float num = dot3(s.b.x, s.b.y, s.b.z, wx, wy, wz);
    const float tau = num * __builtin_amdgcn_rcpf(den);  // den == 0: +-inf or NaN, rejected by the window
    const float px = fmaf(tau, r.dx, -wx), py = fmaf(tau, r.dy, -wy), pz = fmaf(tau, r.dz, -wz);
    const float u = dot3(px, py, pz, s.c.x, s.c.y, s.c.z);
    const float v = dot3(px, py, pz, s.d.x, s.d.y, s.d.z);
    *tau_out = tau;
    *rho2_out = fmaf(u, u, v * v);
}

// A hit: inside (t_min, t_max) (n.r_d == 0 gives +-inf or NaN, rejected) and
// inside the support rho2 <= rho2_max.
__device__ __forceinline__ bool hit_test(const SurfelRec& s, const Ray& r, float t_min, float t_max,
                                         float* tau_out, float* rho2_out)
{
    plane_hit(s, r, tau_out, rho2_out);
    return (*tau_out > t_min && *tau_out < t_max) && (*rho2_out <= s.b.w);
}

// alpha = o exp(-rho2 / 2) (Eq. 7 times the opacity).
__device__ __forceinline__ float alpha_of(const SurfelRec& s, float rho2) { return s.a.w * __expf(-0.5f * rho2); }

__device__ __forceinline__ SurfelRec load_rec(const SurfelRec* __restrict__ rec, int i)
{
    const float4* p = reinterpret_cast<const float4*>(rec + i);
    SurfelRec s;
    s.a = p[0];
    s.b = p[1];
    s.c = p[2];
    s.d = p[3];
    return s;
}

// Hit keys: (tau, leaf position) packed into one 64-bit integer whose
// unsigned order is the lexicographic order.  tau maps to a 32-bit unsigned
// m of the same order (sign-flipped when negative); the key is the top bit,
// then m, then the 31-bit position.  With the top bit set every key read as
// a double is negative, finite and normal (m's high bits equal to all ones or
// all zeros would need a NaN tau), so the FP64 order of keys is the reverse
// of their integer order: the k-buffer merges with FP64 min and max.
__device__ __forceinline__ uint64_t hit_key(float tau, int pos)
{
    const uint32_t u = __float_as_uint(tau);
    const uint32_t m = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return 0x8000000000000000ull | (static_cast<uint64_t>(m) << 31) | static_cast<uint32_t>(pos);
}

__device__ __forceinline__ float key_tau(uint64_t k)
{
    const uint32_t m = static_cast<uint32_t>(k >> 31);
    return __uint_as_float((m & 0x80000000u) ? (m & 0x7fffffffu) : ~m);
}

__device__ __forceinline__ int key_pos(uint64_t k) { return static_cast<int>(static_cast<uint32_t>(k) & 0x7fffffffu); }

// Above every key as an integer (a finite tau gives at most 0xFFBF...), and
// -inf read as a double.  Key 0 (below every key) marks a ray's first round.
constexpr uint64_t kKeyNone = 0xFFF0000000000000ull;

// The root node's box: the union of its non-empty child slots (lo > hi
// when the scene is empty).
__device__ __forceinline__ void root_box(const WideNode* __restrict__ root, float lo[3], float hi[3])
{
    const float inf = __int_as_float(0x7f800000);
    const float* w = reinterpret_cast<const float*>(root);  // lo_x[4], lo_y[4], lo_z[4], hi_x[4], hi_y[4], hi_z[4]
    for (int a = 0; a < 3; ++a) {
        lo[a] = inf;
        hi[a] = -inf;
    }
    for (int c = 0; c < 4; ++c) {
        if (w[c] == inf) continue;  // empty slot
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], w[4 * a + c]);
            hi[a] = fmaxf(hi[a], w[12 + 4 * a + c]);
        }
    }
}

// 30-bit Morton code (10 bits per axis) of point x in the box [lo, hi],
// clamped to the box.
__device__ __forceinline__ uint32_t morton30(const float x[3], const float lo[3], const float hi[3])
{
    uint32_t code = 0;
    for (int a = 0; a < 3; ++a) {
        const float ext = hi[a] - lo[a];
        const float u = ext > 0.0f ? (x[a] - lo[a]) / ext : 0.0f;
        const uint32_t q = static_cast<uint32_t>(fminf(fmaxf(u * 1024.0f, 0.0f), 1023.0f));
        uint32_t v = q;  // spread 10 bits to every third position
        v = (v | (v << 16)) & 0x030000ffu;
        v = (v | (v << 8)) & 0x0300f00fu;
        v = (v | (v << 4)) & 0x030c30c3u;
        v = (v | (v << 2)) & 0x09249249u;
        code |= v << (2 - a);
    }
    return code;
}

// Slab tests take the ray as (inverse direction i, no = -o * i) so that each
// slab distance is one fma: (l - o) / d == l * i + no.  The fused form
// rounds differently from (l - o) * i by less than an ulp of o * i, far
// inside the padding every leaf box carries (at least 1e-5 (1 + |mu|) per
// axis), so a box never loses a hit it contains.
struct SlabRay {
    float ix, iy, iz, nox, noy, noz;
};

// Slab test of a ray against a box, returning the entry distance; the box is
// accepted when it overlaps [lo, hi] along the ray.  `hi` must be finite.
// An empty box is stored with every coordinate = +inf, which this test
// always rejects (the +inf slab of an axis with positive inverse direction
// pushes the entry to +inf, and with all inverse directions negative the
// exit drops to -inf).
__device__ __forceinline__ bool box_hit(float lx, float ly, float lz, float hx, float hy, float hz,
                                        const SlabRay& q, float lo, float hi, float* t_enter)
{
    const float t0x = fmaf(lx, q.ix, q.nox), t1x = fmaf(hx, q.ix, q.nox);
    const float t0y = fmaf(ly, q.iy, q.noy), t1y = fmaf(hy, q.iy, q.noy);
    const float t0z = fmaf(lz, q.iz, q.noz), t1z = fmaf(hz, q.iz, q.noz);
    const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), lo));
    const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), hi));
    *t_enter = tn;
    return tn <= tf;
}

// Entry and exit distance of a ray in a box, clamped to [lo, hi]; the box is
// crossed inside the window when *tn <= *tf.  Same arithmetic as box_hit.
__device__ __forceinline__ void box_span(float lx, float ly, float lz, float hx, float hy, float hz,
                                         const SlabRay& q, float lo, float hi, float* tn, float* tf)
{
    const float t0x = fmaf(lx, q.ix, q.nox), t1x = fmaf(hx, q.ix, q.nox);
    const float t0y = fmaf(ly, q.iy, q.noy), t1y = fmaf(hy, q.iy, q.noy);
    const float t0z = fmaf(lz, q.iz, q.noz), t1z = fmaf(hz, q.iz, q.noz);
    *tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), lo));
    *tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), hi));
}

// View-dependent colour (Sec. 3.1: each surfel's colour is modelled by
// spherical harmonics; the trace uses that colour).  `k` holds RGB
// coefficients of the real SH basis up to degree `deg`, coefficient-major
// (k[3 j + c], j = l^2 + l + m); the colour seen along direction (dx, dy, dz)
// (normalised here) is max(sum_j Y_j k[3 j + c] + 1/2, 0) per channel.  The
// basis is sqrt(2) Re / sqrt(2) Im of the complex harmonics with the
// Condon-Shortley phase (m > 0 / m < 0), written out as polynomials in the
// unit direction; the constants are sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!)
// times the polynomial's own factor.
__device__ __forceinline__ void sh_basis(float dx, float dy, float dz, int deg, float* Y)
{
    const float inv = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    const float x = dx * inv, y = dy * inv, z = dz * inv;
    Y[0] = 0.28209479177387814f;  // 1 / (2 sqrt(pi))
    if (deg < 1) return;
    const float c1 = 0.48860251190291992f;  // sqrt(3 / (4 pi))
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792f * (x * y);          // sqrt(15 / (4 pi))
    Y[5] = -1.0925484305920792f * (y * z);
    Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);  // sqrt(5 / (16 pi))
    Y[7] = -1.0925484305920792f * (x * z);
    Y[8] = 0.54627421529603959f * (xx - yy);       // sqrt(15 / (16 pi))
    if (deg < 3) return;
    Y[9] = -0.59004358992664352f * (y * (3.0f * xx - yy));   // sqrt(35 / (32 pi))
    Y[10] = 2.8906114426405538f * (x * y * z);               // sqrt(105 / (4 pi))
    Y[11] = -0.45704579946446577f * (y * (5.0f * zz - 1.0f)); // sqrt(21 / (32 pi))
    Y[12] = 0.37317633259011540f * (z * (5.0f * zz - 3.0f));  // sqrt(7 / (16 pi))
    Y[13] = -0.45704579946446577f * (x * (5.0f * zz - 1.0f));
    Y[14] = 1.4453057213202769f * (z * (xx - yy));           // sqrt(105 / (16 pi))
    Y[15] = -0.59004358992664352f * (x * (xx - 3.0f * yy));
}

// Raw colour sum_j Y_j k[3 j + c] + 1/2 (before the clamp at 0).
__device__ __forceinline__ void sh_raw(const float* __restrict__ k, int deg, const float* Y, float* raw)
{
    const int nb = (deg + 1) * (deg + 1);
    raw[0] = raw[1] = raw[2] = 0.5f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j < nb) {
            raw[0] = fmaf(Y[j], k[3 * j], raw[0]);
            raw[1] = fmaf(Y[j], k[3 * j + 1], raw[1]);
            raw[2] = fmaf(Y[j], k[3 * j + 2], raw[2]);
        }
    }
}

__device__ __forceinline__ float safe_inv(float d)
{
    const float tiny = 1e-20f;
    float dd = fabsf(d) < tiny ? copysignf(tiny, d) : d;
    return 1.0f / dd;
}

__device__ __forceinline__ SlabRay slab_ray(const Ray& r)
{
    SlabRay q;
    q.ix = safe_inv(r.dx), q.iy = safe_inv(r.dy), q.iz = safe_inv(r.dz);
    q.nox = -(r.ox * q.ix), q.noy = -(r.oy * q.iy), q.noz = -(r.oz * q.iz);
    return q;
}

}  // namespace irgs
