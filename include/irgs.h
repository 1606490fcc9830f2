/*
 * irgs.h -- C ABI of the MI355X (gfx950) 2D Gaussian ray tracer.
 *
 * The library implements Trace(r_o, r_d) -> (c_rt, o_rt) of Sec. 3.2
 * (Eq. 8) and its use as the visibility / indirect-radiance query
 * (L_ind, 1 - V) <- Trace(x, w_i) of Sec. 3.3 (Eq. 14):
 *   - a ray meets a surfel's plane at tau = n.(mu - r_o) / n.r_d   (Eq. 6);
 *   - at p = r_o + tau r_d, u = (p-mu).t_u / s_u, v = (p-mu).t_v / s_v and
 *     alpha = o exp(-(u^2+v^2)/2)                                   (Eq. 7);
 *   - hits are collected by k-buffer marching (the k nearest after the last
 *     composited hit, per round) in exact depth order (hits at equal tau in
 *     the order of the surfels' leaf positions in the tree) and
 *     alpha-blended front to back (Eq. 2), stopping once the transmittance
 *     T < T_min;
 *   - the surfel frame (t_u, t_v, n) is the column set of the rotation of
 *     the unit quaternion q = (w, x, y, z) (Sec. 3.1: quaternion + scaling
 *     parameterisation; Sec. 3.2: two tangents and their cross product).
 * A software LBVH over each surfel's support box stands in for the hardware
 * BVH over icosahedron proxies of Eq. 5 (rebuilt or refit per iteration,
 * Sec. 4 implementation details).
 *
 * Conventions for every entry point:
 *   - pointers are DEVICE pointers unless stated otherwise; arrays are FP32
 *     (or int32), row-major and contiguous;
 *   - `stream` is a hipStream_t (NULL = the default stream); work is queued
 *     asynchronously and no entry point synchronises the stream except
 *     irgs_scene_build (it reads the tree depth back to the host);
 *   - a return value < 0 is an error; nothing is thrown across the ABI;
 *     irgs_last_error() returns a thread-local message about the last
 *     failure on the calling thread.  Argument errors are reported before
 *     any work is queued.  Kernel faults surface at the caller's next sync.
 */
#ifndef IRGS_H
#define IRGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IRGS_OK = 0,
    IRGS_E_INVALID = -1, /* bad argument: null required pointer, size, k, F */
    IRGS_E_OOM = -2,     /* device allocation failed */
    IRGS_E_HIP = -3,     /* a HIP call or kernel launch failed */
    IRGS_E_STATE = -4,   /* scene not built, or built with other alpha_min/sigma */
    IRGS_E_BUSY = -5     /* reserved */
} irgs_status;

typedef struct irgs_scene_s* irgs_scene; /* opaque, owned by the library */

/* Surfel parameters, BORROWED by a scene (the caller keeps them alive):
 *   mu (N x 3) centres; quat (N x 4) raw quaternions (w,x,y,z), normalised
 *   inside; scale (N x 2) activated scales (s_u, s_v) > 0; opacity (N)
 *   activated opacity in [0,1]; feat (N x F) per-surfel features blended
 *   along the ray (RGB, albedo, roughness, ...).  A surfel with a non-finite
 *   value, a zero quaternion or a non-positive scale is never hit. */
typedef struct {
    const float* mu;
    const float* quat;
    const float* scale;
    const float* opacity;
    const float* feat;
} irgs_surfels;

/* Trace parameters.
 *   k             k-buffer size, one of 1, 2, 4, 8, 16, 32, 64 (results do
 *                 not depend on k; it only changes the work per round)
 *   feature_dim   F, must equal the scene's F (1..64)
 *   alpha_min     minimum alpha of a hit (the alpha_min of Eq. 5)
 *   T_min         stop once the transmittance falls below this
 *   t_min, t_max  hits need t_min < tau < t_max
 *   support_sigma hits need u^2 + v^2 <= support_sigma^2
 *   flags         IRGS_FLAG_* below
 *   leaf_size     build only: surfels per BVH leaf cluster, 1..16 (0 = 12)
 * alpha_min and support_sigma are fixed at build time (they size the boxes);
 * tracing with other values returns IRGS_E_STATE. */
typedef struct {
    int32_t k;
    int32_t feature_dim;
    float alpha_min;
    float T_min;
    float t_min;
    float t_max;
    float support_sigma;
    uint32_t flags;
    int32_t leaf_size;
} irgs_params;

#define IRGS_FLAG_BRUTE_FORCE 1u /* trace: test every surfel, no BVH */
#define IRGS_FLAG_RECOMPUTE 2u   /* backward: trace again instead of reading saved hits */
/* trace / backward: view-dependent colour (Sec. 3.1 models each surfel's
 * colour with spherical harmonics; the trace uses that colour, Sec. 3.3).
 * The F = 3 (deg + 1)^2 features of a surfel (deg <= 3: F = 3, 12, 27, 48)
 * are RGB coefficients of the real SH basis, coefficient-major
 * (feat[i][3 j + c], j = l^2 + l + m; Y_lm = sqrt(2) Re / sqrt(2) Im of the
 * complex harmonics with the Condon-Shortley phase for m > 0 / m < 0); each
 * hit contributes, per channel, max(sum_j Y_j(d) k_j + 1/2, 0) with d the
 * normalised ray direction.  out->feat and grad_in->g_feat are then R x 3;
 * grads->feat stays N x F.  k must be 16, 32 or 64; not for irgs_trace_packed. */
#define IRGS_FLAG_SH 4u
/* trace and backward (relighting details: the trace alpha-blends albedo,
 * roughness and the normal with the same weights, Eq. 18): after the
 * F <= 5 features, 3 more composited channels hold each hit's unit normal,
 * negated where it points along the ray (n . r_d > 0) so that it faces the
 * ray; out->feat and grad_in->g_feat are R x (F + 3), and the backward
 * carries the normal channels' gradient through n to the raw quaternion
 * (the turn itself is piecewise constant).  Exclusive with IRGS_FLAG_SH;
 * k must be 16, 32 or 64; not for the packed launch. */
#define IRGS_FLAG_NORMAL 8u
/* scene build only: the binary tree under the 4-wide BVH is Karras' radix
 * tree over the sorted Morton codes (leaves stay in Morton order) instead
 * of the default PLOC clustering (Meister and Bittner 2018: mutually
 * nearest clusters by union surface area within 8 positions of the Morton
 * order merge, iterated; the leaves are then renumbered depth first).  Both
 * trees give the same hits; the PLOC tree bounds them with less box area,
 * so traversals test fewer surfels, at a slower build. */
#define IRGS_FLAG_RADIX_TREE 16u
/* trace and backward (BVH traces of one scene): the call first sorts the
 * rays by the Morton code of their origin in the scene's box, on the
 * device, and hands rays to the traversal in that order, so that rays
 * traced side by side start near each other and share cached nodes and
 * surfels.  Outputs stay in the caller's order and every ray's result is
 * the same bit for bit; it pays when the scene's working set outgrows the
 * caches and the caller's rays are spatially incoherent (5M surfels, random
 * surface points: forward -11% at k = 64).  Extra scratch: 24 bytes per ray
 * plus the sort's tile counts (irgs_trace_bytes).  Ignored by
 * irgs_trace_packed, by brute-force traces and by calls of more than
 * 2^31 - 1 rays (traced in the caller's order). */
#define IRGS_FLAG_SORT_RAYS 32u

/* Outputs of a trace, caller-allocated (R = number of rays):
 *   opacity (R)      accumulated opacity O = sum T_i alpha_i (o_rt of Eq. 8;
 *                    visibility V = 1 - O, Eq. 14)
 *   feat (R x F)     blended features sum T_i alpha_i f_i (c_rt / L_ind)
 *   depth (R)        UNnormalised depth sum T_i alpha_i tau_i (normalised
 *                    depth of Eq. 9 is depth / opacity)
 *   T (R)            final transmittance, optional (NULL)
 *   n_hits (R)       number of composited hits, optional; required by
 *                    irgs_trace_backward
 *   hit_ids (R x H_cap)  ids of the first H_cap composited hits in order,
 *                    optional; entries past n_hits are left untouched
 *   hit_T (R x H_cap)    transmittance before each of those hits, optional
 *                    (needs hit_ids)
 *   counters (R x 4) work counters, optional: BVH nodes visited, surfels
 *                    tested, k-buffer insertions, rounds
 * A ray with a non-finite component or a zero direction gets O = 0, F = 0,
 * D = 0, T = 1, n_hits = 0. */
typedef struct {
    float* opacity;
    float* feat;
    float* depth;
    float* T;
    int32_t* n_hits;
    int32_t* hit_ids;
    float* hit_T;
    int32_t H_cap;
    int32_t* counters;
} irgs_out;

/* Upstream gradients dL/dO (R), dL/dF (R x F), dL/dD (R); any may be NULL
 * (treated as zero).  Rays whose upstream gradients are all zero are
 * skipped. */
typedef struct {
    const float* g_opacity;
    const float* g_feat;
    const float* g_depth;
} irgs_grad_in;

/* Gradient outputs, ACCUMULATED (+=) so the caller zeroes them; any may be
 * NULL to skip it.  Shapes as irgs_surfels; quat is the gradient with
 * respect to the raw (unnormalised) quaternion. */
typedef struct {
    float* mu;
    float* quat;
    float* scale;
    float* opacity;
    float* feat;
} irgs_grads;

/* One work item of a packed launch: rays [ray_begin, ray_begin+ray_count)
 * of ro/rd (R x 3 each), traced against scenes[scene]; outputs are written
 * at the same ray indices of `out` (its feat has the scene's F columns). */
typedef struct {
    int32_t scene;
    int32_t pad;
    int64_t ray_begin;
    int64_t ray_count;
    const float* ro;
    const float* rd;
    irgs_out out;
} irgs_work;

/* Bytes the library allocates for a scene of n surfels (records, nodes,
 * build scratch), and the per-call scratch of a trace of R rays with the
 * given flags (with IRGS_FLAG_RECOMPUTE: of the backward that traces the
 * rays again). */
size_t irgs_scene_bytes(int64_t n, int32_t F);
size_t irgs_trace_bytes(int64_t R, int32_t F, uint32_t flags);

/* Create a scene over borrowed parameters (no device work, no allocation
 * beyond the handle).  0 <= n <= 2^27 (134,217,728), 1 <= F <= 64. */
irgs_status irgs_scene_create(int64_t n, int32_t F, const irgs_surfels* params, irgs_scene* out);

/* Point the scene at other parameter buffers of the same shape (the tree
 * must be refit or rebuilt before the next trace). */
irgs_status irgs_scene_set_params(irgs_scene scene, const irgs_surfels* params);

/* Build (Sec. 3.2: the surfels are wrapped in bounding proxies of their
 * alpha_min support, Eq. 5, and organised in a BVH that the ray tracer
 * traverses; here each proxy is the exact box of the support ellipse):
 * per-surfel records and support boxes, Morton codes, radix sort,
 * hierarchy (PLOC, or the radix tree with IRGS_FLAG_RADIX_TREE), level-by-level
 * boxes, the 4-wide collapse.  Allocates the scene's device buffers on first
 * use.  Uses params->alpha_min, support_sigma, leaf_size and that flag.
 * Reads level sizes and the tree depth back (synchronises `stream`). */
irgs_status irgs_scene_build(irgs_scene scene, const irgs_params* params, void* stream);

/* Refit after the parameters changed in place (Sec. 4, implementation
 * details: the BVH is updated at every training iteration, because the
 * surfels move): records, leaf boxes and internal boxes recomputed, tree
 * topology kept.  Asynchronous. */
irgs_status irgs_scene_refit(irgs_scene scene, void* stream);

/* Forward trace of R rays, ro and rd (R x 3, directions need not be unit:
 * tau is measured in units of r_d).  Uses the BVH unless
 * IRGS_FLAG_BRUTE_FORCE is set (then the scene must still be built, for the
 * records). */
irgs_status irgs_trace(irgs_scene scene, const irgs_params* params, int64_t R, const float* ro, const float* rd,
                       const irgs_out* out, void* stream);

/* irgs_trace for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (bit for bit) as irgs_trace, but the call
 * allocates nothing: its scratch (the ray-claim counter, each persistent
 * thread's traversal-stack overflow and deferred-work lists) lives in one
 * 64 MiB array inside the library's code object, one copy per device, held
 * until the process ends.  The launch fits its grid and deferred-list length
 * into that array (resident blocks are dropped only when even 32 entries per
 * list do not fit them all), so any R is accepted; a scene whose tree is so
 * deep that one block's stack overflow does not fit returns IRGS_E_INVALID.
 * IRGS_FLAG_SORT_RAYS needs a per-ray workspace and returns IRGS_E_INVALID.
 * The claim counter is cleared by a fill kernel on `stream` before each
 * launch (no memset node).  Every call on one device shares that device's
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and give undefined results; order them on one stream. */
irgs_status irgs_trace_noalloc(irgs_scene scene, const irgs_params* params, int64_t R, const float* ro,
                               const float* rd, const irgs_out* out, void* stream);

/* Backward of irgs_trace over the same rays (Sec. 3.3, Stage II: the
 * indirect radiance and visibility returned by the trace are differentiated
 * with respect to the surfels every iteration; the "detach indirect"
 * ablation of Sec. 4.2 turns exactly this off): accumulates parameter
 * gradients.  `saved` is the irgs_out of the forward call: n_hits is
 * required; with hit_ids and hit_T present (and IRGS_FLAG_RECOMPUTE unset)
 * rays with n_hits <= H_cap replay their saved hits, every other ray
 * re-marches its hits.  Without saved lists (or with IRGS_FLAG_RECOMPUTE)
 * the call traces the rays again, in equal batches whose hit lists (256 per
 * ray) fit a transient 4 GiB workspace, replays those lists and re-marches rays
 * with more hits; results are the same either way up to the order of the
 * gradient sums.  Parameters must not have changed since the forward
 * trace. */
irgs_status irgs_trace_backward(irgs_scene scene, const irgs_params* params, int64_t R, const float* ro,
                                const float* rd, const irgs_out* saved, const irgs_grad_in* grad_in,
                                irgs_grads* grads, void* stream);

/* One persistent launch over the work items of several built scenes
 * (`items` is a HOST array, copied by the call).  Every scene must share
 * alpha_min/support_sigma with `params`; params->feature_dim must be >= the
 * largest F.  k must be 16 or 32. */
irgs_status irgs_trace_packed(const irgs_scene* scenes, int32_t n_scenes, const irgs_params* params,
                              const irgs_work* items, int32_t n_items, void* stream);

/* Tree statistics of a built scene (host outputs, any may be NULL):
 * number of internal nodes, maximum leaf depth. */
irgs_status irgs_scene_info(irgs_scene scene, int64_t* n_internal, int32_t* max_depth);

/* Copy the tree of a built scene into caller DEVICE buffers (any NULL is
 * skipped): order (N, int32: leaf position -> surfel id), nodes
 * ((N-1) x 16 int32 words: 12 box floats as bits, child0, child1, parent,
 * 0), leaf_parent (N).  For structural tests. */
irgs_status irgs_scene_export(irgs_scene scene, int32_t* order, int32_t* nodes, int32_t* leaf_parent,
                              void* stream);

irgs_status irgs_scene_destroy(irgs_scene scene);

/* ---- Monte Carlo rendering-equation consumer of the trace (Sec. 3.3,
 * "Rendering": Eq. 15 with the light decomposition of Eq. 13-14 and the
 * BRDF of Eq. 4).  Per pixel p, N = S_t * S_p incident directions; ray
 * p * N + i carries sample i of pixel p. */

/* Rays of stratified uniform hemisphere sampling: sample i = s * S_p + t has
 * cos(theta) = (s + u[p][i][0]) / S_t, phi = 2 pi (t + u[p][i][1]) / S_p in
 * the frame (t1, t2, n_p), (t1, t2) the branchless orthonormal basis of
 * Duff et al. 2017 (t1 = (1 + s nx^2 a, s b, -s nx), t2 = (b, s + ny^2 a,
 * -ny), s = sign(nz) with sign(0) = 1, a = -1 / (s + nz), b = nx ny a).
 * Origin x_p + offset n_p.  x, n: P x 3 (n unit); u: P x N x 2 uniforms;
 * ro, rd: (P N) x 3 written.  S_t, S_p >= 1; P >= 0. */
irgs_status irgs_mc_rays(int64_t P, int32_t S_t, int32_t S_p, const float* x, const float* n, const float* u,
                         float offset, float* ro, float* rd, void* stream);

/* Shading inputs (DEVICE pointers, borrowed). */
typedef struct {
    int64_t P;            /* pixels */
    int32_t N;            /* samples per pixel */
    int32_t E;            /* cubemap face resolution (E x E texels) */
    const float* n;       /* P x 3 unit normals */
    const float* wo;      /* P x 3 unit directions towards the viewer */
    const float* albedo;  /* P x 3 diffuse albedo a */
    const float* rough;   /* P roughness r */
    const float* wi;      /* P x N x 3 incident directions (the rays' rd) */
    const float* O;       /* P x N opacity of each ray's trace (V = 1 - O) */
    const float* Lind;    /* P x N x 3 colour of each ray's trace (L_ind) */
    const float* env;     /* 6 x E x E x 3 cubemap L_dir: faces +x, -x, +y, -y, +z, -z */
    const float* wgt;     /* P x N per-sample weights 1 / (N pdf) of another sampling density
                             (irgs_env_rays), or NULL: 2 pi / N each (uniform hemisphere) */
} irgs_shade_in;

/* c[p] = 2 pi / N sum_i (a / pi + f_s) (V_i L_dir(w_i) + L_ind,i) (w_i . n)
 * (Eq. 15; with wgt, wgt[p, i] in place of 2 pi / N),
 * f_s = D F G / (4 (w_i . n)(w_o . n)): D GGX with alpha = r^2, F Schlick
 * with F0 = 0.04, G Smith with Schlick-GGX G1 and k = (r + 1)^2 / 8; both
 * cosines clamped below at 1e-4 inside G and the denominator.  L_dir is the
 * nearest texel: major axis picks the face (ties to x, then y), face
 * coordinates (s, t) = (-z, -y)/|x|, (z, -y)/|x|, (x, z)/|y|, (x, -z)/|y|,
 * (x, -y)/|z|, (-x, -y)/|z|, texel row floor((t + 1) E / 2), column
 * floor((s + 1) E / 2), clamped.  c: P x 3 written. */
irgs_status irgs_mc_shade(const irgs_shade_in* in, float* c, void* stream);

/* Gradients of sum(g_c * c) (g_c: P x 3): albedo (P x 3), rough (P) and env
 * (6 x E x E x 3) are accumulated (+=, caller zeroes; env by atomics); O
 * (P x N) and Lind (P x N x 3) are written -- they are the upstream
 * gradients of the trace's opacity and colour for irgs_trace_backward.  Any
 * pointer may be NULL (skipped). */
typedef struct {
    float* albedo;
    float* rough;
    float* env;
    float* O;
    float* Lind;
} irgs_shade_grads;
irgs_status irgs_mc_shade_backward(const irgs_shade_in* in, const float* g_c, irgs_shade_grads* grads,
                                   void* stream);

/* ---- Relighting variant (the paper's relighting details): the trace with
 * IRGS_FLAG_NORMAL blends albedo (3), roughness (1) and the ray-facing
 * normal with weights T_i alpha_i (normalised here by O), and each ray's
 * indirect radiance is shaded in one query with the split-sum
 * approximation; the result feeds irgs_mc_shade as L_ind. */

/* Pre-integrated sky (DEVICE buffers): irr (6 x E x E x 3) = irradiance
 * sum_w L(w) max(w . c, 0) dOmega(w) at every texel centre c (NULL: skip);
 * pref (M x 6 x E x E x 3) = the sky prefiltered with the GGX lobe of
 * roughness r_l = (l + 1) / M around c (normal = view = c):
 * sum L(w) D_r(c . h) max(w . c, 0) dOmega / the same sum without L,
 * h = normalise(w + c).  Texel centres and solid angles
 * 4 / (E^2 (1 + s^2 + t^2)^{3/2}) follow the cube addressing of
 * irgs_mc_shade.  1 <= E <= 256, 0 <= M <= 32. */
irgs_status irgs_env_prefilter(int32_t E, const float* env, int32_t M, float* irr, float* pref, void* stream);

/* Split-sum BRDF table (S x S x 2, DEVICE) at cell centres
 * (n.v, r) = ((i + 1/2)/S, (j + 1/2)/S): (S_A, S_B) estimated with GGX
 * importance sampling over 256 Hammersley points ((k + 1/2)/256, bit-reversed
 * k / 2^32); per sample with n.l > 0, g = G (v.h) / ((n.h)(n.v)),
 * F_c = (1 - v.h)^5, S_A += (1 - F_c) g, S_B += F_c g; G as in
 * irgs_mc_shade.  1 <= S <= 1024. */
irgs_status irgs_brdf_table(int32_t S, float* table, void* stream);

/* Indirect radiance (R x 3, written) of each ray from its trace outputs O (R)
 * and Fo (R x 7: albedo, roughness, normal channels of IRGS_FLAG_NORMAL):
 * A = Fo[0:3] / O, R = clamp(Fo[3] / O, 0, 1), N = normalise(Fo[4:7]), v = -d,
 * L_ind = A / pi E(N) + P_R(reflect(d, N)) (0.04 S_A(n.v, R) + S_B(n.v, R))
 * with nearest texel, level clamp(floor(R M + 1/2) - 1, 0, M - 1) and table
 * cell (floor(n.v S), floor(R S)); 0 for a ray with O = 0. */
irgs_status irgs_relight_lind(int64_t R, const float* O, const float* Fo, const float* rd, int32_t E, const float* irr,
                              int32_t M, const float* pref, int32_t S, const float* table, float* lind, void* stream);

/* Importance sampling of the sky by its intensity, which the paper's
 * relighting uses in place of the stratified hemisphere.
 * irgs_env_cdf: cdf (6 E^2, DEVICE, written) = the inclusive running sum,
 * in texel order (face, row, col), of max(mean RGB, 0) times the texel's
 * solid angle 4 / (E^2 (1 + s^2 + t^2)^{3/2}) at its centre (a NaN texel
 * weighs 0), accumulated in FP64 and rounded once to FP32.  The sky must be
 * finite.  1 <= E <= 256. */
irgs_status irgs_env_cdf(int32_t E, const float* env, float* cdf, void* stream);

/* Rays drawn from a sky CDF: sample (p, i) with uniforms u[p, i] = (u0, u1,
 * u2) in [0, 1) takes the first texel j whose cdf exceeds u0 * total (FP32
 * product; total = cdf[6 E^2 - 1]), the point (s, t) = ((col + u1), (row +
 * u2)) 2 / E - 1 of that texel (uniform in the face coordinates of
 * irgs_mc_shade), rd = its unit direction, ro = x_p + offset n_p, and
 * wgt = 1 / (N pdf) with pdf = p_j E^2 / 4 (1 + s^2 + t^2)^{3/2},
 * p_j = (cdf[j] - cdf[j - 1]) / total; wgt = 0 where rd . n_p <= 0 or the
 * sky's total weight is not positive.  Texels of zero intensity are never
 * drawn.  x, n: P x 3; u: P x N x 3; ro, rd: (P N) x 3 and wgt: P N,
 * written.  N >= 1, P >= 0, 1 <= E <= 256. */
irgs_status irgs_env_rays(int64_t P, int32_t N, const float* x, const float* n, const float* u, int32_t E,
                          const float* cdf, float offset, float* ro, float* rd, float* wgt, void* stream);

const char* irgs_status_str(irgs_status status);
const char* irgs_last_error(void);
const char* irgs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IRGS_H */
