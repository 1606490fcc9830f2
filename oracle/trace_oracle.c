/*
 * FP64 brute-force oracle for 2D Gaussian ray tracing (2DGRT).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the package smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP library.
 *
 * What it computes (the plain definition of the trace, Sec. 3.2):
 *   every ray is tested against every surfel; the accepted hits are sorted
 *   by depth and alpha-composited front to back (Eq. 2) until the
 *   transmittance falls below a cutoff.  The k-buffer marching of the paper
 *   only reorganises this work ("exact ordering of intersected Gaussians",
 *   Sec. 3.2), so the plain definition is the oracle.
 *
 * Surfel frame (Sec. 3.1 quaternion parameterisation, Sec. 3.2 tangents):
 *   q = (w,x,y,z) is normalised; t_u, t_v are the first two columns of the
 *   rotation matrix of q, and n = t_u x t_v (Eq. 6).
 * Ray-splat intersection (Eq. 6):  tau = n.(mu - r_o) / n.(r_d),
 *   p = r_o + tau r_d.
 * Influence (Eq. 7):  u = (p-mu).t_u / s_u,  v = (p-mu).t_v / s_v,
 *   G = exp(-(u^2+v^2)/2),  alpha = o G.
 * Readings where the paper gives no value or rule:
 *   - a hit needs t_min < tau < t_max, u^2+v^2 <= sigma^2 and
 *     alpha >= alpha_min (both inclusive); n.r_d == 0 or a non-finite tau is
 *     a miss;
 *   - hits are ordered by (tau, surfel index), ascending;
 *   - compositing includes a hit, then stops once T < T_min (strict);
 *   - the depth output is the unnormalised sum of T_i alpha_i tau_i;
 *   - a ray with a non-finite component or a zero direction misses
 *     everything; a surfel with a non-finite parameter, a zero quaternion or
 *     a non-positive scale is never hit.
 *
 * View-dependent colour (Sec. 3.1: each Gaussian's colour is modelled by
 * spherical harmonics, and the trace uses that colour, Sec. 3.3): with
 * sh_deg >= 0 the F features of a surfel are RGB coefficients of the real SH
 * basis up to degree sh_deg, coefficient-major (F = 3 (sh_deg + 1)^2), and
 * the colour a ray sees is, per channel, max(sum_j Y_j(d) k_j + 1/2, 0) with
 * d the normalised ray direction.  Readings (the paper names SH only): the
 * basis is sqrt(2) Re / sqrt(2) Im of the complex harmonics with the
 * Condon-Shortley phase for m > 0 / m < 0, index j = l^2 + l + m; the 1/2
 * offset and the clamp at 0 are those of the Gaussian-splatting colour
 * model; the composited feature output then has 3 channels.
 *
 * Normal channels (relighting: the trace blends albedo, roughness and the
 * normal): with with_normal = 1 each hit also contributes its unit normal
 * n, negated when n . r_d > 0 so that it faces the ray, as 3 more channels
 * after the features.
 *
 * All inputs are FP64 (callers widen FP32 data exactly).  OpenMP over rays.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double alpha_min;
    double T_min;
    double t_min;
    double t_max;
    double sigma; /* support radius in units of the scales */
    int32_t sh_deg; /* -1: plain features; 0..3: RGB SH coefficients */
    int32_t with_normal; /* 1: 3 more channels, each hit's unit normal turned to face the ray */
} orc_params;

typedef struct {
    double mu[3], tu[3], tv[3], n[3];
    double su, sv, o;
    int valid;
} orc_surfel;

typedef struct {
    double tau;
    double alpha;
    int32_t id;
} orc_hit;

static const double kPi = 3.14159265358979323846;

static int finite3(const double* v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Columns of the rotation matrix of the unit quaternion (w,x,y,z). */
static void quat_columns(const double* q_in, double* c0, double* c1, double* valid_norm)
{
    double nrm = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    *valid_norm = nrm;
    double w = q_in[0] / nrm, x = q_in[1] / nrm, y = q_in[2] / nrm, z = q_in[3] / nrm;
    c0[0] = 1.0 - 2.0 * (y * y + z * z);
    c0[1] = 2.0 * (x * y + w * z);
    c0[2] = 2.0 * (x * z - w * y);
    c1[0] = 2.0 * (x * y - w * z);
    c1[1] = 1.0 - 2.0 * (x * x + z * z);
    c1[2] = 2.0 * (y * z + w * x);
}

static void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void make_surfel(const double* mu, const double* q, const double* s, double o, orc_surfel* out)
{
    double qn;
    memcpy(out->mu, mu, sizeof(double) * 3);
    quat_columns(q, out->tu, out->tv, &qn);
    cross3(out->tu, out->tv, out->n);
    out->su = s[0];
    out->sv = s[1];
    out->o = o;
    out->valid = finite3(mu) && isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]) &&
                 qn > 0.0 && isfinite(qn) && isfinite(s[0]) && isfinite(s[1]) && s[0] > 0.0 && s[1] > 0.0 &&
                 isfinite(o);
}

void orc_surfel_frames(int64_t N, const double* quat, double* tu, double* tv, double* nrm)
{
    for (int64_t i = 0; i < N; ++i) {
        double qn;
        quat_columns(quat + 4 * i, tu + 3 * i, tv + 3 * i, &qn);
        cross3(tu + 3 * i, tv + 3 * i, nrm + 3 * i);
    }
}

/* Associated Legendre function P_l^m(x), 0 <= m <= l, with the
 * Condon-Shortley phase, by the standard upward recurrence in l. */
static double legendre(int l, int m, double x)
{
    double pmm = 1.0;
    const double sx = sqrt(fmax(0.0, 1.0 - x * x));
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * sx;
    if (l == m) return pmm;
    double p1 = x * (2.0 * m + 1.0) * pmm; /* P_{m+1}^m */
    if (l == m + 1) return p1;
    double p0 = pmm, pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((2.0 * ll - 1.0) * x * p1 - (ll + m - 1.0) * p0) / (ll - m);
        p0 = p1;
        p1 = pl;
    }
    return pl;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* Real SH basis of the unit direction d (normalised here), degrees 0..deg:
 * Y[l*l + l + m].  Polar angle from +z, azimuth from +x towards +y. */
static void sh_basis(const double* d_in, int deg, double* Y)
{
    const double nrm = sqrt(dot3(d_in, d_in));
    const double ct = d_in[2] / nrm;
    const double phi = atan2(d_in[1], d_in[0]);
    for (int l = 0; l <= deg; ++l) {
        for (int m = 0; m <= l; ++m) {
            const double N = sqrt((2.0 * l + 1.0) / (4.0 * kPi) * factorial(l - m) / factorial(l + m));
            const double P = legendre(l, m, ct);
            if (m == 0) {
                Y[l * l + l] = N * P;
            } else {
                Y[l * l + l + m] = sqrt(2.0) * N * P * cos(m * phi);
                Y[l * l + l - m] = sqrt(2.0) * N * P * sin(m * phi);
            }
        }
    }
}

void orc_sh_basis(int64_t n, const double* dirs, int32_t deg, double* Y)
{
    const int nb = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < n; ++i) sh_basis(dirs + 3 * i, deg, Y + i * nb);
}

/* Unit normal of surfel S turned to face the ray direction d. */
static void facing_normal(const orc_surfel* S, const double* d, double* out)
{
    const double s = dot3(S->n, d) > 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < 3; ++k) out[k] = s * S->n[k];
}

/* Colour of one surfel seen along the ray whose basis is Y (3 channels). */
static void sh_colour(const double* k, int deg, const double* Y, double* col)
{
    const int nb = (deg + 1) * (deg + 1);
    for (int c = 0; c < 3; ++c) {
        double v = 0.5;
        for (int j = 0; j < nb; ++j) v += Y[j] * k[3 * j + c];
        col[c] = v > 0.0 ? v : 0.0;
    }
}

static int ray_ok(const double* ro, const double* rd)
{
    return finite3(ro) && finite3(rd) && (rd[0] != 0.0 || rd[1] != 0.0 || rd[2] != 0.0);
}

/* Eq. 6-7 for one (ray, surfel) pair.  Returns 1 when tau is finite and
 * inside (t_min, t_max): a candidate.  *is_hit tells whether it also passes
 * the support and alpha_min tests. */
static int evaluate(const orc_surfel* S, const double* ro, const double* rd, const orc_params* P,
                    double* tau_out, double* rho2_out, double* alpha_out, int* is_hit)
{
    *is_hit = 0;
    if (!S->valid) return 0;
    double den = dot3(S->n, rd);
    if (den == 0.0) return 0;
    double dm[3] = {S->mu[0] - ro[0], S->mu[1] - ro[1], S->mu[2] - ro[2]};
    double tau = dot3(S->n, dm) / den;
    if (!isfinite(tau)) return 0;
    if (!(tau > P->t_min && tau < P->t_max)) return 0;
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = ro[k] + tau * rd[k] - S->mu[k];
    double u = dot3(d, S->tu) / S->su;
    double v = dot3(d, S->tv) / S->sv;
    double rho2 = u * u + v * v;
    double alpha = S->o * exp(-0.5 * rho2);
    *tau_out = tau;
    *rho2_out = rho2;
    *alpha_out = alpha;
    *is_hit = (rho2 <= P->sigma * P->sigma) && (alpha >= P->alpha_min);
    return 1;
}

static int cmp_hit(const void* a, const void* b)
{
    const orc_hit* x = (const orc_hit*)a;
    const orc_hit* y = (const orc_hit*)b;
    if (x->tau < y->tau) return -1;
    if (x->tau > y->tau) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

static orc_surfel* build_surfels(int64_t N, const double* mu, const double* quat, const double* scale,
                                 const double* opac)
{
    orc_surfel* S = (orc_surfel*)malloc(sizeof(orc_surfel) * (size_t)(N > 0 ? N : 1));
    if (!S) return NULL;
    for (int64_t i = 0; i < N; ++i) make_surfel(mu + 3 * i, quat + 4 * i, scale + 2 * i, opac[i], &S[i]);
    return S;
}

static void set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Full trace of R rays.  Outputs (FP64): O (R), Fo (R*F), D (R), T (R),
 * n_hits (R).  When hits != NULL the first hit_cap composited surfel indices
 * of each ray are written to hits[r*hit_cap ...] (rest filled with -1).
 * Returns 0, or -1 on allocation failure. */
int orc_trace(int64_t N, int32_t F, const double* mu, const double* quat, const double* scale,
              const double* opac, const double* feat, int64_t R, const double* ro, const double* rd,
              const orc_params* P, double* O, double* Fo, double* D, double* T, int32_t* n_hits,
              int32_t hit_cap, int32_t* hits, int32_t nthreads)
{
    orc_surfel* S = build_surfels(N, mu, quat, scale, opac);
    if (!S) return -1;
    set_threads(nthreads);
    int failed = 0;
#pragma omp parallel
    {
        size_t cap = 256;
        orc_hit* buf = (orc_hit*)malloc(sizeof(orc_hit) * cap);
        if (!buf) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < R; ++r) {
            if (!buf) continue;
            const double* o_r = ro + 3 * r;
            const double* d_r = rd + 3 * r;
            double acc_O = 0.0, acc_D = 0.0, trans = 1.0;
            const int FC = P->sh_deg >= 0 ? 3 : F;
            const int FO = FC + (P->with_normal ? 3 : 0);
            double* acc_F = Fo + (size_t)r * FO;
            for (int c = 0; c < FO; ++c) acc_F[c] = 0.0;
            double Y[16];
            if (P->sh_deg >= 0 && ray_ok(o_r, d_r)) sh_basis(d_r, P->sh_deg, Y);
            int32_t* my_hits = hits ? hits + (size_t)r * hit_cap : NULL;
            if (my_hits)
                for (int32_t h = 0; h < hit_cap; ++h) my_hits[h] = -1;
            size_t nh = 0;
            if (ray_ok(o_r, d_r)) {
                for (int64_t i = 0; i < N; ++i) {
                    double tau, rho2, alpha;
                    int is_hit;
                    if (!evaluate(&S[i], o_r, d_r, P, &tau, &rho2, &alpha, &is_hit) || !is_hit) continue;
                    if (nh == cap) {
                        cap *= 2;
                        orc_hit* nb = (orc_hit*)realloc(buf, sizeof(orc_hit) * cap);
                        if (!nb) {
#pragma omp atomic write
                            failed = 1;
                            break;
                        }
                        buf = nb;
                    }
                    buf[nh].tau = tau;
                    buf[nh].alpha = alpha;
                    buf[nh].id = (int32_t)i;
                    ++nh;
                }
                qsort(buf, nh, sizeof(orc_hit), cmp_hit);
            }
            int32_t count = 0;
            for (size_t h = 0; h < nh; ++h) {
                double w = trans * buf[h].alpha;
                acc_O += w;
                const double* f = feat + (size_t)buf[h].id * F;
                if (P->sh_deg >= 0) {
                    double col[3];
                    sh_colour(f, P->sh_deg, Y, col);
                    for (int c = 0; c < 3; ++c) acc_F[c] += w * col[c];
                } else {
                    for (int c = 0; c < F; ++c) acc_F[c] += w * f[c];
                }
                if (P->with_normal) {
                    double nf[3];
                    facing_normal(&S[buf[h].id], d_r, nf);
                    for (int c = 0; c < 3; ++c) acc_F[FC + c] += w * nf[c];
                }
                acc_D += w * buf[h].tau;
                trans *= (1.0 - buf[h].alpha);
                if (my_hits && count < hit_cap) my_hits[count] = buf[h].id;
                ++count;
                if (trans < P->T_min) break;
            }
            O[r] = acc_O;
            D[r] = acc_D;
            T[r] = trans;
            n_hits[r] = count;
        }
        free(buf);
    }
    free(S);
    return failed ? -1 : 0;
}

/* Near-hit candidates of R rays: every surfel with a finite tau in
 * (t_min, t_max) whose u^2+v^2 is at most sigma^2 (1 + band) and whose alpha
 * is at least alpha_min (1 - band) -- the hits plus the non-hits that lie
 * within `band` (relative) of a threshold.  Per ray up to `cap` entries
 * (ids, tau, rho2, alpha, hit flag) in surfel order; counts[r] is the true
 * number (may exceed cap). */
int orc_candidates(int64_t N, const double* mu, const double* quat, const double* scale, const double* opac,
                   int64_t R, const double* ro, const double* rd, const orc_params* P, double band, int32_t cap,
                   int32_t* ids, double* tau, double* rho2, double* alpha, int8_t* hit, int32_t* counts,
                   int32_t nthreads)
{
    orc_surfel* S = build_surfels(N, mu, quat, scale, opac);
    if (!S) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < R; ++r) {
        const double* o_r = ro + 3 * r;
        const double* d_r = rd + 3 * r;
        int32_t cnt = 0;
        if (ray_ok(o_r, d_r)) {
            for (int64_t i = 0; i < N; ++i) {
                double t, p2, a;
                int is_hit;
                if (!evaluate(&S[i], o_r, d_r, P, &t, &p2, &a, &is_hit)) continue;
                if (!is_hit && !(p2 <= P->sigma * P->sigma * (1.0 + band) && a >= P->alpha_min * (1.0 - band)))
                    continue;
                if (cnt < cap) {
                    size_t k = (size_t)r * cap + cnt;
                    ids[k] = (int32_t)i;
                    tau[k] = t;
                    rho2[k] = p2;
                    alpha[k] = a;
                    hit[k] = (int8_t)is_hit;
                }
                ++cnt;
            }
        }
        counts[r] = cnt;
    }
    free(S);
    return 0;
}

/* FP64 replay of given ordered hit lists: list[r*H ... ] holds len[r] surfel
 * indices, composited in that order with no threshold and no early stop.
 * Outputs O, Fo, D, T after the whole list; Tpre[r*H + h] = transmittance
 * after hit h; tau_out/alpha_out per hit (NULL to skip). */
int orc_replay(int64_t N, int32_t F, const double* mu, const double* quat, const double* scale,
               const double* opac, const double* feat, int64_t R, const double* ro, const double* rd,
               int32_t H, const int32_t* list, const int32_t* len, double* O, double* Fo, double* D, double* T,
               double* Tpost, double* tau_out, double* alpha_out, int32_t sh_deg, int32_t with_normal,
               int32_t nthreads)
{
    orc_surfel* S = build_surfels(N, mu, quat, scale, opac);
    if (!S) return -1;
    set_threads(nthreads);
    orc_params loose = {0.0, 0.0, -INFINITY, INFINITY, INFINITY, sh_deg, with_normal};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < R; ++r) {
        const double* o_r = ro + 3 * r;
        const double* d_r = rd + 3 * r;
        double acc_O = 0.0, acc_D = 0.0, trans = 1.0;
        const int FC = sh_deg >= 0 ? 3 : F;
        const int FO = FC + (with_normal ? 3 : 0);
        double* acc_F = Fo + (size_t)r * FO;
        for (int c = 0; c < FO; ++c) acc_F[c] = 0.0;
        double Y[16];
        if (sh_deg >= 0 && ray_ok(o_r, d_r)) sh_basis(d_r, sh_deg, Y);
        for (int32_t h = 0; h < len[r] && h < H; ++h) {
            int32_t id = list[(size_t)r * H + h];
            double t = NAN, p2, a = NAN;
            int is_hit;
            if (id >= 0 && id < N) evaluate(&S[id], o_r, d_r, &loose, &t, &p2, &a, &is_hit);
            double w = trans * a;
            acc_O += w;
            const double* f = feat + (size_t)id * F;
            if (sh_deg >= 0) {
                double col[3];
                sh_colour(f, sh_deg, Y, col);
                for (int c = 0; c < 3; ++c) acc_F[c] += w * col[c];
            } else {
                for (int c = 0; c < F; ++c) acc_F[c] += w * f[c];
            }
            if (with_normal && id >= 0 && id < N) {
                double nf[3];
                facing_normal(&S[id], d_r, nf);
                for (int c = 0; c < 3; ++c) acc_F[FC + c] += w * nf[c];
            }
            acc_D += w * t;
            trans *= (1.0 - a);
            if (Tpost) Tpost[(size_t)r * H + h] = trans;
            if (tau_out) tau_out[(size_t)r * H + h] = t;
            if (alpha_out) alpha_out[(size_t)r * H + h] = a;
        }
        O[r] = acc_O;
        D[r] = acc_D;
        T[r] = trans;
    }
    free(S);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
