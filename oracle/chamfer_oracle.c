/*
 * CPU oracle for the near-linear Chamfer estimator (Bakshi, Indyk, Jayaram,
 * Silwal, Waingarten, "A Near-Linear Time Algorithm for the Chamfer Distance").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Nothing in the product path may include,
 * link or call it; it shares no source with the GPU library.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 *        -fno-fast-math chamfer_oracle.c -lm
 * (-ffp-contract=off: every float operation below is one IEEE operation,
 *  rounded to nearest even; fused multiply-adds appear only where fmaf is
 *  written, and they are part of the definition there.)
 *
 * Conventions fixed here (each is a reading of the paper; the paper leaves
 * them open):
 *   - distances are not squared (footnote to the definition of CH in the
 *     introduction);
 *   - "dist32" is the canonical single-precision distance: k ascending,
 *     l1: acc = acc + |a_k - b_k|, l2: acc = fmaf(t, t, acc) with
 *     t = a_k - b_k, then sqrtf(acc).  It is used where a float decides an
 *     integer (the crude distance D_a, and arg-mins);
 *   - the exact Chamfer distance is computed in double precision from the
 *     float inputs (which convert exactly), l2 by direct differences.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_L1 1
#define OR_L2 2

/* Threads the OpenMP loops below use (1 without OpenMP). */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (n >= 1; no-op without OpenMP). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Purposes of the counter-based random streams (third counter word). */
#define PURPOSE_GRID 1u
#define PURPOSE_EMBED 2u
#define PURPOSE_SAMPLE 3u

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC 2011).  Ten rounds of two 64x64->128 multiplies,    */
/* with the key bumped by the Weyl constants between rounds.                */
/* ------------------------------------------------------------------------ */
void or_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw_rep(uint64_t seed, uint64_t c0, uint64_t c1, uint32_t purpose, uint64_t rep,
                     uint64_t out[4])
{
    uint64_t ctr[4] = {c0, c1, (uint64_t)purpose, rep};
    uint64_t key[2] = {seed, 0};
    or_philox4x64(ctr, key, out);
}

static void draw(uint64_t seed, uint64_t c0, uint64_t c1, uint32_t purpose, uint64_t out[4])
{
    uint64_t ctr[4] = {c0, c1, (uint64_t)purpose, 0};
    uint64_t key[2] = {seed, 0};
    or_philox4x64(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Hash family at every scale (appendix lemma constructing an LSH at every  */
/* scale): h(x)_k = ceil((x_k + z_k) / r) with z ~ U[0, r]^k.  Written in   */
/* cell units with floor: floor(x_k / r + z'_k), z'_k = z_k / r ~ U[0, 1)   */
/* (floor and ceil differ by one except on the cell boundaries, a set the   */
/* shift hits with probability 0, so the two grids are the same family).    */
/* For scale i and hashed coordinate k the oracle draws                    */
/*   z'_ik = (word0 >> 40) * 2^-24            (24-bit lattice in [0, 1))     */
/*   M_ik  = M1 | M2 << 32, two odd 24-bit key multipliers:                  */
/*           M1 = (word1 & 0xffffff) | 1, M2 = ((word1 >> 32) & 0xffffff) | 1 */
/* from the counter (k, i, GRID, rep): rep numbers the independent LSH      */
/* structures of the repeated variant (0 for the single structure).         */
/* zfrac and mult are [L][kh].                                               */
/* ------------------------------------------------------------------------ */
static uint64_t key_multipliers(uint64_t word1)
{
    uint64_t m1 = (word1 & 0xffffffull) | 1ull;
    uint64_t m2 = ((word1 >> 32) & 0xffffffull) | 1ull;
    return m1 | (m2 << 32);
}

void or_grid_tables_rep(uint64_t seed, uint64_t rep, int L, int kh, float *zfrac, uint64_t *mult)
{
    for (int i = 0; i < L; ++i)
        for (int k = 0; k < kh; ++k) {
            uint64_t w[4];
            draw_rep(seed, (uint64_t)k, (uint64_t)i, PURPOSE_GRID, rep, w);
            zfrac[(size_t)i * kh + k] = ldexpf((float)(w[0] >> 40), -24);
            mult[(size_t)i * kh + k] = key_multipliers(w[1]);
        }
}

void or_grid_tables(uint64_t seed, int L, int kh, float *zfrac, uint64_t *mult)
{
    for (int i = 0; i < L; ++i)
        for (int k = 0; k < kh; ++k) {
            uint64_t w[4];
            draw(seed, (uint64_t)k, (uint64_t)i, PURPOSE_GRID, w);
            zfrac[(size_t)i * kh + k] = ldexpf((float)(w[0] >> 40), -24);
            mult[(size_t)i * kh + k] = key_multipliers(w[1]);
        }
}

/* ------------------------------------------------------------------------ */
/* l2 -> l1 embedding (appendix theorem on embedding l2 into l1):           */
/* T(x)_j = (1 / (beta k)) sum_i Z_ji x_i, beta = sqrt(2/pi), Z Gaussian.   */
/* Finite-precision form: the Gaussian entries are quantised to integers,  */
/* Zq_jk = clamp(rint(32 g_jk), -127, 127), with g_jk from Box-Muller on    */
/* the counter (j*d + k, 0, EMBED):                                          */
/*   u1 = ((w0 >> 11) + 1) 2^-53 in (0, 1], u2 = (w1 >> 11) 2^-53 in [0, 1)*/
/*   g  = sqrt(-2 ln u1) cos(2 pi u2)                                        */
/* so that the embedding of quantised coordinates is an exact integer dot   */
/* product (hashed_coords below).  Zq is [ke][d].                            */
/* ------------------------------------------------------------------------ */
#define EMBED_SCALE 32.0 /* Zq ~ 32 g */
#define EMBED_QBITS 24   /* coordinates quantised to 24 bits of the span */

void or_embedding(uint64_t seed, int d, int ke, int8_t *Zq)
{
    const double two_pi = 2.0 * 3.14159265358979323846;
    for (int j = 0; j < ke; ++j)
        for (int k = 0; k < d; ++k) {
            uint64_t w[4];
            draw(seed, (uint64_t)j * (uint64_t)d + (uint64_t)k, 0, PURPOSE_EMBED, w);
            double u1 = ldexp((double)((w[0] >> 11) + 1), -53);
            double u2 = ldexp((double)(w[1] >> 11), -53);
            double g = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
            double q = rint(EMBED_SCALE * g);
            if (q > 127.0) q = 127.0;
            if (q < -127.0) q = -127.0;
            Zq[(size_t)j * d + k] = (int8_t)q;
        }
}

/* smallest integer e with 2^e >= x, for x > 0 */
static int ceil_log2_double(double x)
{
    int e;
    double m = frexp(x, &e); /* x = m 2^e, m in [0.5, 1) */
    return (m == 0.5) ? e - 1 : e;
}

/* Default number of scales: L = ceil(log2(max(nA, nB) / eps)), the
 * L = O(log(n/eps)) of the CrudeNN figure, clamped to [1, 64]. */
int or_default_scales(int64_t nA, int64_t nB, double eps)
{
    int64_t n = nA > nB ? nA : nB;
    if (n < 1) n = 1;
    int L = ceil_log2_double((double)n / eps);
    if (L < 1) L = 1;
    if (L > 64) L = 64;
    return L;
}

/* Default number of samples: T = ceil(ceil(log2 nA) / eps^2), the
 * T = O(log(n)/eps^2) of the main theorem's proof, at least 1. */
int64_t or_default_samples(int64_t nA, double eps)
{
    int q = 0;
    while (((int64_t)1 << q) < nA) ++q;
    int64_t T = (int64_t)ceil((double)q / (eps * eps));
    return T < 1 ? 1 : T;
}

/* ------------------------------------------------------------------------ */
/* Scale calibration.  The CrudeNN figure assumes distances in             */
/* [1, poly(n/eps)] and uses r_i = 2^i; this oracle instead takes the top   */
/* scale from the data: lo_k/hi_k = per-coordinate min/max over A u B,      */
/* S = sum_k (hi_k - lo_k) (double, k ascending) bounds every l1 (hence l2) */
/* distance, e_top = smallest e with 2^e >= S (0 if S == 0), and scale i of */
/* L (0 = finest) has side r_i = 2^(e_top - (L - 1 - i)).                   */
/* ------------------------------------------------------------------------ */
void or_calibrate(const float *A, int64_t nA, const float *B, int64_t nB, int d,
                  float *lo, float *hi, double *S_out, int *e_top_out)
{
    for (int k = 0; k < d; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int64_t r = 0; r < nA + nB; ++r) {
        const float *x = r < nA ? A + (size_t)r * d : B + (size_t)(r - nA) * d;
        for (int k = 0; k < d; ++k) {
            if (x[k] < lo[k]) lo[k] = x[k];
            if (x[k] > hi[k]) hi[k] = x[k];
        }
    }
    double S = 0.0;
    for (int k = 0; k < d; ++k) S = S + ((double)hi[k] - (double)lo[k]);
    *S_out = S;
    *e_top_out = (S > 0.0) ? ceil_log2_double(S) : 0;
}

/* Coordinates that get hashed.  l1: y = x - lo (d of them, float32).
 * l2 (ke of them): the coordinates quantised to 24 bits of the span,
 *   u_k = floor(min((x_k - lo_k) 2^(24 - e_top), 2^24 - 1))
 * (x_k - lo_k a float32 subtraction, the scaling exact), their exact
 * integer embedding Y_j = sum_k Zq_jk u_k, and
 *   y_j = (float)((Y_j 2^(e_top - 24)) / (beta ke 32))
 * with the division a multiplication by 1 / (beta ke 32) in double
 * (Y_j 2^(e_top - 24) is exact in double, |Y_j| < 2^53), so y approximates
 * the embedding T(x - lo) of the theorem. */
static void hashed_coords(const float *x, int d, int metric, const float *lo, int e_top,
                          const int8_t *Zq, int ke, float *y)
{
    if (metric == OR_L1) {
        for (int k = 0; k < d; ++k) y[k] = x[k] - lo[k];
        return;
    }
    const double inv = 1.0 / (sqrt(2.0 / 3.14159265358979323846) * (double)ke * EMBED_SCALE);
    for (int j = 0; j < ke; ++j) {
        int64_t Y = 0;
        for (int k = 0; k < d; ++k) {
            float v = ldexpf(x[k] - lo[k], EMBED_QBITS - e_top);
            int64_t u = (int64_t)floorf(fminf(v, 16777215.0f));
            Y += (int64_t)Zq[(size_t)j * d + k] * u;
        }
        y[j] = (float)(ldexp((double)Y, e_top - EMBED_QBITS) * inv);
    }
}

/* The hashed coordinates of every point of X, Y[n][kh] (kh = d for l1,
 * ke for l2); exported so the embedding step can be checked on its own. */
void or_hashed_coords(const float *X, int64_t n, int d, int metric, const float *lo, int e_top,
                      const int8_t *Zq, int ke, float *Y)
{
    int kh = metric == OR_L1 ? d : ke;
    for (int64_t p = 0; p < n; ++p)
        hashed_coords(X + (size_t)p * d, d, metric, lo, e_top, Zq, ke, Y + (size_t)p * kh);
}

/* Grid cell of a shifted coordinate q = y / r + z' (float): floor(q) as a
 * 32-bit integer, saturated at the int32 range (q is clamped first, NaN
 * going to the upper bound), so every float maps to one cell. */
static int32_t cell_of(float q)
{
    q = fminf(q, 2147483520.0f); /* the largest float below 2^31 */
    q = fmaxf(q, -2147483648.0f);
    return (int32_t)floorf(q);
}

/* Bucket key of point y at scale i (side 2^e):
 *   cell_k = cell_of(fmaf(y_k, 2^-e, z'_ik))   (y_k 2^-e is exact, so one
 *                                              rounding, of the sum)
 *   K1 = sum_k (cell_k mod 2^24) M1_ik mod 2^32,
 *   K2 = sum_k (cell_k mod 2^24) M2_ik mod 2^32,
 *   key = (K1 2^32 + K2) >> 1
 * (cell_k mod 2^24: the low 24 bits of its two's complement).  Equal cells
 * give equal keys.  Distinct cells whose indices differ in one coordinate
 * by less than 2^24 never share a key (the multipliers are odd); with
 * several differing coordinates they share one with probability about
 * 2^-48 over the multipliers.  Keys fit in 63 bits. */
static uint64_t bucket_key(const float *y, int kh, int e, const float *zf, const uint64_t *M)
{
    const float p = ldexpf(1.0f, -e);
    uint32_t k1 = 0, k2 = 0;
    for (int k = 0; k < kh; ++k) {
        uint32_t c = (uint32_t)cell_of(fmaf(y[k], p, zf[k])) & 0xffffffu;
        k1 += (uint32_t)((uint64_t)c * (M[k] & 0xffffffffull));
        k2 += (uint32_t)((uint64_t)c * (M[k] >> 32));
    }
    return (((uint64_t)k1 << 32) | (uint64_t)k2) >> 1;
}

/* keys[i * n + p] for every point p of X and scale i < L. */
void or_hash_keys(const float *X, int64_t n, int d, int metric, const float *lo,
                  const int8_t *Zs, int ke, int L, int e_top, const float *zfrac,
                  const uint64_t *mult, uint64_t *keys)
{
    int kh = metric == OR_L1 ? d : ke;
    /* points are independent; the loop is split over threads */
#pragma omp parallel
    {
        float *y = (float *)malloc(sizeof(float) * (size_t)kh);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            hashed_coords(X + (size_t)p * d, d, metric, lo, e_top, Zs, ke, y);
            for (int i = 0; i < L; ++i) {
                int e = e_top - (L - 1 - i);
                keys[(size_t)i * n + p] =
                    bucket_key(y, kh, e, zfrac + (size_t)i * kh, mult + (size_t)i * kh);
            }
        }
        free(y);
    }
}

/* Canonical single-precision distance (see header). */
float or_dist32(const float *a, const float *b, int d, int metric)
{
    float acc = 0.0f;
    if (metric == OR_L1) {
        for (int k = 0; k < d; ++k) acc = acc + fabsf(a[k] - b[k]);
        return acc;
    }
    for (int k = 0; k < d; ++k) {
        float t = a[k] - b[k];
        acc = fmaf(t, t, acc);
    }
    return sqrtf(acc);
}

/* Squared accumulator for l2 (before the square root), the l1 sum for l1. */
static float acc32(const float *a, const float *b, int d, int metric)
{
    float acc = 0.0f;
    if (metric == OR_L1) {
        for (int k = 0; k < d; ++k) acc = acc + fabsf(a[k] - b[k]);
        return acc;
    }
    for (int k = 0; k < d; ++k) {
        float t = a[k] - b[k];
        acc = fmaf(t, t, acc);
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* CrudeNN (CrudeNN figure, step 3): for each a the smallest scale i with   */
/* some b in a's bucket; the candidate is the lowest-index such b, and      */
/* D_a = dist32(a, b).  If no scale collides, the candidate is b = 0 (any   */
/* b keeps D_a >= min_b d(a, b)) and the scale is reported as L.            */
/* The join sorts B's (key, index) pairs per scale and binary-searches.     */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t key; int64_t idx; } kv_t;

static int kv_cmp(const void *x, const void *y)
{
    const kv_t *a = (const kv_t *)x, *b = (const kv_t *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

void or_crude_nn(const uint64_t *keysA, int64_t nA, const uint64_t *keysB, int64_t nB,
                 int L, const float *A, const float *B, int d, int metric,
                 int32_t *scale_out, int32_t *nn_out, float *D_out)
{
    kv_t *tab = (kv_t *)malloc(sizeof(kv_t) * (size_t)(nB > 0 ? nB : 1));
    for (int64_t a = 0; a < nA; ++a) { scale_out[a] = -1; nn_out[a] = 0; }
    for (int i = 0; i < L; ++i) {
        for (int64_t b = 0; b < nB; ++b) { tab[b].key = keysB[(size_t)i * nB + b]; tab[b].idx = b; }
        qsort(tab, (size_t)nB, sizeof(kv_t), kv_cmp);
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < nA; ++a) {
            if (scale_out[a] >= 0) continue;
            uint64_t k = keysA[(size_t)i * nA + a];
            int64_t lo = 0, hi = nB; /* first entry with key >= k */
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (tab[mid].key < k) lo = mid + 1; else hi = mid;
            }
            if (lo < nB && tab[lo].key == k) { scale_out[a] = i; nn_out[a] = (int32_t)tab[lo].idx; }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nA; ++a) {
        if (scale_out[a] < 0) { scale_out[a] = L; nn_out[a] = 0; }
        D_out[a] = or_dist32(A + (size_t)a * d, B + (size_t)nn_out[a] * d, d, metric);
    }
    free(tab);
}

/* ------------------------------------------------------------------------ */
/* Window form of the crude join (the large-scale variant of the            */
/* experiments, with window W): walk a's buckets finest scale first and     */
/* retrieve the first W distinct points of B, taking a bucket's points in   */
/* increasing index order; the candidate is the retrieved b with the        */
/* smallest dist32 (ties to the lower b) and D_a that distance.  If no      */
/* scale collides, the window is b = 0 .. min(W, n_B) - 1 and the scale is  */
/* reported as L; otherwise the scale is the first one that collides.       */
/* ------------------------------------------------------------------------ */
void or_crude_window(const uint64_t *keysA, int64_t nA, const uint64_t *keysB, int64_t nB,
                     int L, int W, const float *A, const float *B, int d, int metric,
                     int32_t *scale_out, int32_t *nn_out, float *D_out)
{
    kv_t *tab = (kv_t *)malloc(sizeof(kv_t) * (size_t)(nB > 0 ? nB : 1));
    int64_t *got = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nA > 0 ? nA : 1) * (size_t)W);
    int *ngot = (int *)calloc((size_t)(nA > 0 ? nA : 1), sizeof(int));
    for (int64_t a = 0; a < nA; ++a) scale_out[a] = L;
    for (int i = 0; i < L; ++i) {
        for (int64_t b = 0; b < nB; ++b) { tab[b].key = keysB[(size_t)i * nB + b]; tab[b].idx = b; }
        qsort(tab, (size_t)nB, sizeof(kv_t), kv_cmp);
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < nA; ++a) {
            if (ngot[a] >= W) continue;
            uint64_t k = keysA[(size_t)i * nA + a];
            int64_t lo = 0, hi = nB; /* first entry with key >= k */
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (tab[mid].key < k) lo = mid + 1; else hi = mid;
            }
            int64_t *mine = got + (size_t)a * W;
            for (int64_t e = lo; e < nB && tab[e].key == k && ngot[a] < W; ++e) {
                int seen = 0;
                for (int j = 0; j < ngot[a]; ++j) seen |= mine[j] == tab[e].idx;
                if (!seen) {
                    if (ngot[a] == 0) scale_out[a] = i;
                    mine[ngot[a]++] = tab[e].idx;
                }
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nA; ++a) {
        int64_t *mine = got + (size_t)a * W;
        if (ngot[a] == 0)
            for (int64_t b = 0; b < W && b < nB; ++b) mine[ngot[a]++] = b;
        float best = 0.0f;
        int64_t arg = -1;
        for (int j = 0; j < ngot[a]; ++j) {
            float v = or_dist32(A + (size_t)a * d, B + (size_t)mine[j] * d, d, metric);
            if (arg < 0 || v < best || (v == best && mine[j] < arg)) { best = v; arg = mine[j]; }
        }
        nn_out[a] = (int32_t)arg;
        D_out[a] = best;
    }
    free(ngot);
    free(got);
    free(tab);
}

/* ------------------------------------------------------------------------ */
/* Exact nearest neighbours (the definition of CH in the introduction).     */
/* or_nn_f64: min over b in double precision, l2 by direct differences,     */
/*            arg-min ties to the lower b.                                   */
/* or_nn_f32: min over b of (dist32 accumulator, b), i.e. the canonical     */
/*            float arg-min; returns dist32 of the winner.                   */
/* rows (nullable) selects rows of X.                                        */
/* ------------------------------------------------------------------------ */
void or_nn_f64(const float *X, int64_t nx, const int32_t *rows, const float *B, int64_t nb,
               int d, int metric, double *mind, int32_t *arg)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nx; ++r) {
        const float *x = X + (size_t)(rows ? rows[r] : r) * d;
        double best = INFINITY;
        int64_t bi = 0;
        for (int64_t b = 0; b < nb; ++b) {
            const float *y = B + (size_t)b * d;
            double s = 0.0;
            if (metric == OR_L1) {
                for (int k = 0; k < d; ++k) s += fabs((double)x[k] - (double)y[k]);
            } else {
                for (int k = 0; k < d; ++k) {
                    double t = (double)x[k] - (double)y[k];
                    s += t * t;
                }
                s = sqrt(s);
            }
            if (s < best) { best = s; bi = b; }
        }
        mind[r] = best;
        arg[r] = (int32_t)bi;
    }
}

void or_nn_f32(const float *X, int64_t nx, const int32_t *rows, const float *B, int64_t nb,
               int d, int metric, float *mind, int32_t *arg)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nx; ++r) {
        const float *x = X + (size_t)(rows ? rows[r] : r) * d;
        float best = INFINITY;
        int64_t bi = 0;
        for (int64_t b = 0; b < nb; ++b) {
            float s = acc32(x, B + (size_t)b * d, d, metric);
            if (s < best) { best = s; bi = b; }
        }
        mind[r] = metric == OR_L1 ? best : sqrtf(best);
        arg[r] = (int32_t)bi;
    }
}

/* ------------------------------------------------------------------------ */
/* Importance-sampling distribution (Chamfer-Estimate figure, steps 1-2) in */
/* 64-bit fixed point.  With maxD = max_a D_a in [2^(e-1), 2^e) and         */
/* q = ceil(log2 nA):  s = 47 - q - e,  w_a = ceil(D_a 2^s) (exact),         */
/* P = inclusive prefix of w, W = P[nA-1] <= 2^47.  Pr[x = a] = w_a / W and */
/* D = W 2^-s.  Returns 0, or 1 when every D_a is 0 (then w = P = W = 0).   */
/* ------------------------------------------------------------------------ */
int or_weights(const float *D, int64_t nA, int *s_out, uint64_t *w, uint64_t *P, uint64_t *W_out)
{
    float maxD = 0.0f;
    for (int64_t a = 0; a < nA; ++a) if (D[a] > maxD) maxD = D[a];
    if (!(maxD > 0.0f)) {
        for (int64_t a = 0; a < nA; ++a) { w[a] = 0; P[a] = 0; }
        *s_out = 0; *W_out = 0;
        return 1;
    }
    int e;
    frexp((double)maxD, &e);
    int q = 0;
    while (((int64_t)1 << q) < nA) ++q;
    int s = 47 - q - e;
    uint64_t run = 0;
    for (int64_t a = 0; a < nA; ++a) {
        w[a] = (uint64_t)ceil(ldexp((double)D[a], s));
        run += w[a];
        P[a] = run;
    }
    *s_out = s;
    *W_out = run;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* T i.i.d. draws x ~ w/W (Chamfer-Estimate figure, step 3).  Draw l uses   */
/* word0 of the counter (l, attempt, SAMPLE) and Lemire's bounded-integer   */
/* method (ACM TOMACS 2019): m = x W (128-bit), reject while the low half   */
/* is below (2^64 - W) mod W, u = m >> 64 is uniform on [0, W); the sample  */
/* is the first a with P[a] > u.                                             */
/* ------------------------------------------------------------------------ */
void or_sample(uint64_t seed, const uint64_t *P, int64_t nA, uint64_t W, int64_t T, int32_t *idx)
{
    for (int64_t l = 0; l < T; ++l) {
        uint64_t u = 0;
        for (uint64_t attempt = 0;; ++attempt) {
            uint64_t w4[4];
            draw(seed, (uint64_t)l, attempt, PURPOSE_SAMPLE, w4);
            unsigned __int128 m = (unsigned __int128)w4[0] * W;
            uint64_t low = (uint64_t)m;
            if (low < W) {
                uint64_t t = (0 - W) % W;
                if (low < t) continue;
            }
            u = (uint64_t)(m >> 64);
            break;
        }
        int64_t lo = 0, hi = nA - 1; /* first a with P[a] > u */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (P[mid] > u) hi = mid; else lo = mid + 1;
        }
        idx[l] = (int32_t)lo;
    }
}

/* ------------------------------------------------------------------------ */
/* Reduction to bounded aspect ratio (lemma on the reduction to poly(n/eps)  */
/* aspect ratio and its proof in the appendix).                             */
/*                                                                          */
/* p-stable direction g (d doubles) from the counter (j, 0, SKETCH):       */
/*   l1: Cauchy  g_j = tan(pi (u - 1/2)),  u = ((w0 >> 11) + 1/2) 2^-53     */
/*   l2: Gaussian, Box-Muller as the embedding: u1 = ((w0>>11)+1) 2^-53,    */
/*       u2 = (w1 >> 11) 2^-53, g_j = sqrt(-2 ln u1) cos(2 pi u2).          */
/* ------------------------------------------------------------------------ */
#define PURPOSE_SKETCH 4u
#define PURPOSE_PART 5u
#define PURPOSE_PAD 6u

void or_sketch_direction(uint64_t seed, int d, int metric, double *g)
{
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < d; ++j) {
        uint64_t w[4];
        draw(seed, (uint64_t)j, 0, PURPOSE_SKETCH, w);
        if (metric == OR_L1) {
            double u = ldexp((double)(w[0] >> 11) + 0.5, -53);
            g[j] = tan(pi * (u - 0.5));
        } else {
            double u1 = ldexp((double)((w[0] >> 11) + 1), -53);
            double u2 = ldexp((double)(w[1] >> 11), -53);
            g[j] = sqrt(-2.0 * log(u1)) * cos(2.0 * pi * u2);
        }
    }
}

/* p_i = <x_i, g> in double: acc = fma((double) x_ij, g_j, acc), j ascending
 * from acc = 0. */
void or_project(const float *X, int64_t n, int d, const double *g, double *p)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < d; ++j) acc = fma((double)X[(size_t)i * d + j], g[j], acc);
        p[i] = acc;
    }
}

/* Partition grid (one scale): z'_k = (w0 >> 40) 2^-24, M_k = w1 | 1 from the
 * counter (k, 0, PART). */
void or_part_tables(uint64_t seed, int kh, float *zfrac, uint64_t *mult)
{
    for (int k = 0; k < kh; ++k) {
        uint64_t w[4];
        draw(seed, (uint64_t)k, 0, PURPOSE_PART, w);
        zfrac[k] = ldexpf((float)(w[0] >> 40), -24);
        mult[k] = w[1] | 1ull;
    }
}

/* Partition key of every point at cell side 2^e: the hashed coordinates y
 * as for the bucket keys (float), then in double
 *   cell_k = ceil(ldexp((double) y_k, -e) + (double) z'_k),
 * clamped to [-2^62, 2^62] (0 when y_k is NaN), and
 *   key = (sum_k (uint64) (int64) cell_k * M_k mod 2^64) >> 1. */
void or_part_keys(const float *X, int64_t n, int d, int metric, const float *lo, int e_top,
                  const int8_t *Zs, int ke, int e, const float *zfrac, const uint64_t *mult,
                  uint64_t *keys)
{
    int kh = metric == OR_L1 ? d : ke;
    float *y = (float *)malloc(sizeof(float) * (size_t)kh);
    const double lim = ldexp(1.0, 62);
    for (int64_t p = 0; p < n; ++p) {
        hashed_coords(X + (size_t)p * d, d, metric, lo, e_top, Zs, ke, y);
        uint64_t acc = 0;
        for (int k = 0; k < kh; ++k) {
            double c = ceil(ldexp((double)y[k], -e) + (double)zfrac[k]);
            if (c != c) c = 0.0;
            if (c > lim) c = lim;
            if (c < -lim) c = -lim;
            acc += (uint64_t)(int64_t)c * mult[k];
        }
        keys[p] = acc >> 1;
    }
    free(y);
}

/* Padded copy: row i of X (n x d) followed by m coordinates +-q, the sign of
 * coordinate j being bit (j mod 64) of word j / 64 of the block at the
 * counter (i, side, PAD) (set bit: -q).  side is 0 for A and 1 for B. */
void or_pad(const float *X, int64_t n, int d, int m, int side, uint64_t seed, float q,
            float *out)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t w[4];
        draw(seed, (uint64_t)i, (uint64_t)side, PURPOSE_PAD, w);
        float *o = out + (size_t)i * (d + m);
        for (int j = 0; j < d; ++j) o[j] = X[(size_t)i * d + j];
        for (int j = 0; j < m; ++j) o[d + j] = ((w[j / 64] >> (j % 64)) & 1u) ? -q : q;
    }
}
