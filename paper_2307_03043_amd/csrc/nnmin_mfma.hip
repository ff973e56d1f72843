// Exact l2 nearest neighbours on the matrix cores (gfx950 v_mfma_f32_16x16x4f32),
// returning the same canonical float32 result as the VALU form: the minimum
// over b of (fma-chain accumulator of (x_k - b_k)^2 in ascending k, b), ties
// to the lower b.
//
// 1. Scores.  The MFMA tiles compute s(b) = |b|^2 - 2 x.b for every (b, x)
//    pair (the |x|^2 term is common to a row and dropped).  B rows are the
//    MFMA "A" operand, streamed through LDS 32 rows at a time and shared by
//    the 4 wavefronts of a workgroup; each wavefront keeps 16*NB queries as
//    the "B" operand in VGPRs for the whole sweep.  The K dimension is
//    permuted so that each 16-lane group walks a contiguous quarter of the
//    coordinates, which makes every LDS read a 16-byte vector read.
// 2. Candidates.  Each lane sees a quarter of the rows of each 16-row block
//    for one query; it keeps its best score (with its b) and its second-best
//    score.  The four lane-group bests are the candidates.
// 3. Re-rank.  Candidates are re-evaluated with the canonical float32
//    distance, which is what the result reports.
// 4. Certificate.  With u = 2^-24, the computed score is within
//    E = c (|b|max^2 + 2 |x| |b|max) of the exact one, and the canonical
//    accumulator is within a relative (d+4)u of the exact squared distance,
//    so every non-candidate b has accumulator >= LB = (1-r)(cut - E + |x|^2)
//    where cut is the smallest second-best score.  If LB exceeds the best
//    candidate (or the best already recorded for the query), no non-candidate
//    can be the canonical minimum.  Otherwise the (query, chunk) pair is
//    rescanned exactly by the whole wavefront.  A chunk whose best score
//    already rules it out against the recorded best is skipped.
// The per-query result is merged over chunks with a 64-bit integer
// atomicMin of (accumulator bits << 32 | b), so the outcome is the canonical
// minimum whatever the order of the chunks.
#include <cfloat>
#include <cmath>

#include "internal.h"

namespace chamfer {

typedef float v4f __attribute__((ext_vector_type(4)));

#ifndef CH_MFMA_MB
#define CH_MFMA_MB 2
#endif
constexpr int kMB = CH_MFMA_MB;          // 16-row MFMA blocks per LDS tile
constexpr int kTileRows = 16 * kMB;      // B rows per LDS tile
// Launch shape, chosen by measurement on MI355X (l2, d = 128): one block of
// 16 queries per wavefront keeps the VGPR count low enough for two
// wavefronts per SIMD, and ~4096 workgroups give chunks of a few hundred
// rows for T = 2000 draws against 10^5 points.
#ifndef CH_MFMA_TARGET_WGS
#define CH_MFMA_TARGET_WGS 4096
#endif
#ifndef CH_MFMA_NB128
#define CH_MFMA_NB128 1
#endif
constexpr int kMfmaTargetWGs = CH_MFMA_TARGET_WGS;  // workgroups a launch aims for
constexpr int kMfmaNB128 = CH_MFMA_NB128;           // 16-query blocks per wavefront, d <= 128

__device__ __forceinline__ unsigned long long pack_acc(float v, int64_t b) {
    return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(uint32_t)b;
}

__device__ __forceinline__ float unpack_acc(unsigned long long p) {
    const uint32_t hi = (uint32_t)(p >> 32);
    return hi == 0xffffffffu ? INFINITY : __uint_as_float(hi);
}

// Canonical float32 squared accumulator (fma chain, k ascending).
__device__ __forceinline__ float acc32_l2(const float *__restrict__ x,
                                          const float *__restrict__ b, int d) {
    return canon_acc<CHAMFER_L2>(x, b, d);
}

// |b|^2 per row (float32) and its maximum over B; one thread per row with
// 16-byte loads (independent, so many are in flight per thread).
__global__ __launch_bounds__(256) void k_rownorm(const float *__restrict__ B, int64_t nB, int d,
                                                 float *nb2, DevParams *p) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float v = 0.0f;
    if (r < nB) {
        const float *b = B + r * d;
        if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0) {
            const float4 *b4 = reinterpret_cast<const float4 *>(b);
            for (int k = 0; k < (d >> 2); ++k) {
                const float4 u = b4[k];
                v = fmaf(u.x, u.x, v);
                v = fmaf(u.y, u.y, v);
                v = fmaf(u.z, u.z, v);
                v = fmaf(u.w, u.w, v);
            }
        } else {
            for (int k = 0; k < d; ++k) v = fmaf(b[k], b[k], v);
        }
        nb2[r] = v;
    }
    uint32_t m = __float_as_uint(v);
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(&p->b2max_bits, m);
}

hipError_t launch_rownorm(const float *B, int64_t nB, int d, float *nb2, DevParams *p,
                          hipStream_t st) {
    if (nB <= 0) return hipSuccess;
    k_rownorm<<<(unsigned)((nB + 255) / 256), 256, 0, st>>>(B, nB, d, nb2, p);
    return hipGetLastError();
}

template <int DP, int NB>
__device__ __forceinline__ void nnmin_l2_mfma(
    const float *__restrict__ X, const int32_t *__restrict__ rows, int64_t nx,
    const float *__restrict__ B, int64_t nB, int d, const float *__restrict__ nb2,
    int64_t chunk, int nchunk, unsigned long long *best, DevParams *p, Blk blk) {
    constexpr int KQ = DP / 4;                // coordinates per 16-lane group
    constexpr int LDR = DP + 4;               // padded LDS row (floats)
    constexpr int NV4 = kTileRows * DP / 4;   // float4 per tile
    constexpr int PER_T = (NV4 + 255) / 256;  // float4 per thread per tile
    __shared__ __attribute__((aligned(16))) float tile[kTileRows * LDR];
    __shared__ float tn2[kTileRows];

    if (p->status != CHAMFER_OK) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    int cb;
    int64_t qb;
    chunk_major(blk.id, (nx + 64 * NB - 1) / (64 * NB), nchunk, cb, qb);
    const int64_t qbase = (qb * 4 + wave) * (16 * NB);
    const int64_t b0 = (int64_t)cb * chunk;
    const int64_t b1 = min(nB, b0 + chunk);
    if (b0 >= b1) return;  // uniform over the workgroup
    const bool wave_active = qbase < nx;
    const bool vec_ok = (d & 3) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;

    // Query fragments: lane (g, j) holds coordinates [g*KQ, (g+1)*KQ) of
    // query qbase + nb*16 + j; padding coordinates are zero.
    float qf[NB][KQ];
    float qn2[NB];
    int64_t qrow[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t qi = qbase + nb * 16 + j;
        const int64_t r = qi < nx ? (rows ? (int64_t)ro(rows)[qi] : qi) : 0;
        qrow[nb] = r;
        const auto *xr = ro(X) + r * d;
        float s2 = 0.0f;
#pragma unroll
        for (int s = 0; s < KQ; ++s) {
            const int k = g * KQ + s;
            qf[nb][s] = k < d ? xr[k] : 0.0f;
            s2 = fmaf(qf[nb][s], qf[nb][s], s2);
        }
        s2 += __shfl_xor(s2, 16);
        s2 += __shfl_xor(s2, 32);
        qn2[nb] = s2;
    }

    float bestv[NB], second[NB];
    int32_t bidx[NB];  // B has at most 2^31 - 1 rows
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        bestv[nb] = INFINITY;
        second[nb] = INFINITY;
        bidx[nb] = (int32_t)b0;
    }

    // Register prefetch of one tile (PER_T float4 per thread) and its norms.
    float4 pf[PER_T];
    float pn2 = INFINITY;
    auto fetch = [&](int64_t t0) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int v = tid + i * 256;
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (v < NV4) {
                const int row = v / (DP / 4);
                const int k0 = (v - row * (DP / 4)) * 4;
                const int64_t br = t0 + row;
                if (br < b1 && k0 < d) {
                    const CH_RO float *src = ro(B) + br * d + k0;
                    if (vec_ok) {
                        val = ld(reinterpret_cast<const CH_RO float4 *>(src));
                    } else {
                        val.x = src[0];
                        if (k0 + 1 < d) val.y = src[1];
                        if (k0 + 2 < d) val.z = src[2];
                        if (k0 + 3 < d) val.w = src[3];
                    }
                }
            }
            pf[i] = val;
        }
        if (tid < kTileRows) pn2 = (t0 + tid < b1) ? ro(nb2)[t0 + tid] : INFINITY;
    };

    int64_t t0 = b0;
    fetch(t0);
    for (;;) {
        __syncthreads();  // the previous tile is no longer being read
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int v = tid + i * 256;
            if (v < NV4) {
                const int row = v / (DP / 4);
                const int k0 = (v - row * (DP / 4)) * 4;
                *reinterpret_cast<float4 *>(&tile[row * LDR + k0]) = pf[i];
            }
        }
        if (tid < kTileRows) tn2[tid] = pn2;
        __syncthreads();
        const int64_t next = t0 + kTileRows;
        if (next < b1) fetch(next);

        if (wave_active) {
            v4f acc[kMB][NB];
#pragma unroll
            for (int m = 0; m < kMB; ++m)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[m][nb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < KQ / 4; ++t) {
                float a[kMB][4];
#pragma unroll
                for (int m = 0; m < kMB; ++m) {
                    const float4 f = *reinterpret_cast<const float4 *>(
                        &tile[(16 * m + j) * LDR + g * KQ + 4 * t]);
                    a[m][0] = f.x;
                    a[m][1] = f.y;
                    a[m][2] = f.z;
                    a[m][3] = f.w;
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int m = 0; m < kMB; ++m)
                            acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                a[m][s], qf[nb][4 * t + s], acc[m][nb], 0, 0, 0);
            }
            // Lane (g, j) holds rows 16m + 4g + r of the tile for query j.
#pragma unroll
            for (int m = 0; m < kMB; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int lr = 16 * m + 4 * g + r;
                    const float n2 = tn2[lr];
                    const int32_t brow = (int32_t)(t0 + lr);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        const float sc = fmaf(acc[m][nb][r], -2.0f, n2);
                        const float bv = bestv[nb];
                        second[nb] = fminf(second[nb], fmaxf(bv, sc));
                        const bool lt = sc < bv;
                        bestv[nb] = lt ? sc : bv;
                        bidx[nb] = lt ? brow : bidx[nb];
                    }
                }
        }
        t0 = next;
        if (t0 >= b1) break;
    }
    if (!wave_active) return;

    // ---- re-rank and certificate, per block of 16 queries ----
    constexpr double kU = 1.0 / 16777216.0;  // 2^-24
    const double rho = (double)(d + 4) * kU * 1.1;
    const double crel = (double)(2 * DP + 8) * kU * 1.1;
    const double cabs = (double)DP * 7.52316384526264e-37;  // DP * 2^-120
    const double b2m = (double)__uint_as_float(p->b2max_bits) * (1.0 + rho);
    const double bm = sqrt(b2m);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t qi = qbase + nb * 16 + j;
        const bool valid = qi < nx;
        // recorded best for the query, read once (group 0) and shared
        float gacc = INFINITY;
        if (g == 0 && valid)
            gacc = unpack_acc(__hip_atomic_load(&best[qi], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT));
        gacc = __shfl(gacc, j);
        float bmin = bestv[nb];
        bmin = fminf(bmin, __shfl_xor(bmin, 16));
        bmin = fminf(bmin, __shfl_xor(bmin, 32));
        float cut = second[nb];
        cut = fminf(cut, __shfl_xor(cut, 16));
        cut = fminf(cut, __shfl_xor(cut, 32));
        const double xn2 = (double)qn2[nb];
        const double E = cabs + crel * (b2m + 2.0 * sqrt(xn2 * (1.0 + rho)) * bm);
        const double xlo = xn2 * (1.0 - rho);
        const double lb_all = (1.0 - rho) * ((double)bmin - E + xlo);
        const bool need = valid && !(lb_all > (double)gacc);
        unsigned long long mine = ~0ull;
        if (need && bestv[nb] < INFINITY)
            mine = pack_acc(acc32_l2(X + qrow[nb] * d, B + (int64_t)bidx[nb] * d, d), bidx[nb]);
        mine = min(mine, (unsigned long long)__shfl_xor(mine, 16));
        mine = min(mine, (unsigned long long)__shfl_xor(mine, 32));
        const double thr = fmin((double)unpack_acc(mine), (double)gacc);
        const double lb_nc = (1.0 - rho) * ((double)cut - E + xlo);
        const bool rescan = need && !(lb_nc > thr);
        if (need && g == 0 && mine != ~0ull) atomicMin(&best[qi], mine);
        unsigned long long mask = __ballot(rescan && g == 0);
        while (mask) {
            const int jj = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            const int64_t q2 = qbase + nb * 16 + jj;
            const int64_t xr = rows ? (int64_t)rows[q2] : q2;
            unsigned long long lb = ~0ull;
            for (int64_t b = b0 + lane; b < b1; b += 64)
                lb = min(lb, pack_acc(acc32_l2(X + xr * d, B + b * d, d), b));
            for (int off = 32; off > 0; off >>= 1)
                lb = min(lb, (unsigned long long)__shfl_xor(lb, off));
            if (lane == 0) {
                atomicMin(&best[q2], lb);
                atomicAdd(&p->fallbacks, 1u);
            }
        }
    }
}

template <int DP, int NB>
__global__ __launch_bounds__(256) void k_nnmin_l2_mfma(
    const float *__restrict__ X, const int32_t *__restrict__ rows, int64_t nx,
    const float *__restrict__ B, int64_t nB, int d, const float *__restrict__ nb2,
    int64_t chunk, int nchunk, unsigned long long *best, DevParams *p) {
    nnmin_l2_mfma<DP, NB>(X, rows, nx, B, nB, d, nb2, chunk, nchunk, best, p, grid_blk());
}

bool mfma_supported(int d, int metric) { return metric == CHAMFER_L2 && d >= 12 && d <= 256; }

// Queries per 16-lane group (NB) of the padded-dimension class of d.
static int mfma_nb(int d) {
    if (d <= 64) return 2;
    if (d <= 128) return kMfmaNB128;
    return 1;
}

NNGeom mfma_geom(int64_t nx, int64_t nB, int d, int64_t target) {
    const int64_t per_wg = 64 * mfma_nb(d);
    const int64_t nq = (nx + per_wg - 1) / per_wg;
    // enough workgroups to fill 256 CUs several times; chunks of 256..8192 rows
    if (target <= 0) target = kMfmaTargetWGs;
    int64_t nc = (target + nq - 1) / nq;
    const int64_t cmin = (nB + 8191) / 8192, cmax = (nB + 255) / 256;
    if (nc < cmin) nc = cmin;
    if (nc > cmax) nc = cmax;
    if (nc < 1) nc = 1;
    if (nc > 1) nc = (nc + 7) / 8 * 8;  // one chunk's workgroups share an XCD
    NNGeom g;
    g.chunk = (nB + nc - 1) / nc;
    g.nchunk = (int)((nB + g.chunk - 1) / g.chunk);
    g.blocks = nq * g.nchunk;
    return g;
}

template <int DP, int NB>
static hipError_t go_mfma(const float *X, const int32_t *rows, int64_t nx, const float *B,
                          int64_t nB, int d, unsigned long long *best, const float *nb2,
                          DevParams *p, hipStream_t st) {
    const NNGeom g = mfma_geom(nx, nB, d);
    k_nnmin_l2_mfma<DP, NB><<<(unsigned)g.blocks, 256, 0, st>>>(X, rows, nx, B, nB, d, nb2, g.chunk,
                                                                 g.nchunk, best, p);
    return hipGetLastError();
}

hipError_t launch_nnmin_mfma(const float *X, const int32_t *rows, int64_t nx, const float *B,
                             int64_t nB, int d, unsigned long long *best, const float *nb2,
                             DevParams *p, hipStream_t st) {
    if (nx <= 0) return hipSuccess;
    if (d <= 16) return go_mfma<16, 2>(X, rows, nx, B, nB, d, best, nb2, p, st);
    if (d <= 32) return go_mfma<32, 2>(X, rows, nx, B, nB, d, best, nb2, p, st);
    if (d <= 64) return go_mfma<64, 2>(X, rows, nx, B, nB, d, best, nb2, p, st);
    if (d <= 128) return go_mfma<128, kMfmaNB128>(X, rows, nx, B, nB, d, best, nb2, p, st);
    return go_mfma<256, 1>(X, rows, nx, B, nB, d, best, nb2, p, st);
}

// ---------------------------------------------------------------- batched

constexpr unsigned kGridNNMfma = 2048;

template <int DP, int NB>
__global__ __launch_bounds__(256) void kb_nn_mfma(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsNN, [&](const Job &J, Blk b) {
        nnmin_l2_mfma<DP, NB>(J.A, J.idx, J.T, J.B, J.nB, J.d, J.nb2, J.nn_chunk, J.nn_nchunk,
                              J.best, J.p, b);
    });
}

hipError_t launch_batch_mfma(const Batch *bt, int d, hipStream_t st) {
    if (d <= 16)
        kb_nn_mfma<16, 2><<<kGridNNMfma, 256, 0, st>>>(bt);
    else if (d <= 32)
        kb_nn_mfma<32, 2><<<kGridNNMfma, 256, 0, st>>>(bt);
    else if (d <= 64)
        kb_nn_mfma<64, 2><<<kGridNNMfma, 256, 0, st>>>(bt);
    else if (d <= 128)
        kb_nn_mfma<128, kMfmaNB128><<<kGridNNMfma, 256, 0, st>>>(bt);
    else
        kb_nn_mfma<256, 1><<<kGridNNMfma, 256, 0, st>>>(bt);
    return hipGetLastError();
}

}  // namespace chamfer
