// Low-precision l2 nearest neighbours: distance tiles on BF16 or FP8-E4M3
// matrix cores with FP32 accumulation, then an exact float32 re-rank.
//
// Rows of X (the queries) and B are first cast once per call
// (k_cast_rows): BF16 by round-to-nearest-even; FP8-E4M3 after scaling each
// row by s_r = max|x_r| / 240 (240 is representable in every E4M3 variant),
// with the scale kept in float32.  The norm |q(b)|^2 of each dequantised
// row is kept too, so the score
//     s(b) = |q(b)|^2 - 2 s_x s_b <q(x), q(b)>
// ranks B by the exact squared distance between the quantised points, up to
// FP32 accumulation error.  Each lane keeps the two best scores it sees for
// its query (so 4 lane groups x 2 = 8 candidates per query and chunk); the
// candidates are re-evaluated with the canonical float32 distance on the
// original float32 rows, and the per-query minimum over chunks is merged with
// a 64-bit integer atomicMin of (accumulator bits << 32 | b).  The result is
// the exact float32 distance to a row of B that may not be the nearest one
// when the true nearest row is outside every chunk's top 8 under the
// low-precision score; callers report that error against float64.
#include <cfloat>
#include <cmath>

#include "internal.h"

namespace chamfer {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

constexpr int kLpTileRows = 32;
constexpr float kFp8Range = 240.0f;

// Row length after zero padding to whole MFMA K steps (32 BF16 / 128 FP8).
__host__ __device__ inline int padded_dim(int d, int precision) {
    if (precision == CHAMFER_BF16) return (d + 31) / 32 * 32;
    return (d + 127) / 128 * 128;
}

int lowp_dpad(int d, int precision) { return padded_dim(d, precision); }

bool lowp_supported(int d, int metric, int precision) {
    return metric == CHAMFER_L2 && precision != CHAMFER_FP32 && d >= 12 && d <= 256;
}

size_t lowp_row_bytes(int d, int precision) {
    return (size_t)lowp_dpad(d, precision) * (precision == CHAMFER_BF16 ? 2 : 1);
}

__device__ __forceinline__ uint16_t to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_float(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

// One wavefront per row: lane l takes coordinates 4l .. 4l+3 (dpad <= 256).
template <int PREC>
__device__ __forceinline__ void cast_rows(const float *__restrict__ X,
                                          const int32_t *__restrict__ rows, int64_t n, int d,
                                          int dpad, uint8_t *out, float *scale, float *n2,
                                          const DevParams *p, Blk blk) {
    if (p->status != CHAMFER_OK) return;
    const int lane = threadIdx.x & 63;
    const int64_t r = blk.id * 4 + (threadIdx.x >> 6);
    if (r >= n) return;  // whole wavefront
    const int64_t src = rows ? (int64_t)ro(rows)[r] : r;
    const auto *x = ro(X) + src * d;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = lane * 4 + i;
        v[i] = k < d ? x[k] : 0.0f;
    }
    float sq = 0.0f;
    if (PREC == CHAMFER_BF16) {
        uint16_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            h[i] = to_bf16_rne(v[i]);
            const float f = bf16_to_float(h[i]);
            sq = fmaf(f, f, sq);
        }
        if (lane * 4 < dpad) {
            uint2 w;
            w.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
            w.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
            *reinterpret_cast<uint2 *>(out + ((size_t)r * dpad + lane * 4) * 2) = w;
        }
        if (lane == 0) scale[r] = 1.0f;
    } else {
        float m = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        const float s = m > 0.0f ? m / kFp8Range : 1.0f;
        const float inv = 1.0f / s;
        const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0] * inv, v[1] * inv, 0, false);
        const int pk = __builtin_amdgcn_cvt_pk_fp8_f32(v[2] * inv, v[3] * inv, lo, true);
        const float f[4] = {__builtin_amdgcn_cvt_f32_fp8(pk, 0) * s,
                            __builtin_amdgcn_cvt_f32_fp8(pk, 1) * s,
                            __builtin_amdgcn_cvt_f32_fp8(pk, 2) * s,
                            __builtin_amdgcn_cvt_f32_fp8(pk, 3) * s};
#pragma unroll
        for (int i = 0; i < 4; ++i) sq = fmaf(f[i], f[i], sq);
        if (lane * 4 < dpad) *reinterpret_cast<int *>(out + (size_t)r * dpad + lane * 4) = pk;
        if (lane == 0) scale[r] = s;
    }
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (lane == 0) n2[r] = sq;
}

template <int PREC>
__global__ __launch_bounds__(256) void k_cast_rows(const float *__restrict__ X,
                                                   const int32_t *__restrict__ rows, int64_t n,
                                                   int d, int dpad, uint8_t *out, float *scale,
                                                   float *n2, const DevParams *p) {
    cast_rows<PREC>(X, rows, n, d, dpad, out, scale, n2, p, grid_blk());
}

int64_t cast_blocks(int64_t n) { return (n + 3) / 4; }

hipError_t launch_cast_rows(int precision, const float *X, const int32_t *rows, int64_t n, int d,
                            uint8_t *out, float *scale, float *n2, const DevParams *p,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int dpad = lowp_dpad(d, precision);
    const unsigned blocks = (unsigned)cast_blocks(n);
    if (precision == CHAMFER_BF16)
        k_cast_rows<CHAMFER_BF16><<<blocks, 256, 0, st>>>(X, rows, n, d, dpad, out, scale, n2, p);
    else
        k_cast_rows<CHAMFER_FP8><<<blocks, 256, 0, st>>>(X, rows, n, d, dpad, out, scale, n2, p);
    return hipGetLastError();
}

__device__ __forceinline__ unsigned long long pack_lp(float v, int64_t b) {
    return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(uint32_t)b;
}

// Queries q < nx are rows of Xq (cast), their float32 originals rows[q] of X.
template <int PREC, int DP, int NB>
__device__ __forceinline__ void nnmin_l2_lowp(
    const uint8_t *__restrict__ Xq, const float *__restrict__ xsc, int64_t nx,
    const float *__restrict__ X, const int32_t *__restrict__ rows,
    const uint8_t *__restrict__ Bq, const float *__restrict__ bsc,
    const float *__restrict__ bn2, const float *__restrict__ B, int64_t nB, int d,
    int64_t chunk, int nchunk, unsigned long long *best, const DevParams *__restrict__ p,
    Blk blk) {
    constexpr int ES = PREC == CHAMFER_BF16 ? 2 : 1;  // bytes per element
    constexpr int RB = DP * ES;                       // bytes per row
    constexpr int QB = RB / 4;                        // bytes per 16-lane group
    constexpr int SB = PREC == CHAMFER_BF16 ? 16 : 32;  // bytes per lane per MFMA
    constexpr int NS = QB / SB;                       // MFMA steps over K
    constexpr int LDR = RB + 16;                      // padded LDS row (bytes)
    constexpr int NV = kLpTileRows * RB / 16;         // 16-byte units per tile
    constexpr int PER_T = (NV + 255) / 256;
    __shared__ __attribute__((aligned(16))) uint8_t tile[kLpTileRows * LDR];
    __shared__ float tn2[kLpTileRows], tsc[kLpTileRows];

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
    if (b0 >= b1) return;
    const bool wave_active = qbase < nx;

    // query fragments: lane (g, j) holds bytes [g QB, (g+1) QB) of its query
    uint4 qf[NB][QB / 16];
    float qs[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t qi = qbase + nb * 16 + j;
        const int64_t r = qi < nx ? qi : 0;
        const auto *src = reinterpret_cast<const CH_RO uint4 *>(ro(Xq) + (size_t)r * RB + g * QB);
#pragma unroll
        for (int u = 0; u < QB / 16; ++u) qf[nb][u] = ld(src + u);
        qs[nb] = ro(xsc)[r];
    }
    float b1v[NB], b2v[NB];
    int32_t b1i[NB], b2i[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        b1v[nb] = INFINITY;
        b2v[nb] = INFINITY;
        b1i[nb] = -1;
        b2i[nb] = -1;
    }

    uint4 pf[PER_T];
    float pn2 = INFINITY, psc = 0.0f;
    auto fetch = [&](int64_t t0) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int v = tid + i * 256;
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            if (v < NV) {
                const int row = v / (RB / 16);
                const int u = v - row * (RB / 16);
                if (t0 + row < b1)
                    val = ld(reinterpret_cast<const CH_RO uint4 *>(ro(Bq) + (size_t)(t0 + row) * RB) + u);
            }
            pf[i] = val;
        }
        if (tid < kLpTileRows) {
            const bool ok = t0 + tid < b1;
            pn2 = ok ? ro(bn2)[t0 + tid] : INFINITY;
            psc = ok ? ro(bsc)[t0 + tid] : 0.0f;
        }
    };

    int64_t t0 = b0;
    fetch(t0);
    for (;;) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int v = tid + i * 256;
            if (v < NV) {
                const int row = v / (RB / 16);
                const int u = v - row * (RB / 16);
                *reinterpret_cast<uint4 *>(&tile[row * LDR + u * 16]) = pf[i];
            }
        }
        if (tid < kLpTileRows) {
            tn2[tid] = pn2;
            tsc[tid] = psc;
        }
        __syncthreads();
        const int64_t next = t0 + kLpTileRows;
        if (next < b1) fetch(next);

        if (wave_active) {
            v4f acc[2][NB];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[m][nb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < NS; ++s) {
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const uint8_t *ap = &tile[(16 * m + j) * LDR + g * QB + s * SB];
                    if (PREC == CHAMFER_BF16) {
                        const uint4 a4 = *reinterpret_cast<const uint4 *>(ap);
                        const v8bf a = __builtin_bit_cast(v8bf, a4);
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) {
                            const v8bf b = __builtin_bit_cast(v8bf, qf[nb][s]);
                            acc[m][nb] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[m][nb], 0, 0, 0);
                        }
                    } else {
                        const uint4 a0 = *reinterpret_cast<const uint4 *>(ap);
                        const uint4 a1 = *reinterpret_cast<const uint4 *>(ap + 16);
                        const v8i a = v8i{(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w,
                                          (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) {
                            const uint4 q0 = qf[nb][2 * s], q1 = qf[nb][2 * s + 1];
                            const v8i b = v8i{(int)q0.x, (int)q0.y, (int)q0.z, (int)q0.w,
                                              (int)q1.x, (int)q1.y, (int)q1.z, (int)q1.w};
                            acc[m][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                                a, b, acc[m][nb], 0, 0, 0, 127, 0, 127);
                        }
                    }
                }
            }
            // epilogue: lane (g, j) holds rows 16m + 4g + r for query j
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                float sc[8];
                float mn = INFINITY;
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int lr = 16 * m + 4 * g + r;
                        const float mul = PREC == CHAMFER_BF16 ? -2.0f : -2.0f * qs[nb] * tsc[lr];
                        const float v = fmaf(acc[m][nb][r], mul, tn2[lr]);
                        sc[4 * m + r] = v;
                        mn = fminf(mn, v);
                    }
                if (__ballot(mn < b2v[nb]) != 0) {  // uniform skip when nothing improves
#pragma unroll
                    for (int m = 0; m < 2; ++m)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float v = sc[4 * m + r];
                            const int32_t row = (int32_t)(t0 + 16 * m + 4 * g + r);
                            const bool c1 = v < b1v[nb], c2 = v < b2v[nb];
                            b2v[nb] = c1 ? b1v[nb] : (c2 ? v : b2v[nb]);
                            b2i[nb] = c1 ? b1i[nb] : (c2 ? row : b2i[nb]);
                            b1v[nb] = c1 ? v : b1v[nb];
                            b1i[nb] = c1 ? row : b1i[nb];
                        }
                }
            }
        }
        t0 = next;
        if (t0 >= b1) break;
    }
    if (!wave_active) return;

    // exact float32 re-rank of each lane's two candidates, merged over the
    // four lane groups of a query
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t qi = qbase + nb * 16 + j;
        const bool valid = qi < nx;
        const int64_t xr = valid ? (rows ? (int64_t)ro(rows)[qi] : qi) : 0;
        unsigned long long mine = ~0ull;
        if (valid && b1i[nb] >= 0)
            mine = pack_lp(canon_acc<CHAMFER_L2>(X + xr * d, B + (int64_t)b1i[nb] * d, d), b1i[nb]);
        if (valid && b2i[nb] >= 0)
            mine = min(mine, pack_lp(canon_acc<CHAMFER_L2>(X + xr * d, B + (int64_t)b2i[nb] * d, d),
                                     b2i[nb]));
        mine = min(mine, (unsigned long long)__shfl_xor(mine, 16));
        mine = min(mine, (unsigned long long)__shfl_xor(mine, 32));
        if (valid && g == 0 && mine != ~0ull) atomicMin(&best[qi], mine);
    }
}

template <int PREC, int DP, int NB>
__global__ __launch_bounds__(256) void k_nnmin_l2_lowp(
    const uint8_t *__restrict__ Xq, const float *__restrict__ xsc, int64_t nx,
    const float *__restrict__ X, const int32_t *__restrict__ rows,
    const uint8_t *__restrict__ Bq, const float *__restrict__ bsc,
    const float *__restrict__ bn2, const float *__restrict__ B, int64_t nB, int d,
    int64_t chunk, int nchunk, unsigned long long *best, const DevParams *__restrict__ p) {
    nnmin_l2_lowp<PREC, DP, NB>(Xq, xsc, nx, X, rows, Bq, bsc, bn2, B, nB, d, chunk, nchunk, best,
                                p, grid_blk());
}

// 16-query blocks per wavefront for (precision, padded dimension).
static int lowp_nb(int precision, int dp) {
    if (precision == CHAMFER_BF16) return dp <= 64 ? 4 : 2;
    return dp == 128 ? 4 : 2;
}

NNGeom lowp_geom(int64_t nx, int64_t nB, int d, int precision) {
    const int64_t per_wg = 64 * lowp_nb(precision, lowp_dpad(d, precision));
    const int64_t nq = (nx + per_wg - 1) / per_wg;
    // large chunks (the re-rank runs once per chunk), enough workgroups
    int64_t nc = (2048 + nq - 1) / nq;
    const int64_t cmax = (nB + 2047) / 2048;
    if (nc > cmax) nc = cmax;
    if (nc < 1) nc = 1;
    if (nc > 1) nc = (nc + 7) / 8 * 8;
    NNGeom g;
    g.chunk = (nB + nc - 1) / nc;
    g.nchunk = (int)((nB + g.chunk - 1) / g.chunk);
    g.blocks = nq * g.nchunk;
    return g;
}

template <int PREC, int DP, int NB>
static hipError_t go_lowp(const uint8_t *Xq, const float *xsc, int64_t nx, const float *X,
                          const int32_t *rows, const uint8_t *Bq, const float *bsc,
                          const float *bn2, const float *B, int64_t nB, int d,
                          unsigned long long *best, const DevParams *p, hipStream_t st) {
    const NNGeom g = lowp_geom(nx, nB, d, PREC);
    k_nnmin_l2_lowp<PREC, DP, NB><<<(unsigned)g.blocks, 256, 0, st>>>(
        Xq, xsc, nx, X, rows, Bq, bsc, bn2, B, nB, d, g.chunk, g.nchunk, best, p);
    return hipGetLastError();
}

hipError_t launch_nnmin_lowp(int precision, const uint8_t *Xq, const float *xsc, int64_t nx,
                             const float *X, const int32_t *rows, const uint8_t *Bq,
                             const float *bsc, const float *bn2, const float *B, int64_t nB,
                             int d, unsigned long long *best, const DevParams *p,
                             hipStream_t st) {
    if (nx <= 0) return hipSuccess;
    const int dp = lowp_dpad(d, precision);
#define LP_ARGS Xq, xsc, nx, X, rows, Bq, bsc, bn2, B, nB, d, best, p, st
    if (precision == CHAMFER_BF16) {
        switch (dp) {
            case 32: return go_lowp<CHAMFER_BF16, 32, 4>(LP_ARGS);
            case 64: return go_lowp<CHAMFER_BF16, 64, 4>(LP_ARGS);
            case 96: return go_lowp<CHAMFER_BF16, 96, 2>(LP_ARGS);
            case 128: return go_lowp<CHAMFER_BF16, 128, 2>(LP_ARGS);
            case 160: return go_lowp<CHAMFER_BF16, 160, 2>(LP_ARGS);
            case 192: return go_lowp<CHAMFER_BF16, 192, 2>(LP_ARGS);
            case 224: return go_lowp<CHAMFER_BF16, 224, 2>(LP_ARGS);
            default: return go_lowp<CHAMFER_BF16, 256, 2>(LP_ARGS);
        }
    }
    if (dp == 128) return go_lowp<CHAMFER_FP8, 128, 4>(LP_ARGS);
    return go_lowp<CHAMFER_FP8, 256, 2>(LP_ARGS);
#undef LP_ARGS
}

// ---------------------------------------------------------------- batched
// Low-precision copies of each job's B and sampled rows, then the pass.  The
// float sidecars of a job live at lpf: scale and |.|^2 of B (nB each), then
// of the samples (T each).

constexpr unsigned kGridCast = 1024, kGridNNLowp = 2048;

template <int PREC>
__global__ __launch_bounds__(256) void kb_cast(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsCast, [&](const Job &J, Blk b) {
        const int dpad = padded_dim(J.d, PREC);
        float *bsc = J.lpf, *bn2 = J.lpf + J.nB, *xsc = J.lpf + 2 * J.nB, *xn2 = xsc + J.T;
        if (b.id < J.nb_castB)
            cast_rows<PREC>(J.B, nullptr, J.nB, J.d, dpad, J.bq, bsc, bn2, J.p,
                            Blk{b.id, J.nb_castB});
        else
            cast_rows<PREC>(J.A, J.idx, J.T, J.d, dpad, J.xq, xsc, xn2, J.p,
                            Blk{b.id - J.nb_castB, J.nb_castX});
    });
}

template <int PREC, int DP, int NB>
__global__ __launch_bounds__(256) void kb_nn_lowp(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsNN, [&](const Job &J, Blk b) {
        const float *bsc = J.lpf, *bn2 = J.lpf + J.nB, *xsc = J.lpf + 2 * J.nB;
        nnmin_l2_lowp<PREC, DP, NB>(J.xq, xsc, J.T, J.A, J.idx, J.bq, bsc, bn2, J.B, J.nB, J.d,
                                    J.nn_chunk, J.nn_nchunk, J.best, J.p, b);
    });
}

hipError_t launch_batch_cast(const Batch *bt, int d, int precision, hipStream_t st) {
    (void)d;
    if (precision == CHAMFER_BF16)
        kb_cast<CHAMFER_BF16><<<kGridCast, 256, 0, st>>>(bt);
    else
        kb_cast<CHAMFER_FP8><<<kGridCast, 256, 0, st>>>(bt);
    return hipGetLastError();
}

hipError_t launch_batch_lowp(const Batch *bt, int d, int precision, hipStream_t st) {
    const int dp = lowp_dpad(d, precision);
    if (precision == CHAMFER_BF16) {
        switch (dp) {
            case 32: kb_nn_lowp<CHAMFER_BF16, 32, 4><<<kGridNNLowp, 256, 0, st>>>(bt); break;
            case 64: kb_nn_lowp<CHAMFER_BF16, 64, 4><<<kGridNNLowp, 256, 0, st>>>(bt); break;
            case 96: kb_nn_lowp<CHAMFER_BF16, 96, 2><<<kGridNNLowp, 256, 0, st>>>(bt); break;
            case 128: kb_nn_lowp<CHAMFER_BF16, 128, 2><<<kGridNNLowp, 256, 0, st>>>(bt); break;
            case 160: kb_nn_lowp<CHAMFER_BF16, 160, 2><<<kGridNNLowp, 256, 0, st>>>(bt); break;
            case 192: kb_nn_lowp<CHAMFER_BF16, 192, 2><<<kGridNNLowp, 256, 0, st>>>(bt); break;
            case 224: kb_nn_lowp<CHAMFER_BF16, 224, 2><<<kGridNNLowp, 256, 0, st>>>(bt); break;
            default: kb_nn_lowp<CHAMFER_BF16, 256, 2><<<kGridNNLowp, 256, 0, st>>>(bt); break;
        }
    } else if (dp == 128) {
        kb_nn_lowp<CHAMFER_FP8, 128, 4><<<kGridNNLowp, 256, 0, st>>>(bt);
    } else {
        kb_nn_lowp<CHAMFER_FP8, 256, 2><<<kGridNNLowp, 256, 0, st>>>(bt);
    }
    return hipGetLastError();
}

}  // namespace chamfer
