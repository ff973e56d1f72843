// Exact l2 nearest neighbours on the BF16 matrix cores (gfx950
// v_mfma_f32_16x16x32_bf16) with every float32 coordinate split in two
// BF16 terms, returning the same canonical float32 result as the VALU form:
// the minimum over b of (fma-chain accumulator of (x_k - b_k)^2 in
// ascending k, b), ties to the lower b.
//
// Split.  v = h + m + r with h = bf16(v), m = bf16(v - h) (round to nearest
// even; v - h is exact in float32), so |m| <= 2^-8 (1 + 2^-8) |v| and
// |r| <= 2^-16 |v|.  B and the queries are split once per call into
// row-major tables of [h[0..DP), m[0..DP)] per row (zero padded), the
// queries' (in query order) with their |x|^2.
//
// Scores.  s(b) = |b|^2 - 2 x~.b~ with x~.b~ = xh.bh + xm.bh + xh.bm (three
// BF16 MFMAs per 32 coordinates, TERMS = 3) or that plus xm.bm (TERMS = 4).
// The accumulator of each (b, x) starts at -|b|^2 / 2 (exact), so it ends at
// v = -s / 2 and the selection keeps the largest v.  BF16 products are
// exact in float32.  Error of the computed score against |b|^2 - 2 x.b
// (split_score_bound below; every term is a sum of magnitudes):
//   - dropped split terms, at most c_tr |x| |b| (Cauchy-Schwarz over k):
//     (xh + xm).rb + rx.(bh + bm) + rx.rb gives 2.01 * 2^-16 and xm.bm adds
//     at most 1.02 * 2^-16 (TERMS = 3);
//   - the accumulation, under the assumed model of the matrix cores: every
//     product is added to the float32 accumulator with one rounding to
//     nearest, which errs by at most u = 2^-24 times the partial sum.
//     TERMS = 3 accumulates all 3 DP products in one register (partial sums
//     at most |b|^2 / 2 + 1.02 |x||b|): (3 DP + 8) u (|b|^2 + 2.04 |x||b|)
//     after doubling.  TERMS = 4 keeps the leading products xh.bh (DP
//     additions) apart from the three small ones (3 DP additions, partial
//     sums at most 0.008 |x||b|) and adds the two at the end:
//     (DP + 8) u (|b|^2 + 2.04 |x||b|);
//   - the float32 |b|^2 the accumulator starts from, an fma chain over the
//     d coordinates: at most (d + 1) u |b|^2;
//   - c_abs and c_den absorb flushes of subnormal operands, products and
//     sums to zero.
// The factors 1.1 cover the second-order terms.  With |b|^2 and |x| taken
// at their largest values this gives
//   E = c_abs + c_den (|x| + |b|max) + c_rel (|b|max^2 + 2.04 |x| |b|max)
//       + c_nrm |b|max^2 + 2 c_tr |x| |b|max,
// c_rel = (N + 8) u 1.1 (N = 3 DP or DP), c_nrm = (d + 1) u 1.1.
// TERMS = 4 has the smaller E (fewer exact rescans) and TERMS = 3 the fewer
// registers and MFMAs; launches over many queries take TERMS = 4.
//
// Candidates and certificate: each lane keeps its best score (with its b)
// and its second-best score per query; the four lane-group bests are
// re-evaluated with the canonical float32 distance; a (query, chunk) pair
// whose non-candidates cannot be proved worse than the best candidate (or
// the best already recorded) is rescanned exactly by the whole wavefront;
// chunks merge with a 64-bit atomicMin of (accumulator bits << 32 | b).
// Overflow of any norm makes E infinite, which sends every chunk to the
// exact rescan.
//
// Deferred form (the estimator's draws): the pass only records, per (query,
// chunk), the chunk's largest v, its row, the second largest v of the whole
// chunk and the chunk's index; k_split_resolve then takes each query in one wavefront,
// bounds its minimum from above over all chunks, evaluates the canonical
// distance of only those chunk candidates whose lower bound reaches that
// bound (one per query on most data, instead of four per chunk), and lists
// the chunks whose other rows it cannot exclude; k_split_redo rescans them
// in pieces spread over the whole device.
#include <cfloat>
#include <cmath>

#include "internal.h"

namespace chamfer {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kSplitMB = 2;                    // 16-row MFMA blocks per LDS tile
constexpr int kSplitTileRows = 16 * kSplitMB;  // B rows per LDS tile
// Launch shape by padded dimension, chosen by measured sweeps on MI355X:
// two 16-query blocks per wavefront (half the LDS reads per MFMA) up to
// d_pad = 128, one at 256 (registers: three wavefronts per SIMD either way),
// and a workgroup target that is a whole number of resident rounds of
// 256 CUs x 3 workgroups: 3 rounds (2304) up to d_pad = 64, 6 (4608) at 128
// (the 10^6-point exact pass of the 2000 draws at d = 128: 1.45 ms, against
// 1.57 with 3 rounds and 2.1 with one query block and 4096 workgroups).
__host__ __device__ constexpr int split_nb(int dp) { return dp <= 128 ? 2 : 1; }
constexpr int64_t split_target(int dp) { return dp <= 64 ? 2304 : dp <= 128 ? 4608 : 4096; }

// Launches with at least this many queries take the four-product form: they
// split B into few, long chunks, where near-ties inside a chunk (and so
// exact rescans, each reading the whole chunk) are frequent.
constexpr int64_t kSplitManyQueries = 16384;

// Certificate constants of a launch and the bound E of one query (see the
// header): |computed score - (|b|^2 - 2 x.b)| <= E for every row b, given
// the float32 |x|^2 of the query and the float32 maximum of |b|^2 over B.
// rho bounds the relative error of the canonical float32 accumulator (and
// of the float32 norms) against the exact squared distance (norm).
__host__ __device__ inline double split_rho(int d) {
    return (double)(d + 4) * (1.0 / 16777216.0) * 1.1;
}

__host__ __device__ inline double split_score_bound(int d, int dp, int terms, double xn2,
                                                    double b2max) {
    constexpr double kU = 1.0 / 16777216.0;           // 2^-24
    constexpr double kTiny = 1.1754943508222875e-38;  // 2^-126
    const double rho = split_rho(d);
    const double crel = (double)((terms == 4 ? 1 : 3) * dp + 8) * kU * 1.1;
    const double cnrm = (double)(d + 1) * kU * 1.1;
    const double ctr = (terms == 4 ? 2.01 : 3.03) / 65536.0 * 1.1;
    const double cabs = (double)(20 * dp + 16) * kTiny * 1.1;
    const double cden = 8.0 * sqrt((double)dp) * kTiny * 1.1;
    const double b2m = b2max * (1.0 + rho);
    const double bm = sqrt(b2m);
    const double xabs = sqrt(xn2 * (1.0 + rho));
    return cabs + cden * (xabs + bm) + crel * (b2m + 2.04 * xabs * bm) + cnrm * b2m +
           2.0 * ctr * xabs * bm;
}

size_t split_table_bytes(int64_t nB, int d) { return (size_t)nB * split_dpad(d) * 4; }

__device__ __forceinline__ unsigned long long pack_sp(float v, int64_t b) {
    return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(uint32_t)b;
}

__device__ __forceinline__ float unpack_sp(unsigned long long p) {
    const uint32_t hi = (uint32_t)(p >> 32);
    return hi == 0xffffffffu ? INFINITY : __uint_as_float(hi);
}

// Split table of n rows (row i is X[rows[i]], or X[i] without rows): thread
// t of the blk.n blocks of 256 handles 4 coordinates of one row.  With n2,
// also |row|^2 (float32; the d_pad / 4 threads of a row are consecutive
// lanes of one wavefront, d_pad / 4 a power of two).
__device__ __forceinline__ void split_rows(const float *__restrict__ X,
                                           const int32_t *__restrict__ rows, int64_t n, int d,
                                           int dp, uint16_t *out, float *n2, const DevParams *p,
                                           Blk blk) {
    if (p->status != CHAMFER_OK) return;
    const int per_row = dp / 4;
    const int64_t t = blk.id * 256 + threadIdx.x;
    if (t >= n * per_row) return;
    const int64_t r = t / per_row;
    const int k0 = (int)(t - r * per_row) * 4;
    const int64_t src = rows ? (int64_t)ro(rows)[r] : r;
    const auto *x = ro(X) + src * d;
    uint32_t h[4], m[4];
    float s2 = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float v = k0 + i < d ? x[k0 + i] : 0.0f;
        s2 = fmaf(v, v, s2);
        split2(v, h[i], m[i]);
    }
    uint16_t *row = out + (size_t)r * (2 * dp);
    *reinterpret_cast<uint2 *>(row + k0) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    *reinterpret_cast<uint2 *>(row + dp + k0) =
        make_uint2(m[0] | (m[1] << 16), m[2] | (m[3] << 16));
    if (n2) {
        for (int off = per_row / 2; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
        if (k0 == 0) n2[r] = s2;
    }
}

__global__ __launch_bounds__(256) void k_split_rows(const float *__restrict__ X,
                                                    const int32_t *__restrict__ rows, int64_t n,
                                                    int d, int dp, uint16_t *out, float *n2,
                                                    const DevParams *p) {
    split_rows(X, rows, n, d, dp, out, n2, p, grid_blk());
}

int64_t split_blocks(int64_t nB, int d) { return (nB * (split_dpad(d) / 4) + 255) / 256; }

hipError_t launch_split_rows(const float *B, int64_t nB, int d, uint16_t *out, const DevParams *p,
                             hipStream_t st) {
    if (nB <= 0) return hipSuccess;
    k_split_rows<<<(unsigned)split_blocks(nB, d), 256, 0, st>>>(B, nullptr, nB, d, split_dpad(d),
                                                                out, nullptr, p);
    return hipGetLastError();
}

hipError_t launch_split_queries(const float *X, const int32_t *rows, int64_t nx, int d,
                                uint16_t *out, float *n2, const DevParams *p, hipStream_t st) {
    if (nx <= 0) return hipSuccess;
    k_split_rows<<<(unsigned)split_blocks(nx, d), 256, 0, st>>>(X, rows, nx, d, split_dpad(d),
                                                                out, n2, p);
    return hipGetLastError();
}

// |b|^2 per row (float32 fma chain in ascending k) and its maximum over B
// (p->b2max_rep); one thread per row with 16-byte loads.
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
    if ((threadIdx.x & 63) == 0) rep_max(p->b2max_rep, blockIdx.x, m);
}

hipError_t launch_rownorm(const float *B, int64_t nB, int d, float *nb2, DevParams *p,
                          hipStream_t st) {
    if (nB <= 0) return hipSuccess;
    k_rownorm<<<(unsigned)((nB + 255) / 256), 256, 0, st>>>(B, nB, d, nb2, p);
    return hipGetLastError();
}

bool mfma_supported(int d, int metric) { return metric == CHAMFER_L2 && d >= 12 && d <= 256; }

// Xs and xn2 hold the queries' split table and |x|^2, in query order.
// DEFER: write the (query, chunk) record to rec[query * nchunk + chunk]
// instead of the re-rank and certificate (k_split_resolve completes them).
template <int DP, int NB, int TERMS, bool DEFER = false>
__device__ __forceinline__ void nnmin_l2_split(
    const float *__restrict__ X, const int32_t *__restrict__ rows, int64_t nx,
    const uint16_t *__restrict__ Xs, const float *__restrict__ xn2,
    const float *__restrict__ B, const uint16_t *__restrict__ Bs, int64_t nB, int d,
    const float *__restrict__ nb2, int64_t chunk, int nchunk, unsigned long long *best,
    DevParams *p, Blk blk, uint4 *__restrict__ rec = nullptr) {
    constexpr int KQ = DP / 4;                   // coordinates per 16-lane group
    constexpr int NS = KQ / 8;                   // MFMA steps (8 coordinates per lane)
    constexpr int RB = 4 * DP;                   // bytes per split row (h then m)
    constexpr int LDR = RB + 16;                 // padded LDS row (bytes)
    constexpr int NV = kSplitTileRows * RB / 16;  // 16-byte units per tile
    constexpr int PER_T = (NV + 255) / 256;
    constexpr int NBUF = DP <= 128 ? 2 : 1;  // LDS tile buffers (three workgroups per CU)
    __shared__ __attribute__((aligned(16))) uint8_t tile[NBUF * kSplitTileRows * LDR];
    __shared__ __attribute__((aligned(16))) float tn2[NBUF * kSplitTileRows];  // -|b|^2 / 2

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

    // Query fragments: lane (g, j) holds coordinates [g KQ, (g+1) KQ) of
    // query qbase + nb 16 + j, split, 8 per MFMA step; padding is zero.
    uint4 qh[NB][NS], qm[NB][NS];
    float qn2[NB];
    int64_t qrow[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t qi = qbase + nb * 16 + j;
        qrow[nb] = qi < nx ? (rows ? (int64_t)ro(rows)[qi] : qi) : 0;
        const auto *xs = reinterpret_cast<const CH_RO uint4 *>(
            ro(Xs) + (size_t)(qi < nx ? qi : 0) * (2 * DP) + g * KQ);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            qh[nb][s] = ld(xs + s);
            qm[nb][s] = ld(xs + DP / 8 + s);
        }
        qn2[nb] = qi < nx ? ro(xn2)[qi] : 0.0f;
    }

    // Per lane and query: the largest v = x~.b~ - |b|^2 / 2 over the lane's
    // rows (v = -s / 2, so the smallest score), its row, and the second
    // largest v.  The MFMA accumulators start at -|b|^2 / 2 of their rows.
    float bestv[NB], second[NB];
    int32_t bidx[NB];  // B has at most 2^31 - 1 rows
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        bestv[nb] = -INFINITY;
        second[nb] = -INFINITY;
        bidx[nb] = (int32_t)b0;
    }

    // Register prefetch of one tile: thread tid takes the 16-byte unit
    // u = tid % UPR of the rows tid / UPR + i RPI (i < PER_T), and threads
    // below kSplitTileRows take |b|^2 of one row.  Rows past the chunk are
    // read at its last row, so every load is in bounds and unconditional
    // (no register defaults that would make the loop wait on the loads in
    // flight); store() writes them as zero rows with -|b|^2 / 2 = -inf.
    constexpr int UPR = RB / 16;  // 16-byte units per split row
    constexpr int RPI = 256 / UPR;
    static_assert(RPI * PER_T == kSplitTileRows, "one tile per 256 threads and PER_T passes");
    const int r0 = tid / UPR, u0 = tid - (tid / UPR) * UPR;
    // Tiles are addressed by their first row t relative to b0 (a chunk has
    // fewer than 2^31 rows).
    const int len = (int)(b1 - b0);
    const CH_RO uint4 *cbase = reinterpret_cast<const CH_RO uint4 *>(ro(Bs)) + b0 * UPR + u0;
    const CH_RO float *cn2 = ro(nb2) + b0;
    uint4 pf[PER_T];
    float pn2 = 0.0f;
    auto fetch = [&](int t) {
        if (tid < kSplitTileRows) pn2 = cn2[min(t + tid, len - 1)];
        if (t + kSplitTileRows <= len) {  // whole tile (uniform)
            const CH_RO uint4 *src = cbase + (size_t)(t + r0) * UPR;
#pragma unroll
            for (int i = 0; i < PER_T; ++i) pf[i] = ld(src + i * RPI * UPR);
        } else {
#pragma unroll
            for (int i = 0; i < PER_T; ++i)
                pf[i] = ld(cbase + (size_t)min(t + r0 + i * RPI, len - 1) * UPR);
        }
    };
    auto store = [&](int buf, int t) {
        uint8_t *tb = tile + buf * (kSplitTileRows * LDR);
        if (t + kSplitTileRows <= len) {
#pragma unroll
            for (int i = 0; i < PER_T; ++i)
                *reinterpret_cast<uint4 *>(&tb[(r0 + i * RPI) * LDR + u0 * 16]) = pf[i];
        } else {
#pragma unroll
            for (int i = 0; i < PER_T; ++i)
                *reinterpret_cast<uint4 *>(&tb[(r0 + i * RPI) * LDR + u0 * 16]) =
                    t + r0 + i * RPI < len ? pf[i] : make_uint4(0u, 0u, 0u, 0u);
        }
        if (tid < kSplitTileRows)
            tn2[buf * kSplitTileRows + tid] = t + tid < len ? -0.5f * pn2 : -INFINITY;
    };
    // MFMA scores of the tile in buffer buf (rows b0 + t...) and the
    // running best / second-best per lane and query
    auto compute = [&](int buf, int t) {
        if (!wave_active) return;
        const uint8_t *tb = tile + buf * (kSplitTileRows * LDR);
        const int32_t rbase = (int32_t)b0 + t + 4 * g;
        const float *tnb = tn2 + buf * kSplitTileRows;
        // TERMS = 3: every product into hi; TERMS = 4: the small ones into lo
        constexpr int NL = TERMS == 4 ? kSplitMB : 1;
        v4f hi[kSplitMB][NB], lo[NL][NB];
#pragma unroll
        for (int m = 0; m < kSplitMB; ++m) {
            const v4f h0 = *reinterpret_cast<const v4f *>(&tnb[16 * m + 4 * g]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) hi[m][nb] = h0;
        }
#pragma unroll
        for (int m = 0; m < NL; ++m)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) lo[m][nb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            v8bf ah[kSplitMB], am[kSplitMB];
#pragma unroll
            for (int m = 0; m < kSplitMB; ++m) {
                const uint8_t *ap = &tb[(16 * m + j) * LDR + (g * KQ + 8 * s) * 2];
                ah[m] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4 *>(ap));
                am[m] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4 *>(ap + 2 * DP));
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const v8bf xh = __builtin_bit_cast(v8bf, qh[nb][s]);
                const v8bf xm = __builtin_bit_cast(v8bf, qm[nb][s]);
#pragma unroll
                for (int m = 0; m < kSplitMB; ++m)
                    hi[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], xh, hi[m][nb],
                                                                        0, 0, 0);
                if constexpr (TERMS == 4) {
#pragma unroll
                    for (int m = 0; m < kSplitMB; ++m) {
                        lo[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], xm,
                                                                            lo[m][nb], 0, 0, 0);
                        lo[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[m], xh,
                                                                            lo[m][nb], 0, 0, 0);
                        lo[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[m], xm,
                                                                            lo[m][nb], 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < kSplitMB; ++m)
                        hi[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], xm,
                                                                            hi[m][nb], 0, 0, 0);
#pragma unroll
                    for (int m = 0; m < kSplitMB; ++m)
                        hi[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[m], xh,
                                                                            hi[m][nb], 0, 0, 0);
                }
            }
        }
        // Lane (g, j) holds rows 16m + 4g + r of the tile for query j,
        // taken in pairs (r, r + 1): the pair's larger value (the lower
        // row on a tie) against the best, and the second largest of
        // {best, pair} = med3 against the second.
#pragma unroll
        for (int m = 0; m < kSplitMB; ++m)
#pragma unroll
            for (int r = 0; r < 4; r += 2) {
                const int32_t row0 = rbase + 16 * m + r;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    float v0 = hi[m][nb][r], v1 = hi[m][nb][r + 1];
                    if constexpr (TERMS == 4) {
                        v0 += lo[m][nb][r];
                        v1 += lo[m][nb][r + 1];
                    }
                    const float bv = bestv[nb];
                    const bool up = v1 > v0;
                    const float pm = up ? v1 : v0;
                    second[nb] = fmaxf(second[nb], __builtin_amdgcn_fmed3f(bv, v0, v1));
                    const bool gt = pm > bv;
                    bestv[nb] = gt ? pm : bv;
                    bidx[nb] = gt ? row0 + (int32_t)up : bidx[nb];
                }
            }
    };

    // One barrier per tile with two buffers: tile i + 1 is written to the
    // buffer that tile i - 1 occupied, which every wavefront finished
    // reading before the barrier that ended step i - 1.  With one buffer
    // (d_pad = 256: LDS) the tile is written between two barriers.
    int t = 0, buf = 0;
    fetch(t);
    if constexpr (NBUF == 2) {
        store(0, t);
        __syncthreads();
    }
    for (; t + kSplitTileRows < len; t += kSplitTileRows) {
        if constexpr (NBUF == 1) {
            __syncthreads();  // the previous tile is no longer being read
            store(0, t);
            __syncthreads();
        }
        fetch(t + kSplitTileRows);
        compute(buf, t);
        if constexpr (NBUF == 2) {
            buf ^= 1;
            store(buf, t + kSplitTileRows);
            __syncthreads();
        }
    }
    if constexpr (NBUF == 1) {
        __syncthreads();
        store(0, t);
        __syncthreads();
    }
    compute(buf, t);
    if (!wave_active) return;

    if constexpr (DEFER) {
        // the chunk's largest v over the four lane groups (the lower row on
        // a tie) and the largest v of every other row of the chunk: the
        // groups' second-best values and the other groups' best ones
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            float v1 = bestv[nb], v2 = second[nb];
            int32_t i1 = bidx[nb];
#pragma unroll
            for (int off = 16; off <= 32; off <<= 1) {
                const float o1 = __shfl_xor(v1, off), o2 = __shfl_xor(v2, off);
                const int32_t oi = __shfl_xor(i1, off);
                v2 = fmaxf(fmaxf(v2, o2), fminf(v1, o1));
                const bool take = o1 > v1 || (o1 == v1 && oi < i1);
                i1 = take ? oi : i1;
                v1 = take ? o1 : v1;
            }
            const int64_t qi = qbase + nb * 16 + j;
            if (g == 0 && qi < nx)
                rec[(size_t)qi * nchunk + cb] = make_uint4(
                    __float_as_uint(v1), (uint32_t)i1, __float_as_uint(v2), (uint32_t)cb);
        }
        return;
    }

    // ---- re-rank and certificate, per block of 16 queries ----
    const double rho = split_rho(d);
    const double b2max = (double)__uint_as_float(rep_fold(p->b2max_rep));
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t qi = qbase + nb * 16 + j;
        const bool valid = qi < nx;
        // recorded best for the query, read once (group 0) and shared
        float gacc = INFINITY;
        if (g == 0 && valid)
            gacc = unpack_sp(__hip_atomic_load(&best[qi], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT));
        gacc = __shfl(gacc, j);
        // smallest score (and smallest second-best score) over the lane groups
        float vmax = bestv[nb];
        vmax = fmaxf(vmax, __shfl_xor(vmax, 16));
        vmax = fmaxf(vmax, __shfl_xor(vmax, 32));
        float vcut = second[nb];
        vcut = fmaxf(vcut, __shfl_xor(vcut, 16));
        vcut = fmaxf(vcut, __shfl_xor(vcut, 32));
        const double bmin = -2.0 * (double)vmax, cut = -2.0 * (double)vcut;
        const double xn2 = (double)qn2[nb];
        const double E = split_score_bound(d, DP, TERMS, xn2, b2max);
        const double xlo = xn2 * (1.0 - rho);
        const double lb_all = (1.0 - rho) * (bmin - E + xlo);
        const bool need = valid && !(lb_all > (double)gacc);
        unsigned long long mine = ~0ull;
        if (need && bestv[nb] > -INFINITY)
            mine = pack_sp(canon_acc<CHAMFER_L2>(X + qrow[nb] * d, B + (int64_t)bidx[nb] * d, d),
                           bidx[nb]);
        mine = min(mine, (unsigned long long)__shfl_xor(mine, 16));
        mine = min(mine, (unsigned long long)__shfl_xor(mine, 32));
        const double thr = fmin((double)unpack_sp(mine), (double)gacc);
        const double lb_nc = (1.0 - rho) * (cut - E + xlo);
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
                lb = min(lb, pack_sp(canon_acc<CHAMFER_L2>(X + xr * d, B + b * d, d), b));
            for (int off = 32; off > 0; off >>= 1)
                lb = min(lb, (unsigned long long)__shfl_xor(lb, off));
            if (lane == 0) {
                atomicMin(&best[q2], lb);
                atomicAdd(&p->fallbacks, 1u);
            }
        }
    }
}

// Three wavefronts per SIMD with the accumulators in VGPRs: the epilogue
// reads them without AGPR copies.
template <int DP, int NB, int TERMS, bool DEFER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_nnmin_l2_split(
    const float *__restrict__ X, const int32_t *__restrict__ rows, int64_t nx,
    const uint16_t *__restrict__ Xs, const float *__restrict__ xn2,
    const float *__restrict__ B, const uint16_t *__restrict__ Bs, int64_t nB, int d,
    const float *__restrict__ nb2, int64_t chunk, int nchunk, unsigned long long *best,
    DevParams *p, uint4 *__restrict__ rec) {
    nnmin_l2_split<DP, NB, TERMS, DEFER>(X, rows, nx, Xs, xn2, B, Bs, nB, d, nb2, chunk, nchunk,
                                         best, p, grid_blk(), rec);
}

// Second phase of the deferred form: one wavefront per query q (4 per
// workgroup) over the nchunk records of q, with the bound E of the
// three-product form.  (1) ub = the smallest upper bound (1 + 2 rho)
// (s + E + |x|^2 (1 + 2 rho)) over the chunk candidates, s = -2 v: the
// canonical minimum is at most ub.  (2) Every candidate whose lower bound
// (1 - rho)(s - E + |x|^2 (1 - rho)) does not exceed ub is evaluated with the
// canonical float32 distance; the others cannot reach the minimum, and thr
// is the smallest value found.  (3) A chunk whose other rows have the lower
// bound (1 - rho)(cut - E + |x|^2 (1 - rho)) > thr, cut = -2 v2, is settled;
// the others are rescanned here when chunks are short (redo null), else
// listed in redo (p->nredo entries) for k_split_redo.  best[q] = the
// smallest (value, row) found.
// K > 0: the query's records are read once into K registers per lane
// (nchunk <= 64 K), so the three passes over them wait on one round of
// loads; the candidates of (2) and the chunks to rescan of (3) are first
// listed in LDS and then evaluated in one loop each, which keeps a single
// copy of the canonical distance in the kernel (unrolled over the K
// records it would not fit the instruction cache).  K = 0 reads the
// records from memory in each pass.
// The rescans queued by a workgroup's four wavefronts (rq[0 .. *nrq), draw
// slot << 24 | chunk): every wavefront takes pieces of 64 rows in turn and
// merges the canonical minimum of each piece into slot_min of its draw.
// xoff: this wavefront's draw row offset (row * d), or -1 without a draw.
// Every wavefront of the workgroup calls it (two barriers); slot_min holds
// the merged minima when it returns.
__device__ __forceinline__ void resolve_rescans(const float *__restrict__ X,
                                                const float *__restrict__ B, int64_t nB, int d,
                                                int64_t chunk, const uint32_t *rq, const int *nrq,
                                                unsigned long long *slot_min, int64_t *slot_x,
                                                int wv, int lane, int64_t xoff) {
    if (lane == 0) slot_x[wv] = xoff < 0 ? 0 : xoff;
    __syncthreads();  // the queue, the row offsets and the minima are initialised
    const int64_t P = (chunk + 63) / 64;
    const int64_t total = (int64_t)*nrq * P;
    for (int64_t id = wv; id < total; id += 4) {
        const uint32_t e = rq[id / P];
        const int ws = (int)(e >> 24);
        const int64_t c = (int64_t)(e & 0xffffffu);
        const int64_t b1 = min(nB, c * chunk + chunk);
        const int64_t b = c * chunk + (id % P) * 64 + lane;
        unsigned long long mm = ~0ull;
        if (b < b1) mm = pack_sp(canon_acc<CHAMFER_L2, 16>(X + slot_x[ws], B + b * d, d), b);
        for (int off = 32; off > 0; off >>= 1) mm = min(mm, (unsigned long long)__shfl_xor(mm, off));
        if (lane == 0 && mm != ~0ull) atomicMin(&slot_min[ws], mm);
    }
    __syncthreads();  // every piece merged
}

template <int K>
__global__ __launch_bounds__(256) void k_split_resolve(
    const float *__restrict__ X, const int32_t *__restrict__ rows, int64_t nx,
    const float *__restrict__ xn2, const float *__restrict__ B, int64_t nB, int d, int DP,
    int64_t chunk, int nchunk, const uint4 *__restrict__ rec, uint2 *__restrict__ redo,
    unsigned long long *best, DevParams *p) {
    __shared__ int lists[4][K > 0 ? 64 * K : 1];
    // K > 0 without a redo list: the flagged chunks of the workgroup's four
    // draws (draw slot << 24 | chunk) are rescanned by all four wavefronts,
    // in pieces of 64 rows, their minima merged per draw in LDS
    __shared__ uint32_t rq[K > 0 ? 4 * 64 * K : 1];
    __shared__ int nrq;
    __shared__ unsigned long long slot_min[4];
    __shared__ int64_t slot_x[4];
    if (p->status != CHAMFER_OK) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * 4 + wv;
    const bool coop = K > 0 && redo == nullptr;  // uniform over the grid
    if (coop) {
        if (threadIdx.x == 0) nrq = 0;
        if (lane == 0) slot_min[wv] = ~0ull;
        __syncthreads();
    }
    if (q >= nx) {  // uniform over the wavefront
        if (!coop) return;
        resolve_rescans(X, B, nB, d, chunk, rq, &nrq, slot_min, slot_x, wv, lane, -1);
        return;
    }
    int *list = lists[wv];
    const unsigned long long below = (1ull << lane) - 1;
    const CH_RO uint4 *r = ro(rec) + (size_t)q * nchunk;
    // records past nchunk read as empty chunks (v = v2 = -inf); a record
    // is (v, row, v2, chunk), and all four words stay in use, so no load's
    // destination is reused while it is in flight
    const uint4 none = make_uint4(0xff800000u, 0u, 0xff800000u, 0u);
    uint4 w[K > 0 ? K : 1];
    if constexpr (K > 0) {
        // every load in bounds and unconditional, so they are all in flight
        // together; the records past nchunk are replaced afterwards
#pragma unroll
        for (int i = 0; i < K; ++i) w[i] = ld(r + min(i * 64 + lane, nchunk - 1));
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i * 64 + lane >= nchunk) w[i] = none;
    }
    auto rec_at = [&](int i) -> uint4 {
        if constexpr (K > 0) return w[i];
        return i * 64 + lane < nchunk ? ld(r + i * 64 + lane) : none;
    };
    const int iters = K > 0 ? K : (nchunk + 63) / 64;
    constexpr int kUnroll = K > 0 ? K : 1;

    const double rho = split_rho(d);
    const double xn = (double)ro(xn2)[q];
    const double E =
        split_score_bound(d, DP, 3, xn, (double)__uint_as_float(rep_fold(p->b2max_rep)));
    const double xlo = xn * (1.0 - rho), xhi = xn * (1.0 + 2.0 * rho);
    const float *x = X + (rows ? (int64_t)ro(rows)[q] : q) * d;
    auto dist = [&](int64_t b) {
        return pack_sp(canon_acc<CHAMFER_L2, 16>(x, B + b * d, d), b);
    };

    double ub = INFINITY;
#pragma unroll kUnroll
    for (int i = 0; i < iters; ++i) {
        const float v = __uint_as_float(rec_at(i).x);
        if (v > -INFINITY) ub = fmin(ub, (1.0 + 2.0 * rho) * (-2.0 * (double)v + E + xhi));
    }
    for (int off = 32; off > 0; off >>= 1) ub = fmin(ub, __shfl_xor(ub, off));

    auto is_cand = [&](uint4 c) {
        const float v = __uint_as_float(c.x);
        return v > -INFINITY && !((1.0 - rho) * (-2.0 * (double)v - E + xlo) > ub);
    };
    unsigned long long m = ~0ull;
    if constexpr (K > 0) {
        int n = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const uint4 c = w[i];
            const bool cand = is_cand(c);
            const unsigned long long mk = __ballot(cand);
            if (cand) list[n + __popcll(mk & below)] = (int)c.y;
            n += __popcll(mk);
        }
        for (int t = lane; t < n; t += 64) m = min(m, dist(list[t]));
    } else {
        for (int i = 0; i < iters; ++i) {
            const uint4 c = rec_at(i);
            if (is_cand(c)) m = min(m, dist(c.y));
        }
    }
    for (int off = 32; off > 0; off >>= 1) m = min(m, (unsigned long long)__shfl_xor(m, off));
    const double thr = (double)unpack_sp(m);

    // chunks whose other rows are not settled: rescanned below (redo null)
    // or listed for k_split_redo
    auto rescan = [&](int64_t c) {
        const int64_t b0 = c * chunk, b1 = min(nB, b0 + chunk);
        for (int64_t b = b0 + lane; b < b1; b += 64) m = min(m, dist(b));
    };
    int nf = 0;
#pragma unroll kUnroll
    for (int i = 0; i < iters; ++i) {
        const uint4 c = rec_at(i);
        const float v2 = __uint_as_float(c.z);
        const bool flag =
            i * 64 + lane < nchunk && !((1.0 - rho) * (-2.0 * (double)v2 - E + xlo) > thr);
        unsigned long long mask = __ballot(flag);
        if (mask == 0) continue;
        if (lane == 0) atomicAdd(&p->fallbacks, (uint32_t)__popcll(mask));
        if (redo == nullptr) {
            if constexpr (K > 0) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&nrq, (uint32_t)__popcll(mask));
                base = __shfl(base, 0);
                if (flag) rq[base + (uint32_t)__popcll(mask & below)] = ((uint32_t)wv << 24) | c.w;
            } else {
                while (mask) {
                    const int jj = __ffsll((long long)mask) - 1;
                    mask &= mask - 1;
                    rescan(i * 64 + jj);
                }
            }
            continue;
        }
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&p->nredo, (uint32_t)__popcll(mask));
        base = __shfl(base, 0);
        if (flag) redo[base + (uint32_t)__popcll(mask & below)] = make_uint2((uint32_t)q, c.w);
    }
    (void)nf;
    if (coop) {
        const int64_t xr = rows ? (int64_t)ro(rows)[q] : q;
        resolve_rescans(X, B, nB, d, chunk, rq, &nrq, slot_min, slot_x, wv, lane, xr * d);
        m = min(m, slot_min[wv]);
    } else if (redo == nullptr) {
        for (int off = 32; off > 0; off >>= 1) m = min(m, (unsigned long long)__shfl_xor(m, off));
    }
    if (lane == 0) best[q] = m;
}

// Rescans of the deferred form: each listed (query, chunk) pair is cut into
// pieces of kRedoRows rows dealt to the wavefronts of a fixed grid, so a
// few long chunks do not serialise on one wavefront; each piece merges its
// canonical minimum into best[query] with a 64-bit atomicMin.  A piece is one
// row per lane (with four rows per lane, each lane's rows were four chains of
// dependent loads one after another).
constexpr int64_t kRedoRows = 64;
constexpr unsigned kGridRedo = 256;
// Chunks up to this many rows are rescanned by the resolving wavefront
// itself (a third launch costs more than such rescans at 10^5 points: 347-row
// chunks); longer ones go to k_split_redo (3472-row chunks at 10^6).
constexpr int64_t kRedoInlineRows = 512;
// Records per lane that k_split_resolve keeps in registers (up to 512
// chunks: 288 for the 2000 draws at d <= 128).
constexpr int kResolveRegs = 8;

__global__ __launch_bounds__(256) void k_split_redo(
    const float *__restrict__ X, const int32_t *__restrict__ rows, const float *__restrict__ B,
    int64_t nB, int d, int64_t chunk, const uint2 *__restrict__ redo,
    unsigned long long *best, const DevParams *p) {
    if (p->status != CHAMFER_OK) return;
    const int lane = threadIdx.x & 63;
    const int64_t pieces = (chunk + kRedoRows - 1) / kRedoRows;
    const int64_t total = (int64_t)p->nredo * pieces;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); t < total; t += nw) {
        // (query, chunk) as the low and high words of one 64-bit load
        const unsigned long long it =
            ro(reinterpret_cast<const unsigned long long *>(redo))[t / pieces];
        const int64_t q = (uint32_t)it, c = (uint32_t)(it >> 32);
        const int64_t b0 = c * chunk + (t % pieces) * kRedoRows;
        const int64_t b1 = min(min(nB, (c + 1) * chunk), b0 + kRedoRows);
        const float *x = X + (rows ? (int64_t)ro(rows)[q] : q) * d;
        unsigned long long m = ~0ull;
        for (int64_t b = b0 + lane; b < b1; b += 64)
            m = min(m, pack_sp(canon_acc<CHAMFER_L2, 16>(x, B + b * d, d), b));
        for (int off = 32; off > 0; off >>= 1)
            m = min(m, (unsigned long long)__shfl_xor(m, off));
        if (lane == 0 && m != ~0ull) atomicMin(&best[q], m);
    }
}

int64_t split_target_wgs(int d) { return split_target(split_dpad(d)); }

NNGeom split_geom(int64_t nx, int64_t nB, int d, int64_t target) {
    const int64_t per_wg = 64 * split_nb(split_dpad(d));
    const int64_t nq = (nx + per_wg - 1) / per_wg;
    if (target <= 0) target = split_target(split_dpad(d));
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

size_t split_record_bytes(int64_t nx, int64_t nB, int d) {
    if (nx <= 0 || nB <= 0 || nx >= kSplitManyQueries) return 0;
    // a record per (query, chunk), then room to list every pair for rescan
    return (size_t)nx * (size_t)split_geom(nx, nB, d, 0).nchunk * (sizeof(uint4) + sizeof(uint2));
}

template <int DP>
static hipError_t go_split(const float *X, const int32_t *rows, int64_t nx, const uint16_t *Xs,
                           const float *xn2, const float *B, const uint16_t *Bs, int64_t nB,
                           int d, unsigned long long *best, const float *nb2, DevParams *p,
                           uint4 *rec, hipStream_t st) {
    const NNGeom g = split_geom(nx, nB, d, 0);
    if (nx >= kSplitManyQueries) {
        k_nnmin_l2_split<DP, split_nb(DP), 4, false><<<(unsigned)g.blocks, 256, 0, st>>>(
            X, rows, nx, Xs, xn2, B, Bs, nB, d, nb2, g.chunk, g.nchunk, best, p, nullptr);
    } else if (rec != nullptr) {
        k_nnmin_l2_split<DP, split_nb(DP), 3, true><<<(unsigned)g.blocks, 256, 0, st>>>(
            X, rows, nx, Xs, xn2, B, Bs, nB, d, nb2, g.chunk, g.nchunk, best, p, rec);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint2 *redo = g.chunk > kRedoInlineRows
                          ? reinterpret_cast<uint2 *>(rec + (size_t)nx * g.nchunk)
                          : nullptr;
        const unsigned nbr = (unsigned)((nx + 3) / 4);
        if (g.nchunk <= 64 * kResolveRegs)
            k_split_resolve<kResolveRegs><<<nbr, 256, 0, st>>>(
                X, rows, nx, xn2, B, nB, d, DP, g.chunk, g.nchunk, rec, redo, best, p);
        else
            k_split_resolve<0><<<nbr, 256, 0, st>>>(X, rows, nx, xn2, B, nB, d, DP, g.chunk,
                                                    g.nchunk, rec, redo, best, p);
        if (redo != nullptr)
            k_split_redo<<<kGridRedo, 256, 0, st>>>(X, rows, B, nB, d, g.chunk, redo, best, p);
    } else {
        k_nnmin_l2_split<DP, split_nb(DP), 3, false><<<(unsigned)g.blocks, 256, 0, st>>>(
            X, rows, nx, Xs, xn2, B, Bs, nB, d, nb2, g.chunk, g.nchunk, best, p, nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_nnmin_split(const float *X, const int32_t *rows, int64_t nx, const uint16_t *Xs,
                              const float *xn2, const float *B, const uint16_t *Bs, int64_t nB,
                              int d, unsigned long long *best, const float *nb2, DevParams *p,
                              hipStream_t st, uint4 *rec) {
    if (nx <= 0) return hipSuccess;
    if (Xs == nullptr || xn2 == nullptr) return hipErrorInvalidValue;
#define CH_SPLIT_ARGS X, rows, nx, Xs, xn2, B, Bs, nB, d, best, nb2, p, rec, st
    switch (split_dpad(d)) {
        case 32: return go_split<32>(CH_SPLIT_ARGS);
        case 64: return go_split<64>(CH_SPLIT_ARGS);
        case 128: return go_split<128>(CH_SPLIT_ARGS);
        default: return go_split<256>(CH_SPLIT_ARGS);
    }
#undef CH_SPLIT_ARGS
}

// ---------------------------------------------------------------- batched
// A job's split tables live at J.bq (B) and J.xsplit, J.xn2 (the draws); its
// cast stage fills them.  Served batches take the three-product form.

constexpr unsigned kGridSplit = 1024, kGridNNSplit = 2048;

__global__ __launch_bounds__(256) void kb_split_rows(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsCast, [&](const Job &J, Blk b) {
        if (b.id < J.nb_castB)
            split_rows(J.B, nullptr, J.nB, J.d, split_dpad(J.d),
                       reinterpret_cast<uint16_t *>(J.bq), nullptr, J.p, Blk{b.id, J.nb_castB});
        else
            split_rows(J.A, J.idx, J.T, J.d, split_dpad(J.d), J.xsplit, J.xn2, J.p,
                       Blk{b.id - J.nb_castB, J.nb_castX});
    });
}

template <int DP>
__global__ __launch_bounds__(256) void kb_nn_split(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsNN, [&](const Job &J, Blk b) {
        nnmin_l2_split<DP, split_nb(DP), 3>(J.A, J.idx, J.T, J.xsplit, J.xn2, J.B,
                                            reinterpret_cast<const uint16_t *>(J.bq), J.nB, J.d,
                                            J.nb2, J.nn_chunk, J.nn_nchunk, J.best, J.p, b);
    });
}

hipError_t launch_batch_split_rows(const Batch *bt, hipStream_t st) {
    kb_split_rows<<<kGridSplit, 256, 0, st>>>(bt);
    return hipGetLastError();
}

hipError_t launch_batch_split(const Batch *bt, int d, hipStream_t st) {
    switch (split_dpad(d)) {
        case 32: kb_nn_split<32><<<kGridNNSplit, 256, 0, st>>>(bt); break;
        case 64: kb_nn_split<64><<<kGridNNSplit, 256, 0, st>>>(bt); break;
        case 128: kb_nn_split<128><<<kGridNNSplit, 256, 0, st>>>(bt); break;
        default: kb_nn_split<256><<<kGridNNSplit, 256, 0, st>>>(bt); break;
    }
    return hipGetLastError();
}

}  // namespace chamfer

extern "C" double chamfer_split_score_bound(int32_t d, int32_t terms, float xn2, float b2max) {
    if (d < 1 || d > 256 || (terms != 3 && terms != 4)) return -1.0;
    return chamfer::split_score_bound(d, chamfer::split_dpad(d), terms, (double)xn2,
                                      (double)b2max);
}
