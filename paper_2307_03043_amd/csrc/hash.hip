// CrudeNN on the GPU (the CrudeNN figure and the appendix lemma on the grid
// hash at every scale): scale calibration, per-scale shifts and key
// multipliers, the open-addressing bucket tables of B, and the probe of A
// that yields the first colliding scale, the candidate b and D_a.
//
// Layout: one workgroup of four wavefronts per tile of 64 consecutive
// points, one point per lane; the wavefronts split the scales.  The tile's
// hashed coordinates are staged in LDS with an odd row stride, so the
// per-lane reads of row p, coordinate k hit 64 distinct banks.  Shifts and
// multipliers are indexed only by the (wave-uniform) scale and coordinate,
// so they are read through the scalar cache.  B's keys are written once,
// [L][n_B], and its tables built from them region by region in LDS (the
// partitioned build below; the serving path and the window tables insert
// directly); A's keys are never written: they are recomputed scale by
// scale until the first hit.
#include <climits>

#include "internal.h"

namespace chamfer {

// ------------------------------------------------------------- parameters

__device__ __forceinline__ void init_params(DevParams *p, uint32_t *lohi, int d, Blk b) {
    const int64_t t = b.id * blockDim.x + threadIdx.x;
    if (t == 0) {
        p->status = CHAMFER_OK;
        p->e_top = 0;
        p->s = 0;
        p->all_zero = 0;
        p->nonfinite = 0;
        p->W = 0;
        p->S = 0.0;
        p->fallbacks = 0;
        p->nredo = 0;
    }
    for (int64_t k = t; k < 2 * kMaxRepl; k += b.n * blockDim.x)
        (k < kMaxRepl ? p->max_d_rep : p->b2max_rep)[(k % kMaxRepl) * kReplStride] = 0u;
    if (lohi != nullptr)
        for (int64_t k = t; k < (int64_t)kLohiReps * 2 * d; k += b.n * blockDim.x)
            lohi[k] = (k % (2 * d)) < d ? 0xffffffffu : 0u;  // running min / max (ordered)
}

__global__ void k_init_params(DevParams *p, uint32_t *lohi, int d) {
    init_params(p, lohi, d, grid_blk());
}

int64_t init_blocks(int d) { return ((int64_t)kLohiReps * 2 * d + 255) / 256; }

hipError_t launch_init_params(DevParams *p, uint32_t *lohi, int d, hipStream_t st) {
    const int blocks = lohi ? (int)init_blocks(d) : 1;
    k_init_params<<<blocks, 256, 0, st>>>(p, lohi, d);
    return hipGetLastError();
}

// Key multipliers from the second Philox word: two odd 24-bit values.
__host__ __device__ inline uint64_t key_multipliers(uint64_t w1) {
    return ((w1 & 0xffffffull) | 1ull) | ((((w1 >> 32) & 0xffffffull) | 1ull) << 32);
}

// Shifts z'_ik (cell units, 24-bit lattice in [0,1)) and key multipliers
// M_ik from Philox4x64-10, counter (k, i, GRID, rep), key (seed, 0).
__device__ __forceinline__ void grid_tables(uint64_t seed, int L, int kh, float *zfrac,
                                            uint64_t *mult, int rep, Blk b) {
    const int t = (int)(b.id * blockDim.x + threadIdx.x);
    if (t >= L * kh) return;
    const int i = t / kh, k = t - i * kh;
    uint64_t c[4] = {(uint64_t)k, (uint64_t)i, (uint64_t)kPurposeGrid, (uint64_t)rep};
    philox4x64_10(c, seed, 0);
    zfrac[t] = ldexpf((float)(uint32_t)(c[0] >> 40), -24);
    mult[t] = key_multipliers(c[1]);
}

__global__ void k_grid_tables(uint64_t seed, int L, int kh, float *zfrac, uint64_t *mult,
                              int rep) {
    grid_tables(seed, L, kh, zfrac, mult, rep, grid_blk());
}

int64_t grid_table_blocks(int L, int kh) { return ((int64_t)L * kh + 255) / 256; }

hipError_t launch_grid_tables(uint64_t seed, int L, int kh, float *zfrac, uint64_t *mult,
                              int rep, hipStream_t st) {
    k_grid_tables<<<(unsigned)grid_table_blocks(L, kh), 256, 0, st>>>(seed, L, kh, zfrac, mult,
                                                                      rep);
    return hipGetLastError();
}

// Per-coordinate min and max over a point set, and a non-finite flag.  The
// flat element e has coordinate e mod d; the grid stride is a multiple of d,
// so every thread keeps one coordinate.  Min/max use integer atomics on an
// order-preserving encoding, whose result does not depend on their order.
__device__ __forceinline__ void minmax(const float *__restrict__ X, int64_t total, int d,
                                       int64_t stride, uint32_t *lohi, DevParams *p, Blk b) {
    extern __shared__ uint32_t sm[];
    const bool use_lds = d <= 2048;
    if (use_lds) {
        for (int i = threadIdx.x; i < d; i += blockDim.x) {
            sm[i] = 0xffffffffu;
            sm[d + i] = 0u;
        }
        __syncthreads();
    }
    const int64_t g = b.id * blockDim.x + threadIdx.x;
    uint32_t lo = 0xffffffffu, hi = 0u;
    int bad = 0;
    if (g < stride) {
        for (int64_t e = g; e < total; e += stride) {
            const float v = ro(X)[e];
            bad |= !isfinite(v);
            const uint32_t o = float_to_ordered(v);
            lo = min(lo, o);
            hi = max(hi, o);
        }
        const int k = (int)(g % d);
        if (use_lds) {
            atomicMin(&sm[k], lo);
            atomicMax(&sm[d + k], hi);
        } else {
            uint32_t *rep = lohi + (b.id % kLohiReps) * 2 * d;
            atomicMin(&rep[k], lo);
            atomicMax(&rep[d + k], hi);
        }
    }
    if (bad) atomicOr(&p->nonfinite, 1u);
    if (use_lds) {
        __syncthreads();
        uint32_t *rep = lohi + (b.id % kLohiReps) * 2 * d;
        for (int i = threadIdx.x; i < d; i += blockDim.x) {
            if (sm[i] != 0xffffffffu) atomicMin(&rep[i], sm[i]);
            if (sm[d + i] != 0u) atomicMax(&rep[d + i], sm[d + i]);
        }
    }
}

__global__ __launch_bounds__(256) void k_minmax(const float *__restrict__ X, int64_t total,
                                                int d, int64_t stride, uint32_t *lohi,
                                                DevParams *p) {
    minmax(X, total, d, stride, lohi, p, grid_blk());
}

// Same with 16-byte loads when d is a multiple of 4: thread g keeps the four
// coordinates of float4 column (g mod d/4).
__device__ __forceinline__ void minmax4(const float4 *__restrict__ X4, int64_t total4, int d,
                                        int64_t stride4, uint32_t *lohi, DevParams *p, Blk b) {
    extern __shared__ uint32_t sm[];
    const int d4 = d >> 2;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        sm[i] = 0xffffffffu;
        sm[d + i] = 0u;
    }
    __syncthreads();
    const int64_t g = b.id * blockDim.x + threadIdx.x;
    uint32_t lo[4] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu};
    uint32_t hi[4] = {0u, 0u, 0u, 0u};
    int bad = 0;
    auto take = [&](const float4 v) {
        const float c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bad |= !isfinite(c[i]);
            const uint32_t o = float_to_ordered(c[i]);
            lo[i] = min(lo[i], o);
            hi[i] = max(hi[i], o);
        }
    };
    if (g < stride4) {
        int64_t e = g;
        const auto *Xr = ro(X4);
        // up to 16 loads per thread (10^5 x 128 points: exactly 16) eight go
        // out together; on longer runs eight at a time was slower (10^6:
        // 0.21 -> 0.23 ms), so those keep four
        if (total4 <= 16 * stride4)
            for (; e + 7 * stride4 < total4; e += 8 * stride4) {
                float4 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = ld(Xr + e + u * stride4);
#pragma unroll
                for (int u = 0; u < 8; ++u) take(v[u]);
            }
        for (; e + 3 * stride4 < total4; e += 4 * stride4) {
            const float4 v0 = ld(Xr + e), v1 = ld(Xr + e + stride4),
                         v2 = ld(Xr + e + 2 * stride4), v3 = ld(Xr + e + 3 * stride4);
            take(v0);
            take(v1);
            take(v2);
            take(v3);
        }
        for (; e < total4; e += stride4) take(ld(Xr + e));
        const int k0 = (int)(g % d4) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            atomicMin(&sm[k0 + i], lo[i]);
            atomicMax(&sm[d + k0 + i], hi[i]);
        }
    }
    if (bad) atomicOr(&p->nonfinite, 1u);
    __syncthreads();
    uint32_t *rep = lohi + (b.id % kLohiReps) * 2 * d;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        if (sm[i] != 0xffffffffu) atomicMin(&rep[i], sm[i]);
        if (sm[d + i] != 0u) atomicMax(&rep[d + i], sm[d + i]);
    }
}

__global__ __launch_bounds__(256) void k_minmax4(const float4 *__restrict__ X4, int64_t total4,
                                                 int d, int64_t stride4, uint32_t *lohi,
                                                 DevParams *p) {
    minmax4(X4, total4, d, stride4, lohi, p, grid_blk());
}

// Both point sets in one launch: blocks [0, nbA) take A, the rest B.
__global__ __launch_bounds__(256) void k_minmax4_pair(const float4 *__restrict__ A4,
                                                      int64_t totalA4, int64_t strideA4,
                                                      int64_t nbA, const float4 *__restrict__ B4,
                                                      int64_t totalB4, int64_t strideB4, int d,
                                                      uint32_t *lohi, DevParams *p) {
    const int64_t b = blockIdx.x;
    if (b < nbA)
        minmax4(A4, totalA4, d, strideA4, lohi, p, Blk{b, nbA});
    else
        minmax4(B4, totalB4, d, strideB4, lohi, p, Blk{b - nbA, (int64_t)gridDim.x - nbA});
}

bool minmax_vec4(const float *X, int d) {
    return (d & 3) == 0 && d <= 2048 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
}

void minmax_geom(int64_t n, int d, bool vec4, int64_t *blocks_out, int64_t *stride_out) {
    const int64_t total = n * (int64_t)d;
    int64_t blocks;
    // about 64 coordinates per thread: each block ends with 2d global atomics
    // on the same 2d words, so small inputs want few blocks
    if (vec4) {
        const int64_t total4 = total / 4;
        const int d4 = d / 4;
        blocks = (total4 + 4095) / 4096;
        if (blocks > 1024) blocks = 1024;
        const int64_t min_blocks = (d4 + 255) / 256;
        if (blocks < min_blocks) blocks = min_blocks;
        *stride_out = (blocks * 256 / d4) * d4;
    } else {
        blocks = (total + 16383) / 16384;
        if (blocks > 2048) blocks = 2048;
        const int64_t min_blocks = (d + 255) / 256;
        if (blocks < min_blocks) blocks = min_blocks;
        *stride_out = (blocks * 256 / d) * d;
    }
    *blocks_out = blocks;
}

hipError_t launch_minmax(const float *X, int64_t n, int d, uint32_t *lohi, DevParams *p,
                         hipStream_t st) {
    const int64_t total = n * (int64_t)d;
    int64_t blocks, stride;
    if (minmax_vec4(X, d)) {
        minmax_geom(n, d, true, &blocks, &stride);
        k_minmax4<<<(unsigned)blocks, 256, 2 * (size_t)d * sizeof(uint32_t), st>>>(
            reinterpret_cast<const float4 *>(X), total / 4, d, stride, lohi, p);
        return hipGetLastError();
    }
    minmax_geom(n, d, false, &blocks, &stride);
    const size_t lds = d <= 2048 ? 2 * (size_t)d * sizeof(uint32_t) : 0;
    k_minmax<<<(unsigned)blocks, 256, lds, st>>>(X, total, d, stride, lohi, p);
    return hipGetLastError();
}

hipError_t launch_minmax_pair(const float *A, int64_t nA, const float *B, int64_t nB, int d,
                              uint32_t *lohi, DevParams *p, hipStream_t st) {
    if (nA <= 0 || !minmax_vec4(A, d) || !minmax_vec4(B, d)) {
        hipError_t e = nA > 0 ? launch_minmax(A, nA, d, lohi, p, st) : hipSuccess;
        return e != hipSuccess ? e : launch_minmax(B, nB, d, lohi, p, st);
    }
    int64_t nbA, sA, nbB, sB;
    minmax_geom(nA, d, true, &nbA, &sA);
    minmax_geom(nB, d, true, &nbB, &sB);
    k_minmax4_pair<<<(unsigned)(nbA + nbB), 256, 2 * (size_t)d * sizeof(uint32_t), st>>>(
        reinterpret_cast<const float4 *>(A), nA * (int64_t)d / 4, sA, nbA,
        reinterpret_cast<const float4 *>(B), nB * (int64_t)d / 4, sB, d, lohi, p);
    return hipGetLastError();
}

// Fold the kLohiReps copies of the running min/max into the first.
__device__ __forceinline__ void fold_lohi(uint32_t *lohi, int d) {
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        uint32_t lo = lohi[k], hi = lohi[d + k];
        for (int r = 1; r < kLohiReps; ++r) {
            lo = min(lo, lohi[(size_t)r * 2 * d + k]);
            hi = max(hi, lohi[(size_t)r * 2 * d + d + k]);
        }
        lohi[k] = lo;
        lohi[d + k] = hi;
    }
    __syncthreads();
}

__global__ void k_calib_final_wide(uint32_t *lohi, int d, DevParams *p) {
    fold_lohi(lohi, d);
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double S = 0.0;
    for (int k = 0; k < d; ++k)
        S = S + ((double)ordered_to_float(lohi[d + k]) - (double)ordered_to_float(lohi[k]));
    p->S = S;
    p->e_top = S > 0.0 ? ceil_log2_pos(S) : 0;
    if (p->nonfinite) p->status = CHAMFER_ENONFINITE;
}

// S = sum_k (hi_k - lo_k) in double, k ascending; e_top = ceil(log2 S).
// The per-coordinate spans are gathered in parallel; one thread sums them
// in order.
__device__ __forceinline__ void calib_final(uint32_t *lohi, int d, DevParams *p) {
    extern __shared__ double span[];
    fold_lohi(lohi, d);
    for (int k = threadIdx.x; k < d; k += blockDim.x)
        span[k] = (double)ordered_to_float(lohi[d + k]) - (double)ordered_to_float(lohi[k]);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double S = 0.0;
    for (int k = 0; k < d; ++k) S = S + span[k];
    p->S = S;
    p->e_top = S > 0.0 ? ceil_log2_pos(S) : 0;
    if (p->nonfinite) p->status = CHAMFER_ENONFINITE;
}

__global__ __launch_bounds__(256) void k_calib_final(uint32_t *lohi, int d, DevParams *p) {
    calib_final(lohi, d, p);
}

hipError_t launch_calib_final(uint32_t *lohi, int d, DevParams *p, hipStream_t st) {
    if ((size_t)d * sizeof(double) > 60000) {
        // very wide points: spans recomputed by the summing thread
        k_calib_final_wide<<<1, 64, 0, st>>>(lohi, d, p);
        return hipGetLastError();
    }
    k_calib_final<<<1, 256, (size_t)d * sizeof(double), st>>>(lohi, d, p);
    return hipGetLastError();
}

// Empty W = 1 tables: `count` buckets (key EMPTY, value INT_MAX), then the
// count fingerprint bytes that follow them (0 = empty slot).
__device__ __forceinline__ void table_fill(Bucket *t, size_t count, Blk b) {
    const size_t stride = (size_t)b.n * blockDim.x;
    for (size_t i = (size_t)b.id * blockDim.x + threadIdx.x; i < count; i += stride) {
        Bucket b;
        b.key = kEmptyKey;
        b.val = INT_MAX;
        b.pad = 0;
        t[i] = b;
    }
    uint4 *fp = reinterpret_cast<uint4 *>(t + count);
    for (size_t i = (size_t)b.id * blockDim.x + threadIdx.x; i < count / 16; i += stride)
        fp[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_table_fill(Bucket *t, size_t count) { table_fill(t, count, grid_blk()); }

int64_t table_fill_blocks(size_t count) {
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    return (int64_t)blocks;
}

// Parameter block, lo/hi, shifts and multipliers of structure 0 and (tables
// non-null) the empty W = 1 tables in one launch: the three independent
// bodies over consecutive block ranges.
__global__ __launch_bounds__(256) void k_setup(DevParams *p, uint32_t *lohi, int d, uint64_t seed,
                                               int L, int kh, float *zfrac, uint64_t *mult,
                                               Bucket *tables, size_t count, int nb_init,
                                               int nb_grid, int nb_fill) {
    const int64_t b = blockIdx.x;
    if (b < nb_init) {
        init_params(p, lohi, d, Blk{b, nb_init});
    } else if (b < nb_init + nb_grid) {
        grid_tables(seed, L, kh, zfrac, mult, 0, Blk{b - nb_init, nb_grid});
    } else {
        table_fill(tables, count, Blk{b - nb_init - nb_grid, nb_fill});
    }
}

hipError_t launch_setup(DevParams *p, uint32_t *lohi, int d, uint64_t seed, int L, int kh,
                        float *zfrac, uint64_t *mult, Bucket *tables, size_t count,
                        hipStream_t st) {
    const int nb_init = (int)init_blocks(d), nb_grid = (int)grid_table_blocks(L, kh);
    const int nb_fill = tables ? (int)table_fill_blocks(count) : 0;
    k_setup<<<(unsigned)(nb_init + nb_grid + nb_fill), 256, 0, st>>>(
        p, lohi, d, seed, L, kh, zfrac, mult, tables, count, nb_init, nb_grid, nb_fill);
    return hipGetLastError();
}

hipError_t launch_table_fill(Bucket *tables, size_t count, hipStream_t st) {
    k_table_fill<<<(unsigned)table_fill_blocks(count), 256, 0, st>>>(tables, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------ keys

// Key of hashed coordinates y (stride 1) at the scale of side 2^e:
// cell_k = floor(fma(y_k, 2^-e, z'_k)) as an int32 (y_k 2^-e is exact, so one
// rounding, of the sum), K1 = sum_k (cell_k mod 2^24) M1_k mod 2^32, K2 the
// same with M2_k, key = (K1 2^32 + K2) >> 1; M_k = M1_k | M2_k << 32 (odd
// 24-bit multipliers).  Four VALU operations per coordinate: one fma, the
// floor conversion and two 24-bit multiply-adds.  CLAMP: saturate the
// shifted coordinate at the int32 range first (NaN to the upper bound);
// needed only when a cell index can leave that range: more than 30 scales,
// or sides below 2^-126 (2^-e not finite).  Sums are mod 2^32 and split
// over two accumulator pairs to shorten the dependent chains.
template <bool CLAMP>
__device__ __forceinline__ uint32_t cell24(float q) {
    if (CLAMP) q = fmaxf(fminf(q, 2147483520.0f), -2147483648.0f);
    return (uint32_t)(int32_t)floorf(q);
}

template <bool CLAMP, class PZ, class PM>
__device__ __forceinline__ unsigned long long bucket_key(const float *y, int kh, int e, PZ zf,
                                                         PM M) {
    const float p = ldexpf(1.0f, -e);
    uint32_t a1 = 0, a2 = 0, b1 = 0, b2 = 0;
    int k = 0;
    for (; k + 2 <= kh; k += 2) {
        const uint32_t c0 = cell24<CLAMP>(fmaf(y[k], p, zf[k]));
        const uint32_t c1 = cell24<CLAMP>(fmaf(y[k + 1], p, zf[k + 1]));
        const unsigned long long m0 = M[k], m1 = M[k + 1];
        a1 += __umul24(c0, (uint32_t)m0);
        a2 += __umul24(c0, (uint32_t)(m0 >> 32));
        b1 += __umul24(c1, (uint32_t)m1);
        b2 += __umul24(c1, (uint32_t)(m1 >> 32));
    }
    if (k < kh) {
        const uint32_t c0 = cell24<CLAMP>(fmaf(y[k], p, zf[k]));
        const unsigned long long m0 = M[k];
        a1 += __umul24(c0, (uint32_t)m0);
        a2 += __umul24(c0, (uint32_t)(m0 >> 32));
    }
    return (((unsigned long long)(a1 + b1) << 32) | (unsigned long long)(a2 + b2)) >> 1;
}

// Same, with y_k = x_k - lo_k read from HBM (l1 with d too large for LDS).
template <bool CLAMP, class PX, class PL, class PZ, class PM>
__device__ __forceinline__ unsigned long long bucket_key_global(PX x, PL lohi, int kh, int e,
                                                                PZ zf, PM M) {
    const float p = ldexpf(1.0f, -e);
    uint32_t a1 = 0, a2 = 0;
    for (int k = 0; k < kh; ++k) {
        const float y = x[k] - ordered_to_float(lohi[k]);
        const uint32_t c = cell24<CLAMP>(fmaf(y, p, zf[k]));
        const unsigned long long m = M[k];
        a1 += __umul24(c, (uint32_t)m);
        a2 += __umul24(c, (uint32_t)(m >> 32));
    }
    return (((unsigned long long)a1 << 32) | (unsigned long long)a2) >> 1;
}

// Home slot: the top bits of the key times an odd 64-bit constant (the
// golden-ratio multiplier), which carries the well-mixed low bits of the two
// 32-bit sums into the top (the top bits of a sum of small cells times
// 24-bit multipliers are not uniform by themselves).  The fingerprint of a
// key is the next 8 bits of the same product, 0 mapped to 1 (0 marks an
// empty slot in the fingerprint bytes that follow a W = 1 table).
__device__ __forceinline__ uint64_t home_slot(unsigned long long key, int log2cap) {
    return (uint64_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - log2cap));
}

__device__ __forceinline__ uint32_t key_fp(unsigned long long key, int log2cap) {
    const uint32_t f = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (56 - log2cap)) & 0xffu;
    return f ? f : 1u;
}

// Fingerprint bytes of scale i of W = 1 tables of 2^log2cap buckets per scale.
__device__ __forceinline__ uint8_t *table_fps(Bucket *tables, int L, int log2cap, int i) {
    return reinterpret_cast<uint8_t *>(tables + ((size_t)L << log2cap)) + ((size_t)i << log2cap);
}

// Insert (key -> b) keeping the lowest b per key.  Linear probing; a slot's
// key changes only from EMPTY, by CAS, so each key owns exactly one slot,
// and the lane that claims it writes the key's fingerprint byte.  The slot
// is read first, so a key already present costs a load (and an atomicMin
// only when b is lower than the stored value).
__device__ void table_insert(Bucket *tab, uint8_t *fps, int log2cap, unsigned long long key,
                             int b) {
    const uint64_t mask = (1ull << log2cap) - 1;
    uint64_t slot = home_slot(key, log2cap);
    for (;;) {
        Bucket *e = tab + slot;
        unsigned long long cur =
            __hip_atomic_load(&e->key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == kEmptyKey) {
            const unsigned long long prev = atomicCAS(&e->key, kEmptyKey, key);
            if (prev == kEmptyKey || prev == key) {
                if (prev == kEmptyKey) fps[slot] = (uint8_t)key_fp(key, log2cap);
                atomicMin(&e->val, b);
                return;
            }
            cur = prev;
        }
        if (cur == key) {
            if (__hip_atomic_load(&e->val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > b)
                atomicMin(&e->val, b);
            return;
        }
        slot = (slot + 1) & mask;
    }
}

// Lowest b stored under key, or -1.  Runs in a later kernel than every
// insert.  The probe walks the fingerprint bytes, 16 per load, and reads a
// bucket only where the fingerprint matches: a missing key (most probes
// below a point's first colliding scale) touches only the fingerprints,
// 1/16 of the table's bytes.
__device__ __forceinline__ int table_probe(const CH_RO Bucket *tab, const CH_RO uint8_t *fps,
                                           int log2cap, unsigned long long key) {
    const uint64_t mask = (1ull << log2cap) - 1;
    const uint32_t f = key_fp(key, log2cap);
    uint64_t slot = home_slot(key, log2cap);
    for (;;) {
        const uint64_t base = slot & ~15ull;
        const uint4 w = ld(reinterpret_cast<const CH_RO uint4 *>(fps + base));
        for (int q = (int)(slot - base); q < 16; ++q) {
            const uint32_t word = q < 4 ? w.x : q < 8 ? w.y : q < 12 ? w.z : w.w;
            const uint32_t byte = (word >> (8 * (q & 3))) & 0xffu;
            if (byte == 0) return -1;
            if (byte == f) {
                const uint4 bk = ld(reinterpret_cast<const CH_RO uint4 *>(tab + base + q));
                const unsigned long long k =
                    (unsigned long long)bk.x | ((unsigned long long)bk.y << 32);
                if (k == key) return (int)bk.z;
            }
        }
        slot = (base + 16) & mask;
    }
}

// Window tables (multi-probe CrudeNN): a bucket holds its key and the W
// smallest b inserted under it, ascending, INT_MAX for empty positions.
// W smallest suffice: a probe that has seen s < W points at finer scales
// needs W - s unseen points of the bucket, and at most s of its W smallest
// are seen, so the W - s smallest unseen ones are among them.
// The insert runs b through the W positions as a chain of atomicMin: each
// position keeps the smaller of its value and the incoming one and passes
// the larger on, so position j ends with the (j+1)-th smallest b inserted,
// whatever the interleaving.  A position already below b is skipped (values
// only decrease), and an empty position ends the chain.
__device__ void wide_insert(unsigned long long *keys, int *mem, int log2cap,
                            unsigned long long key, int b, int W) {
    const uint64_t mask = (1ull << log2cap) - 1;
    uint64_t slot = home_slot(key, log2cap);
    for (;;) {
        unsigned long long cur =
            __hip_atomic_load(&keys[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == kEmptyKey) {
            const unsigned long long prev = atomicCAS(&keys[slot], kEmptyKey, key);
            if (prev == kEmptyKey || prev == key) break;
            cur = prev;
        }
        if (cur == key) break;
        slot = (slot + 1) & mask;
    }
    int *m = mem + slot * (uint64_t)W;
    int x = b;
    for (int j = 0; j < W; ++j) {
        if (__hip_atomic_load(&m[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < x) continue;
        const int old = atomicMin(&m[j], x);
        if (old == INT_MAX) return;  // x took an empty position
        x = max(old, x);             // the larger one moves on
    }
}

// Bucket index of key in a window table, or -1.
__device__ __forceinline__ int64_t wide_find(const CH_RO unsigned long long *keys, int log2cap,
                                             unsigned long long key) {
    const uint64_t mask = (1ull << log2cap) - 1;
    uint64_t slot = home_slot(key, log2cap);
    for (;;) {
        const unsigned long long k = keys[slot];
        if (k == key) return (int64_t)slot;
        if (k == kEmptyKey) return -1;
        slot = (slot + 1) & mask;
    }
}

// Canonical float32 distance (square root of the accumulator for l2).
template <int METRIC>
__device__ __forceinline__ float dist32(const float *__restrict__ a, const float *__restrict__ b,
                                        int d) {
    const float acc = canon_acc<METRIC, 4>(a, b, d);
    return METRIC == CHAMFER_L1 ? acc : sqrtf(acc);
}

constexpr int kTile = 64;        // points per workgroup
constexpr int kWaves = 4;        // wavefronts per workgroup; they split the scales
constexpr int kThreads = 64 * kWaves;
constexpr int kEmbedChunk = 64;  // coordinates of x - lo staged per pass (l2), by default

// Copy rows [np][kc] of the tile (row stride d, from column k0) into LDS
// rows of stride ldr, less lo_k (the ordered-int lower corner) when lo is
// given: each thread issues a batch of loads before it stores any of them,
// so a tile costs a few memory round trips instead of one per element.  The
// loads are in bounds and unconditional (rows past np and elements past the
// tile read its last element, and are not stored), so the batch is in flight
// at once; in the float4 form a thread always takes the same quad of
// columns, whose lo it loads once, first.
template <int BATCH>
__device__ __forceinline__ void stage_rows(const float *__restrict__ X, int64_t p0, int np, int d,
                                           int k0, int kc, float *dst, int ldr,
                                           const uint32_t *__restrict__ lo) {
    const auto *Xr = ro(X);
    if (kc == 64 && (d & 3) == 0 && (k0 & 3) == 0 &&
        (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
        // 64 coordinates per row as 16 float4 loads (row r, quad c of
        // element e: r = e / 16, c = e % 16 = thread % 16), four per thread
        // in one batch
        const auto *X4 = reinterpret_cast<const CH_RO float4 *>(Xr);
        constexpr int kRowsPerPass = kThreads / 16;
        const int c = (int)threadIdx.x & 15, r0 = (int)threadIdx.x >> 4;
        // without lo the quad is read from X itself and not used
        const bool sub = lo != nullptr;
        const auto *lr = sub ? ro(lo) + k0 + 4 * c : ro(reinterpret_cast<const uint32_t *>(X));
        const uint32_t l0 = lr[0], l1 = lr[1], l2 = lr[2], l3 = lr[3];
        float4 v[kTile * 16 / kThreads];
#pragma unroll
        for (int i = 0; i < kTile * 16 / kThreads; ++i) {
            const int r = min(i * kRowsPerPass + r0, np - 1);
            v[i] = ld(X4 + (((p0 + r) * d + k0) >> 2) + c);
        }
        const float4 off = sub ? make_float4(ordered_to_float(l0), ordered_to_float(l1),
                                             ordered_to_float(l2), ordered_to_float(l3))
                               : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int i = 0; i < kTile * 16 / kThreads; ++i) {
            const int r = i * kRowsPerPass + r0;
            if (r < np) {
                float *o = dst + r * ldr + 4 * c;
                o[0] = v[i].x - off.x;
                o[1] = v[i].y - off.y;
                o[2] = v[i].z - off.z;
                o[3] = v[i].w - off.w;
            }
        }
        return;
    }
    const int total = np * kc;
    const bool sub = lo != nullptr;
    const auto *lr = sub ? ro(lo) + k0 : ro(reinterpret_cast<const uint32_t *>(X));
    for (int base = 0; base < total; base += BATCH * kThreads) {
        float v[BATCH];
        uint32_t o[BATCH];
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int e = min(base + i * kThreads + (int)threadIdx.x, total - 1);
            const int r = e / kc, k = e - r * kc;
            v[i] = Xr[(p0 + r) * d + k0 + k];
            o[i] = lr[sub ? k : 0];
        }
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int e = base + i * kThreads + (int)threadIdx.x;
            if (e < total) {
                const int r = e / kc, k = e - r * kc;
                dst[r * ldr + k] = v[i] - (sub ? ordered_to_float(o[i]) : 0.0f);
            }
        }
    }
}

// Probe grids of at least this many tiles compute the candidate distances
// with all four wavefronts (l2, d = 128, tile_dist against the gather by
// wavefront 0: gather faster by 10% at 1563 tiles and 4% at 3907, tile_dist
// faster by 1% at 6250 tiles and 4% at 15625; quad_dist 2% faster again at
// 15625, and 8% for l1 at d = 64).
constexpr int64_t kCoopDistTiles = 5000;

// Canonical float32 distance of each point of the tile to its candidate row
// cand[p] of B (an LDS list; rows past np are never used): the workgroup
// stages t = x_k - b_k for 64 coordinates of all points at a time into LDS
// (rows read whole by consecutive lanes, both rows of a point in one batch
// of loads; when d is a multiple of 64 the next chunk's loads are in flight
// while the current one is summed), and lane p of wavefront 0 adds point p's
// terms in coordinate order, so the result is the one dist32 computes.  tb:
// LDS of kTile rows of (min(d, 64) | 1) floats.  Every thread of the
// workgroup must call it; the distance is returned in wavefront 0's lanes.
template <int METRIC>
__device__ __forceinline__ float tile_dist(const float *__restrict__ X, int64_t p0, int np, int d,
                                           const float *__restrict__ Bpts, const int *cand,
                                           float *tb) {
    const auto *Xr = ro(X);
    const auto *Br = ro(Bpts);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ldt = min(d, 64) | 1;
    float acc = 0.0f;
    auto term = [&](float t) { acc = METRIC == CHAMFER_L1 ? acc + fabsf(t) : fmaf(t, t, acc); };
    if ((d & 63) == 0) {
        // element (row 4 i + wave, coordinate lane): rows are wave-uniform
        constexpr int kPer = kTile * 64 / kThreads;
        float a[kPer], b[kPer];
        auto load = [&](int k0) {
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int r = min(kThreads / 64 * i + wave, np - 1);
                const int c = __builtin_amdgcn_readfirstlane(cand[r]);
                a[i] = Xr[(p0 + r) * d + k0 + lane];
                b[i] = Br[(int64_t)c * d + k0 + lane];
            }
        };
        load(0);
        for (int k0 = 0; k0 < d; k0 += 64) {
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int r = kThreads / 64 * i + wave;
                if (r < np) tb[r * ldt + lane] = a[i] - b[i];
            }
            __syncthreads();
            if (k0 + 64 < d) load(k0 + 64);
            if (wave == 0 && lane < np) {
                const float *t = tb + lane * ldt;
#pragma unroll
                for (int k = 0; k < 64; k += 16) {
                    float v[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) v[j] = t[k + j];
#pragma unroll
                    for (int j = 0; j < 16; ++j) term(v[j]);
                }
            }
            __syncthreads();
        }
    } else {
        constexpr int kPer = 8;  // elements per thread per batch
        float a[kPer], b[kPer];
        for (int k0 = 0; k0 < d; k0 += 64) {
            const int kc = min(64, d - k0);
            const int total = np * kc;
            for (int base = 0; base < total; base += kPer * kThreads) {
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int e = min(base + i * kThreads + (int)threadIdx.x, total - 1);
                    const int r = e / kc, k = e - r * kc;
                    a[i] = Xr[(p0 + r) * d + k0 + k];
                    b[i] = Br[(int64_t)cand[r] * d + k0 + k];
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int e = base + i * kThreads + (int)threadIdx.x;
                    if (e < total) {
                        const int r = e / kc, k = e - r * kc;
                        tb[r * ldt + k] = a[i] - b[i];
                    }
                }
            }
            __syncthreads();
            if (wave == 0 && lane < np)
                for (int k = 0; k < kc; ++k) term(tb[lane * ldt + k]);
            __syncthreads();
        }
    }
    return METRIC == CHAMFER_L1 ? acc : sqrtf(acc);
}

// Canonical float32 distance of the tile's point pp to B's row c with four
// lanes: lane 4 j + s holds quarter s of both rows (coordinates
// [s S, (s + 1) S), S = ceil(d / 4) <= kQuadCols, all loaded in one batch)
// and continues the sum of quarter s - 1, which moves one lane up between
// quarters, so the terms are added in coordinate order as dist32 adds them.
// The distance is returned in lane 4 j + 3.  All 64 lanes must call it.
constexpr int kQuadCols = 32;
template <int METRIC>
__device__ __forceinline__ float quad_dist(const float *__restrict__ X, int64_t p0, int pp, int d,
                                           const float *__restrict__ Bpts, int c) {
    const int lane = threadIdx.x & 63, s = lane & 3;
    const int S = (d + 3) >> 2;
    const int k0 = s * S, k1 = min(d, k0 + S);
    const auto *xr = ro(X) + (p0 + pp) * d;
    const auto *br = ro(Bpts) + (int64_t)c * d;
    float t[kQuadCols];
    if ((S & 3) == 0 && (d & 3) == 0 &&
        ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Bpts)) & 15) == 0) {
        // quarters of whole 16-byte quads (d a multiple of 16)
        float4 xv[kQuadCols / 4], bv[kQuadCols / 4];
#pragma unroll
        for (int i = 0; i < kQuadCols / 4; ++i) {
            const int k = min(k0 + 4 * i, d - 4);
            xv[i] = ld(reinterpret_cast<const CH_RO float4 *>(xr + k));
            bv[i] = ld(reinterpret_cast<const CH_RO float4 *>(br + k));
        }
#pragma unroll
        for (int i = 0; i < kQuadCols / 4; ++i) {
            t[4 * i] = xv[i].x - bv[i].x;
            t[4 * i + 1] = xv[i].y - bv[i].y;
            t[4 * i + 2] = xv[i].z - bv[i].z;
            t[4 * i + 3] = xv[i].w - bv[i].w;
        }
    } else {
        float xv[kQuadCols], bv[kQuadCols];
#pragma unroll
        for (int i = 0; i < kQuadCols; ++i) {
            const int k = min(k0 + i, d - 1);
            xv[i] = xr[k];
            bv[i] = br[k];
        }
#pragma unroll
        for (int i = 0; i < kQuadCols; ++i) t[i] = xv[i] - bv[i];
    }
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float prev = __shfl_up(acc, 1, 4);  // quarter q - 1's sum, in the lane below
        if (s == q) {
            acc = q == 0 ? 0.0f : prev;
#pragma unroll
            for (int i = 0; i < kQuadCols; ++i)
                if (k0 + i < k1) acc = METRIC == CHAMFER_L1 ? acc + fabsf(t[i]) : fmaf(t[i], t[i], acc);
        }
    }
    return METRIC == CHAMFER_L1 ? acc : sqrtf(acc);
}

// MODE 0: insert the tile's points (B) into the L tables.
// MODE 1: probe (A): first scale with a hit, candidate, D_a; max D_a.
// MODE 2: write keys[L][n].
// MODE 5: write keys[L][n] of B for the partitioned table build: a lane
//         whose key a lower lane of its wavefront also holds writes the
//         empty key instead (it cannot be the lowest index of its bucket),
//         and the l2 row norms are computed as in MODE 0.
// MODE 3: insert into window tables (W smallest b per bucket).
// MODE 4: probe window tables: the first W distinct b over the scales, finest
//         first (wavefront 0 walks the scales of its lane's point; the
//         retrieved b are kept in LDS), candidate = the closest of them.
// With kProbeMerge a probe keeps the better of its candidate and the one
// already stored for the point (an earlier LSH structure), by (D_a, b); the
// max of D_a is reduced only with kProbeLast.
// KE: embedding dimension for l2 (0 for l1).  YG: l1 coordinates from HBM.
// Lane p of every wavefront works on point p of the tile; wavefront w takes
// scales w, w + 4, w + 8, ...  For the probe each wavefront stops at its own
// first hit (or once another wavefront has hit at a finer scale); the first
// colliding scale is the smallest over the four.
// EC: coordinates of x staged per pass of the l2 embedding.
// B's split table for the l2 exact pass, written from the staged rows while B
// is hashed (B is read once): row r of the table holds h = bf16(x_k) for
// k < split_dp, then m = bf16(x_k - h) (zero past d), as the separate split
// pass writes them.  Coordinates [k0, k0 + kc) of the tile's np points are
// staged at xs[point * ld + k - k0]; the last chunk also writes the padding
// [k0 + kc, split_dp).  Thread t takes 16 consecutive coordinates of point
// t / 4 per 64-coordinate step.
__device__ __forceinline__ void split_staged(const float *xs, int ld, int64_t p0, int np, int k0,
                                             int kc, bool last, int split_dp, uint16_t *out) {
    const int pp = threadIdx.x >> 2;
    if (pp >= np) return;
    uint16_t *row = out + (size_t)(p0 + pp) * (2 * split_dp);
    const int kend = last ? split_dp : k0 + kc;
    for (int c = k0 + (threadIdx.x & 3) * 16; c < kend; c += 64) {
        uint32_t hw[8], mw[8];
#pragma unroll
        for (int e = 0; e < 16; e += 2) {
            const int a = c + e - k0;
            const float v0 = a < kc ? xs[pp * ld + a] : 0.0f;
            const float v1 = a + 1 < kc ? xs[pp * ld + a + 1] : 0.0f;
            uint32_t h0, m0, h1, m1;
            split2(v0, h0, m0);
            split2(v1, h1, m1);
            hw[e / 2] = h0 | (h1 << 16);
            mw[e / 2] = m0 | (m1 << 16);
        }
        uint4 *hd = reinterpret_cast<uint4 *>(row + c);
        uint4 *md = reinterpret_cast<uint4 *>(row + split_dp + c);
        hd[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        hd[1] = make_uint4(hw[4], hw[5], hw[6], hw[7]);
        md[0] = make_uint4(mw[0], mw[1], mw[2], mw[3]);
        md[1] = make_uint4(mw[4], mw[5], mw[6], mw[7]);
    }
}

template <int METRIC, int MODE, int KE, bool YG, int EC = kEmbedChunk>
__device__ __forceinline__ void hash_tile(
    const float *__restrict__ X, int64_t n, const float *__restrict__ Bpts, int d, int L,
    const uint32_t *__restrict__ lohi, const int8_t *__restrict__ embed,
    const float *__restrict__ zfrac, const uint64_t *__restrict__ mult, Bucket *tables,
    int log2cap, unsigned long long *keys_out, float *D_out, int32_t *nn_out,
    int32_t *scale_out, float *nb2_out, DevParams *p, int64_t nB, int W, int flags, Blk blk,
    uint16_t *split_out = nullptr, int split_dp = 0) {
    extern __shared__ float smem[];
    __shared__ float los[EC > kEmbedChunk ? EC : kEmbedChunk];
    __shared__ int hit_scale[kTile];
    __shared__ int hit_cand[kWaves][kTile];
    __shared__ int wave_scale[kWaves][kTile];
    const int tid = threadIdx.x;
    // wave-uniform by construction; readfirstlane lets the compiler know, so
    // the per-scale tables and the embedding columns go through scalar loads
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t p0 = blk.id * kTile;
    const int np = (int)min<int64_t>(kTile, n - p0);
    const int64_t pt = p0 + lane;
    const bool active = lane < np;

    if (p->status != CHAMFER_OK) {
        if ((MODE == 1 || MODE == 4) && wave == 0 && active) {
            D_out[pt] = __builtin_nanf("");
            nn_out[pt] = -1;
            if (scale_out) scale_out[pt] = -1;
        }
        return;
    }
    const int kh = METRIC == CHAMFER_L1 ? d : KE;
    const int khp = kh | 1;  // odd row stride: lanes read distinct banks
    float *ys = smem;        // [kTile][khp]
    const int e_top = p->e_top;

    if (METRIC == CHAMFER_L1) {
        if (!YG) {
            stage_rows<16>(X, p0, np, d, 0, d, ys, khp, lohi);
        }
    } else {
        // The quantised embedding: u_k = floor(min((x_k - lo_k) 2^(24 - e_top),
        // 2^24 - 1)), Y_j = sum_k Zq_jk u_k exactly, on the int8 matrix cores:
        // wavefront w takes points 16 w + i of the tile (A rows: the three
        // bytes of u offset by -128, 16 coordinates per lane), B is Zq^T from
        // the packed table (16-column tiles of j, 64-coordinate steps), one
        // int32 accumulator per byte; then Y_j = sum_a 2^(8a) (acc_a + 128 R_j)
        // with R_j = sum_k Zq_jk, and y_j = (float)((Y_j 2^(e_top - 24)) inv),
        // inv = 1 / (beta KE 32).  The raw rows are staged 64 coordinates at a
        // time; for B, wavefront 0 also accumulates |x|^2 per row (fma chain,
        // coordinates ascending) for the l2 nearest-neighbour pass.
        constexpr int NT = (KE + 15) / 16;
        constexpr int ECM = kEmbedChunk;  // one 64-coordinate MFMA step per staged chunk
        const int nks = (d + ECM - 1) / ECM;
        const int i16 = lane & 15, g4 = lane >> 4;
        float *xs = smem + kTile * khp;  // [kTile][ECM + 1]
        typedef int v4i __attribute__((ext_vector_type(4)));
        v4i acc[3][NT];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[a][t] = v4i{0, 0, 0, 0};
        const auto *zpk = reinterpret_cast<const CH_RO uint4 *>(ro(embed));
        float n2 = 0.0f;
        const bool want_n2 =
            (MODE == 0 || MODE == 3 || MODE == 5) && nb2_out != nullptr && wave == 0;
        for (int ks = 0; ks < nks; ++ks) {
            const int k0 = ks * ECM;
            const int kc = min(ECM, d - k0);
            __syncthreads();
            stage_rows<16>(X, p0, np, d, k0, kc, xs, ECM + 1, nullptr);
            if (tid < kc) los[tid] = ordered_to_float(ro(lohi)[k0 + tid]);
            __syncthreads();
            if (want_n2 && active)
                for (int k = 0; k < kc; ++k) {
                    const float xraw = xs[lane * (ECM + 1) + k];
                    n2 = fmaf(xraw, xraw, n2);
                }
            if ((MODE == 0 || MODE == 3 || MODE == 5) && split_out != nullptr)
                split_staged(xs, ECM + 1, p0, np, k0, kc, ks == nks - 1, split_dp, split_out);
            // A: 16 coordinates k0 + 16 g4 + e of point 16 wave + i16, as the
            // three bytes of u, each offset by -128 (xor 0x80); four
            // coordinates at a time give one dword of each byte's operand
            v4i ab[3];
            const float *xr = xs + (16 * wave + i16) * (ECM + 1) + 16 * g4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t u[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * g4 + 4 * q + e;
                    const float v = ldexpf(xr[4 * q + e] - los[k < kc ? k : 0], 24 - e_top);
                    u[e] = k < kc ? (uint32_t)(int32_t)floorf(fminf(v, 16777215.0f)) : 0u;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const uint32_t sel = (uint32_t)a | ((uint32_t)(4 + a) << 8);
                    const uint32_t lo2 = __builtin_amdgcn_perm(u[1], u[0], sel);
                    const uint32_t hi2 = __builtin_amdgcn_perm(u[3], u[2], sel);
                    ab[a][q] = (int)(__builtin_amdgcn_perm(hi2, lo2, 0x05040100u) ^ 0x80808080u);
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const uint4 bz = ld(zpk + ((size_t)(t * nks + ks) * 64 + lane));
                const v4i bv = v4i{(int)bz.x, (int)bz.y, (int)bz.z, (int)bz.w};
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    acc[a][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ab[a], bv, acc[a][t], 0, 0, 0);
            }
        }
        // lane (g4, i16) holds points 16 wave + 4 g4 + r of column j = 16 t + i16
        const auto *rsum = reinterpret_cast<const CH_RO int32_t *>(ro(embed) + (size_t)NT * nks * 1024);
        const double inv = 1.0 / (sqrt(2.0 / 3.14159265358979323846) * (double)KE * 32.0);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = 16 * t + i16;
            const int32_t r128 = 128 * rsum[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t Y = (int64_t)(acc[0][t][r] + r128) +
                                  ((int64_t)(acc[1][t][r] + r128) << 8) +
                                  ((int64_t)(acc[2][t][r] + r128) << 16);
                if (j < KE)
                    ys[(16 * wave + 4 * g4 + r) * khp + j] =
                        (float)(ldexp((double)Y, e_top - 24) * inv);
            }
        }
        if (want_n2 && active) nb2_out[pt] = n2;
        if (want_n2) {
            uint32_t m = __float_as_uint(n2);
            for (int off = 32; off > 0; off >>= 1)
                m = max(m, (uint32_t)__shfl_xor((int)m, off));
            if (lane == 0) rep_max(p->b2max_rep, blk.id, m);
        }
    }
    if (MODE == 1 && wave == 0) hit_scale[lane] = L;
    __syncthreads();

    const float *yrow = ys + lane * khp;
    const float *xrow = X + pt * d;
    // cell indices can leave the int32 range only with more than 30 scales
    // or sides below 2^-126
    const bool clamp = L > 30 || e_top - (L - 1) <= -127;
    auto key_at = [&](int i) -> unsigned long long {
        const int e = e_top - (L - 1 - i);
        const auto zi = ro(zfrac) + (size_t)i * kh;
        const auto mi = ro(mult) + (size_t)i * kh;
        if (METRIC == CHAMFER_L1 && YG)
            return clamp ? bucket_key_global<true>(ro(xrow), ro(lohi), kh, e, zi, mi)
                         : bucket_key_global<false>(ro(xrow), ro(lohi), kh, e, zi, mi);
        return clamp ? bucket_key<true>(yrow, kh, e, zi, mi) : bucket_key<false>(yrow, kh, e, zi, mi);
    };

    if (MODE == 0) {
        // At coarse scales most lanes share a bucket.  A lane skips its
        // insert when a lower lane holds the same key (it has a lower index),
        // so the lowest index per bucket is unchanged and the hot buckets see
        // one access per wavefront instead of one per point.
        // Up to kLeaders distinct keys of the wavefront are deduplicated by
        // leader election (the leader is the lowest lane holding the key);
        // all remaining inserts then run in parallel.
        constexpr int kLeaders = 4;
        for (int i = wave; i < L; i += kWaves) {
            const unsigned long long key = active ? key_at(i) : kEmptyKey;
            unsigned long long rest = __ballot(active);
            bool mine = false;
            for (int it = 0; it < kLeaders && rest != 0; ++it) {
                const int leader = __ffsll((long long)rest) - 1;
                const unsigned long long lk = lane_u64(key, leader);
                rest &= ~__ballot(active && key == lk);
                mine |= lane == leader;
            }
            mine |= ((rest >> lane) & 1ull) != 0;
            if (mine)
                table_insert(tables + ((size_t)i << log2cap), table_fps(tables, L, log2cap, i),
                             log2cap, key, (int)pt);
        }
        return;
    }
    if (MODE == 5) {
        constexpr int kLeaders = 4;
        for (int i = wave; i < L; i += kWaves) {
            const unsigned long long key = active ? key_at(i) : kEmptyKey;
            unsigned long long rest = __ballot(active);
            bool mine = false;
            for (int it = 0; it < kLeaders && rest != 0; ++it) {
                const int leader = __ffsll((long long)rest) - 1;
                const unsigned long long lk = lane_u64(key, leader);
                rest &= ~__ballot(active && key == lk);
                mine |= lane == leader;
            }
            mine |= ((rest >> lane) & 1ull) != 0;
            if (active) keys_out[(size_t)i * n + pt] = mine ? key : kEmptyKey;
        }
        return;
    }
    if (MODE == 2) {
        if (active)
            for (int i = wave; i < L; i += kWaves) keys_out[(size_t)i * n + pt] = key_at(i);
        return;
    }
    // keep the better of (D, c, s) and the stored result of an earlier
    // structure; then store, and reduce max D on the last structure
    // store (D, c, s) for point ptx of the tile's points when act; with
    // wave_max, the wavefront's max of the stored D goes to p->max_d_rep
    // (kProbeLast).  Returns the stored D.
    auto finish_at = [&](int64_t ptx, bool act, float D, int c, int s, bool wave_max) {
        if (act) {
            if (flags & kProbeMerge) {
                const float Dp = D_out[ptx];
                const int cp = nn_out[ptx];
                if (Dp < D || (Dp == D && cp < c)) {
                    D = Dp;
                    c = cp;
                }
                if (scale_out) s = min(s, scale_out[ptx]);
            }
            D_out[ptx] = D;
            nn_out[ptx] = c;
            if (scale_out) scale_out[ptx] = s;
        }
        if (wave_max && (flags & kProbeLast)) {
            // wavefront max of D (D >= 0, so its bits order as floats)
            uint32_t m = act ? __float_as_uint(D) : 0u;
            for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
            if (lane == 0) rep_max(p->max_d_rep, blk.id, m);
        }
        return D;
    };
    auto finish = [&](float D, int c, int s) { finish_at(pt, active, D, c, s, true); };
    if (MODE == 3) {
        unsigned long long *wkeys = reinterpret_cast<unsigned long long *>(tables);
        int *wmem = reinterpret_cast<int *>(wkeys + ((size_t)L << log2cap));
        // lanes sharing a key: only the W lowest (smallest b) can be among
        // the bucket's W smallest; the rest skip, as in MODE 0
        constexpr int kLeaders = 4;
        for (int i = wave; i < L; i += kWaves) {
            const unsigned long long key = active ? key_at(i) : kEmptyKey;
            unsigned long long rest = __ballot(active);
            bool mine = false;
            for (int it = 0; it < kLeaders && rest != 0; ++it) {
                const int leader = __ffsll((long long)rest) - 1;
                const unsigned long long lk = lane_u64(key, leader);
                const unsigned long long same = __ballot(active && key == lk);
                if ((same >> lane) & 1ull) mine = __popcll(same & ((1ull << lane) - 1)) < W;
                rest &= ~same;
            }
            mine |= ((rest >> lane) & 1ull) != 0;
            if (mine)
                wide_insert(wkeys + ((size_t)i << log2cap), wmem + ((size_t)i << log2cap) * W,
                            log2cap, key, (int)pt, W);
        }
        return;
    }
    if (MODE == 4) {
        if (wave != 0) return;  // no barrier follows
        const auto *wk = reinterpret_cast<const unsigned long long *>(tables);
        const auto *wkeys = ro(wk);
        const auto *wmem = ro(reinterpret_cast<const int *>(wk + ((size_t)L << log2cap)));
        const int lds_floats = METRIC == CHAMFER_L1 ? (YG ? 0 : kTile * khp)
                                                    : kTile * (khp + EC + 1);
        int *got = reinterpret_cast<int *>(smem + lds_floats) + lane * W;
        int ng = 0, first = L;
        float D = 0.0f;
        int c = 0;
        if (active) {
            for (int i = 0; i < L && ng < W; ++i) {
                const int64_t s = wide_find(wkeys + ((size_t)i << log2cap), log2cap, key_at(i));
                if (s < 0) continue;
                const auto *m = wmem + (((size_t)i << log2cap) + (size_t)s) * W;
                for (int j = 0; j < W && ng < W; ++j) {
                    const int b = m[j];
                    if (b == INT_MAX) break;
                    bool seen = false;
                    for (int t = 0; t < ng; ++t) seen |= got[t] == b;
                    if (!seen) {
                        if (ng == 0) first = i;
                        got[ng++] = b;
                    }
                }
            }
            if (ng == 0)  // no collision at any scale: the window is b = 0 .. W - 1
                for (int b = 0; b < W && b < nB; ++b) got[ng++] = b;
            c = -1;
            for (int t = 0; t < ng; ++t) {
                const int b = got[t];
                const float v = dist32<METRIC>(xrow, Bpts + (size_t)b * d, d);
                if (c < 0 || v < D || (v == D && b < c)) {
                    D = v;
                    c = b;
                }
            }
        }
        finish(D, c, first);
        return;
    }
    // MODE 1: probe.
    int found = L, cand = 0;
    if (active) {
        for (int i = wave; i < L; i += kWaves) {
            if (i > __hip_atomic_load(&hit_scale[lane], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP))
                break;  // a finer scale already collided
            const int v = table_probe(ro((const Bucket *)tables) + ((size_t)i << log2cap),
                                      ro((const uint8_t *)table_fps(tables, L, log2cap, i)),
                                      log2cap, key_at(i));
            if (v >= 0) {
                found = i;
                cand = v;
                atomicMin(&hit_scale[lane], i);
                break;
            }
        }
    }
    wave_scale[wave][lane] = found;
    hit_cand[wave][lane] = cand;
    __syncthreads();
    // Small grids (about one round of resident workgroups) finish sooner when
    // wavefront 0 gathers both rows itself and the other three leave at once;
    // large ones are faster with all four wavefronts on the distances: four
    // lanes per point (quad_dist, d <= 128) or coalesced chunks (tile_dist).
    const bool coop = !(METRIC == CHAMFER_L1 && YG) && (n + kTile - 1) / kTile >= kCoopDistTiles;
    if (coop && d <= 4 * kQuadCols) {
        // wavefront w: points 16 w + j, four lanes each
        const int pq = 16 * wave + (lane >> 2);
        int sq = L, cq = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w)
            if (wave_scale[w][pq] < sq) {
                sq = wave_scale[w][pq];
                cq = hit_cand[w][pq];
            }
        const bool aq = (lane & 3) == 3 && pq < np;
        const float Dq = finish_at(p0 + pq, aq,
                                   quad_dist<METRIC>(X, p0, min(pq, np - 1), d, Bpts, cq), cq, sq,
                                   false);
        if (flags & kProbeLast) {  // one atomic per tile: the wavefronts' maxima meet in LDS
            uint32_t m = aq ? __float_as_uint(Dq) : 0u;
            for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
            if (lane == 0) hit_scale[wave] = (int)m;
            __syncthreads();
            if (tid == 0)
                rep_max(p->max_d_rep, blk.id,
                        max(max((uint32_t)hit_scale[0], (uint32_t)hit_scale[1]),
                            max((uint32_t)hit_scale[2], (uint32_t)hit_scale[3])));
        }
        return;
    }
    // the finest colliding scale over the four wavefronts (every wavefront
    // computes it for its lane's point; wavefront 0 keeps it)
    int best_s = L, best_c = 0;
    if (active) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w)
            if (wave_scale[w][lane] < best_s) {
                best_s = wave_scale[w][lane];
                best_c = hit_cand[w][lane];
            }
    }
    if (!coop) {
        if (wave != 0) return;
        finish(active ? dist32<METRIC>(xrow, Bpts + (size_t)best_c * d, d) : 0.0f, best_c,
               best_s);
        return;
    }
    if (wave == 0) hit_scale[lane] = best_c;  // the scale walk is over: reuse as the row list
    __syncthreads();
    const float D = tile_dist<METRIC>(X, p0, np, d, Bpts, hit_scale, smem);
    if (wave != 0) return;
    finish(active ? D : 0.0f, best_c, best_s);
}

int64_t hash_blocks(int64_t n) { return (n + kTile - 1) / kTile; }

// WAVES: wavefronts per SIMD the register allocation must allow.
template <int METRIC, int MODE, int KE, bool YG, int EC, int WAVES>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_hash(
    const float *__restrict__ X, int64_t n, const float *__restrict__ Bpts, int d, int L,
    const uint32_t *__restrict__ lohi, const int8_t *__restrict__ embed,
    const float *__restrict__ zfrac, const uint64_t *__restrict__ mult, Bucket *tables,
    int log2cap, unsigned long long *keys_out, float *D_out, int32_t *nn_out,
    int32_t *scale_out, float *nb2_out, DevParams *p, int64_t nB, int W, int flags,
    uint16_t *split_out, int split_dp) {
    hash_tile<METRIC, MODE, KE, YG, EC>(X, n, Bpts, d, L, lohi, embed, zfrac, mult, tables,
                                        log2cap, keys_out, D_out, nn_out, scale_out, nb2_out, p,
                                        nB, W, flags, grid_blk(), split_out, split_dp);
}


template <int METRIC, int KE, bool YG, int EC = kEmbedChunk>
static size_t hash_lds(int d) {
    const int kh = METRIC == CHAMFER_L1 ? d : KE;
    if (METRIC == CHAMFER_L1) return YG ? 0 : (size_t)kTile * (kh | 1) * sizeof(float);
    return (size_t)kTile * ((kh | 1) + EC + 1) * sizeof(float);
}

template <int METRIC, int KE, bool YG>
static hipError_t launch_hash_t(int mode, const float *X, int64_t n, const float *Bpts,
                                int64_t nB, int d, int L, const uint32_t *lohi,
                                const int8_t *embed, const float *zfrac, const uint64_t *mult,
                                Bucket *tables, int log2cap, uint64_t *keys_out, float *D_out,
                                int32_t *nn_out, int32_t *scale_out, float *nb2_out,
                                DevParams *p, int W, int flags, hipStream_t st,
                                uint16_t *split_out, int split_dp) {
    const unsigned blocks = (unsigned)hash_blocks(n);
    auto *ko = reinterpret_cast<unsigned long long *>(keys_out);
#define CH_KARGS X, n, Bpts, d, L, lohi, embed, zfrac, mult, tables, log2cap, ko, D_out, nn_out, \
                 scale_out, nb2_out, p, nB, W, flags, split_out, split_dp
    // Four wavefronts per SIMD for every mode: measured against six and
    // eight (l2, 10^5 points: probe 90, 117 and 141 us; keys and insert
    // within noise or slower).
    const size_t lds = hash_lds<METRIC, KE, YG>(d);
    switch (mode) {
        case 0: k_hash<METRIC, 0, KE, YG, kEmbedChunk, 4><<<blocks, kThreads, lds, st>>>(CH_KARGS); break;
        case 1: k_hash<METRIC, 1, KE, YG, kEmbedChunk, 4><<<blocks, kThreads, lds, st>>>(CH_KARGS); break;
        case 2: k_hash<METRIC, 2, KE, YG, kEmbedChunk, 4><<<blocks, kThreads, lds, st>>>(CH_KARGS); break;
        case 3: k_hash<METRIC, 3, KE, YG, kEmbedChunk, 4><<<blocks, kThreads, lds, st>>>(CH_KARGS); break;
        case 4:  // retrieved b per lane after the tile
            k_hash<METRIC, 4, KE, YG, kEmbedChunk, 4>
                <<<blocks, kThreads, lds + (size_t)kTile * W * sizeof(int), st>>>(CH_KARGS);
            break;
        case 5: k_hash<METRIC, 5, KE, YG, kEmbedChunk, 4><<<blocks, kThreads, lds, st>>>(CH_KARGS); break;
        default: return hipErrorInvalidValue;
    }
#undef CH_KARGS
    return hipGetLastError();
}

size_t table_bytes(int L, int log2cap, int W) {
    const size_t buckets = (size_t)L << log2cap;
    // W = 1: buckets, then a fingerprint byte per bucket
    return W <= 1 ? buckets * (sizeof(Bucket) + 1) : buckets * (sizeof(uint64_t) + (size_t)W * 4);
}

hipError_t launch_tables_empty(Bucket *tables, int L, int log2cap, int W, hipStream_t st) {
    const size_t buckets = (size_t)L << log2cap;
    if (W <= 1) return launch_table_fill(tables, buckets, st);
    auto *keys = reinterpret_cast<unsigned long long *>(tables);
    hipError_t e = launch_fill_u64(keys, (int64_t)buckets, ~0ull, st);
    if (e != hipSuccess) return e;
    // members: INT_MAX in both halves of each 64-bit word (W * buckets is even)
    return launch_fill_u64(keys + buckets, (int64_t)(buckets * W / 2), 0x7fffffff7fffffffull, st);
}

// kMaxLdsL1Dim: largest l1 dimension whose tile (64 x (d|1) floats) plus the
// static LDS fits the default 64 KiB.

hipError_t launch_hash(int mode, const float *X, int64_t n, const float *Bpts, int64_t nB,
                       int d, int metric, int L, int ke, const uint32_t *lohi,
                       const int8_t *embed, const float *zfrac, const uint64_t *mult,
                       Bucket *tables, int log2cap, uint64_t *keys_out, float *D_out,
                       int32_t *nn_out, int32_t *scale_out, float *nb2_out, DevParams *p,
                       int W, int flags, hipStream_t st, uint16_t *split_out, int split_dp) {
    if (n <= 0) return hipSuccess;
    if (W < 1 || W > kMaxWindow) return hipErrorInvalidValue;
    // the split table is written from the l2 embedding's staged rows (B's
    // hashing modes only; split_dp a multiple of 64 at or above d, or 32)
    if (split_out != nullptr &&
        (metric != CHAMFER_L2 || !(mode == 0 || mode == 3 || mode == 5) || split_dp < d ||
         (split_dp % 64 != 0 && split_dp != 32)))
        return hipErrorInvalidValue;
#define CH_ARGS mode, X, n, Bpts, nB, d, L, lohi, embed, zfrac, mult, tables, log2cap, keys_out, \
                D_out, nn_out, scale_out, nb2_out, p, W, flags, st, split_out, split_dp
    if (metric == CHAMFER_L1) {
        // the window probe also keeps W ints per lane in LDS
        const int room = mode == 4 ? kMaxLdsL1Dim - W : kMaxLdsL1Dim;
        if (d <= room) return launch_hash_t<CHAMFER_L1, 0, false>(CH_ARGS);
        return launch_hash_t<CHAMFER_L1, 0, true>(CH_ARGS);
    }
    switch (ke) {
        case 8: return launch_hash_t<CHAMFER_L2, 8, false>(CH_ARGS);
        case 16: return launch_hash_t<CHAMFER_L2, 16, false>(CH_ARGS);
        case 32: return launch_hash_t<CHAMFER_L2, 32, false>(CH_ARGS);
        case 64: return launch_hash_t<CHAMFER_L2, 64, false>(CH_ARGS);
        default: return hipErrorInvalidValue;
    }
#undef CH_ARGS
}

// ------------------------------------------------------ partitioned build
// The W = 1 tables of the direct path, built without global atomics.  A
// table of 2^c slots is cut into regions of S = 2^min(c, 11) slots, and a
// key's region is the top bits of its home slot.  From B's keys (hash mode
// 5, a wavefront's duplicate keys dropped): per scale, each block of
// kPartBlock keys counts its keys per region (k_part_hist), the counts
// become offsets (small partitions: inside k_part_scatter, each workgroup
// from its scale's counts; large ones: k_part_scan_rows and k_part_base),
// the blocks write their (key, b) pairs grouped by region (k_part_scatter,
// runs of a region contiguous), and one workgroup per (scale, region)
// inserts the region's pairs into a table in LDS -- linear probing from
// the home slot, lowest b per key, LDS atomics only -- and writes all S
// slots out (k_region_build).  The LDS build never wraps: a pair whose
// probe reaches the region's end is kept aside and inserted afterwards with
// the global insert (k_spill_insert), which continues into the next region
// like any linear probe; the probe then finds every key as after the global
// insert.
// A region holds at most S keys against about S / 2 expected (tables are
// at most half full), so on hashed keys few pairs spill.

constexpr int kRegionBits = 11;
constexpr int kPartBlock = 4096;   // keys per histogram / scatter workgroup
constexpr int kMaxRegions = 1024;  // regions per scale the scan and scatter hold in LDS

__host__ __device__ inline int region_bits(int log2cap) {
    return log2cap < kRegionBits ? log2cap : kRegionBits;
}

__host__ __device__ inline int64_t part_regions(int log2cap) {
    return (int64_t)1 << (log2cap - region_bits(log2cap));
}
int64_t part_blocks(int64_t nB) { return (nB + kPartBlock - 1) / kPartBlock; }
bool part_build_ok(int log2cap) { return part_regions(log2cap) <= kMaxRegions; }

static_assert(sizeof(uint3) == 12, "a (key, b) pair is three words");

size_t part_work_bytes(int L, int64_t nB, int log2cap, PartWork *w, char *base) {
    const int64_t R = part_regions(log2cap), nblk = part_blocks(nB);
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t b_keys = al((size_t)L * nB * sizeof(uint64_t));
    const size_t b_offs = al((size_t)L * nblk * R * sizeof(uint32_t));
    const size_t b_bins = al((size_t)L * R * 3 * sizeof(uint32_t));
    const size_t b_ent = al((size_t)L * nB * sizeof(uint3));
    if (w) {
        w->keys = reinterpret_cast<uint64_t *>(base);
        w->offs = reinterpret_cast<uint32_t *>(base + b_keys);
        w->bins = reinterpret_cast<uint32_t *>(base + b_keys + b_offs);
        w->entries = reinterpret_cast<uint3 *>(base + b_keys + b_offs + b_bins);
        w->spilled = reinterpret_cast<uint32_t *>(base + b_keys + b_offs + b_bins + b_ent);
    }
    return b_keys + b_offs + b_bins + b_ent + 256;
}

__device__ __forceinline__ uint32_t key_region(unsigned long long key, int log2cap) {
    return (uint32_t)(home_slot(key, log2cap) >> region_bits(log2cap));
}

// In-place exclusive prefix sum of v[0..R) (R <= 1024) by a workgroup of
// 256 threads; returns the total.  Each thread sums up to four consecutive
// values, the 256 partial sums are scanned by wavefront shuffles (tmp: the
// four wavefronts' totals), then written back.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t *v, int R, uint32_t *tmp) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int per = (R + 255) / 256;
    uint32_t loc[4] = {0, 0, 0, 0};
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (q < per && t * per + q < R) {
            loc[q] = v[t * per + q];
            sum += loc[q];
        }
    // inclusive scan of the groups' sums: shuffles in each wavefront, then
    // the totals of the wavefronts before
    uint32_t x = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) tmp[wv] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wv; ++w) before += tmp[w];
    const uint32_t total = tmp[0] + tmp[1] + tmp[2] + tmp[3];
    uint32_t run = before + x - sum;  // exclusive prefix of this thread's group
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (q < per && t * per + q < R) {
            v[t * per + q] = run;
            run += loc[q];
        }
    __syncthreads();
    return total;
}

// Counts per (scale i, block j, region): offs[(i nblk + j) R + g].
__global__ __launch_bounds__(256) void k_part_hist(const uint64_t *__restrict__ keys, int64_t nB,
                                                   int log2cap, int64_t nblk, uint32_t *offs) {
    extern __shared__ uint32_t cnt[];
    const int R = (int)part_regions(log2cap);
    const int64_t i = blockIdx.x / nblk, j = blockIdx.x - i * nblk;
    for (int g = threadIdx.x; g < R; g += 256) cnt[g] = 0;
    __syncthreads();
    const CH_RO uint64_t *kr = ro(keys) + i * nB;
    // all of the thread's keys are loaded (in bounds, unconditionally, so
    // the loads are in flight together) before any is counted
    constexpr int kPer = kPartBlock / 256;
    unsigned long long k[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) k[t] = kr[min(j * kPartBlock + t * 256 + threadIdx.x, nB - 1)];
#pragma unroll
    for (int t = 0; t < kPer; ++t)
        if (j * kPartBlock + t * 256 + threadIdx.x < nB && k[t] != kEmptyKey)
            atomicAdd(&cnt[key_region(k[t], log2cap)], 1u);
    __syncthreads();
    uint32_t *o = offs + (size_t)(i * nblk + j) * R;
    for (int g = threadIdx.x; g < R; g += 256) o[g] = cnt[g];
}

// Large partitions (many blocks and regions): the counts become offsets in
// two launches (offs: the exclusive prefix over blocks of each region's
// counts; bins[(i R + g) 3 + {0, 1, 2}] = the region's first entry in the
// scale's [nB] span of entries, its count, and 0, the spill count):
// k_part_scan_rows takes 64 regions of one scale per workgroup, each
// wavefront a contiguous quarter of the blocks (loads coalesced over the
// regions, eight in flight per lane), and writes the regions' totals;
// k_part_base scans the totals of each scale into the regions' first
// entries and clears the spill flag.
__global__ __launch_bounds__(256) void k_part_scan_rows(int log2cap, int64_t nblk,
                                                        uint32_t *offs, uint32_t *bins) {
    __shared__ uint32_t part[4][64];
    const int R = (int)part_regions(log2cap);
    const int gpb = (R + 63) / 64;  // workgroups per scale
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = blockIdx.x / gpb;
    const int g = (int)(blockIdx.x % gpb) * 64 + lane;
    const bool live = g < R;
    const int64_t q = (nblk + 3) / 4;
    const int64_t j0 = min(nblk, w * q), j1 = min(nblk, j0 + q);
    uint32_t *o = offs + (size_t)i * nblk * R + g;
    uint32_t sum = 0;
    if (live) {
        int64_t j = j0;
        for (; j + 8 <= j1; j += 8) {
            uint32_t c[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) c[e] = o[(j + e) * R];
#pragma unroll
            for (int e = 0; e < 8; ++e) sum += c[e];
        }
        for (; j < j1; ++j) sum += o[j * R];
    }
    part[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, tot = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint32_t x = part[v][lane];
        run += v < w ? x : 0u;
        tot += x;
    }
    if (!live) return;
    int64_t j = j0;
    for (; j + 8 <= j1; j += 8) {
        uint32_t c[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) c[e] = o[(j + e) * R];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            o[(j + e) * R] = run;
            run += c[e];
        }
    }
    for (; j < j1; ++j) {
        const uint32_t c = o[j * R];
        o[j * R] = run;
        run += c;
    }
    if (w == 0) {
        bins[((size_t)i * R + g) * 3 + 1] = tot;
        bins[((size_t)i * R + g) * 3 + 2] = 0;
    }
}

__global__ __launch_bounds__(256) void k_part_base(int log2cap, uint32_t *bins,
                                                   uint32_t *spilled) {
    __shared__ uint32_t tot[kMaxRegions + 256];
    const int R = (int)part_regions(log2cap);
    const int64_t i = blockIdx.x;
    if (i == 0 && threadIdx.x == 0) *spilled = 0;  // read after the region builds
    for (int g = threadIdx.x; g < R; g += 256) tot[g] = bins[((size_t)i * R + g) * 3 + 1];
    __syncthreads();
    block_exclusive_scan(tot, R, tot + R);
    for (int g = threadIdx.x; g < R; g += 256) bins[((size_t)i * R + g) * 3 + 0] = tot[g];
}

// The block's (key, b) pairs grouped by region: counted in LDS, placed in
// LDS in region order, then written so that consecutive threads write
// consecutive entries of a region's run.
// fused (small partitions, nblk x R <= kPartScanOneGroup): offs holds the
// raw counts of k_part_hist; the workgroup derives its offsets in every
// region and the regions' first entries from its scale's counts itself,
// and workgroup j = 0 of each scale writes the scale's bins and workgroup 0
// clears the spill flag (what k_part_scan_rows and k_part_base do for large
// partitions).
__global__ __launch_bounds__(256) void k_part_scatter(const uint64_t *__restrict__ keys,
                                                      int64_t nB, int log2cap, int64_t nblk,
                                                      const uint32_t *__restrict__ offs,
                                                      uint32_t *bins, uint3 *entries,
                                                      uint32_t *spilled, int fused) {
    extern __shared__ uint32_t sm[];
    const int R = (int)part_regions(log2cap);
    uint32_t *cnt = sm;               // [R] counts, then the block's region starts
    uint32_t *fill = sm + R;          // [R + 256] scan scratch, then positions per region
    auto *sk = reinterpret_cast<unsigned long long *>(sm + 2 * R + 256);  // [kPartBlock]
    int32_t *sb = reinterpret_cast<int32_t *>(sk + kPartBlock);                      // [kPartBlock]
    uint32_t *gbase = reinterpret_cast<uint32_t *>(sb + kPartBlock);  // [R] fused: first entry
    uint32_t *gtot = gbase + R;                                        // [R] fused: region totals
    __shared__ uint32_t total;
    const int64_t i = blockIdx.x / nblk, j = blockIdx.x - i * nblk;
    if (fused) {
        if (i == 0 && j == 0 && threadIdx.x == 0) *spilled = 0;  // read after the region builds
        for (int g = threadIdx.x; g < R; g += 256) {
            const CH_RO uint32_t *o = ro(offs) + (size_t)i * nblk * R + g;
            uint32_t before = 0, all = 0;
#pragma unroll 8
            for (int64_t b = 0; b < nblk; ++b) {
                const uint32_t c = o[b * R];
                before += b < j ? c : 0u;
                all += c;
            }
            gbase[g] = before;
            gtot[g] = all;
            if (j == 0) {
                bins[((size_t)i * R + g) * 3 + 1] = all;
                bins[((size_t)i * R + g) * 3 + 2] = 0;
            }
        }
        __syncthreads();
        block_exclusive_scan(gtot, R, fill);
        for (int g = threadIdx.x; g < R; g += 256) {
            gbase[g] += gtot[g];
            if (j == 0) bins[((size_t)i * R + g) * 3 + 0] = gtot[g];
        }
    }
    for (int g = threadIdx.x; g < R; g += 256) cnt[g] = 0;
    __syncthreads();
    constexpr int kPer = kPartBlock / 256;
    unsigned long long k[kPer];
    const CH_RO uint64_t *kr = ro(keys) + i * nB;
    // loads first (in bounds, unconditional: in flight together), then the
    // counts; keys past n_B become the empty key
#pragma unroll
    for (int t = 0; t < kPer; ++t) k[t] = kr[min(j * kPartBlock + t * 256 + threadIdx.x, nB - 1)];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        if (j * kPartBlock + t * 256 + threadIdx.x >= nB) k[t] = kEmptyKey;
        if (k[t] != kEmptyKey) atomicAdd(&cnt[key_region(k[t], log2cap)], 1u);
    }
    __syncthreads();
    const uint32_t tsum = block_exclusive_scan(cnt, R, fill);  // fill: scan scratch
    for (int g = threadIdx.x; g < R; g += 256) fill[g] = cnt[g];
    if (threadIdx.x == 0) total = tsum;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        if (k[t] == kEmptyKey) continue;
        const uint32_t pos = atomicAdd(&fill[key_region(k[t], log2cap)], 1u);
        sk[pos] = k[t];
        sb[pos] = (int32_t)(j * kPartBlock + t * 256 + threadIdx.x);
    }
    __syncthreads();
    const uint32_t n = total;
    const uint32_t *o = offs + (size_t)(i * nblk + j) * R;
    const uint32_t *bn = bins + (size_t)i * R * 3;
    for (uint32_t pos = threadIdx.x; pos < n; pos += 256) {
        const unsigned long long key = sk[pos];
        const uint32_t g = key_region(key, log2cap);
        const uint32_t first = fused ? gbase[g] : bn[g * 3] + o[g];
        const size_t dst = (size_t)i * nB + first + (pos - cnt[g]);
        entries[dst] = make_uint3((uint32_t)key, (uint32_t)(key >> 32), (uint32_t)sb[pos]);
    }
}

// One workgroup per (scale, region): the region's pairs into an LDS table of
// S slots (lowest b per key), then all S slots written to the table.  Pairs
// whose probe reaches the region's end are compacted to the front of the
// region's run of entries, counted in bins[.. + 2] and flagged in *spilled.
// Up to kRegionPrefetch pairs per
// thread are read before any is inserted (one round of loads).
constexpr int kRegionPrefetch = 8;

__global__ __launch_bounds__(256) void k_region_build(uint3 *entries, int64_t nB, int L,
                                                      int log2cap, Bucket *tables, uint32_t *bins,
                                                      uint32_t *spilled) {
    extern __shared__ unsigned long long tk[];  // [S] keys, then [S] values
    const int qb = region_bits(log2cap);
    const int S = 1 << qb;
    int32_t *tv = reinterpret_cast<int32_t *>(tk + S);
    __shared__ uint32_t nspill;
    const int64_t R = part_regions(log2cap);
    const int64_t i = blockIdx.x / R, g = blockIdx.x - i * R;
    const uint32_t start = bins[(i * R + g) * 3], count = bins[(i * R + g) * 3 + 1];
    for (int s = threadIdx.x; s < S; s += 256) {
        tk[s] = kEmptyKey;
        tv[s] = INT_MAX;
    }
    if (threadIdx.x == 0) nspill = 0;
    uint3 *run = entries + (size_t)i * nB + start;
    const int lane = threadIdx.x & 63;
    for (uint32_t base = 0; base < count; base += 256 * kRegionPrefetch) {
        uint3 e[kRegionPrefetch];
#pragma unroll
        for (int q = 0; q < kRegionPrefetch; ++q) {
            const uint32_t at = base + q * 256 + threadIdx.x;
            e[q] = at < count ? run[at] : make_uint3(0xffffffffu, 0xffffffffu, 0u);
        }
        __syncthreads();  // the table is initialised; every pair read before spills overwrite
#pragma unroll
        for (int q = 0; q < kRegionPrefetch; ++q) {
            const unsigned long long key = (unsigned long long)e[q].x |
                                           ((unsigned long long)e[q].y << 32);
            const bool valid = key != kEmptyKey;
            int b = (int)e[q].z;
            // the lowest lane's key: its lanes fold their b into it (a key
            // repeated across wavefronts at coarse scales goes in once per
            // wavefront); the others insert on their own
            const unsigned long long vm = __ballot(valid);
            const int first = vm ? __ffsll((long long)vm) - 1 : 0;  // wave-uniform
            const unsigned long long lk = lane_u64(key, first);
            const bool same = valid && key == lk;
            // the lowest b among the lanes holding the first valid lane's key
            const int mb = __ockl_wfred_min_i32(same ? b : INT_MAX);
            const bool leader = same && lane == first;
            if (leader) b = mb;
            if (!valid || (same && !leader)) continue;
            int s = (int)(home_slot(key, log2cap) & (uint64_t)(S - 1));
            bool done = false;
            for (; s < S; ++s) {
                unsigned long long cur = tk[s];
                if (cur == kEmptyKey) cur = atomicCAS(&tk[s], kEmptyKey, key);
                if (cur == kEmptyKey || cur == key) {
                    atomicMin(&tv[s], b);
                    done = true;
                    break;
                }
            }
            if (!done) {
                const uint32_t r = atomicAdd(&nspill, 1u);
                run[r] = make_uint3((uint32_t)key, (uint32_t)(key >> 32), (uint32_t)b);
            }
        }
        __syncthreads();
    }
    // an empty region skips the loop: the fingerprints below read slots that
    // other threads initialised
    __syncthreads();
    Bucket *out = tables + ((size_t)i << log2cap) + ((size_t)g << qb);
    uint8_t *ofp = table_fps(tables, L, log2cap, (int)i) + ((size_t)g << qb);
    for (int s = threadIdx.x; s < S; s += 256) {
        Bucket bk;
        bk.key = tk[s];
        bk.val = tv[s];
        bk.pad = 0;
        out[s] = bk;
    }
    for (int s4 = threadIdx.x; s4 < S / 4; s4 += 256) {
        uint32_t w = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned long long k = tk[4 * s4 + q];
            w |= (k == kEmptyKey ? 0u : key_fp(k, log2cap)) << (8 * q);
        }
        reinterpret_cast<uint32_t *>(ofp)[s4] = w;
    }
    if (threadIdx.x == 0) {
        bins[(i * R + g) * 3 + 2] = nspill;
        if (nspill) atomicOr(spilled, 1u);
    }
}

// The pairs the LDS builds kept aside, inserted with the global insert; a
// single flag word says whether there are any.
__global__ __launch_bounds__(256) void k_spill_insert(const uint32_t *__restrict__ bins,
                                                      const uint3 *__restrict__ entries,
                                                      int64_t nB, int L, int log2cap,
                                                      Bucket *tables, const uint32_t *spilled) {
    if (*spilled == 0) return;
    const int64_t R = part_regions(log2cap);
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < (int64_t)L * R; r += nw) {
        const uint32_t ns = bins[r * 3 + 2];
        if (ns == 0) continue;
        const int64_t i = r / R;
        const uint3 *run = entries + (size_t)i * nB + bins[r * 3];
        for (uint32_t e = lane; e < ns; e += 64) {
            const uint3 v = run[e];
            table_insert(tables + ((size_t)i << log2cap), table_fps(tables, L, log2cap, (int)i),
                         log2cap, (unsigned long long)v.x | ((unsigned long long)v.y << 32),
                         (int)v.z);
        }
    }
}

// Largest count table (blocks x regions) of one scale that each scatter
// workgroup reads and scans itself (10^5 points: 25 x 128); above it the
// two-launch scan (10^6 points, 245 x 1024: 88 us in one workgroup per
// scale, about 15 us in two launches).
constexpr int64_t kPartScanOneGroup = 16384;

hipError_t launch_part_build(const PartWork &w, int64_t nB, int L, int log2cap, Bucket *tables,
                             hipStream_t st) {
    if (nB <= 0 || L <= 0) return hipSuccess;
    if (!part_build_ok(log2cap)) return hipErrorInvalidValue;
    const int64_t R = part_regions(log2cap), nblk = part_blocks(nB);
    const int S = 1 << region_bits(log2cap);
    k_part_hist<<<(unsigned)(L * nblk), 256, (size_t)R * sizeof(uint32_t), st>>>(
        w.keys, nB, log2cap, nblk, w.offs);
    const bool fused = nblk * R <= kPartScanOneGroup;  // the scatter scans the counts itself
    if (!fused) {
        k_part_scan_rows<<<(unsigned)(L * ((R + 63) / 64)), 256, 0, st>>>(log2cap, nblk, w.offs,
                                                                         w.bins);
        k_part_base<<<(unsigned)L, 256, 0, st>>>(log2cap, w.bins, w.spilled);
    }
    const size_t lds_sc = (2 * (size_t)R + 256) * sizeof(uint32_t) + (size_t)kPartBlock * 12 +
                          (fused ? 2 * (size_t)R * sizeof(uint32_t) : 0);
    k_part_scatter<<<(unsigned)(L * nblk), 256, lds_sc, st>>>(
        w.keys, nB, log2cap, nblk, w.offs, w.bins, w.entries, w.spilled, fused ? 1 : 0);
    k_region_build<<<(unsigned)(L * R), 256, (size_t)S * 12, st>>>(w.entries, nB, L, log2cap,
                                                                   tables, w.bins, w.spilled);
    // a wavefront per (scale, region): most have nothing kept aside, and a
    // wavefront that walked several regions waited on each one's inserts
    k_spill_insert<<<(unsigned)((L * R + 3) / 4), 256, 0, st>>>(w.bins, w.entries, nB, L,
                                                                 log2cap, tables, w.spilled);
    return hipGetLastError();
}

// ---------------------------------------------------------------- batched
// Persistent grids over all jobs of a batch (see batch_loop).  A job's
// blocks are the blocks of its direct launches, so every job computes what
// chamfer_estimate computes for it alone.

constexpr unsigned kGridSetup = 512, kGridMinmax = 1024, kGridCalib = kBatchMax,
                   kGridHash = 2048;

__global__ __launch_bounds__(256) void kb_setup(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsSetup, [&](const Job &J, Blk b) {
        if (b.id < J.nb_init) {
            init_params(J.p, J.lohi, J.d, Blk{b.id, J.nb_init});
            return;
        }
        int64_t r = b.id - J.nb_init;
        if (r < J.nb_grid) {
            grid_tables(J.seed, J.L, J.kh, J.zfrac, J.mult, 0, Blk{r, J.nb_grid});
            return;
        }
        r -= J.nb_grid;
        table_fill(J.tables, (size_t)J.table_count, Blk{r, J.nb_fill});
    });
}

__global__ __launch_bounds__(256) void kb_minmax(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsMinmax, [&](const Job &J, Blk b) {
        const bool isA = b.id < J.nb_mmA;
        const float *X = isA ? J.A : J.B;
        const int64_t total = (isA ? J.nA : J.nB) * (int64_t)J.d;
        const int64_t stride = isA ? J.mm_strideA : J.mm_strideB;
        const Blk c = isA ? Blk{b.id, J.nb_mmA} : Blk{b.id - J.nb_mmA, J.nb_mmB};
        if (J.mm_vec4)
            minmax4(reinterpret_cast<const float4 *>(X), total / 4, J.d, stride, J.lohi, J.p, c);
        else
            minmax(X, total, J.d, stride, J.lohi, J.p, c);
    });
}

__global__ __launch_bounds__(256) void kb_calib(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsCalib, [&](const Job &J, Blk) { calib_final(J.lohi, J.d, J.p); });
}

template <int METRIC, int MODE, int KE, bool YG>
__global__ __launch_bounds__(kThreads) void kb_hash(const Batch *__restrict__ bt) {
    batch_loop(bt, MODE == 0 ? kBsInsert : kBsProbe, [&](const Job &J, Blk b) {
        if (MODE == 0)
            hash_tile<METRIC, 0, KE, YG>(J.B, J.nB, J.B, J.d, J.L, J.lohi, J.embed, J.zfrac,
                                         J.mult, J.tables, J.log2cap, nullptr, nullptr, nullptr,
                                         nullptr, J.nb2, J.p, J.nB, 1, 0, b);
        else
            hash_tile<METRIC, 1, KE, YG>(J.A, J.nA, J.B, J.d, J.L, J.lohi, J.embed, J.zfrac,
                                         J.mult, J.tables, J.log2cap, nullptr, J.D, J.nn,
                                         nullptr, nullptr, J.p, J.nB, 1, kProbeLast, b);
    });
}

hipError_t launch_batch_setup(const Batch *bt, hipStream_t st) {
    kb_setup<<<kGridSetup, 256, 0, st>>>(bt);
    return hipGetLastError();
}

hipError_t launch_batch_minmax(const Batch *bt, int d, hipStream_t st) {
    if (d > 2048) return hipErrorInvalidValue;
    kb_minmax<<<kGridMinmax, 256, 2 * (size_t)d * sizeof(uint32_t), st>>>(bt);
    return hipGetLastError();
}

hipError_t launch_batch_calib(const Batch *bt, int d, hipStream_t st) {
    if (d > 2048) return hipErrorInvalidValue;
    kb_calib<<<kGridCalib, 256, (size_t)d * sizeof(double), st>>>(bt);
    return hipGetLastError();
}

template <int METRIC, int KE, bool YG>
static hipError_t launch_batch_hash_t(int mode, const Batch *bt, int d, hipStream_t st) {
    const size_t lds = hash_lds<METRIC, KE, YG>(d);
    if (mode == 0)
        kb_hash<METRIC, 0, KE, YG><<<kGridHash, kThreads, lds, st>>>(bt);
    else
        kb_hash<METRIC, 1, KE, YG><<<kGridHash, kThreads, lds, st>>>(bt);
    return hipGetLastError();
}

hipError_t launch_batch_hash(int mode, const Batch *bt, int d, int metric, int ke,
                             hipStream_t st) {
    if (mode != 0 && mode != 1) return hipErrorInvalidValue;
    if (metric == CHAMFER_L1) {
        if (d <= kMaxLdsL1Dim) return launch_batch_hash_t<CHAMFER_L1, 0, false>(mode, bt, d, st);
        return launch_batch_hash_t<CHAMFER_L1, 0, true>(mode, bt, d, st);
    }
    switch (ke) {
        case 8: return launch_batch_hash_t<CHAMFER_L2, 8, false>(mode, bt, d, st);
        case 16: return launch_batch_hash_t<CHAMFER_L2, 16, false>(mode, bt, d, st);
        case 32: return launch_batch_hash_t<CHAMFER_L2, 32, false>(mode, bt, d, st);
        case 64: return launch_batch_hash_t<CHAMFER_L2, 64, false>(mode, bt, d, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace chamfer
