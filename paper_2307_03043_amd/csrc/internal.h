// Internal declarations of libchamfer: device helpers, the per-call device
// parameter block, the workspace layout and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "chamfer.h"

namespace chamfer {

constexpr uint32_t kPurposeGrid = 1;    // shifts z' and key multipliers M
constexpr uint32_t kPurposeEmbed = 2;   // Gaussian embedding matrix
constexpr uint32_t kPurposeSample = 3;  // importance-sampling draws
constexpr uint64_t kEmptyKey = ~0ull;   // bucket keys are < 2^63
constexpr int kMaxScales = 64;

// Device-resident parameters of one call; written by the kernels, read by
// later kernels of the same call (no host round trip).
struct DevParams {
    int32_t status;      // CHAMFER_OK / CHAMFER_ENONFINITE
    int32_t e_top;       // top grid scale exponent
    int32_t s;           // fixed-point exponent of the weights
    int32_t all_zero;    // every D_a == 0
    uint32_t max_d_bits; // bits of max_a D_a (D_a >= 0, so bits order as floats)
    uint32_t nonfinite;  // an input coordinate is NaN or Inf
    uint64_t W;          // fixed-point total
    double S;            // sum_k (hi_k - lo_k)
    uint32_t b2max_bits; // bits of max_b |b|^2 (float32, >= 0)
    uint32_t fallbacks;  // (query, chunk) pairs rescanned exactly by the MFMA pass
    uint64_t pad[2];
};

// One bucket of a scale's open-addressing table: key -> lowest b index.
struct alignas(16) Bucket {
    unsigned long long key;
    int32_t val;
    int32_t pad;
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint32_t float_to_ordered(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ordered_to_float(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011): key (k0, k1),
// counter c[0..3]; returns the four output words in c.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull, kMul1 = 0xCA5A826395121157ull;
    constexpr uint64_t kBump0 = 0x9E3779B97F4A7C15ull, kBump1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t h0 = __umul64hi(kMul0, c[0]), l0 = kMul0 * c[0];
        const uint64_t h1 = __umul64hi(kMul1, c[2]), l1 = kMul1 * c[2];
        const uint64_t x0 = h1 ^ c[1] ^ k0, x2 = h0 ^ c[3] ^ k1;
        c[0] = x0;
        c[1] = l1;
        c[2] = x2;
        c[3] = l0;
        k0 += kBump0;
        k1 += kBump1;
    }
}

// Canonical float32 distance accumulator between rows a and b: k ascending,
// one rounding per operation; l1: acc + |a_k - b_k|, l2: fma(t, t, acc) with
// t = a_k - b_k (the caller takes the square root for l2).  Loads are issued
// in batches of 8 x 16 bytes ahead of the (sequential) arithmetic, so a row
// costs a few memory round trips instead of one per 16 bytes.
template <int METRIC>
__device__ __forceinline__ float canon_acc(const float *__restrict__ a,
                                           const float *__restrict__ b, int d) {
    float acc = 0.0f;
    auto step = [&](float x, float y) {
        const float t = x - y;
        acc = METRIC == CHAMFER_L1 ? acc + fabsf(t) : fmaf(t, t, acc);
    };
    if ((d & 3) == 0 &&
        ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0) {
        const float4 *a4 = reinterpret_cast<const float4 *>(a);
        const float4 *b4 = reinterpret_cast<const float4 *>(b);
        const int d4 = d >> 2;
        constexpr int kBatch = 8;
        for (int k0 = 0; k0 < d4; k0 += kBatch) {
            float4 u[kBatch], v[kBatch];
#pragma unroll
            for (int i = 0; i < kBatch; ++i)
                if (k0 + i < d4) {
                    u[i] = a4[k0 + i];
                    v[i] = b4[k0 + i];
                }
#pragma unroll
            for (int i = 0; i < kBatch; ++i)
                if (k0 + i < d4) {
                    step(u[i].x, v[i].x);
                    step(u[i].y, v[i].y);
                    step(u[i].z, v[i].z);
                    step(u[i].w, v[i].w);
                }
        }
        return acc;
    }
    constexpr int kBatch = 16;
    for (int k0 = 0; k0 < d; k0 += kBatch) {
        float u[kBatch], v[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            if (k0 + i < d) {
                u[i] = a[k0 + i];
                v[i] = b[k0 + i];
            }
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            if (k0 + i < d) step(u[i], v[i]);
    }
    return acc;
}

// smallest e with 2^e >= x (x > 0)
__device__ __forceinline__ int ceil_log2_pos(double x) {
    int e;
    const double m = frexp(x, &e);
    return m == 0.5 ? e - 1 : e;
}

// ------------------------------------------------------------ workspace

struct Plan {
    // problem
    int64_t nA, nB, T;
    int32_t d, metric, L, ke, kh, q, precision;
    uint64_t seed;
    int log2cap;  // per-scale table capacity is 2^log2cap
    // byte offsets into the workspace
    size_t off_params, off_lohi, off_zfrac, off_mult, off_embed, off_tables, off_D,
        off_nn, off_scale, off_blocksums, off_P, off_idx, off_best, off_partial, off_nb2, off_fallback,
        off_bq, off_xq, off_lpf, total;
};

// Row block of the fixed-point scan: 256 threads x 4 items.
constexpr int kScanItems = 4;
constexpr int kScanThreads = 256;
constexpr int kScanBlock = kScanItems * kScanThreads;

// --------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipGetLastError().

hipError_t launch_init_params(DevParams *p, uint32_t *lohi, int d, hipStream_t st);
hipError_t launch_grid_tables(uint64_t seed, int L, int kh, float *zfrac, uint64_t *mult,
                              hipStream_t st);
hipError_t launch_minmax(const float *X, int64_t n, int d, uint32_t *lohi, DevParams *p,
                         hipStream_t st);
hipError_t launch_calib_final(uint32_t *lohi, int d, DevParams *p, hipStream_t st);
hipError_t launch_table_fill(Bucket *tables, size_t count, hipStream_t st);
// mode 0: insert B into the tables (l2: also |b|^2 into nb2_out and
// p->b2max_bits when nb2_out is set); 1: probe A (CrudeNN); 2: write keys
hipError_t launch_hash(int mode, const float *X, int64_t n, const float *Bpts, int64_t nB,
                       int d, int metric, int L, int ke, const uint32_t *lohi,
                       const float *embed_t, const float *zfrac, const uint64_t *mult,
                       Bucket *tables, int log2cap, uint64_t *keys_out, float *D_out,
                       int32_t *nn_out, int32_t *scale_out, float *nb2_out, DevParams *p,
                       hipStream_t st);
hipError_t launch_weights(const float *D, int64_t nA, int q, uint64_t *blocksums, uint64_t *P,
                          DevParams *p, hipStream_t st);
hipError_t launch_sample(uint64_t seed, const uint64_t *P, int64_t nA, int64_t T, int32_t *idx,
                         unsigned long long *best, DevParams *p, hipStream_t st);
hipError_t launch_estimate_final(const unsigned long long *best, const int32_t *idx,
                                 const float *D, int64_t T, int metric, DevParams *p,
                                 double *eta_out, chamfer_aux aux, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                           hipStream_t st);
// Exact nearest neighbours; nb2 (float [nB], or nullptr) selects the l2 MFMA
// form, which needs launch_rownorm to have filled nb2 and p->b2max_bits.
hipError_t launch_nnmin(const float *X, const int32_t *rows, int64_t nx, const float *B,
                        int64_t nB, int d, int metric, unsigned long long *best,
                        const float *nb2, DevParams *p, hipStream_t st);
hipError_t launch_rownorm(const float *B, int64_t nB, int d, float *nb2, DevParams *p,
                          hipStream_t st);
bool mfma_supported(int d, int metric);
hipError_t launch_nnmin_mfma(const float *X, const int32_t *rows, int64_t nx, const float *B,
                             int64_t nB, int d, unsigned long long *best, const float *nb2,
                             DevParams *p, hipStream_t st);
// Low-precision (BF16 / FP8-E4M3) l2 nearest neighbours with float32 re-rank.
int lowp_dpad(int d, int precision);
bool lowp_supported(int d, int metric, int precision);
size_t lowp_row_bytes(int d, int precision);
hipError_t launch_cast_rows(int precision, const float *X, const int32_t *rows, int64_t n, int d,
                            uint8_t *out, float *scale, float *n2, const DevParams *p,
                            hipStream_t st);
hipError_t launch_nnmin_lowp(int precision, const uint8_t *Xq, const float *xsc, int64_t nx,
                             const float *X, const int32_t *rows, const uint8_t *Bq,
                             const float *bsc, const float *bn2, const float *B, int64_t nB,
                             int d, unsigned long long *best, const DevParams *p,
                             hipStream_t st);
hipError_t launch_nn_finalize(const unsigned long long *best, int64_t nx, int metric,
                              float *min_out, int32_t *arg_out, double *partial,
                              const DevParams *p, hipStream_t st);
hipError_t launch_sum_final(const double *partial, int64_t nparts, const DevParams *p,
                            double *out, hipStream_t st);
hipError_t launch_copy_status(const DevParams *p, int32_t *status_out, hipStream_t st);
int nn_finalize_blocks(int64_t nx);

}  // namespace chamfer
