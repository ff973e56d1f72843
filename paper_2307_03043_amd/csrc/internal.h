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
constexpr uint32_t kPurposeSketch = 4;  // p-stable direction of the reduction
constexpr uint32_t kPurposePart = 5;    // shifts and multipliers of the partition grid
constexpr uint32_t kPurposePad = 6;     // signs of the padding coordinates
constexpr uint64_t kEmptyKey = ~0ull;   // bucket keys are < 2^63
constexpr int kMaxScales = 64;
// The per-coordinate min/max is accumulated in kLohiReps copies (workgroup
// id mod kLohiReps picks one) so that the global atomics of many workgroups
// do not queue on the same 2d words; the calibration folds the copies into
// the first, [lo(d) | hi(d)], which every later kernel reads.
constexpr int kLohiReps = 8;
inline size_t lohi_bytes(int d) { return (size_t)kLohiReps * 2 * (size_t)d * sizeof(uint32_t); }
constexpr int kMaxWindow = 32;          // W of the multi-probe CrudeNN
constexpr int kMaxReps = 64;            // k of the multi-probe CrudeNN
// flags of the probe launches of the multi-probe CrudeNN
constexpr int kProbeMerge = 1;  // keep the better of this and the previous structure's result
constexpr int kProbeLast = 2;   // last structure: also reduce max D_a

constexpr int kMaxRepl = 64;     // replicas of the per-workgroup maxima (one per lane)
constexpr int kReplStride = 32;  // uint32 words between replicas: one 128-byte line each

// Device-resident parameters of one call; written by the kernels, read by
// later kernels of the same call (no host round trip).
struct DevParams {
    int32_t status;      // CHAMFER_OK / CHAMFER_ENONFINITE
    int32_t e_top;       // top grid scale exponent
    int32_t s;           // fixed-point exponent of the weights
    int32_t all_zero;    // every D_a == 0
    uint32_t nonfinite;  // an input coordinate is NaN or Inf
    uint64_t W;          // fixed-point total
    double S;            // sum_k (hi_k - lo_k)
    uint32_t fallbacks;  // (query, chunk) pairs rescanned exactly by the MFMA pass
    uint32_t nredo;      // (query, chunk) pairs listed for the deferred pass's rescan
    uint32_t pad32[2];
    uint64_t pad[1];
    // The maxima of D_a and |b|^2 reduced over thousands of workgroups: each
    // workgroup's atomicMax goes to replica (id mod kMaxRepl), one 128-byte
    // line each, since atomics queued on one address serialise at its cache
    // channel; readers take the max over the replicas (rep_fold).
    uint32_t max_d_rep[kMaxRepl * kReplStride];
    uint32_t b2max_rep[kMaxRepl * kReplStride];
};

__device__ __forceinline__ void rep_max(uint32_t *rep, int64_t id, uint32_t m) {
    atomicMax(&rep[(id % kMaxRepl) * kReplStride], m);
}

// Max over the replicas (unsigned: the bits of non-negative floats order as
// the floats); a whole wavefront calls it, lane r reading replica r.
__device__ __forceinline__ uint32_t rep_fold(const uint32_t *rep) {
    uint32_t m = rep[(threadIdx.x & 63) * kReplStride];
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    return m;
}

// Lane l's 64-bit value in every lane (l wave-uniform; a scalar register
// read, no LDS round trip).
__device__ __forceinline__ unsigned long long lane_u64(unsigned long long v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

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
    int32_t d, metric, L, ke, kh, q, precision, window, reps, sampling;
    uint64_t seed;
    int log2cap;  // per-scale table capacity is 2^log2cap
    bool part;    // B's tables come from the partitioned build (W = 1)
    // byte offsets into the workspace
    size_t off_params, off_lohi, off_zfrac, off_mult, off_embed, off_tables, off_D,
        off_nn, off_scale, off_blocksums, off_P, off_idx, off_best, off_partial, off_nb2, off_bsplit, off_xsplit, off_xn2, off_srec, off_part,
        off_bq, off_xq, off_lpf, total;
};

// Row block of the fixed-point scan: 256 threads x 4 items.
constexpr int kScanItems = 4;
constexpr int kScanThreads = 256;
constexpr int kScanBlock = kScanItems * kScanThreads;

// ------------------------------------------------------- block coordinates
// Every stage kernel is a device body over workgroup coordinates (id, n): a
// direct launch runs it with (blockIdx.x, gridDim.x); a batched launch runs
// the blocks of every request of a batch with request-local coordinates.
struct Blk {
    int64_t id, n;
};
__device__ __forceinline__ Blk grid_blk() { return Blk{(int64_t)blockIdx.x, (int64_t)gridDim.x}; }

// Work order of the exact passes (nq query blocks x nchunk chunks of B):
// workgroup ids are dealt to the 8 XCDs round-robin, so id runs on XCD
// id % 8 as its (id / 8)-th workgroup.  With nchunk a multiple of 8, XCD x
// takes the chunks cb = 8c + x in turn and, for each, all its query blocks
// one after the other: the workgroups of one chunk run on one XCD at about
// the same time and read the chunk through that XCD's L2 once.  Otherwise
// the chunk varies fastest.
__device__ __forceinline__ void chunk_major(int64_t id, int64_t nq, int nchunk, int &cb,
                                            int64_t &qb) {
    if ((nchunk & 7) == 0) {
        const int64_t s = id >> 3;
        cb = (int)((s / nq) * 8 + (id & 7));
        qb = s % nq;
    } else {
        cb = (int)(id % nchunk);
        qb = id / nchunk;
    }
}

// ---------------------------------------------------------------- batches
// One request of a batched estimate: its inputs, workspace regions, output
// slots and the block counts of each of its launches (the same counts its
// direct launch would use).
struct Job {
    const float *A, *B;
    int64_t nA, nB, T;
    uint64_t seed;
    int32_t d, metric, L, ke, kh, q, log2cap, precision;
    DevParams *p;
    uint32_t *lohi;
    float *zfrac;
    uint64_t *mult;
    const int8_t *embed;
    Bucket *tables;
    int64_t table_count;
    float *D;
    int32_t *nn;
    unsigned long long *blocksums, *P;  // block totals (then offsets); in-block prefixes
    int32_t *idx;
    unsigned long long *best;
    float *nb2;
    uint8_t *bq, *xq;  // low precision: cast B and draws; float32 l2: B's split table at bq
    float *lpf;
    uint16_t *xsplit;  // float32 l2: the draws' split table and |x|^2
    float *xn2;
    double *eta;
    chamfer_aux aux;
    // geometry
    int32_t nb_init, nb_grid, nb_fill;
    int32_t nb_mmA, nb_mmB, mm_vec4;
    int64_t mm_strideA, mm_strideB;
    int32_t nb_hashB, nb_hashA, nb_scan, nb_sample;
    int32_t nb_castB, nb_castX, nn_nchunk, nb_nn;
    int64_t nn_chunk;
};

// Stages of a batched estimate, one launch each.
enum BatchStage {
    kBsSetup,   // parameter block, shifts and multipliers, empty tables
    kBsMinmax,  // per-coordinate min/max of A and of B
    kBsCalib,   // S and e_top
    kBsInsert,  // B into the tables
    kBsProbe,   // CrudeNN of A
    kBsWsum,    // fixed-point weights: block sums
    kBsWscan,   // scan of the block sums, W and s
    kBsSample,  // T draws
    kBsCast,    // low-precision copies of B and of the sampled rows, or B's split table
    kBsNN,      // exact nearest neighbours of the samples
    kBsFinal,   // eta and the per-request outputs
    kBsCount
};

constexpr int kBatchMax = 256;

struct alignas(16) Batch {
    int32_t njobs;
    int32_t pad[3];
    int32_t start[kBsCount][kBatchMax + 1];  // prefix of the jobs' block counts
    Job job[kBatchMax];
};

// Pointers read from a batch descriptor are generic to the compiler (flat
// loads and stores).  glb() states that one points to global memory, so the
// accesses compile as they do from a kernel argument; ro() also states that
// the memory is not written while the kernel runs, so loads at wave-uniform
// addresses go through the scalar cache (which every dispatch invalidates
// at its start).
template <class T>
__device__ __forceinline__ T *glb(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)p;
}
#define CH_RO __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const CH_RO T *ro(const T *p) {
    return (const CH_RO T *)p;
}
// 16-byte loads through such a pointer (HIP's vector classes cannot be
// copied out of another address space).
__device__ __forceinline__ float4 ld(const CH_RO float4 *p) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *reinterpret_cast<const CH_RO v4 *>(p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 ld(const CH_RO uint4 *p) {
    typedef unsigned v4 __attribute__((ext_vector_type(4)));
    const v4 v = *reinterpret_cast<const CH_RO v4 *>(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Padded dimension of the split tables of the l2 exact pass (12 <= d <= 256).
__host__ __device__ inline int split_dpad(int d) {
    return d <= 32 ? 32 : d <= 64 ? 64 : d <= 128 ? 128 : 256;
}

// BF16 bits of f, round to nearest even (f finite or infinite).
__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// The two-term split of the l2 exact pass: (h, m) of v as BF16 bit patterns,
// h = bf16(v), m = bf16(v - h) (v - h is exact in float32).
__device__ __forceinline__ void split2(float v, uint32_t &h, uint32_t &m) {
    h = bf16_rne_bits(v);
    m = bf16_rne_bits(v - __uint_as_float(h << 16));
}

// Canonical float32 distance accumulator between rows a and b: k ascending,
// one rounding per operation; l1: acc + |a_k - b_k|, l2: fma(t, t, acc) with
// t = a_k - b_k (the caller takes the square root for l2).  Loads are issued
// in batches of BATCH x 16 bytes ahead of the (sequential) arithmetic, so a
// row costs a few memory round trips instead of one per 16 bytes (kernels
// with registers to spare take BATCH = 16: two round trips at d = 128).
// Both rows must be read-only for the kernel that calls it (they are read
// through the constant address space).
template <int METRIC, int BATCH = 8>
__device__ __forceinline__ float canon_acc(const float *__restrict__ a,
                                           const float *__restrict__ b, int d) {
    float acc = 0.0f;
    auto step = [&](float x, float y) {
        const float t = x - y;
        acc = METRIC == CHAMFER_L1 ? acc + fabsf(t) : fmaf(t, t, acc);
    };
    if ((d & 3) == 0 &&
        ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0) {
        const auto *a4 = reinterpret_cast<const CH_RO float4 *>(ro(a));
        const auto *b4 = reinterpret_cast<const CH_RO float4 *>(ro(b));
        const int d4 = d >> 2;
        constexpr int kBatch = BATCH;
        int k0 = 0;
        for (; k0 + kBatch <= d4; k0 += kBatch) {  // whole batches: no guards
            float4 u[kBatch], v[kBatch];
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                u[i] = ld(a4 + k0 + i);
                v[i] = ld(b4 + k0 + i);
            }
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                step(u[i].x, v[i].x);
                step(u[i].y, v[i].y);
                step(u[i].z, v[i].z);
                step(u[i].w, v[i].w);
            }
        }
        if (k0 < d4) {  // the last, partial batch: loads clamped in bounds
            float4 u[kBatch], v[kBatch];
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                u[i] = ld(a4 + min(k0 + i, d4 - 1));
                v[i] = ld(b4 + min(k0 + i, d4 - 1));
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
                u[i] = ro(a)[k0 + i];
                v[i] = ro(b)[k0 + i];
            }
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            if (k0 + i < d) step(u[i], v[i]);
    }
    return acc;
}

// Persistent loop of a batched stage: workgroup g takes the batch's blocks
// g, g + gridDim.x, ... of the stage (jobs in order, each job's blocks
// consecutive) and runs body(job, request-local coordinates).  The bodies
// have no barrier after a wave-dependent return, so the barrier that closes
// each iteration is reached by every wavefront.
template <class Body>
__device__ __forceinline__ void batch_loop(const Batch *__restrict__ bt, int stage, Body &&body) {
    __shared__ int32_t st[kBatchMax + 1];
    const int nj = bt->njobs;
    for (int i = threadIdx.x; i <= nj; i += blockDim.x) st[i] = bt->start[stage][i];
    __syncthreads();
    const int total = st[nj];
    int j = 0;
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        while (st[j + 1] <= v) ++j;
        j = __builtin_amdgcn_readfirstlane(j);
        body(bt->job[j], Blk{(int64_t)(v - st[j]), (int64_t)(st[j + 1] - st[j])});
        __syncthreads();
    }
}

// --------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipGetLastError().

hipError_t launch_init_params(DevParams *p, uint32_t *lohi, int d, hipStream_t st);
// init_params, the rep-0 grid tables and (tables non-null) the empty W = 1
// tables of `count` buckets, in one launch
hipError_t launch_setup(DevParams *p, uint32_t *lohi, int d, uint64_t seed, int L, int kh,
                        float *zfrac, uint64_t *mult, Bucket *tables, size_t count,
                        hipStream_t st);
// rep: index of the independent LSH structure (0 for the single one)
hipError_t launch_grid_tables(uint64_t seed, int L, int kh, float *zfrac, uint64_t *mult,
                              int rep, hipStream_t st);
hipError_t launch_minmax(const float *X, int64_t n, int d, uint32_t *lohi, DevParams *p,
                         hipStream_t st);
// The same over A and then B in one launch (two launches when either set
// is not 16-byte aligned with d a multiple of 4).
hipError_t launch_minmax_pair(const float *A, int64_t nA, const float *B, int64_t nB, int d,
                              uint32_t *lohi, DevParams *p, hipStream_t st);
hipError_t launch_calib_final(uint32_t *lohi, int d, DevParams *p, hipStream_t st);
hipError_t launch_table_fill(Bucket *tables, size_t count, hipStream_t st);
// mode 0: insert B into the tables (l2: also |b|^2 into nb2_out and
// p->b2max_rep when nb2_out is set); 1: probe A (CrudeNN); 2: write keys;
// 5: write B's keys for launch_part_build (duplicates within a wavefront
// dropped; |b|^2 as mode 0);
// 3 / 4: insert / probe with a window of W points per bucket (the tables
// are then keys [L][cap] followed by members [L][cap][W]).  flags: kProbe*.
hipError_t launch_hash(int mode, const float *X, int64_t n, const float *Bpts, int64_t nB,
                       int d, int metric, int L, int ke, const uint32_t *lohi,
                       const int8_t *embed, const float *zfrac, const uint64_t *mult,
                       Bucket *tables, int log2cap, uint64_t *keys_out, float *D_out,
                       int32_t *nn_out, int32_t *scale_out, float *nb2_out, DevParams *p,
                       int W, int flags, hipStream_t st, uint16_t *split_out = nullptr,
                       int split_dp = 0);
// Bytes of the tables of L scales of 2^log2cap buckets with window W.
size_t table_bytes(int L, int log2cap, int W);
// The partitioned build of the W = 1 tables (no global atomics): keys of B
// from launch_hash mode 5 into w.keys, then launch_part_build.  Usable when
// part_build_ok(log2cap) (at most 4096 regions of 4096 slots per scale).
struct PartWork {
    uint64_t *keys;    // [L][nB] (the empty key for a dropped duplicate)
    uint32_t *offs;    // [L][blocks][regions]
    uint32_t *bins;    // [L][regions][3]: first entry, count, spilled
    uint3 *entries;    // [L][nB] (key lo, key hi, b) grouped by region
    uint32_t *spilled; // [1] some region kept pairs aside for the global insert
};
bool part_build_ok(int log2cap);
// Workspace bytes of the build; with w, also lays the regions out from base.
size_t part_work_bytes(int L, int64_t nB, int log2cap, PartWork *w = nullptr,
                       char *base = nullptr);
hipError_t launch_part_build(const PartWork &w, int64_t nB, int L, int log2cap, Bucket *tables,
                             hipStream_t st);
// Empty tables (window W).
hipError_t launch_tables_empty(Bucket *tables, int L, int log2cap, int W, hipStream_t st);
// Weights: per-block totals into blocksums (scanned in place to the blocks'
// offsets) and each point's in-block inclusive prefix into Ploc [n_A].
hipError_t launch_weights(const float *D, int64_t nA, int q, uint64_t *blocksums, uint64_t *Ploc,
                          DevParams *p, hipStream_t st);
// Draws from P_a = offs[a / kScanBlock] + Ploc_a (launch_weights' outputs;
// q as for launch_weights).
hipError_t launch_sample(uint64_t seed, const uint64_t *Ploc, const uint64_t *offs, int64_t nA,
                         int64_t T, int q, int32_t *idx, unsigned long long *best, DevParams *p,
                         hipStream_t st);
hipError_t launch_estimate_final(const unsigned long long *best, const int32_t *idx,
                                 const float *D, int64_t T, int metric, DevParams *p,
                                 double *eta_out, chamfer_aux aux, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                           hipStream_t st);
// Exact nearest neighbours on the vector ALU (l1, and l2 outside the
// matrix-core dimensions).
hipError_t launch_nnmin(const float *X, const int32_t *rows, int64_t nx, const float *B,
                        int64_t nB, int d, int metric, unsigned long long *best, DevParams *p,
                        hipStream_t st);
// The l2 exact pass on the BF16 matrix cores (12 <= d <= 256) with a two-term
// split of every coordinate: launch_rownorm (or the hash of B) fills nb2 and
// p->b2max_rep, launch_split_rows (or the hash of B) the split table of B
// (split_table_bytes), then launch_nnmin_split returns the canonical float32
// minima.
bool mfma_supported(int d, int metric);
hipError_t launch_rownorm(const float *B, int64_t nB, int d, float *nb2, DevParams *p,
                          hipStream_t st);
size_t split_table_bytes(int64_t nB, int d);
int64_t split_blocks(int64_t nB, int d);
hipError_t launch_split_rows(const float *B, int64_t nB, int d, uint16_t *out,
                             const DevParams *p, hipStream_t st);
// The queries' split table (rows X[rows[i]], i < nx) and their |x|^2.
hipError_t launch_split_queries(const float *X, const int32_t *rows, int64_t nx, int d,
                                uint16_t *out, float *n2, const DevParams *p, hipStream_t st);
// Xs, xn2: the queries' split table and norms (launch_split_queries).
// rec (may be null): split_record_bytes(nx, nB, d) bytes for the deferred
// form of launches over fewer than 16384 queries (the pass records its
// chunk candidates, a second kernel certifies them per query and lists the
// chunks to rescan, a third rescans them); null, or a launch over more
// queries, certifies inside the pass.
size_t split_record_bytes(int64_t nx, int64_t nB, int d);
hipError_t launch_nnmin_split(const float *X, const int32_t *rows, int64_t nx, const uint16_t *Xs,
                              const float *xn2, const float *B, const uint16_t *Bs, int64_t nB,
                              int d, unsigned long long *best, const float *nb2, DevParams *p,
                              hipStream_t st, uint4 *rec = nullptr);
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
// Uniform sampling: D_a = 1 for every a (nn, scale = -1 when given) and
// max D_a = 1.
hipError_t launch_unit_weights(float *D, int32_t *nn, int32_t *scale, int64_t nA, DevParams *p,
                               hipStream_t st);
int nn_finalize_blocks(int64_t nx);

// ------------------------------------------------------------ geometry
// Block counts of the direct launches, shared with the batched ones.
int64_t init_blocks(int d);
int64_t grid_table_blocks(int L, int kh);
int64_t table_fill_blocks(size_t count);
// minmax over n rows: float4 form when vec4; stride in elements (or float4)
void minmax_geom(int64_t n, int d, bool vec4, int64_t *blocks, int64_t *stride);
bool minmax_vec4(const float *X, int d);
int64_t hash_blocks(int64_t n);
int64_t scan_blocks(int64_t nA);
int64_t sample_blocks(int64_t T);
int64_t cast_blocks(int64_t n);
struct NNGeom {
    int64_t blocks, chunk;
    int32_t nchunk;
};
// target: workgroups the split of B aims for (0: the direct-launch target)
NNGeom valu_geom(int64_t nx, int64_t nB, int d, int64_t target = 0);
NNGeom split_geom(int64_t nx, int64_t nB, int d, int64_t target = 0);
int64_t split_target_wgs(int d);  // the direct-launch target of split_geom
constexpr int64_t kValuTargetWGs = 4096;
NNGeom lowp_geom(int64_t nx, int64_t nB, int d, int precision);
constexpr int kMaxLdsL1Dim = 240;  // widest l1 tile staged in LDS by the hash

// --------------------------------------------------------- batched launches
// Each launches one persistent grid over every job of *bt (device memory);
// d, metric, ke and precision are the same for every job of the batch.
hipError_t launch_batch_setup(const Batch *bt, hipStream_t st);
hipError_t launch_batch_minmax(const Batch *bt, int d, hipStream_t st);
hipError_t launch_batch_calib(const Batch *bt, int d, hipStream_t st);
hipError_t launch_batch_hash(int mode, const Batch *bt, int d, int metric, int ke,
                             hipStream_t st);
hipError_t launch_batch_weights(const Batch *bt, hipStream_t st);
hipError_t launch_batch_sample(const Batch *bt, hipStream_t st);
hipError_t launch_batch_cast(const Batch *bt, int d, int precision, hipStream_t st);
hipError_t launch_batch_nn(const Batch *bt, int d, int metric, int precision, hipStream_t st);
hipError_t launch_batch_split_rows(const Batch *bt, hipStream_t st);
hipError_t launch_batch_split(const Batch *bt, int d, hipStream_t st);
hipError_t launch_batch_lowp(const Batch *bt, int d, int precision, hipStream_t st);
hipError_t launch_batch_final(const Batch *bt, int metric, hipStream_t st);

// Host side of batching (api.hip): validate a request and fill its job with
// the layout of chamfer_estimate in workspace ws; for l2, embed_host
// receives the packed embedding (embedding_packed, embed_bytes(d, ke)) that
// the caller must place at embed_dev before the batch runs.
int job_prepare(const float *A, const float *B, int64_t nA, int64_t nB, int32_t d,
                int32_t metric, double eps, int64_t T, uint64_t seed, const chamfer_opts *opts,
                void *ws, size_t ws_bytes, double *eta, chamfer_aux aux, const int8_t *embed_dev,
                int8_t *embed_host, Job *job);
// Block counts of every stage of a job.
void job_stage_blocks(const Job &job, int64_t out[kBsCount]);

// Host Philox4x64-10 (counter c, key (k0, k1); output in c), the quantised
// l2 -> l1 embedding matrix ([ke][d] int8) and its packed operand layout for
// the hash kernels (embed_bytes(d, ke) bytes).
void philox_host(uint64_t c[4], uint64_t k0, uint64_t k1);
void embedding_host(uint64_t seed, int d, int ke, int8_t *Z);
size_t embed_bytes(int d, int ke);
void embedding_packed(uint64_t seed, int d, int ke, int8_t *out);

// chamfer_estimate / chamfer_workspace_bytes with opts->reduction set.
size_t reduced_workspace_bytes(int64_t n_A, int64_t n_B, int32_t d, int32_t metric, double eps,
                               int64_t T, const chamfer_opts *opts);
int estimate_reduced(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                     int32_t metric, double eps, int64_t T, uint64_t seed, double *eta_out,
                     chamfer_aux *aux, const chamfer_opts *opts, void *ws, size_t ws_bytes,
                     void *stream);
// Re-split B for the exact pass of a job in a batch: the exact float32
// passes give the exact nearest neighbour for any split, so a batch shares
// one workgroup target among its jobs in proportion to their work instead
// of every job splitting B finely enough to fill the device alone.  The
// low-precision pass keeps the direct split (its candidates depend on it).
void job_share_nn(Job *jobs, int n);
// The launch sequence of a batched estimate (what a captured graph holds).
int launch_estimate_batch(const Batch *bt, int d, int metric, int ke, int precision,
                          hipStream_t st);

}  // namespace chamfer
