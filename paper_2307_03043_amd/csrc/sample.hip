// Importance sampling (the Chamfer-Estimate figure, steps 1-4) on the GPU:
// fixed-point weights w_a = ceil(D_a 2^s), their inclusive prefix P (kept
// as block offsets plus in-block prefixes) and total W (two-level scan),
// T i.i.d. draws u ~ U[0, W) by Lemire's bounded integers on Philox4x64-10
// with the sample index min{a : P_a > u}, and the final reweighted mean
// eta = (1/T) sum_l (W / w_{x_l}) m_l in double.
//
// Everything is integer arithmetic except the final sum, which is a fixed
// order tree in double: results do not depend on scheduling.
#include <cmath>

#include "internal.h"

namespace chamfer {

__device__ __forceinline__ unsigned long long weight_of(float D, int s) {
    return (unsigned long long)ceil(ldexp((double)D, s));
}

// s = 47 - q - e_max with max D in [2^(e_max - 1), 2^e_max).
__device__ __forceinline__ int fixed_point_exponent(uint32_t max_d_bits, int q) {
    int e;
    frexp((double)__uint_as_float(max_d_bits), &e);
    return 47 - q - e;
}

// Blocks (of kScanBlock points) whose offsets the sampler holds in LDS:
// up to n_A = 4 Mi points.
constexpr int64_t kOffsLds = 4096;

// Block-wide inclusive scan of one uint64 per thread: a shuffle scan in each
// wavefront, then each wavefront adds the totals of the wavefronts before it
// (integer sums: the same values as any other order).  buf holds NT / 64
// totals.
template <int NT>
__device__ unsigned long long block_inclusive_scan(unsigned long long v,
                                                   unsigned long long *buf) {
    static_assert(NT % 64 == 0 && NT <= 1024, "whole wavefronts");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, off);
        const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), off);
        if (lane >= off) v += ((unsigned long long)hi << 32) | lo;
    }
    if (lane == 63) buf[wv] = v;
    __syncthreads();
    for (int w = 0; w < wv; ++w) v += buf[w];
    __syncthreads();
    return v;
}

// Block b.id of kScanBlock points: each point's weight w_a and its
// inclusive prefix within the block (Ploc, uint64), and the block's total
// (blocksums[b.id]).  After the scan of the totals, P_a = blocksums[a /
// kScanBlock] + Ploc_a.
__device__ __forceinline__ void weight_blocksum(const float *__restrict__ D, int64_t nA, int q,
                                                unsigned long long *blocksums,
                                                unsigned long long *Ploc, const DevParams *p,
                                                Blk b) {
    __shared__ unsigned long long buf[kScanThreads / 64];
    if (p->status != CHAMFER_OK) return;
    const uint32_t mb = rep_fold(p->max_d_rep);
    const bool pos = __uint_as_float(mb) > 0.0f;  // else every weight is 0
    const int s = pos ? fixed_point_exponent(mb, q) : 0;
    const int64_t base = b.id * kScanBlock + threadIdx.x * kScanItems;
    unsigned long long w[kScanItems];
    unsigned long long own = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        w[j] = (pos && base + j < nA) ? weight_of(ro(D)[base + j], s) : 0ull;
        own += w[j];
    }
    const unsigned long long inc = block_inclusive_scan<kScanThreads>(own, buf);
    unsigned long long run = inc - own;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        run += w[j];
        if (base + j < nA) Ploc[base + j] = run;
    }
    if (threadIdx.x == kScanThreads - 1) blocksums[b.id] = inc;
}

__global__ __launch_bounds__(kScanThreads) void k_weight_blocksum(
    const float *__restrict__ D, int64_t nA, int q, unsigned long long *blocksums,
    unsigned long long *Ploc, const DevParams *p) {
    weight_blocksum(D, nA, q, blocksums, Ploc, p, grid_blk());
}

// Exclusive scan of the block sums in place; W = total.  One block of 1024.
__device__ __forceinline__ void scan_blocksums(unsigned long long *blocksums, int64_t nblk, int q,
                                               DevParams *p) {
    __shared__ unsigned long long buf[1024 / 64];
    if (p->status != CHAMFER_OK) return;
    unsigned long long carry = 0;
    for (int64_t c0 = 0; c0 < nblk; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const unsigned long long v = i < nblk ? blocksums[i] : 0ull;
        const unsigned long long inc = block_inclusive_scan<1024>(v, buf);
        if (i < nblk) blocksums[i] = carry + inc - v;
        // total of this chunk is the last thread's inclusive value
        __shared__ unsigned long long tot;
        if (threadIdx.x == 1023) tot = inc;
        __syncthreads();
        carry += tot;
        __syncthreads();
    }
    const uint32_t mb = rep_fold(p->max_d_rep);
    if (threadIdx.x == 0) {
        const bool zero = !(__uint_as_float(mb) > 0.0f);
        p->W = carry;
        p->s = zero ? 0 : fixed_point_exponent(mb, q);
        p->all_zero = zero ? 1 : 0;
    }
}

__global__ __launch_bounds__(1024) void k_scan_blocksums(unsigned long long *blocksums,
                                                         int64_t nblk, int q, DevParams *p) {
    scan_blocksums(blocksums, nblk, q, p);
}

int64_t scan_blocks(int64_t nA) { return (nA + kScanBlock - 1) / kScanBlock; }

// Up to kOffsLds blocks the sampler scans the block totals itself (one
// launch fewer); above, k_scan_blocksums does.
bool sample_scans(int64_t nA) { return scan_blocks(nA) <= kOffsLds; }

hipError_t launch_weights(const float *D, int64_t nA, int q, uint64_t *blocksums, uint64_t *Ploc,
                          DevParams *p, hipStream_t st) {
    const int64_t nblk = scan_blocks(nA);
    auto *bs = reinterpret_cast<unsigned long long *>(blocksums);
    k_weight_blocksum<<<(unsigned)nblk, kScanThreads, 0, st>>>(
        D, nA, q, bs, reinterpret_cast<unsigned long long *>(Ploc), p);
    if (!sample_scans(nA)) k_scan_blocksums<<<1, 1024, 0, st>>>(bs, nblk, q, p);
    return hipGetLastError();
}

// Draw l: word 0 of Philox4x64-10 at counter (l, attempt, SAMPLE, 0), key
// (seed, 0); Lemire: m = x W, reject while (m mod 2^64) < (2^64 - W) mod W,
// u = m >> 64; idx = min{a : P_a > u}.  Also resets the nearest-neighbour
// slot of the draw.  P_a is the block offset offs[a / kScanBlock] (the
// scanned block totals, held in LDS when there are at most kOffsLds blocks)
// plus the in-block prefix Ploc_a.  The search first finds, in LDS, the
// first of kFences evenly spaced fences P[(i + 1) S - 1] (S = ceil(n_A /
// kFences), the last one P[n_A - 1] = W > u) above u, then searches the S
// entries it closes in memory: the same index with log2 S dependent loads
// instead of log2 n_A.  Every thread of the workgroup must call it (one
// barrier).
constexpr int kFences = 1024;

// local (at most kOffsLds blocks, 256 threads): offs holds the blocks'
// totals, not yet scanned; every workgroup scans them into LDS itself, and
// workgroup 0 stores W, s and all_zero (what k_scan_blocksums stores).
__device__ __forceinline__ void sample(uint64_t seed, const unsigned long long *__restrict__ Ploc,
                                       const unsigned long long *__restrict__ offs, int64_t nA,
                                       int64_t T, int32_t *idx, unsigned long long *best,
                                       DevParams *p, int q, bool local, Blk blk) {
    __shared__ unsigned long long fence[kFences];
    __shared__ unsigned long long boff[kOffsLds];
    __shared__ unsigned long long sbuf[4];
    __shared__ unsigned long long total;
    const int64_t l = blk.id * blockDim.x + threadIdx.x;
    const bool st_ok = p->status == CHAMFER_OK;  // uniform
    const int64_t S = (nA + kFences - 1) / kFences;
    const int64_t nblk = (nA + kScanBlock - 1) / kScanBlock;
    const bool lds_off = nblk <= kOffsLds;  // uniform; true when local
    uint64_t W;
    if (local) {
        // thread t: a run of `per` consecutive totals (loads in flight
        // together), their sum scanned across the workgroup, then the run's
        // exclusive offsets
        constexpr int kPer = kOffsLds / 256;
        const int64_t i0 = (int64_t)threadIdx.x * kPer;
        unsigned long long v[kPer];
        unsigned long long own = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            v[j] = (st_ok && i0 + j < nblk) ? ro(offs)[i0 + j] : 0ull;
            own += v[j];
        }
        const unsigned long long inc = block_inclusive_scan<256>(own, sbuf);
        unsigned long long run = inc - own;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (i0 + j < nblk) boff[i0 + j] = run;
            run += v[j];
        }
        if (threadIdx.x == 255) total = inc;
        const uint32_t mb = rep_fold(p->max_d_rep);
        __syncthreads();
        W = total;
        if (blk.id == 0 && threadIdx.x == 0 && st_ok) {
            const bool zero = !(__uint_as_float(mb) > 0.0f);
            p->W = W;
            p->s = zero ? 0 : fixed_point_exponent(mb, q);
            p->all_zero = zero ? 1 : 0;
        }
    } else {
        W = p->W;
        if (st_ok && W != 0 && lds_off)
            for (int64_t i = threadIdx.x; i < nblk; i += blockDim.x) boff[i] = ro(offs)[i];
    }
    const bool ok = st_ok && W != 0;  // uniform
    if (ok)
        for (int i = threadIdx.x; i < kFences; i += blockDim.x) {
            const int64_t a = min((int64_t)(i + 1) * S - 1, nA - 1);
            const int64_t j = a / kScanBlock;
            fence[i] = (local ? boff[j] : ro(offs)[j]) + ro(Ploc)[a];
        }
    __syncthreads();
    if (l >= T) return;
    best[l] = ~0ull;
    if (!ok) {
        idx[l] = 0;
        return;
    }
    uint64_t u = 0;
    for (uint64_t attempt = 0; attempt < (1ull << 20); ++attempt) {
        uint64_t c[4] = {(uint64_t)l, attempt, (uint64_t)kPurposeSample, 0};
        philox4x64_10(c, seed, 0);
        const uint64_t lo = c[0] * W;
        u = __umul64hi(c[0], W);
        if (lo < W) {
            const uint64_t thr = (0ull - W) % W;
            if (lo < thr) continue;
        }
        break;
    }
    int f0 = 0, f1 = kFences - 1;
    while (f0 < f1) {
        const int mid = (f0 + f1) >> 1;
        if (fence[mid] > u)
            f1 = mid;
        else
            f0 = mid + 1;
    }
    // P[f0 S - 1] <= u < P[min((f0 + 1) S, n_A) - 1]
    int64_t a = (int64_t)f0 * S, b = min((int64_t)(f0 + 1) * S - 1, nA - 1);
    while (a < b) {
        const int64_t mid = a + ((b - a) >> 1);
        const int64_t j = mid / kScanBlock;
        const unsigned long long pm = (lds_off ? boff[j] : ro(offs)[j]) + ro(Ploc)[mid];
        if (pm > u)
            b = mid;
        else
            a = mid + 1;
    }
    idx[l] = (int32_t)a;
}

__global__ __launch_bounds__(256) void k_sample(uint64_t seed,
                                                const unsigned long long *__restrict__ Ploc,
                                                const unsigned long long *__restrict__ offs,
                                                int64_t nA, int64_t T, int32_t *idx,
                                                unsigned long long *best, DevParams *p, int q,
                                                int local) {
    sample(seed, Ploc, offs, nA, T, idx, best, p, q, local != 0, grid_blk());
}

int64_t sample_blocks(int64_t T) { return (T + 255) / 256; }

hipError_t launch_sample(uint64_t seed, const uint64_t *Ploc, const uint64_t *offs, int64_t nA,
                         int64_t T, int q, int32_t *idx, unsigned long long *best, DevParams *p,
                         hipStream_t st) {
    const bool local = sample_scans(nA);
    if (T <= 0 && !local) return hipSuccess;
    // with T <= 0 one workgroup still stores W and s
    k_sample<<<(unsigned)(T > 0 ? sample_blocks(T) : 1), 256, 0, st>>>(
        seed, reinterpret_cast<const unsigned long long *>(Ploc),
        reinterpret_cast<const unsigned long long *>(offs), nA, T, idx, best, p, q,
        local ? 1 : 0);
    return hipGetLastError();
}

// eta = (1/T) sum_l (W / w_{x_l}) m_l; one block, fixed summation order.
__device__ __forceinline__ void estimate_final(const unsigned long long *__restrict__ best,
                                               const int32_t *__restrict__ idx,
                                               const float *__restrict__ D, int64_t T, int metric,
                                               const DevParams *p, double *eta_out,
                                               const chamfer_aux &aux) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int status = p->status;
    const uint64_t W = p->W;
    const int s = p->s;
    double acc = 0.0;
    // kG terms per thread per round: their loads (best, idx, then D[idx])
    // are issued together, then the terms are added in index order
    // (all loads in bounds and unconditional, so each group of them is in
    // flight together: positions past T read draw T - 1, whose idx is a row
    // of A like every draw's)
    constexpr int kG = 8;
    for (int64_t l0 = t; l0 < T; l0 += 256 * kG) {
        unsigned long long bv[kG];
        int32_t ix[kG];
        float dv[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const int64_t l = min(l0 + (int64_t)g * 256, T - 1);
            bv[g] = ro(best)[l];
            ix[g] = ro(idx)[l];
        }
#pragma unroll
        for (int g = 0; g < kG; ++g) dv[g] = ro(D)[ix[g]];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const int64_t l = l0 + (int64_t)g * 256;
            if (l >= T) break;
            const float v = __uint_as_float((uint32_t)(bv[g] >> 32));
            const int32_t nn = (int32_t)(uint32_t)(bv[g] & 0xffffffffu);
            float m = metric == CHAMFER_L2 ? sqrtf(v) : v;
            if (status != CHAMFER_OK) m = __builtin_nanf("");
            if (status == CHAMFER_OK && W != 0) {
                const double w = (double)weight_of(dv[g], s);
                acc += ((double)W / w) * (double)m;
            }
            if (aux.sample_min) aux.sample_min[l] = (status == CHAMFER_OK && W == 0) ? 0.0f : m;
            if (aux.sample_nn) aux.sample_nn[l] = (W == 0) ? 0 : nn;
            if (aux.sample_idx) aux.sample_idx[l] = ix[g];
        }
    }
    red[t] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) {
        double eta = (W == 0 || T == 0) ? 0.0 : red[0] / (double)T;
        if (status != CHAMFER_OK) eta = __builtin_nan("");
        *eta_out = eta;
        if (aux.D) *aux.D = ldexp((double)W, -s);
        if (aux.W) *aux.W = W;
        if (aux.s) *aux.s = s;
        if (aux.status) *aux.status = status;
    }
}

__global__ __launch_bounds__(256) void k_estimate_final(
    const unsigned long long *__restrict__ best, const int32_t *__restrict__ idx,
    const float *__restrict__ D, int64_t T, int metric, const DevParams *p, double *eta_out,
    chamfer_aux aux) {
    estimate_final(best, idx, D, T, metric, p, eta_out, aux);
}

hipError_t launch_estimate_final(const unsigned long long *best, const int32_t *idx,
                                 const float *D, int64_t T, int metric, DevParams *p,
                                 double *eta_out, chamfer_aux aux, hipStream_t st) {
    k_estimate_final<<<1, 256, 0, st>>>(best, idx, D, T, metric, p, eta_out, aux);
    return hipGetLastError();
}

__global__ void k_unit_weights(float *D, int32_t *nn, int32_t *scale, int64_t nA, DevParams *p) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nA; a += stride) {
        D[a] = 1.0f;
        if (nn) nn[a] = -1;
        if (scale) scale[a] = -1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) p->max_d_rep[0] = __float_as_uint(1.0f);
}

hipError_t launch_unit_weights(float *D, int32_t *nn, int32_t *scale, int64_t nA, DevParams *p,
                               hipStream_t st) {
    int64_t blocks = (nA + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    k_unit_weights<<<(unsigned)blocks, 256, 0, st>>>(D, nn, scale, nA, p);
    return hipGetLastError();
}

__global__ void k_copy_status(const DevParams *p, int32_t *out) {
    if (threadIdx.x == 0) *out = p->status;
}

hipError_t launch_copy_status(const DevParams *p, int32_t *status_out, hipStream_t st) {
    k_copy_status<<<1, 64, 0, st>>>(p, status_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- batched

constexpr unsigned kGridScan = 1024, kGridWscan = kBatchMax, kGridSample = 256,
                   kGridFinal = kBatchMax;

__global__ __launch_bounds__(kScanThreads) void kb_wsum(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsWsum, [&](const Job &J, Blk b) {
        weight_blocksum(J.D, J.nA, J.q, J.blocksums, J.P, J.p, b);
    });
}

__global__ __launch_bounds__(1024) void kb_wscan(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsWscan, [&](const Job &J, Blk) {
        scan_blocksums(J.blocksums, J.nb_scan, J.q, J.p);
    });
}

__global__ __launch_bounds__(256) void kb_sample(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsSample, [&](const Job &J, Blk b) {
        sample(J.seed, J.P, J.blocksums, J.nA, J.T, J.idx, J.best, J.p, J.q, false, b);
    });
}

__global__ __launch_bounds__(256) void kb_final(const Batch *__restrict__ bt, int metric) {
    batch_loop(bt, kBsFinal, [&](const Job &J, Blk) {
        estimate_final(J.best, J.idx, J.D, J.T, metric, J.p, J.eta, J.aux);
    });
}

hipError_t launch_batch_weights(const Batch *bt, hipStream_t st) {
    kb_wsum<<<kGridScan, kScanThreads, 0, st>>>(bt);
    kb_wscan<<<kGridWscan, 1024, 0, st>>>(bt);
    return hipGetLastError();
}

hipError_t launch_batch_sample(const Batch *bt, hipStream_t st) {
    kb_sample<<<kGridSample, 256, 0, st>>>(bt);
    return hipGetLastError();
}

hipError_t launch_batch_final(const Batch *bt, int metric, hipStream_t st) {
    kb_final<<<kGridFinal, 256, 0, st>>>(bt, metric);
    return hipGetLastError();
}

}  // namespace chamfer
