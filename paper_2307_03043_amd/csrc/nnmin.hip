// Exact nearest neighbours of a set of query rows against all of B: step 3
// of the Chamfer-Estimate figure (the T sampled rows) and the inner loop of
// brute-force CH (every row of A).
//
// VALU form.  Each lane owns QPL query rows, held in VGPRs for the whole
// sweep; all lanes of a wavefront walk the same rows of B, whose coordinates
// are wave-uniform and so arrive through scalar loads (SGPR operands of the
// vector ALU ops).  No LDS, no shuffles in the inner loop: per coordinate
// and query one subtract and one add (l1, |t| as a source modifier) or one
// fma (l2).  Every (query, b) pair is accumulated over k in ascending order
// with one rounding per operation, so the distance is the canonical float32
// value; ties keep the lower b.  Work is split into (query group, B chunk)
// tiles; the per-row result (distance bits << 32 | b) is merged with a
// 64-bit integer atomicMin, whose result does not depend on the order.
#include <cfloat>

#include "internal.h"

namespace chamfer {

__device__ __forceinline__ unsigned long long pack_best(float v, int b) {
    return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(uint32_t)b;
}

template <int METRIC>
__device__ __forceinline__ float accum(float acc, float q, float b) {
    const float t = q - b;
    return METRIC == CHAMFER_L1 ? acc + fabsf(t) : fmaf(t, t, acc);
}

// B rows per pass of the fixed-dimension form.  The distance of a (query, b)
// pair is one chain of D dependent adds (k ascending), so with one query per
// lane (d = 128) four rows are run at once: four independent chains per lane
// (measured +40% on MI355X); with two or more queries per lane the extra
// registers cost more than the chains gain.
template <int QPL>
constexpr int valu_rows() {
    return QPL == 1 ? 4 : 1;
}

// Exact dimension D known at compile time; QPL queries per lane, RB rows of
// B per pass (rows are still taken in index order, so ties keep the lower b).
template <int METRIC, int D, int QPL>
__device__ __forceinline__ void nnmin_fixed(const float *__restrict__ X,
                                            const int32_t *__restrict__ rows, int64_t nx,
                                            const float *__restrict__ B, int64_t nB, int64_t chunk,
                                            int nchunk, unsigned long long *best,
                                            const DevParams *__restrict__ p, Blk blk) {
    constexpr int RB = valu_rows<QPL>();
    if (p->status != CHAMFER_OK) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int cb;
    int64_t qb;
    chunk_major(blk.id, ((nx + 64 * QPL - 1) / (64 * QPL) + 3) / 4, nchunk, cb, qb);
    const int64_t qg = qb * 4 + wave;
    const int64_t q0 = qg * 64 * QPL;
    if (q0 >= nx) return;
    const int64_t b0 = (int64_t)cb * chunk;
    const int64_t b1 = min(nB, b0 + chunk);
    if (b0 >= b1) return;

    float q[QPL][D];
    int64_t qi[QPL];
#pragma unroll
    for (int j = 0; j < QPL; ++j) {
        qi[j] = q0 + j * 64 + lane;
        const int64_t r = qi[j] < nx ? (rows ? (int64_t)ro(rows)[qi[j]] : qi[j]) : 0;
        const auto *xr = ro(X) + r * D;
#pragma unroll
        for (int k = 0; k < D; ++k) q[j][k] = xr[k];
    }
    float bv[QPL];
    int bi[QPL];
#pragma unroll
    for (int j = 0; j < QPL; ++j) {
        bv[j] = FLT_MAX;
        bi[j] = (int)b0;
    }
    const auto *Bk = ro(B);  // rows are wave-uniform: scalar loads
    bool first = true;
    int64_t b = b0;
    for (; b + RB <= b1; b += RB) {
        float acc[RB][QPL];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int j = 0; j < QPL; ++j) acc[r][j] = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const float bk = Bk[(b + r) * D + k];
#pragma unroll
                for (int j = 0; j < QPL; ++j) acc[r][j] = accum<METRIC>(acc[r][j], q[j][k], bk);
            }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
#pragma unroll
            for (int j = 0; j < QPL; ++j) {
                if (first || acc[r][j] < bv[j]) {
                    bv[j] = acc[r][j];
                    bi[j] = (int)(b + r);
                }
            }
            first = false;
        }
    }
    for (; b < b1; ++b) {  // rows left over from the passes of RB
        const auto *br = Bk + b * D;
        float acc[QPL];
#pragma unroll
        for (int j = 0; j < QPL; ++j) acc[j] = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float bk = br[k];
#pragma unroll
            for (int j = 0; j < QPL; ++j) acc[j] = accum<METRIC>(acc[j], q[j][k], bk);
        }
#pragma unroll
        for (int j = 0; j < QPL; ++j) {
            if (first || acc[j] < bv[j]) {
                bv[j] = acc[j];
                bi[j] = (int)b;
            }
        }
        first = false;
    }
#pragma unroll
    for (int j = 0; j < QPL; ++j)
        if (qi[j] < nx) atomicMin(&best[qi[j]], pack_best(bv[j], bi[j]));
}

template <int METRIC, int D, int QPL>
__global__ __launch_bounds__(256) void k_nnmin_fixed(const float *__restrict__ X,
                                                     const int32_t *__restrict__ rows,
                                                     int64_t nx, const float *__restrict__ B,
                                                     int64_t nB, int64_t chunk, int nchunk,
                                                     unsigned long long *best,
                                                     const DevParams *__restrict__ p) {
    nnmin_fixed<METRIC, D, QPL>(X, rows, nx, B, nB, chunk, nchunk, best, p, grid_blk());
}

// Any dimension: coordinates in chunks of KC held in VGPRs, NB rows of B per
// pass so a query chunk is loaded once per NB rows.
template <int METRIC, int KC, int NB>
__device__ __forceinline__ void nnmin_any(const float *__restrict__ X,
                                          const int32_t *__restrict__ rows, int64_t nx,
                                          const float *__restrict__ B, int64_t nB, int d,
                                          int64_t chunk, int nchunk, unsigned long long *best,
                                          const DevParams *__restrict__ p, Blk blk) {
    if (p->status != CHAMFER_OK) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int cb;
    int64_t qb;
    chunk_major(blk.id, ((nx + 63) / 64 + 3) / 4, nchunk, cb, qb);
    const int64_t qi = (qb * 4 + wave) * 64 + lane;
    if (qi - lane >= nx) return;
    const int64_t b0 = (int64_t)cb * chunk;
    const int64_t b1 = min(nB, b0 + chunk);
    if (b0 >= b1) return;
    const int64_t r = qi < nx ? (rows ? (int64_t)ro(rows)[qi] : qi) : 0;
    const auto *xr = ro(X) + r * d;

    float bv = FLT_MAX;
    int bi = (int)b0;
    bool first = true;
    for (int64_t bb = b0; bb < b1; bb += NB) {
        const int nb = (int)min<int64_t>(NB, b1 - bb);
        float acc[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j] = 0.0f;
        for (int k0 = 0; k0 < d; k0 += KC) {
            const int kc = min(KC, d - k0);
            float qv[KC];
#pragma unroll
            for (int k = 0; k < KC; ++k) qv[k] = k < kc ? xr[k0 + k] : 0.0f;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if (j < nb) {
                    const auto *br = ro(B) + (bb + j) * d + k0;
#pragma unroll
                    for (int k = 0; k < KC; ++k)
                        if (k < kc) acc[j] = accum<METRIC>(acc[j], qv[k], br[k]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < nb && (first || acc[j] < bv)) {
                bv = acc[j];
                bi = (int)(bb + j);
                first = false;
            }
        }
    }
    if (qi < nx) atomicMin(&best[qi], pack_best(bv, bi));
}

template <int METRIC, int KC, int NB>
__global__ __launch_bounds__(256) void k_nnmin_any(const float *__restrict__ X,
                                                   const int32_t *__restrict__ rows, int64_t nx,
                                                   const float *__restrict__ B, int64_t nB,
                                                   int d, int64_t chunk, int nchunk,
                                                   unsigned long long *best,
                                                   const DevParams *__restrict__ p) {
    nnmin_any<METRIC, KC, NB>(X, rows, nx, B, nB, d, chunk, nchunk, best, p, grid_blk());
}

// Split B into chunks so the grid has enough workgroups to fill 256 CUs;
// the chunk count is a multiple of 8 when > 1 so that the work order
// (chunk_major) keeps each chunk's workgroups on one XCD.
static void split_b(int64_t qblocks, int64_t nB, int64_t target, int64_t &chunk, int &nchunk) {
    int64_t nc = (target + qblocks - 1) / qblocks;
    const int64_t maxc = (nB + 63) / 64;
    if (nc > maxc) nc = maxc;
    if (nc > 1) nc = (nc + 7) / 8 * 8;
    if (nc < 1) nc = 1;
    chunk = (nB + nc - 1) / nc;
    nchunk = (int)((nB + chunk - 1) / chunk);
}

// Queries per lane of the fixed-dimension forms (0: the any-dimension form).
static int valu_qpl(int d) {
    switch (d) {
        case 3: return 8;
        case 16: return 4;
        case 32: return 2;
        case 64: return 2;
        case 128: return 1;
        default: return 0;
    }
}

NNGeom valu_geom(int64_t nx, int64_t nB, int d, int64_t target) {
    const int qpl = valu_qpl(d);
    const int64_t per = 64 * (qpl ? qpl : 1);
    const int64_t qblocks = ((nx + per - 1) / per + 3) / 4;
    NNGeom g;
    split_b(qblocks, nB, target > 0 ? target : kValuTargetWGs, g.chunk, g.nchunk);
    g.blocks = qblocks * g.nchunk;
    return g;
}

template <int METRIC, int D, int QPL>
static hipError_t go_fixed(const float *X, const int32_t *rows, int64_t nx, const float *B,
                           int64_t nB, unsigned long long *best, const DevParams *p,
                           hipStream_t st) {
    const NNGeom g = valu_geom(nx, nB, D);
    k_nnmin_fixed<METRIC, D, QPL><<<(unsigned)g.blocks, 256, 0, st>>>(X, rows, nx, B, nB, g.chunk,
                                                                       g.nchunk, best, p);
    return hipGetLastError();
}

template <int METRIC>
static hipError_t go_metric(const float *X, const int32_t *rows, int64_t nx, const float *B,
                            int64_t nB, int d, unsigned long long *best, const DevParams *p,
                            hipStream_t st) {
    switch (d) {
        case 3: return go_fixed<METRIC, 3, 8>(X, rows, nx, B, nB, best, p, st);
        case 16: return go_fixed<METRIC, 16, 4>(X, rows, nx, B, nB, best, p, st);
        case 32: return go_fixed<METRIC, 32, 2>(X, rows, nx, B, nB, best, p, st);
        case 64: return go_fixed<METRIC, 64, 2>(X, rows, nx, B, nB, best, p, st);
        case 128: return go_fixed<METRIC, 128, 1>(X, rows, nx, B, nB, best, p, st);
        default: break;
    }
    const NNGeom g = valu_geom(nx, nB, d);
    k_nnmin_any<METRIC, 32, 8><<<(unsigned)g.blocks, 256, 0, st>>>(X, rows, nx, B, nB, d, g.chunk,
                                                                    g.nchunk, best, p);
    return hipGetLastError();
}

hipError_t launch_nnmin(const float *X, const int32_t *rows, int64_t nx, const float *B,
                        int64_t nB, int d, int metric, unsigned long long *best, DevParams *p,
                        hipStream_t st) {
    if (nx <= 0) return hipSuccess;
    if (metric == CHAMFER_L1) return go_metric<CHAMFER_L1>(X, rows, nx, B, nB, d, best, p, st);
    return go_metric<CHAMFER_L2>(X, rows, nx, B, nB, d, best, p, st);
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill_u64<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

constexpr int kFinThreads = 256;
constexpr int kFinItems = 8;

int nn_finalize_blocks(int64_t nx) {
    return (int)((nx + kFinThreads * kFinItems - 1) / (kFinThreads * kFinItems));
}

// Unpack (distance bits, b) -> min/arg (square root for l2) and a per-block
// double partial sum of the minima in a fixed order.
__global__ __launch_bounds__(kFinThreads) void k_nn_finalize(
    const unsigned long long *__restrict__ best, int64_t nx, int metric, float *min_out,
    int32_t *arg_out, double *partial, const DevParams *__restrict__ p) {
    __shared__ double red[kFinThreads];
    const int t = threadIdx.x;
    const bool bad = p->status != CHAMFER_OK;
    double acc = 0.0;
    const int64_t base = (int64_t)blockIdx.x * kFinThreads * kFinItems;
#pragma unroll
    for (int j = 0; j < kFinItems; ++j) {
        const int64_t r = base + (int64_t)j * kFinThreads + t;
        if (r < nx) {
            const unsigned long long b = best[r];
            const float v = __uint_as_float((uint32_t)(b >> 32));
            float m = metric == CHAMFER_L2 ? sqrtf(v) : v;
            if (bad) m = __builtin_nanf("");
            if (min_out) min_out[r] = m;
            if (arg_out) arg_out[r] = bad ? -1 : (int32_t)(uint32_t)(b & 0xffffffffu);
            acc += (double)m;
        }
    }
    red[t] = acc;
    __syncthreads();
    for (int off = kFinThreads / 2; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0 && partial) partial[blockIdx.x] = red[0];
}

hipError_t launch_nn_finalize(const unsigned long long *best, int64_t nx, int metric,
                              float *min_out, int32_t *arg_out, double *partial,
                              const DevParams *p, hipStream_t st) {
    if (nx <= 0) return hipSuccess;
    k_nn_finalize<<<nn_finalize_blocks(nx), kFinThreads, 0, st>>>(best, nx, metric, min_out,
                                                                   arg_out, partial, p);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sum_final(const double *__restrict__ partial,
                                                   int64_t nparts, const DevParams *p,
                                                   double *out) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int64_t i = t; i < nparts; i += 256) acc += partial[i];
    red[t] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) *out = p->status != CHAMFER_OK ? __builtin_nan("") : red[0];
}

hipError_t launch_sum_final(const double *partial, int64_t nparts, const DevParams *p,
                            double *out, hipStream_t st) {
    k_sum_final<<<1, 256, 0, st>>>(partial, nparts, p, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- batched
// Nearest neighbours of every job's T samples (rows idx of A) against its B.

constexpr unsigned kGridNNValu = 4096;

template <int METRIC, int D, int QPL>
__global__ __launch_bounds__(256) void kb_nn_fixed(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsNN, [&](const Job &J, Blk b) {
        nnmin_fixed<METRIC, D, QPL>(glb(J.A), glb(J.idx), J.T, glb(J.B), J.nB, J.nn_chunk,
                                    J.nn_nchunk, glb(J.best), glb(J.p), b);
    });
}

template <int METRIC>
__global__ __launch_bounds__(256) void kb_nn_any(const Batch *__restrict__ bt) {
    batch_loop(bt, kBsNN, [&](const Job &J, Blk b) {
        nnmin_any<METRIC, 32, 8>(glb(J.A), glb(J.idx), J.T, glb(J.B), J.nB, J.d, J.nn_chunk,
                                 J.nn_nchunk, glb(J.best), glb(J.p), b);
    });
}

template <int METRIC>
static hipError_t batch_valu(const Batch *bt, int d, hipStream_t st) {
    switch (d) {
        case 3: kb_nn_fixed<METRIC, 3, 8><<<kGridNNValu, 256, 0, st>>>(bt); break;
        case 16: kb_nn_fixed<METRIC, 16, 4><<<kGridNNValu, 256, 0, st>>>(bt); break;
        case 32: kb_nn_fixed<METRIC, 32, 2><<<kGridNNValu, 256, 0, st>>>(bt); break;
        case 64: kb_nn_fixed<METRIC, 64, 2><<<kGridNNValu, 256, 0, st>>>(bt); break;
        case 128: kb_nn_fixed<METRIC, 128, 1><<<kGridNNValu, 256, 0, st>>>(bt); break;
        default: kb_nn_any<METRIC><<<kGridNNValu, 256, 0, st>>>(bt); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_nn(const Batch *bt, int d, int metric, int precision, hipStream_t st) {
    if (lowp_supported(d, metric, precision)) return launch_batch_lowp(bt, d, precision, st);
    if (mfma_supported(d, metric)) return launch_batch_split(bt, d, st);
    if (metric == CHAMFER_L1) return batch_valu<CHAMFER_L1>(bt, d, st);
    return batch_valu<CHAMFER_L2>(bt, d, st);
}

}  // namespace chamfer
