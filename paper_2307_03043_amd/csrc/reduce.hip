// Reduction to bounded aspect ratio (the lemma reducing to poly(n/eps)
// aspect ratio, proved in the appendix), on the device:
//   1. a p-stable direction g (host, double; Cauchy for l1, Gaussian for l2);
//   2. p_x = <x, g> for every point (double, fused multiply-adds in
//      ascending coordinate order; rows staged through LDS);
//   3. B's projections sorted (radix sort), t_a = min_b |p_a - p_b| by a
//      binary search per a; M = max t_a (order-free, as 64-bit patterns of
//      non-negative doubles) and ch1 = sum t_a (fixed block order);
//   4. bounds, partition exponent and padding value from the exponent of M
//      (one thread, integer exponent arithmetic and ldexp only);
//   5. partition keys of A and B: one grid of side 2^e_part on the hashed
//      coordinates (x - lo, or the l2 -> l1 embedding), cells in double;
//   6. optional padded copies (m coordinates of +-q, signs from Philox).
// The estimate with the reduction reads the partition on the host once and
// either runs the plain estimate (one part, degenerate, or a part of A
// without points of B) or sums the estimates of the gathered parts.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

using namespace chamfer;

namespace {

// Keys per block of the radix sort of B's projections (below).
constexpr int kSortItems = 8;
constexpr int kSortBlock = 256 * kSortItems;

int64_t sort_blocks(int64_t n) { return (n + kSortBlock - 1) / kSortBlock; }

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int ceil_log2_i64(int64_t x) {
    int k = 0;
    while (k < 63 && (int64_t(1) << k) < x) ++k;
    return k;
}

// Padding coordinates: at least 3 ceil(log2 n), then d + m rounded up to the
// next of 16, 32, 64, 128 (or to a multiple of 16 above 128), the widths the
// exact-pass kernels specialise.
int pad_dims(int64_t nA, int64_t nB, int d) {
    const int64_t n = std::max<int64_t>(std::max(nA, nB), 2);
    int dp = d + 3 * ceil_log2_i64(n);
    if (dp <= 128) {
        int w = 16;
        while (w < dp) w *= 2;
        dp = w;
    } else {
        dp = (dp + 15) / 16 * 16;
    }
    return dp - d;
}

constexpr int kThreads = 256;
constexpr int kNearBlocks = 1024;  // fixed grid of the 1-D search: a fixed sum order
constexpr int kProjCols = 32;      // coordinates per LDS stage of the projection

struct Scratch {
    unsigned long long max_bits;  // bits of max_a t_a (t_a >= 0 orders as its bits)
};

struct RPlan {
    int64_t nA, nB;
    int32_t d, metric, ke, kh, m, la, lb, ln;
    size_t sort_bytes;
    size_t off_info, off_scr, off_g, off_pa, off_pb, off_alt, off_sort, off_partial, off_params,
        off_lohi, off_embed, off_zp, off_mp, off_keysA, off_keysB, total;
};

bool valid_ke(int ke) { return ke == 8 || ke == 16 || ke == 32 || ke == 64; }

int rplan(RPlan &rp, int64_t nA, int64_t nB, int32_t d, int32_t metric,
          const chamfer_opts *opts) {
    std::memset(&rp, 0, sizeof(rp));
    if (nA < 1 || nB < 1 || nA > INT32_MAX || nB > INT32_MAX || d < 1 || d > 2048)
        return CHAMFER_EINVAL;
    if (metric != CHAMFER_L1 && metric != CHAMFER_L2) return CHAMFER_EINVAL;
    chamfer_opts o{};
    if (opts) o = *opts;
    const int ke = o.embed_dim ? o.embed_dim : 32;
    if (!valid_ke(ke)) return CHAMFER_EINVAL;
    rp.nA = nA;
    rp.nB = nB;
    rp.d = d;
    rp.metric = metric;
    rp.ke = ke;
    rp.kh = metric == CHAMFER_L1 ? d : ke;
    const int64_t n = std::max<int64_t>(std::max(nA, nB), 2);
    rp.la = ceil_log2_i64(nA);
    rp.lb = ceil_log2_i64(nB);
    rp.ln = ceil_log2_i64(n);
    rp.m = pad_dims(nA, nB, d);
    // radix sort: a 256-bin count per block of keys, per pass
    rp.sort_bytes = up((size_t)256 * (sort_blocks(nB) + 1) * sizeof(uint32_t));
    size_t o2 = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o2;
        o2 += up(bytes);
        return at;
    };
    rp.off_info = take(sizeof(chamfer_reduction));
    rp.off_scr = take(sizeof(Scratch));
    rp.off_g = take((size_t)d * sizeof(double));
    rp.off_pa = take((size_t)nA * sizeof(double));
    rp.off_pb = take((size_t)nB * sizeof(double));
    rp.off_alt = take((size_t)nB * sizeof(double));
    rp.off_sort = take(rp.sort_bytes);
    rp.off_partial = take(kNearBlocks * sizeof(double));
    rp.off_params = take(sizeof(DevParams));
    rp.off_lohi = take(lohi_bytes(d));
    rp.off_embed = take(metric == CHAMFER_L2 ? (size_t)d * ke : 0);
    rp.off_zp = take((size_t)rp.kh * sizeof(float));
    rp.off_mp = take((size_t)rp.kh * sizeof(uint64_t));
    rp.off_keysA = take((size_t)nA * sizeof(uint64_t));
    rp.off_keysB = take((size_t)nB * sizeof(uint64_t));
    rp.total = o2;
    return CHAMFER_OK;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

#define CH_TRY(expr)                                    \
    do {                                                \
        if ((expr) != hipSuccess) return CHAMFER_EHIP;  \
    } while (0)

// ------------------------------------------------------------- host draws

// g_j from the Philox block (j, 0, SKETCH, 0): l1 Cauchy tan(pi (u - 1/2)),
// u = ((w0 >> 11) + 1/2) 2^-53; l2 Gaussian by Box-Muller, u1 = ((w0 >> 11)
// + 1) 2^-53, u2 = (w1 >> 11) 2^-53, sqrt(-2 ln u1) cos(2 pi u2).
void sketch_direction(uint64_t seed, int d, int metric, double *g) {
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < d; ++j) {
        uint64_t c[4] = {(uint64_t)j, 0, kPurposeSketch, 0};
        philox_host(c, seed, 0);
        if (metric == CHAMFER_L1) {
            const double u = std::ldexp((double)(c[0] >> 11) + 0.5, -53);
            g[j] = std::tan(pi * (u - 0.5));
        } else {
            const double u1 = std::ldexp((double)((c[0] >> 11) + 1), -53);
            const double u2 = std::ldexp((double)(c[1] >> 11), -53);
            g[j] = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * pi * u2);
        }
    }
}

// Partition grid: z'_k = (w0 >> 40) 2^-24, M_k = w1 | 1 from (k, 0, PART, 0).
void part_tables(uint64_t seed, int kh, float *zp, uint64_t *mp) {
    for (int k = 0; k < kh; ++k) {
        uint64_t c[4] = {(uint64_t)k, 0, kPurposePart, 0};
        philox_host(c, seed, 0);
        zp[k] = std::ldexp((float)(c[0] >> 40), -24);
        mp[k] = c[1] | 1ull;
    }
}

// ---------------------------------------------------------------- kernels

// Stage rows r0 .. r0 + rows - 1, coordinates c0 .. c0 + cols - 1, of X
// (row length d) into tile, minus lo when lohi is given.  With d a multiple
// of 4 and X 16-byte aligned each row segment is read as float4 by 8
// consecutive threads.
__device__ __forceinline__ void stage_tile(const float *__restrict__ X, int d, int64_t r0,
                                           int rows, int c0, int cols,
                                           const uint32_t *__restrict__ lohi,
                                           float (*tile)[kProjCols + 1]) {
    if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
        const int c4 = (threadIdx.x & 7) * 4;
        if (c4 < cols) {
            float lo[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (lohi)
                for (int u = 0; u < 4; ++u) lo[u] = ordered_to_float(lohi[c0 + c4 + u]);
            for (int r = threadIdx.x >> 3; r < rows; r += kThreads / 8) {
                const float4 v = *reinterpret_cast<const float4 *>(X + (r0 + r) * d + c0 + c4);
                tile[r][c4 + 0] = v.x - lo[0];
                tile[r][c4 + 1] = v.y - lo[1];
                tile[r][c4 + 2] = v.z - lo[2];
                tile[r][c4 + 3] = v.w - lo[3];
            }
        }
    } else {
        for (int q = threadIdx.x; q < rows * cols; q += kThreads) {
            const int r = q / cols, c = q - r * cols;
            const float x = X[(r0 + r) * d + c0 + c];
            tile[r][c] = lohi ? x - ordered_to_float(lohi[c0 + c]) : x;
        }
    }
}

// p_i = <x_i, g>: 256 rows per block, their coordinates staged through LDS
// kProjCols at a time (contiguous loads), each thread accumulating its row
// in ascending coordinate order.
__global__ __launch_bounds__(kThreads) void k_project(const float *__restrict__ X, int64_t n,
                                                      int d, const double *__restrict__ g,
                                                      double *__restrict__ out) {
    __shared__ float tile[kThreads][kProjCols + 1];
    for (int64_t r0 = (int64_t)blockIdx.x * kThreads; r0 < n; r0 += (int64_t)gridDim.x * kThreads) {
        const int rows = n - r0 < kThreads ? (int)(n - r0) : kThreads;
        double acc = 0.0;
        for (int c0 = 0; c0 < d; c0 += kProjCols) {
            const int cols = d - c0 < kProjCols ? d - c0 : kProjCols;
            __syncthreads();
            stage_tile(X, d, r0, rows, c0, cols, nullptr, tile);
            __syncthreads();
            if ((int)threadIdx.x < rows)
                for (int c = 0; c < cols; ++c)
                    acc = fma((double)tile[threadIdx.x][c], g[c0 + c], acc);
        }
        if ((int)threadIdx.x < rows) out[r0 + threadIdx.x] = acc;
    }
}

// ------------------------------------------------------------- radix sort
// B's projections in ascending order: an LSD radix sort of their
// order-preserving 64-bit codes (sign bit flipped for non-negative doubles,
// every bit for negative ones), eight passes of 8-bit digits.  A pass counts
// the digits of each block of kSortBlock codes into 256 bins (k_sort_hist),
// one workgroup per digit turns its row of the [digit][block] counts into
// exclusive offsets within the digit and the digit's total
// (k_sort_rowscan), and each block adds the digits' exclusive totals and
// writes its codes to their places (k_sort_scatter).  The scatter is stable: codes of one block keep their
// order -- a wavefront ranks equal digits by ballots over the eight digit
// bits, the wavefronts of a round and the rounds of a block are ordered
// through per-digit counters in LDS -- so each pass keeps the order of the
// previous ones among equal digits, and the eight passes sort.
__device__ __forceinline__ unsigned long long dbl_code(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

__device__ __forceinline__ double code_dbl(unsigned long long c) {
    const unsigned long long u = (c >> 63) ? (c & ~(1ull << 63)) : ~c;
    return __longlong_as_double((long long)u);
}

__global__ __launch_bounds__(256) void k_sort_encode(double *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) reinterpret_cast<unsigned long long *>(p)[i] = dbl_code(p[i]);
}

__global__ __launch_bounds__(256) void k_sort_decode(unsigned long long *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) reinterpret_cast<double *>(p)[i] = code_dbl(p[i]);
}

// cnt[digit * nblk + block] = how many codes of the block have that digit.
__global__ __launch_bounds__(256) void k_sort_hist(const unsigned long long *__restrict__ keys,
                                                   int64_t n, int shift, int64_t nblk,
                                                   uint32_t *cnt) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b = blockIdx.x;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t e = b * kSortBlock + it * 256 + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    cnt[(int64_t)threadIdx.x * nblk + b] = h[threadIdx.x];
}

// Exclusive scan of one value per thread of a 256-thread workgroup: the
// thread's exclusive prefix, and the sum of all 256 in *all.  ws: 4 words
// of LDS.  Every thread must call it (two barriers).
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t c, uint32_t *ws, uint32_t *all) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t x = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    uint32_t pre = 0, sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t v = ws[q];
        pre += q < w ? v : 0u;
        sum += v;
    }
    __syncthreads();  // ws is free again
    *all = sum;
    return pre + x - c;
}

// Workgroup d: the counts cnt[d nblk + b] of digit d in place as exclusive
// offsets over the blocks b (256 blocks per step, coalesced), and the
// digit's total in tot[d].
__global__ __launch_bounds__(256) void k_sort_rowscan(uint32_t *cnt, int64_t nblk, uint32_t *tot) {
    __shared__ uint32_t ws[4];
    uint32_t *row = cnt + (int64_t)blockIdx.x * nblk;
    uint32_t carry = 0;
    for (int64_t i0 = 0; i0 < nblk; i0 += 256) {
        const int64_t i = i0 + threadIdx.x;
        const uint32_t c = i < nblk ? row[i] : 0u;
        uint32_t all;
        const uint32_t pre = block_excl_scan256(c, ws, &all);
        if (i < nblk) row[i] = carry + pre;
        carry += all;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(256) void k_sort_scatter(const unsigned long long *__restrict__ in,
                                                      unsigned long long *__restrict__ out,
                                                      int64_t n, int shift, int64_t nblk,
                                                      const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ tot) {
    __shared__ uint32_t base[256];    // next place of each digit for this block
    __shared__ uint32_t wc[4][256];   // per-wavefront digit counts of the round
    __shared__ uint32_t ws[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t b = blockIdx.x;
    uint32_t all;
    base[t] = off[(int64_t)t * nblk + b] + block_excl_scan256(tot[t], ws, &all);
    for (int q = 0; q < 4; ++q) wc[q][t] = 0;
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1;
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t e = b * kSortBlock + it * 256 + t;
        const bool valid = e < n;
        const unsigned long long key = valid ? in[e] : 0ull;
        const uint32_t dg = (uint32_t)(key >> shift) & 255u;
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long bb = __ballot((dg >> bit) & 1u);
            m &= ((dg >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & below);
        if (valid && rank == 0) wc[w][dg] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[dg] + rank;
            for (int q = 0; q < w; ++q) pos += wc[q][dg];
            out[pos] = key;
        }
        __syncthreads();
        base[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        for (int q = 0; q < 4; ++q) wc[q][t] = 0;
        __syncthreads();
    }
}

// Sorts p[0..n) (doubles) ascending; tmp holds n doubles, cnt 256
// (sort_blocks(n) + 1) counts (the last 256: the digits' totals).  The
// sorted values end in p.
hipError_t sort_doubles(double *p, double *tmp, int64_t n, uint32_t *cnt, hipStream_t st) {
    if (n <= 1) return hipSuccess;
    const int64_t nblk = sort_blocks(n);
    const unsigned g256 = (unsigned)((n + 255) / 256);
    auto *a = reinterpret_cast<unsigned long long *>(p);
    auto *b = reinterpret_cast<unsigned long long *>(tmp);
    k_sort_encode<<<g256, 256, 0, st>>>(p, n);
    for (int shift = 0; shift < 64; shift += 8) {
        k_sort_hist<<<(unsigned)nblk, 256, 0, st>>>(a, n, shift, nblk, cnt);
        k_sort_rowscan<<<256, 256, 0, st>>>(cnt, nblk, cnt + 256 * nblk);
        k_sort_scatter<<<(unsigned)nblk, 256, 0, st>>>(a, b, n, shift, nblk, cnt,
                                                     cnt + 256 * nblk);
        std::swap(a, b);
    }
    // eight passes: the sorted codes are back in p
    k_sort_decode<<<g256, 256, 0, st>>>(a, n);
    return hipGetLastError();
}

// t_a = min(succ - p_a, p_a - pred) over B's sorted projections; per block
// the sum (thread order, then a fixed tree) and the maximum bit pattern.
__global__ __launch_bounds__(kThreads) void k_nearest1d(const double *__restrict__ pa,
                                                        int64_t nA,
                                                        const double *__restrict__ pbs,
                                                        int64_t nB, double *__restrict__ t_out,
                                                        double *__restrict__ partial,
                                                        Scratch *scr) {
    __shared__ double ssum[kThreads];
    __shared__ unsigned long long smax[kThreads];
    double sum = 0.0;
    unsigned long long mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nA;
         i += (int64_t)gridDim.x * kThreads) {
        const double x = pa[i];
        int64_t lo = 0, hi = nB;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (pbs[mid] < x)
                lo = mid + 1;
            else
                hi = mid;
        }
        double t = INFINITY;
        if (lo < nB) t = pbs[lo] - x;
        if (lo > 0) {
            const double pred = x - pbs[lo - 1];
            t = pred < t ? pred : t;
        }
        if (t_out) t_out[i] = t;
        sum += t;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(t);
        mx = bits > mx ? bits : mx;
    }
    ssum[threadIdx.x] = sum;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ssum[threadIdx.x] = ssum[threadIdx.x] + ssum[threadIdx.x + s];
            const unsigned long long o = smax[threadIdx.x + s];
            if (o > smax[threadIdx.x]) smax[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = ssum[0];
        if (smax[0] != 0) atomicMax(&scr->max_bits, smax[0]);
    }
}

__global__ void k_reduce_init(Scratch *scr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) scr->max_bits = 0;
}

// ch1, M and the quantities derived from e_M = floor(log2 M).
__global__ __launch_bounds__(kThreads) void k_reduce_finish(const double *__restrict__ partial,
                                                            int nparts, const Scratch *scr,
                                                            int la, int ln, int k_lo, int k_hi,
                                                            int m, double q0,
                                                            chamfer_reduction *info) {
    __shared__ double ssum[kThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kThreads) s += partial[i];
    ssum[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) ssum[threadIdx.x] = ssum[threadIdx.x] + ssum[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double M = __longlong_as_double((long long)scr->max_bits);
    chamfer_reduction r;
    r.ch1 = ssum[0];
    r.max_t = M;
    r.pad_dims = m;
    r.one_part = 1;
    r.degenerate = !(M > 0.0) || isinf(M);
    if (r.degenerate) {
        r.e_M = 0;
        r.e_part = 0;
        r.eta_lo = 0.0;
        r.eta_hi = 0.0;
        r.pad_value = 0.0f;
    } else {
        int e;
        frexp(M, &e);
        r.e_M = e - 1;
        const int e_hi = r.e_M + 1 + la + k_lo;
        const int log2c = e_hi - (r.e_M - k_hi);
        r.e_part = log2c + ln + e_hi;
        r.eta_lo = ldexp(1.0, r.e_M - k_hi);
        r.eta_hi = ldexp(1.0, e_hi);
        r.pad_value = (float)ldexp(q0, r.e_M - k_hi);
    }
    *info = r;
}

// Partition key of each point (see chamfer_aspect_reduce): hashed
// coordinates in float as the bucket keys, the cell in double.  256 rows per
// block; y = x - lo is staged through LDS kProjCols coordinates at a time
// (contiguous loads); l2 accumulates the KE embedded coordinates of its row
// in registers, coordinates ascending.
__device__ __forceinline__ uint64_t part_cell_term(float y, int e, float z, uint64_t mult) {
    const double lim = 4611686018427387904.0;  // 2^62
    double cell = ceil(ldexp((double)y, -e) + (double)z);
    if (cell != cell) cell = 0.0;
    cell = cell > lim ? lim : (cell < -lim ? -lim : cell);
    return (uint64_t)(int64_t)cell * mult;
}

template <int METRIC, int KE>
__global__ __launch_bounds__(kThreads) void k_part_keys(
    const float *__restrict__ X, int64_t n, int d, const uint32_t *__restrict__ lohi,
    const int8_t *__restrict__ zt, const float *__restrict__ zp, const uint64_t *__restrict__ mp,
    const chamfer_reduction *info, const DevParams *pr, uint64_t *__restrict__ keys) {
    __shared__ float tile[kThreads][kProjCols + 1];
    const bool degenerate = info->degenerate != 0;
    const int e = info->e_part;
    const int e_top = pr->e_top;
    const double inv = 1.0 / (sqrt(2.0 / 3.14159265358979323846) * (double)KE * 32.0);
    for (int64_t r0 = (int64_t)blockIdx.x * kThreads; r0 < n; r0 += (int64_t)gridDim.x * kThreads) {
        const int rows = n - r0 < kThreads ? (int)(n - r0) : kThreads;
        if (degenerate) {
            if ((int)threadIdx.x < rows) keys[r0 + threadIdx.x] = 0;
            continue;
        }
        uint64_t acc = 0;
        // l2: the exact integer embedding of the quantised coordinates
        int64_t emb[KE > 0 ? KE : 1];
#pragma unroll
        for (int k = 0; k < (KE > 0 ? KE : 1); ++k) emb[k] = 0;
        for (int c0 = 0; c0 < d; c0 += kProjCols) {
            const int cols = d - c0 < kProjCols ? d - c0 : kProjCols;
            __syncthreads();
            stage_tile(X, d, r0, rows, c0, cols, lohi, tile);
            __syncthreads();
            if ((int)threadIdx.x < rows) {
                for (int c = 0; c < cols; ++c) {
                    const float y = tile[threadIdx.x][c];
                    if (METRIC == CHAMFER_L1) {
                        acc += part_cell_term(y, e, zp[c0 + c], mp[c0 + c]);
                    } else {
                        const int64_t u =
                            (int64_t)floorf(fminf(ldexpf(y, 24 - e_top), 16777215.0f));
                        const int8_t *zrow = zt + (size_t)(c0 + c) * KE;
#pragma unroll
                        for (int k = 0; k < KE; ++k) emb[k] += (int64_t)zrow[k] * u;
                    }
                }
            }
        }
        if ((int)threadIdx.x < rows) {
            if (METRIC == CHAMFER_L2) {
#pragma unroll
                for (int k = 0; k < KE; ++k) {
                    const float yk = (float)(ldexp((double)emb[k], e_top - 24) * inv);
                    acc += part_cell_term(yk, e, zp[k], mp[k]);
                }
            }
            keys[r0 + threadIdx.x] = acc >> 1;
        }
    }
}

hipError_t launch_part_keys(const float *X, int64_t n, int d, int metric, int ke,
                            const uint32_t *lohi, const int8_t *zt, const float *zp,
                            const uint64_t *mp, const chamfer_reduction *info,
                            const DevParams *pr, uint64_t *keys, unsigned grid, hipStream_t st) {
#define CH_PK_ARGS X, n, d, lohi, zt, zp, mp, info, pr, keys
    if (metric == CHAMFER_L1) {
        k_part_keys<CHAMFER_L1, 0><<<grid, kThreads, 0, st>>>(CH_PK_ARGS);
    } else {
        switch (ke) {
            case 8: k_part_keys<CHAMFER_L2, 8><<<grid, kThreads, 0, st>>>(CH_PK_ARGS); break;
            case 16: k_part_keys<CHAMFER_L2, 16><<<grid, kThreads, 0, st>>>(CH_PK_ARGS); break;
            case 32: k_part_keys<CHAMFER_L2, 32><<<grid, kThreads, 0, st>>>(CH_PK_ARGS); break;
            default: k_part_keys<CHAMFER_L2, 64><<<grid, kThreads, 0, st>>>(CH_PK_ARGS); break;
        }
    }
#undef CH_PK_ARGS
    return hipGetLastError();
}

// one_part = 0 if any key differs from A's first.
__global__ __launch_bounds__(kThreads) void k_one_part(const uint64_t *__restrict__ kA,
                                                       int64_t nA,
                                                       const uint64_t *__restrict__ kB,
                                                       int64_t nB, chamfer_reduction *info) {
    const uint64_t ref = kA[0];
    bool differ = false;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nA + nB;
         i += (int64_t)gridDim.x * kThreads)
        differ |= (i < nA ? kA[i] : kB[i - nA]) != ref;
    if (__ballot(differ) != 0 && (threadIdx.x & 63) == 0) atomicAnd(&info->one_part, 0);
}

// Padded copy, coordinates: out[i][j] = X[i][j] for j < d.
__global__ __launch_bounds__(kThreads) void k_pad_copy(const float *__restrict__ X, int64_t n,
                                                       int d, int m, float *__restrict__ out) {
    const int64_t total = n * d;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t i = e / d;
        const int j = (int)(e - i * d);
        out[i * (d + m) + j] = X[e];
    }
}

// Padded copy, appended values: out[i][d + j] = +-q, sign from bit j mod 64
// of word j / 64 of the Philox block (i, side, PAD, 0).  256 rows per block:
// one Philox block per row into LDS, then the block writes the rows' m
// values together (each row's values are contiguous).
__global__ __launch_bounds__(kThreads) void k_pad_signs(int64_t n, int d, int m, int side,
                                                        uint64_t seed,
                                                        const chamfer_reduction *info,
                                                        float *__restrict__ out) {
    __shared__ uint64_t words[kThreads][4];
    const float q = info->pad_value;
    for (int64_t r0 = (int64_t)blockIdx.x * kThreads; r0 < n; r0 += (int64_t)gridDim.x * kThreads) {
        const int rows = n - r0 < kThreads ? (int)(n - r0) : kThreads;
        __syncthreads();
        if ((int)threadIdx.x < rows) {
            uint64_t c[4] = {(uint64_t)(r0 + threadIdx.x), (uint64_t)side, kPurposePad, 0};
            philox4x64_10(c, seed, 0);
            for (int w = 0; w < 4; ++w) words[threadIdx.x][w] = c[w];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < rows * m; e += kThreads) {
            const int r = e / m, j = e - r * m;
            out[(r0 + r) * (d + m) + d + j] = ((words[r][j >> 6] >> (j & 63)) & 1u) ? -q : q;
        }
    }
}

// dst[r] = src[rows[r]] for r < cnt (rows of width w).
__global__ __launch_bounds__(kThreads) void k_gather(const float *__restrict__ src, int w,
                                                     const int32_t *__restrict__ rows,
                                                     int64_t cnt, float *__restrict__ dst) {
    const int64_t total = cnt * w;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t r = e / w;
        dst[e] = src[(int64_t)rows[r] * w + (e - r * w)];
    }
}

// eta = sum of the parts' estimates in part order.
__global__ void k_sum_slots(const double *slots, int64_t n, double *eta) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += slots[i];
    *eta = s;
}

unsigned grid_for(int64_t items, unsigned cap = 4096) {
    int64_t b = (items + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// Steps 1-5 (and 6 when A_pad/B_pad are given) into the reduction workspace.
int run_reduce(const RPlan &rp, const float *A, const float *B, double eps, uint64_t seed,
               double *t_out, uint64_t *keysA, uint64_t *keysB, float *A_pad, float *B_pad,
               void *ws, hipStream_t st) {
    const int d = rp.d;
    chamfer_reduction *info = at<chamfer_reduction>(ws, rp.off_info);
    Scratch *scr = at<Scratch>(ws, rp.off_scr);
    double *g = at<double>(ws, rp.off_g);
    double *pa = at<double>(ws, rp.off_pa);
    double *pb = at<double>(ws, rp.off_pb);
    double *alt = at<double>(ws, rp.off_alt);
    double *partial = at<double>(ws, rp.off_partial);
    DevParams *p = at<DevParams>(ws, rp.off_params);
    uint32_t *lohi = at<uint32_t>(ws, rp.off_lohi);
    int8_t *zt = at<int8_t>(ws, rp.off_embed);
    float *zp = at<float>(ws, rp.off_zp);
    uint64_t *mp = at<uint64_t>(ws, rp.off_mp);

    // host draws: g, the partition grid and (l2) the embedding, one upload
    // each (pageable copies, read before the call returns)
    thread_local std::vector<double> hg;
    thread_local std::vector<float> hz;
    thread_local std::vector<int8_t> hzq, hzt;
    thread_local std::vector<uint64_t> hm;
    hg.resize(d);
    sketch_direction(seed, d, rp.metric, hg.data());
    hz.resize(rp.kh);
    hm.resize(rp.kh);
    part_tables(seed, rp.kh, hz.data(), hm.data());
    CH_TRY(hipMemcpyAsync(g, hg.data(), (size_t)d * sizeof(double), hipMemcpyHostToDevice, st));
    CH_TRY(hipMemcpyAsync(zp, hz.data(), hz.size() * sizeof(float), hipMemcpyHostToDevice, st));
    CH_TRY(hipMemcpyAsync(mp, hm.data(), hm.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    if (rp.metric == CHAMFER_L2) {
        // the quantised matrix transposed to [d][ke] (a row per coordinate)
        hzq.resize((size_t)d * rp.ke);
        hzt.resize((size_t)d * rp.ke);
        embedding_host(seed, d, rp.ke, hzq.data());
        for (int j = 0; j < rp.ke; ++j)
            for (int k = 0; k < d; ++k) hzt[(size_t)k * rp.ke + j] = hzq[(size_t)j * d + k];
        CH_TRY(hipMemcpyAsync(zt, hzt.data(), hzt.size(), hipMemcpyHostToDevice,
                              st));
    }

    // 2-3: projections, sort, 1-D nearest neighbours
    k_reduce_init<<<1, 64, 0, st>>>(scr);
    k_project<<<grid_for(rp.nA, 8192), kThreads, 0, st>>>(A, rp.nA, d, g, pa);
    k_project<<<grid_for(rp.nB, 8192), kThreads, 0, st>>>(B, rp.nB, d, g, pb);
    CH_TRY(hipGetLastError());
    CH_TRY(sort_doubles(pb, alt, rp.nB, at<uint32_t>(ws, rp.off_sort), st));
    const double *pbs = pb;
    const unsigned nb = grid_for(rp.nA, kNearBlocks);
    k_nearest1d<<<nb, kThreads, 0, st>>>(pa, rp.nA, pbs, rp.nB, t_out, partial, scr);
    // 4: bounds; q0 = eps / (2 n m) in double, scaled by 2^(e_M - k_hi) on
    // the device
    const int64_t n = std::max<int64_t>(std::max(rp.nA, rp.nB), 2);
    const double q0 = eps / (double)(2 * n * (int64_t)rp.m);
    k_reduce_finish<<<1, kThreads, 0, st>>>(partial, (int)nb, scr, rp.la, rp.ln,
                                            rp.la + rp.lb + rp.ln, rp.la + rp.ln, rp.m, q0, info);
    CH_TRY(hipGetLastError());

    // 5: calibration (lo of A u B) and the partition keys
    CH_TRY(launch_init_params(p, lohi, d, st));
    CH_TRY(launch_minmax(A, rp.nA, d, lohi, p, st));
    CH_TRY(launch_minmax(B, rp.nB, d, lohi, p, st));
    CH_TRY(launch_calib_final(lohi, d, p, st));
    CH_TRY(launch_part_keys(A, rp.nA, d, rp.metric, rp.ke, lohi, zt, zp, mp, info, p, keysA,
                            grid_for(rp.nA), st));
    CH_TRY(launch_part_keys(B, rp.nB, d, rp.metric, rp.ke, lohi, zt, zp, mp, info, p, keysB,
                            grid_for(rp.nB), st));
    k_one_part<<<grid_for(rp.nA + rp.nB), kThreads, 0, st>>>(keysA, rp.nA, keysB, rp.nB, info);
    CH_TRY(hipGetLastError());

    // 6: padded copies
    for (int side = 0; side < 2; ++side) {
        float *out = side == 0 ? A_pad : B_pad;
        if (!out) continue;
        const float *X = side == 0 ? A : B;
        const int64_t rows = side == 0 ? rp.nA : rp.nB;
        k_pad_copy<<<grid_for(rows * d), kThreads, 0, st>>>(X, rows, d, rp.m, out);
        k_pad_signs<<<grid_for(rows), kThreads, 0, st>>>(rows, d, rp.m, side, seed, info, out);
    }
    CH_TRY(hipGetLastError());
    return CHAMFER_OK;
}

// Workspace of the estimate with the reduction: the reduction's regions,
// padded copies, gathered parts, per-part estimates, row lists, then the
// inner estimate's workspace.
struct EPlan {
    RPlan rp;
    int32_t dp;  // d of the estimated sets (d + m when padded)
    size_t off_Ap, off_Bp, off_At, off_Bt, off_slots, off_rows, off_inner, inner_bytes, total;
};

int eplan(EPlan &ep, int64_t nA, int64_t nB, int32_t d, int32_t metric, double eps, int64_t T,
          const chamfer_opts *opts) {
    if (!opts || (opts->reduction != CHAMFER_REDUCE_PARTITION &&
                  opts->reduction != CHAMFER_REDUCE_PAD))
        return CHAMFER_EINVAL;
    if (!(eps > 0.0 && eps < 1.0)) return CHAMFER_EINVAL;
    int rc = rplan(ep.rp, nA, nB, d, metric, opts);
    if (rc) return rc;
    const bool padded = opts->reduction == CHAMFER_REDUCE_PAD;
    ep.dp = d + (padded ? ep.rp.m : 0);
    if (ep.dp > 2048) return CHAMFER_EINVAL;
    chamfer_opts inner = *opts;
    inner.reduction = CHAMFER_REDUCE_NONE;
    ep.inner_bytes = chamfer_workspace_bytes(nA, nB, ep.dp, metric, eps, T, &inner);
    if (ep.inner_bytes == 0) return CHAMFER_EINVAL;
    size_t o = ep.rp.total;
    auto take = [&](size_t bytes) {
        const size_t a = o;
        o += up(bytes);
        return a;
    };
    ep.off_Ap = take(padded ? (size_t)nA * ep.dp * sizeof(float) : 0);
    ep.off_Bp = take(padded ? (size_t)nB * ep.dp * sizeof(float) : 0);
    ep.off_At = take((size_t)nA * ep.dp * sizeof(float));
    ep.off_Bt = take((size_t)nB * ep.dp * sizeof(float));
    ep.off_slots = take((size_t)nA * sizeof(double));
    ep.off_rows = take((size_t)(nA + nB) * sizeof(int32_t));
    ep.off_inner = take(ep.inner_bytes);
    ep.total = o;
    return CHAMFER_OK;
}

}  // namespace

namespace chamfer {

size_t reduced_workspace_bytes(int64_t n_A, int64_t n_B, int32_t d, int32_t metric, double eps,
                               int64_t T, const chamfer_opts *opts) {
    EPlan ep;
    if (eplan(ep, n_A, n_B, d, metric, eps, T, opts) != CHAMFER_OK) return 0;
    return ep.total;
}

int estimate_reduced(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                     int32_t metric, double eps, int64_t T, uint64_t seed, double *eta_out,
                     chamfer_aux *aux, const chamfer_opts *opts, void *ws, size_t ws_bytes,
                     void *stream) {
    chamfer_opts inner = opts ? *opts : chamfer_opts{};
    inner.reduction = CHAMFER_REDUCE_NONE;
    if (aux != nullptr || eta_out == nullptr || B == nullptr) return CHAMFER_EINVAL;
    if (n_A == 0) {  // nothing to reduce: the plain estimate (eta = 0)
        if (ws_bytes < chamfer_workspace_bytes(0, n_B, d, metric, eps, T, &inner))
            return CHAMFER_EWORKSPACE;
        return chamfer_estimate(A, B, n_A, n_B, d, metric, eps, T, seed, eta_out, nullptr,
                                &inner, ws, ws_bytes, stream);
    }
    EPlan ep;
    int rc = eplan(ep, n_A, n_B, d, metric, eps, T, opts);
    if (rc) return rc;
    if (A == nullptr) return CHAMFER_EINVAL;
    if (ws == nullptr || ws_bytes < ep.total) return CHAMFER_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) return CHAMFER_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const RPlan &rp = ep.rp;
    const bool padded = opts->reduction == CHAMFER_REDUCE_PAD;
    float *Ap = padded ? at<float>(ws, ep.off_Ap) : nullptr;
    float *Bp = padded ? at<float>(ws, ep.off_Bp) : nullptr;
    uint64_t *kA = at<uint64_t>(ws, rp.off_keysA);
    uint64_t *kB = at<uint64_t>(ws, rp.off_keysB);
    if ((rc = run_reduce(rp, A, B, eps, seed, nullptr, kA, kB, Ap, Bp, ws, st))) return rc;
    const float *X = padded ? Ap : A;
    const float *Y = padded ? Bp : B;
    void *inner_ws = at<void>(ws, ep.off_inner);

    chamfer_reduction info;
    CH_TRY(hipMemcpyAsync(&info, at<void>(ws, rp.off_info), sizeof(info), hipMemcpyDeviceToHost,
                          st));
    CH_TRY(hipStreamSynchronize(st));
    auto plain = [&]() {
        return chamfer_estimate(X, Y, n_A, n_B, ep.dp, metric, eps, T, seed, eta_out, nullptr,
                                &inner, inner_ws, ep.inner_bytes, stream);
    };
    if (info.degenerate || info.one_part) return plain();

    // several parts: group rows by key on the host
    std::vector<uint64_t> hA(n_A), hB(n_B);
    CH_TRY(hipMemcpyAsync(hA.data(), kA, n_A * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    CH_TRY(hipMemcpyAsync(hB.data(), kB, n_B * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    CH_TRY(hipStreamSynchronize(st));
    std::vector<int32_t> ra(n_A), rb(n_B);
    std::iota(ra.begin(), ra.end(), 0);
    std::iota(rb.begin(), rb.end(), 0);
    std::stable_sort(ra.begin(), ra.end(), [&](int32_t x, int32_t y) { return hA[x] < hA[y]; });
    std::stable_sort(rb.begin(), rb.end(), [&](int32_t x, int32_t y) { return hB[x] < hB[y]; });
    struct Part {
        int64_t a0, na, b0, nb;
    };
    std::vector<Part> parts;
    int64_t j = 0;
    for (int64_t i = 0; i < n_A;) {
        const uint64_t key = hA[ra[i]];
        int64_t i1 = i;
        while (i1 < n_A && hA[ra[i1]] == key) ++i1;
        while (j < n_B && hB[rb[j]] < key) ++j;
        int64_t j1 = j;
        while (j1 < n_B && hB[rb[j1]] == key) ++j1;
        if (j1 == j) return plain();  // a part of A without points of B
        parts.push_back(Part{i, i1 - i, j, j1 - j});
        i = i1;
        j = j1;
    }
    std::vector<int32_t> rows(n_A + n_B);
    std::copy(ra.begin(), ra.end(), rows.begin());
    std::copy(rb.begin(), rb.end(), rows.begin() + n_A);
    int32_t *drows = at<int32_t>(ws, ep.off_rows);
    // the copy reads the host row list: whatever path leaves this function
    // after it drains the stream first
    struct DrainOnExit {
        hipStream_t st;
        ~DrainOnExit() { (void)hipStreamSynchronize(st); }
    } drain{st};
    CH_TRY(hipMemcpyAsync(drows, rows.data(), rows.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    float *At = at<float>(ws, ep.off_At);
    float *Bt = at<float>(ws, ep.off_Bt);
    double *slots = at<double>(ws, ep.off_slots);
    for (size_t t = 0; t < parts.size(); ++t) {
        const Part &pt = parts[t];
        k_gather<<<grid_for(pt.na * ep.dp), kThreads, 0, st>>>(X, ep.dp, drows + pt.a0, pt.na,
                                                              At);
        k_gather<<<grid_for(pt.nb * ep.dp), kThreads, 0, st>>>(Y, ep.dp, drows + n_A + pt.b0,
                                                              pt.nb, Bt);
        CH_TRY(hipGetLastError());
        if ((rc = chamfer_estimate(At, Bt, pt.na, pt.nb, ep.dp, metric, eps, T, seed, slots + t,
                                   nullptr, &inner, inner_ws, ep.inner_bytes, stream)))
            return rc;
    }
    k_sum_slots<<<1, 64, 0, st>>>(slots, (int64_t)parts.size(), eta_out);
    CH_TRY(hipGetLastError());
    return CHAMFER_OK;
}

}  // namespace chamfer

extern "C" {

int32_t chamfer_pad_dims(int64_t n_A, int64_t n_B, int32_t d) {
    if (d < 1) return -1;
    return pad_dims(n_A, n_B, d);
}

size_t chamfer_reduce_workspace_bytes(int64_t n_A, int64_t n_B, int32_t d, int32_t metric,
                                      const chamfer_opts *opts) {
    RPlan rp;
    if (rplan(rp, n_A, n_B, d, metric, opts) != CHAMFER_OK) return 0;
    return rp.total;
}

int chamfer_aspect_reduce(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                          int32_t metric, double eps, uint64_t seed, const chamfer_opts *opts,
                          chamfer_reduction *info_out, double *t_out, uint64_t *keys_A_out,
                          uint64_t *keys_B_out, float *A_pad_out, float *B_pad_out, void *ws,
                          size_t ws_bytes, void *stream) {
    RPlan rp;
    int rc = rplan(rp, n_A, n_B, d, metric, opts);
    if (rc) return rc;
    if (A == nullptr || B == nullptr || !(eps > 0.0 && eps < 1.0)) return CHAMFER_EINVAL;
    if (ws == nullptr || ws_bytes < rp.total) return CHAMFER_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) return CHAMFER_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint64_t *kA = keys_A_out ? keys_A_out : at<uint64_t>(ws, rp.off_keysA);
    uint64_t *kB = keys_B_out ? keys_B_out : at<uint64_t>(ws, rp.off_keysB);
    if ((rc = run_reduce(rp, A, B, eps, seed, t_out, kA, kB, A_pad_out, B_pad_out, ws, st)))
        return rc;
    if (info_out)
        CH_TRY(hipMemcpyAsync(info_out, at<void>(ws, rp.off_info), sizeof(chamfer_reduction),
                              hipMemcpyDeviceToDevice, st));
    return CHAMFER_OK;
}

}  // extern "C"
