// libchamfer C ABI: argument checks, workspace layout and the launch
// sequence of each entry point.  All device work is enqueued on the
// caller's stream; nothing here waits for the device.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

using namespace chamfer;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int ceil_log2_u64(uint64_t n) {
    int q = 0;
    while (q < 63 && (1ull << q) < n) ++q;
    return q;
}

int ceil_log2_dbl(double x) {
    int e;
    const double m = std::frexp(x, &e);
    return m == 0.5 ? e - 1 : e;
}

}  // namespace

namespace chamfer {

// Host Philox4x64-10 (Salmon et al., SC 2011), for the embedding matrix.
void philox_host(uint64_t c[4], uint64_t k0, uint64_t k1) {
    for (int r = 0; r < 10; ++r) {
        const unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * c[0];
        const unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * c[2];
        const uint64_t x0 = (uint64_t)(p1 >> 64) ^ c[1] ^ k0;
        const uint64_t x2 = (uint64_t)(p0 >> 64) ^ c[3] ^ k1;
        c[1] = (uint64_t)p1;
        c[3] = (uint64_t)p0;
        c[0] = x0;
        c[2] = x2;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

// Zq_jk = clamp(rint(32 g_jk), -127, 127), g_jk by Box-Muller from the words
// of counter (j*d + k, 0, EMBED, 0): u1 = ((w0 >> 11) + 1) 2^-53 in (0, 1],
// u2 = (w1 >> 11) 2^-53, g = sqrt(-2 ln u1) cos(2 pi u2).  Row-major [ke][d]:
// the quantised Gaussian matrix of the l2 -> l1 embedding (the scale
// 1 / (beta ke 32), beta = sqrt(2/pi), is applied after the exact integer
// product).
void embedding_host(uint64_t seed, int d, int ke, int8_t *Z) {
    const double pi = 3.14159265358979323846;
    const double two_pi = 2.0 * pi;
    for (int j = 0; j < ke; ++j)
        for (int k = 0; k < d; ++k) {
            uint64_t c[4] = {(uint64_t)j * (uint64_t)d + (uint64_t)k, 0, kPurposeEmbed, 0};
            philox_host(c, seed, 0);
            const double u1 = std::ldexp((double)((c[0] >> 11) + 1), -53);
            const double u2 = std::ldexp((double)(c[1] >> 11), -53);
            const double g = std::sqrt(-2.0 * std::log(u1)) * std::cos(two_pi * u2);
            const double q = std::fmin(std::fmax(std::rint(32.0 * g), -127.0), 127.0);
            Z[(size_t)j * d + k] = (int8_t)q;
        }
}

size_t embed_bytes(int d, int ke) {
    const size_t nt = (size_t)(ke + 15) / 16, nks = (size_t)(d + 63) / 64;
    return nt * nks * 1024 + nt * 16 * sizeof(int32_t);
}

// The matrix in the operand layout of the hash kernels' int8 matrix-core
// embedding: for each 16-column tile t of j and 64-coordinate step s, lane
// l (= 16 g + i) holds the 16 bytes Zq[16 t + i][64 s + 16 g + e], e < 16
// (zero outside [ke] x [d]); then R_j = sum_k Zq_jk as int32 for the 16 nt
// columns.  embed_bytes(d, ke) bytes.
void embedding_packed(uint64_t seed, int d, int ke, int8_t *out) {
    thread_local std::vector<int8_t> z;
    z.resize((size_t)ke * d);
    embedding_host(seed, d, ke, z.data());
    const int nt = (ke + 15) / 16, nks = (d + 63) / 64;
    for (int t = 0; t < nt; ++t)
        for (int s = 0; s < nks; ++s)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 16; ++e) {
                    const int j = 16 * t + (l & 15), k = 64 * s + 16 * (l >> 4) + e;
                    out[((size_t)(t * nks + s) * 64 + l) * 16 + e] =
                        (j < ke && k < d) ? z[(size_t)j * d + k] : (int8_t)0;
                }
    int32_t *r = reinterpret_cast<int32_t *>(out + (size_t)nt * nks * 1024);
    for (int j = 0; j < 16 * nt; ++j) {
        int32_t acc = 0;
        if (j < ke)
            for (int k = 0; k < d; ++k) acc += z[(size_t)j * d + k];
        r[j] = acc;
    }
}

}  // namespace chamfer

namespace {

bool valid_ke(int ke) { return ke == 8 || ke == 16 || ke == 32 || ke == 64; }

int default_scales(int64_t nA, int64_t nB, double eps) {
    int64_t n = nA > nB ? nA : nB;
    if (n < 1) n = 1;
    int L = ceil_log2_dbl((double)n / eps);
    if (L < 1) L = 1;
    if (L > kMaxScales) L = kMaxScales;
    return L;
}

int64_t default_samples(int64_t nA, double eps) {
    const int q = ceil_log2_u64((uint64_t)(nA < 1 ? 1 : nA));
    const int64_t T = (int64_t)std::ceil((double)q / (eps * eps));
    return T < 1 ? 1 : T;
}

// Validate and lay out the workspace.  estimating: the entry point draws T
// points (needs eps, the weight, prefix and draw regions) and, with
// importance sampling, runs CrudeNN (the table regions); otherwise only the
// regions of the nearest-neighbour pass are laid out, so its total never
// exceeds the estimating total for the same sizes.
int make_plan(Plan &pl, int64_t nA, int64_t nB, int32_t d, int32_t metric, double eps,
              int64_t T, const chamfer_opts *opts, bool estimating) {
    const bool need_eps = estimating;
    std::memset(&pl, 0, sizeof(pl));
    if (d < 1 || (metric != CHAMFER_L1 && metric != CHAMFER_L2)) return CHAMFER_EINVAL;
    if (nA < 0 || nB < 1 || nA > INT32_MAX || nB > INT32_MAX || T < 0 || T > INT32_MAX)
        return CHAMFER_EINVAL;
    if (need_eps && !(eps > 0.0 && eps < 1.0)) return CHAMFER_EINVAL;
    chamfer_opts o{};
    if (opts) o = *opts;
    if (o.n_scales < 0 || o.n_scales > kMaxScales || o.reduction != 0) return CHAMFER_EINVAL;
    if (o.window < 0 || o.window > kMaxWindow || o.reps < 0 || o.reps > kMaxReps)
        return CHAMFER_EINVAL;
    if (o.sampling != CHAMFER_IMPORTANCE && o.sampling != CHAMFER_UNIFORM) return CHAMFER_EINVAL;
    const bool hashing = estimating && o.sampling == CHAMFER_IMPORTANCE;
    if (o.precision < CHAMFER_FP32 || o.precision > CHAMFER_FP8) return CHAMFER_EINVAL;
    const int ke = o.embed_dim ? o.embed_dim : 32;
    if (!valid_ke(ke)) return CHAMFER_EINVAL;
    const double e = (eps > 0.0 && eps < 1.0) ? eps : 0.5;
    pl.nA = nA;
    pl.nB = nB;
    pl.d = d;
    pl.metric = metric;
    pl.precision = o.precision;
    pl.window = o.window ? o.window : 1;
    pl.reps = o.reps ? o.reps : 1;
    pl.sampling = o.sampling;
    pl.L = o.n_scales ? o.n_scales : default_scales(nA, nB, e);
    pl.ke = ke;
    pl.kh = metric == CHAMFER_L1 ? d : ke;
    pl.T = T ? T : default_samples(nA, e);
    pl.q = ceil_log2_u64((uint64_t)(nA < 1 ? 1 : nA));
    int lc = ceil_log2_u64((uint64_t)(2 * nB));
    if (lc < 6) lc = 6;
    pl.log2cap = lc;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return at;
    };
    const int64_t nrow = (estimating && pl.T > nA) ? pl.T : nA;
    const size_t h = hashing ? 1 : 0, e_ = estimating ? 1 : 0;
    pl.off_params = take(sizeof(DevParams));
    pl.off_lohi = take(lohi_bytes(d));
    pl.off_zfrac = take(h * pl.L * pl.kh * sizeof(float));
    pl.off_mult = take(h * pl.L * pl.kh * sizeof(uint64_t));
    pl.off_embed = take(metric == CHAMFER_L2 ? h * embed_bytes(d, ke) : 0);
    pl.off_tables = take(h * table_bytes(pl.L, lc, pl.window));
    pl.part = hashing && pl.window == 1 && part_build_ok(lc);
    pl.off_part = take(pl.part ? part_work_bytes(pl.L, nB, lc) : 0);
    pl.off_D = take(e_ * nA * sizeof(float));
    pl.off_nn = take(h * nA * sizeof(int32_t));
    pl.off_scale = take(h * nA * sizeof(int32_t));
    pl.off_blocksums = take(e_ * ((nA + kScanBlock - 1) / kScanBlock + 1) * 8);
    pl.off_P = take(e_ * nA * sizeof(uint64_t));
    pl.off_idx = take(e_ * pl.T * sizeof(int32_t));
    pl.off_best = take((size_t)nrow * sizeof(uint64_t));
    pl.off_partial = take((size_t)(nn_finalize_blocks(nrow) + 1) * sizeof(double));
    pl.off_nb2 = take(mfma_supported(d, metric) ? (size_t)nB * sizeof(float) : 0);
    // low precision: cast rows of B and of the queries, scales and norms
    const bool lp = lowp_supported(d, metric, pl.precision);
    const bool split = !lp && mfma_supported(d, metric);
    pl.off_bsplit = take(split ? split_table_bytes(nB, d) : 0);
    pl.off_xsplit = take(split ? split_table_bytes(nrow, d) : 0);
    pl.off_xn2 = take(split ? (size_t)nrow * sizeof(float) : 0);
    // the deferred exact pass over the draws: its (draw, chunk) records live
    // in the hash tables' region when that is large enough (the tables are
    // done with before the draws are taken)
    const size_t srec = split && estimating ? split_record_bytes(pl.T, nB, d) : 0;
    pl.off_srec = h && srec <= table_bytes(pl.L, lc, pl.window) ? pl.off_tables : take(srec);
    const size_t rb = lp ? lowp_row_bytes(d, pl.precision) : 0;
    pl.off_bq = take(rb * (size_t)nB);
    pl.off_xq = take(rb * (size_t)nrow);
    pl.off_lpf = take(lp ? 2 * ((size_t)nB + (size_t)nrow) * sizeof(float) : 0);
    pl.total = off;
    return CHAMFER_OK;
}

template <class T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

#define CH_TRY(expr)                                    \
    do {                                                \
        if ((expr) != hipSuccess) return CHAMFER_EHIP;  \
    } while (0)

int check_ws(const Plan &pl, void *ws, size_t ws_bytes) {
    if (ws == nullptr || ws_bytes < pl.total) return CHAMFER_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) return CHAMFER_EINVAL;
    return CHAMFER_OK;
}

// Calibration, tables and (l2) the embedding upload: common prefix of the
// hashing entry points.
int hash_prologue(const Plan &pl, const float *A, const float *B, uint64_t seed, void *ws,
                  hipStream_t st) {
    DevParams *p = at<DevParams>(ws, pl.off_params);
    uint32_t *lohi = at<uint32_t>(ws, pl.off_lohi);
    // parameter block and the structure-0 shifts and multipliers in one
    // launch; the tables are emptied after the min/max pass (emptying them
    // first evicts A and B from the memory-side cache at 10^6 points)
    CH_TRY(launch_setup(p, lohi, pl.d, seed, pl.L, pl.kh, at<float>(ws, pl.off_zfrac),
                        at<uint64_t>(ws, pl.off_mult), nullptr, 0, st));
    if (pl.metric == CHAMFER_L2) {
        // The embedding matrix is drawn on the host (it needs log and cos in
        // double precision) and uploaded in the hash kernels' operand layout
        // from a buffer a later call may overwrite: a captured copy would
        // replay from it, so a capturing stream is refused.  The buffer keeps
        // the last (seed, d, k_e)'s matrix, which repeated calls reuse.
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        CH_TRY(hipStreamIsCapturing(st, &cs));
        if (cs != hipStreamCaptureStatusNone) return CHAMFER_EINVAL;
        thread_local std::vector<int8_t> zt;
        thread_local uint64_t zt_seed = 0;
        thread_local int zt_d = -1, zt_ke = -1;
        if (zt_d != pl.d || zt_ke != pl.ke || zt_seed != seed) {
            zt.resize(embed_bytes(pl.d, pl.ke));
            embedding_packed(seed, pl.d, pl.ke, zt.data());
            zt_seed = seed;
            zt_d = pl.d;
            zt_ke = pl.ke;
        }
        CH_TRY(hipMemcpyAsync(at<int8_t>(ws, pl.off_embed), zt.data(), zt.size(),
                              hipMemcpyHostToDevice, st));
    }
    CH_TRY(launch_minmax_pair(A, pl.nA, B, pl.nB, pl.d, lohi, p, st));
    CH_TRY(launch_calib_final(lohi, pl.d, p, st));
    return CHAMFER_OK;
}

// Record stage event i if the caller asked for stage events.
hipError_t mark(void **ev, int i, hipStream_t st) {
    if (ev == nullptr || ev[i] == nullptr) return hipSuccess;
    return hipEventRecord(static_cast<hipEvent_t>(ev[i]), st);
}

// CrudeNN into D/nn/scale.  nb2 (l2 only, may be null): |b|^2 per row of B,
// computed while B is bucketed, for the nearest-neighbour pass.  With k LSH
// structures (reps) the tables are rebuilt for each structure r (grid stream
// word r) and each probe keeps the better of its candidate and the stored
// one; with a window W the tables hold W points per bucket.
// nb2 given: the hash of B also fills |b|^2 and p->b2max_rep (inputs of the
// l2 exact pass).
int crude_core(const Plan &pl, const float *A, const float *B, uint64_t seed, float *D,
               int32_t *nn, int32_t *scale, void *ws, hipStream_t st, void **ev = nullptr,
               float *nb2 = nullptr, uint16_t *bsplit = nullptr) {
    // bsplit (l2 only, may be null): B's split table for the exact pass,
    // written by the kernel that hashes B (B is read once for both)
    const int sdp = bsplit ? split_dpad(pl.d) : 0;
    CH_TRY(mark(ev, 0, st));
    const int W = pl.window;
    int rc = hash_prologue(pl, A, B, seed, ws, st);
    if (rc) return rc;
    DevParams *p = at<DevParams>(ws, pl.off_params);
    Bucket *tables = at<Bucket>(ws, pl.off_tables);
    const uint32_t *lohi = at<uint32_t>(ws, pl.off_lohi);
    const int8_t *emb = at<int8_t>(ws, pl.off_embed);
    float *zf = at<float>(ws, pl.off_zfrac);
    uint64_t *mt = at<uint64_t>(ws, pl.off_mult);
    PartWork pw{};
    if (pl.part) part_work_bytes(pl.L, pl.nB, pl.log2cap, &pw, at<char>(ws, pl.off_part));
    for (int r = 0; r < pl.reps; ++r) {
        if (r > 0) CH_TRY(launch_grid_tables(seed, pl.L, pl.kh, zf, mt, r, st));
        if (pl.part) {
            // B's keys, then the tables built region by region in LDS (every
            // slot written, so no emptying pass)
            if (r == 0) CH_TRY(mark(ev, 1, st));
            CH_TRY(launch_hash(5, B, pl.nB, B, pl.nB, pl.d, pl.metric, pl.L, pl.ke, lohi, emb, zf,
                               mt, nullptr, pl.log2cap, pw.keys, nullptr, nullptr, nullptr,
                               r == 0 ? nb2 : nullptr, p, 1, 0, st, r == 0 ? bsplit : nullptr,
                               sdp));
            CH_TRY(launch_part_build(pw, pl.nB, pl.L, pl.log2cap, tables, st));
        } else {
            CH_TRY(launch_tables_empty(tables, pl.L, pl.log2cap, W, st));
            if (r == 0) CH_TRY(mark(ev, 1, st));
            CH_TRY(launch_hash(W == 1 ? 0 : 3, B, pl.nB, B, pl.nB, pl.d, pl.metric, pl.L, pl.ke,
                               lohi, emb, zf, mt, tables, pl.log2cap, nullptr, nullptr, nullptr,
                               nullptr, r == 0 ? nb2 : nullptr, p, W, 0, st,
                               r == 0 ? bsplit : nullptr, sdp));
        }
        if (r == 0) CH_TRY(mark(ev, 2, st));
        const int flags = (r > 0 ? kProbeMerge : 0) | (r == pl.reps - 1 ? kProbeLast : 0);
        CH_TRY(launch_hash(W == 1 ? 1 : 4, A, pl.nA, B, pl.nB, pl.d, pl.metric, pl.L, pl.ke, lohi,
                           emb, zf, mt, tables, pl.log2cap, nullptr, D, nn, scale, nullptr, p, W,
                           flags, st));
    }
    CH_TRY(mark(ev, 3, st));
    return CHAMFER_OK;
}

// Exact pass over queries (rows of X, or X[rows[q]]): the low-precision
// form when requested and supported, else the float32 result (split-BF16
// matrix cores for l2 when nb2 is given, vector ALU otherwise).  split_ready:
// the split tables of B and of the queries are already in the workspace.
// draws: X rows are the estimator's draws (the deferred split pass may use
// its record region).
int nn_pass(const Plan &pl, void *ws, const float *X, const int32_t *rows, int64_t nx,
            const float *B, int64_t nB, unsigned long long *best, float *nb2, DevParams *p,
            hipStream_t st, bool split_ready = false, bool draws = false) {
    if (lowp_supported(pl.d, pl.metric, pl.precision)) {
        uint8_t *bq = at<uint8_t>(ws, pl.off_bq);
        uint8_t *xq = at<uint8_t>(ws, pl.off_xq);
        float *lpf = at<float>(ws, pl.off_lpf);
        float *bsc = lpf, *bn2 = lpf + nB, *xsc = lpf + 2 * nB, *xn2 = xsc + nx;
        CH_TRY(launch_cast_rows(pl.precision, B, nullptr, nB, pl.d, bq, bsc, bn2, p, st));
        CH_TRY(launch_cast_rows(pl.precision, X, rows, nx, pl.d, xq, xsc, xn2, p, st));
        CH_TRY(launch_nnmin_lowp(pl.precision, xq, xsc, nx, X, rows, bq, bsc, bn2, B, nB, pl.d,
                                 best, p, st));
        return CHAMFER_OK;
    }
    if (nb2 != nullptr && mfma_supported(pl.d, pl.metric)) {
        uint16_t *bs = at<uint16_t>(ws, pl.off_bsplit);
        uint16_t *xs = at<uint16_t>(ws, pl.off_xsplit);
        float *xn2 = at<float>(ws, pl.off_xn2);
        if (!split_ready) {
            CH_TRY(launch_split_rows(B, nB, pl.d, bs, p, st));
            CH_TRY(launch_split_queries(X, rows, nx, pl.d, xs, xn2, p, st));
        }
        uint4 *rec = draws && split_record_bytes(nx, nB, pl.d) ? at<uint4>(ws, pl.off_srec)
                                                               : nullptr;
        CH_TRY(launch_nnmin_split(X, rows, nx, xs, xn2, B, bs, nB, pl.d, best, nb2, p, st, rec));
        return CHAMFER_OK;
    }
    CH_TRY(launch_nnmin(X, rows, nx, B, nB, pl.d, pl.metric, best, p, st));
    return CHAMFER_OK;
}

// out[0] = out[1] + out[2] (the two directions of a symmetric call).
__global__ void k_sum_pair(double *out) {
    if (threadIdx.x == 0) out[0] = out[1] + out[2];
}

__global__ void k_store_zero(double *out, int32_t *status) {
    if (threadIdx.x == 0) {
        if (out) *out = 0.0;
        if (status) *status = CHAMFER_OK;
    }
}

}  // namespace

// ------------------------------------------------------------ batching

namespace chamfer {

int job_prepare(const float *A, const float *B, int64_t nA, int64_t nB, int32_t d,
                int32_t metric, double eps, int64_t T, uint64_t seed, const chamfer_opts *opts,
                void *ws, size_t ws_bytes, double *eta, chamfer_aux aux, const int8_t *embed_dev,
                int8_t *embed_host, Job *job) {
    Plan pl;
    int rc = make_plan(pl, nA, nB, d, metric, eps, T, opts, true);
    if (rc) return rc;
    if (nA < 1 || d > 2048 || A == nullptr || B == nullptr || eta == nullptr || job == nullptr)
        return CHAMFER_EINVAL;
    // single structure, W = 1, importance sampling
    if (pl.window != 1 || pl.reps != 1 || pl.sampling != CHAMFER_IMPORTANCE) return CHAMFER_EINVAL;
    if (metric == CHAMFER_L2 && embed_dev == nullptr) return CHAMFER_EINVAL;
    if ((rc = check_ws(pl, ws, ws_bytes))) return rc;
    const bool lp = lowp_supported(d, metric, pl.precision);
    Job &J = *job;
    std::memset(&J, 0, sizeof(J));
    J.A = A;
    J.B = B;
    J.nA = nA;
    J.nB = nB;
    J.T = pl.T;
    J.seed = seed;
    J.d = d;
    J.metric = metric;
    J.L = pl.L;
    J.ke = pl.ke;
    J.kh = pl.kh;
    J.q = pl.q;
    J.log2cap = pl.log2cap;
    J.precision = lp ? pl.precision : CHAMFER_FP32;
    J.p = at<DevParams>(ws, pl.off_params);
    J.lohi = at<uint32_t>(ws, pl.off_lohi);
    J.zfrac = at<float>(ws, pl.off_zfrac);
    J.mult = at<uint64_t>(ws, pl.off_mult);
    J.embed = metric == CHAMFER_L2 ? embed_dev : nullptr;
    J.tables = at<Bucket>(ws, pl.off_tables);
    J.table_count = (int64_t)pl.L << pl.log2cap;
    J.D = at<float>(ws, pl.off_D);
    J.nn = at<int32_t>(ws, pl.off_nn);
    J.blocksums = at<unsigned long long>(ws, pl.off_blocksums);
    J.P = at<unsigned long long>(ws, pl.off_P);
    J.idx = at<int32_t>(ws, pl.off_idx);
    J.best = at<unsigned long long>(ws, pl.off_best);
    J.nb2 = mfma_supported(d, metric) ? at<float>(ws, pl.off_nb2) : nullptr;
    // low precision: the cast rows of B; float32 l2: the split table of B
    J.bq = lp ? at<uint8_t>(ws, pl.off_bq)
              : mfma_supported(d, metric) ? at<uint8_t>(ws, pl.off_bsplit) : nullptr;
    J.xq = lp ? at<uint8_t>(ws, pl.off_xq) : nullptr;
    J.lpf = lp ? at<float>(ws, pl.off_lpf) : nullptr;
    J.eta = eta;
    J.aux = aux;
    J.aux.stage_events = nullptr;
    // geometry: the block counts of the direct launches
    J.nb_init = (int32_t)init_blocks(d);
    J.nb_grid = (int32_t)grid_table_blocks(pl.L, pl.kh);
    J.nb_fill = (int32_t)table_fill_blocks((size_t)J.table_count);
    J.mm_vec4 = minmax_vec4(A, d) && minmax_vec4(B, d);
    int64_t blocks, stride;
    minmax_geom(nA, d, J.mm_vec4 != 0, &blocks, &stride);
    J.nb_mmA = (int32_t)blocks;
    J.mm_strideA = stride;
    minmax_geom(nB, d, J.mm_vec4 != 0, &blocks, &stride);
    J.nb_mmB = (int32_t)blocks;
    J.mm_strideB = stride;
    J.nb_hashB = (int32_t)hash_blocks(nB);
    J.nb_hashA = (int32_t)hash_blocks(nA);
    J.nb_scan = (int32_t)scan_blocks(nA);
    J.nb_sample = (int32_t)sample_blocks(pl.T);
    NNGeom g;
    if (lp) {
        J.nb_castB = (int32_t)cast_blocks(nB);
        J.nb_castX = (int32_t)cast_blocks(pl.T);
        g = lowp_geom(pl.T, nB, d, pl.precision);
    } else if (mfma_supported(d, metric)) {
        J.xsplit = at<uint16_t>(ws, pl.off_xsplit);
        J.xn2 = at<float>(ws, pl.off_xn2);
        J.nb_castB = (int32_t)split_blocks(nB, d);
        J.nb_castX = (int32_t)split_blocks(pl.T, d);
        g = split_geom(pl.T, nB, d);
    } else {
        g = valu_geom(pl.T, nB, d);
    }
    J.nn_chunk = g.chunk;
    J.nn_nchunk = g.nchunk;
    J.nb_nn = (int32_t)g.blocks;
    // embed_host NULL: the caller has staged this job's embedding already
    if (metric == CHAMFER_L2 && embed_host) embedding_packed(seed, d, pl.ke, embed_host);
    return CHAMFER_OK;
}

void job_stage_blocks(const Job &J, int64_t out[kBsCount]) {
    out[kBsSetup] = (int64_t)J.nb_init + J.nb_grid + J.nb_fill;
    out[kBsMinmax] = (int64_t)J.nb_mmA + J.nb_mmB;
    out[kBsCalib] = 1;
    out[kBsInsert] = J.nb_hashB;
    out[kBsProbe] = J.nb_hashA;
    out[kBsWsum] = J.nb_scan;
    out[kBsWscan] = 1;
    out[kBsSample] = J.nb_sample;
    out[kBsCast] = (int64_t)J.nb_castB + J.nb_castX;
    out[kBsNN] = J.nb_nn;
    out[kBsFinal] = 1;
}

void job_share_nn(Job *jobs, int n) {
    if (n <= 1) return;
    const Job &J0 = jobs[0];
    if (lowp_supported(J0.d, J0.metric, J0.precision)) return;
    const bool mfma = mfma_supported(J0.d, J0.metric);
    double total = 0.0;
    for (int j = 0; j < n; ++j) total += (double)jobs[j].T * (double)jobs[j].nB;
    const double target = mfma ? (double)split_target_wgs(J0.d) : (double)kValuTargetWGs;
    for (int j = 0; j < n; ++j) {
        Job &J = jobs[j];
        const double share = target * ((double)J.T * (double)J.nB) / total;
        const int64_t t = share < 1.0 ? 1 : (int64_t)std::ceil(share);
        const NNGeom g = mfma ? split_geom(J.T, J.nB, J.d, t) : valu_geom(J.T, J.nB, J.d, t);
        J.nn_chunk = g.chunk;
        J.nn_nchunk = g.nchunk;
        J.nb_nn = (int32_t)g.blocks;
    }
}

int launch_estimate_batch(const Batch *bt, int d, int metric, int ke, int precision,
                          hipStream_t st) {
    CH_TRY(launch_batch_setup(bt, st));
    CH_TRY(launch_batch_minmax(bt, d, st));
    CH_TRY(launch_batch_calib(bt, d, st));
    CH_TRY(launch_batch_hash(0, bt, d, metric, ke, st));
    CH_TRY(launch_batch_hash(1, bt, d, metric, ke, st));
    CH_TRY(launch_batch_weights(bt, st));
    CH_TRY(launch_batch_sample(bt, st));
    if (lowp_supported(d, metric, precision))
        CH_TRY(launch_batch_cast(bt, d, precision, st));
    else if (mfma_supported(d, metric))
        CH_TRY(launch_batch_split_rows(bt, st));
    CH_TRY(launch_batch_nn(bt, d, metric, precision, st));
    CH_TRY(launch_batch_final(bt, metric, st));
    return CHAMFER_OK;
}

}  // namespace chamfer

// ------------------------------------------------------ static scratch
// The workspace of chamfer_estimate_noalloc: one array per device, loaded
// with the code object and kept until the process ends.  Host code never
// passes the array's name to a kernel or a copy: it takes the device
// address from hipGetSymbolAddress, once per device with that device
// current, and uses only that address.

static __device__ __align__(256) uint8_t scratch[CHAMFER_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of `scratch` on the device of `st`.
int scratch_for_stream(hipStream_t st, void **out) {
    int dev = 0, cur = 0;
    if (hipStreamGetDevice(st, &dev) != hipSuccess || hipGetDevice(&cur) != hipSuccess)
        return CHAMFER_EHIP;
    if (dev < 0 || dev >= kMaxScratchDevices) return CHAMFER_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        if (dev != cur && hipSetDevice(dev) != hipSuccess) return CHAMFER_EHIP;
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (dev != cur && hipSetDevice(cur) != hipSuccess) return CHAMFER_EHIP;
        if (e != hipSuccess || ptr == nullptr) return CHAMFER_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CHAMFER_OK;
}

}  // namespace

extern "C" {

size_t chamfer_workspace_bytes(int64_t n_A, int64_t n_B, int32_t d, int32_t metric, double eps,
                               int64_t T, const chamfer_opts *opts) {
    if (opts && opts->reduction != CHAMFER_REDUCE_NONE)
        return reduced_workspace_bytes(n_A, n_B, d, metric, eps, T, opts);
    Plan pl;
    // Without a valid eps only the non-estimating entry points can run.
    const bool estimating = eps > 0.0 && eps < 1.0;
    if (make_plan(pl, n_A, n_B, d, metric, eps, T, opts, estimating) != CHAMFER_OK) return 0;
    return pl.total;
}

int chamfer_exact(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                  int32_t metric, double *ch_out, float *rowmin_out, int32_t *rownn_out,
                  const chamfer_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    Plan pl;
    int rc = make_plan(pl, n_A, n_B, d, metric, 0.5, 0, opts, false);
    if (rc) return rc;
    if (ch_out == nullptr || (A == nullptr && n_A > 0) || B == nullptr) return CHAMFER_EINVAL;
    if ((rc = check_ws(pl, ws, ws_bytes))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_A == 0) {
        k_store_zero<<<1, 64, 0, st>>>(ch_out, nullptr);
        return hipGetLastError() == hipSuccess ? CHAMFER_OK : CHAMFER_EHIP;
    }
    DevParams *p = at<DevParams>(ws, pl.off_params);
    uint32_t *lohi = at<uint32_t>(ws, pl.off_lohi);
    auto *best = at<unsigned long long>(ws, pl.off_best);
    double *partial = at<double>(ws, pl.off_partial);
    CH_TRY(launch_init_params(p, lohi, d, st));
    CH_TRY(launch_minmax_pair(A, n_A, B, n_B, d, lohi, p, st));
    CH_TRY(launch_calib_final(lohi, d, p, st));
    CH_TRY(launch_fill_u64(best, n_A, ~0ull, st));
    float *nb2 = nullptr;
    const bool lp = lowp_supported(d, metric, pl.precision);
    if (!lp && mfma_supported(d, metric)) {
        nb2 = at<float>(ws, pl.off_nb2);
        CH_TRY(launch_rownorm(B, n_B, d, nb2, p, st));
    }
    if ((rc = nn_pass(pl, ws, A, nullptr, n_A, B, n_B, best, nb2, p, st))) return rc;
    CH_TRY(launch_nn_finalize(best, n_A, metric, rowmin_out, rownn_out, partial, p, st));
    CH_TRY(launch_sum_final(partial, nn_finalize_blocks(n_A), p, ch_out, st));
    return CHAMFER_OK;
}

int chamfer_nn_min(const float *X, const int32_t *rows, int64_t n_x, const float *B,
                   int64_t n_B, int32_t d, int32_t metric, float *min_out, int32_t *arg_out,
                   const chamfer_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    Plan pl;
    int rc = make_plan(pl, n_x, n_B, d, metric, 0.5, 0, opts, false);
    if (rc) return rc;
    if ((X == nullptr && n_x > 0) || B == nullptr) return CHAMFER_EINVAL;
    if ((rc = check_ws(pl, ws, ws_bytes))) return rc;
    if (n_x == 0) return CHAMFER_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevParams *p = at<DevParams>(ws, pl.off_params);
    auto *best = at<unsigned long long>(ws, pl.off_best);
    CH_TRY(launch_init_params(p, nullptr, d, st));
    CH_TRY(launch_fill_u64(best, n_x, ~0ull, st));
    float *nb2 = nullptr;
    const bool lp = lowp_supported(d, metric, pl.precision);
    if (!lp && mfma_supported(d, metric)) {
        nb2 = at<float>(ws, pl.off_nb2);
        CH_TRY(launch_rownorm(B, n_B, d, nb2, p, st));
    }
    if ((rc = nn_pass(pl, ws, X, rows, n_x, B, n_B, best, nb2, p, st))) return rc;
    CH_TRY(launch_nn_finalize(best, n_x, metric, min_out, arg_out, nullptr, p, st));
    return CHAMFER_OK;
}

int crude_nn(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
             int32_t metric, double eps, uint64_t seed, float *D_out, int32_t *nn_out,
             int32_t *scale_out, const chamfer_opts *opts, void *ws, size_t ws_bytes,
             void *stream) {
    Plan pl;
    int rc = make_plan(pl, n_A, n_B, d, metric, eps, 0, opts, true);
    if (rc) return rc;
    if ((A == nullptr && n_A > 0) || B == nullptr ||
        (n_A > 0 && (D_out == nullptr || nn_out == nullptr)) ||
        pl.sampling != CHAMFER_IMPORTANCE)
        return CHAMFER_EINVAL;
    if ((rc = check_ws(pl, ws, ws_bytes))) return rc;
    if (n_A == 0) return CHAMFER_OK;
    return crude_core(pl, A, B, seed, D_out, nn_out, scale_out, ws,
                      static_cast<hipStream_t>(stream));
}

int chamfer_estimate(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                     int32_t metric, double eps, int64_t T, uint64_t seed, double *eta_out,
                     chamfer_aux *aux, const chamfer_opts *opts, void *ws, size_t ws_bytes,
                     void *stream) {
    if (opts && opts->reduction != CHAMFER_REDUCE_NONE)
        return estimate_reduced(A, B, n_A, n_B, d, metric, eps, T, seed, eta_out, aux, opts, ws,
                                ws_bytes, stream);
    Plan pl;
    int rc = make_plan(pl, n_A, n_B, d, metric, eps, T, opts, true);
    if (rc) return rc;
    if ((A == nullptr && n_A > 0) || B == nullptr || eta_out == nullptr) return CHAMFER_EINVAL;
    if ((rc = check_ws(pl, ws, ws_bytes))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    chamfer_aux ax{};
    if (aux) ax = *aux;
    if (n_A == 0) {
        k_store_zero<<<1, 64, 0, st>>>(eta_out, ax.status);
        return hipGetLastError() == hipSuccess ? CHAMFER_OK : CHAMFER_EHIP;
    }
    float *D = ax.crude_D ? ax.crude_D : at<float>(ws, pl.off_D);
    int32_t *scale = ax.crude_scale;
    void **ev = ax.stage_events;
    float *nb2 = mfma_supported(d, metric) ? at<float>(ws, pl.off_nb2) : nullptr;
    uint16_t *bsplit = nb2 && !lowp_supported(d, metric, pl.precision)
                           ? at<uint16_t>(ws, pl.off_bsplit)
                           : nullptr;
    DevParams *p = at<DevParams>(ws, pl.off_params);
    if (pl.sampling == CHAMFER_UNIFORM) {
        // the baseline: no CrudeNN, every D_a = 1 (inputs still checked)
        uint32_t *lohi = at<uint32_t>(ws, pl.off_lohi);
        CH_TRY(mark(ev, 0, st));
        CH_TRY(launch_init_params(p, lohi, d, st));
        CH_TRY(launch_minmax_pair(A, n_A, B, n_B, d, lohi, p, st));
        CH_TRY(launch_calib_final(lohi, d, p, st));
        CH_TRY(mark(ev, 1, st));
        if (bsplit) CH_TRY(launch_rownorm(B, n_B, d, nb2, p, st));
        CH_TRY(mark(ev, 2, st));
        CH_TRY(launch_unit_weights(D, ax.crude_nn, scale, n_A, p, st));
        CH_TRY(mark(ev, 3, st));
    } else {
        int32_t *nn = ax.crude_nn ? ax.crude_nn : at<int32_t>(ws, pl.off_nn);
        if ((rc = crude_core(pl, A, B, seed, D, nn, scale, ws, st, ev, nb2, bsplit))) return rc;
    }
    uint64_t *P = at<uint64_t>(ws, pl.off_P);  // in-block prefixes of the weights
    int32_t *idx = at<int32_t>(ws, pl.off_idx);
    auto *best = at<unsigned long long>(ws, pl.off_best);
    CH_TRY(launch_weights(D, n_A, pl.q, at<uint64_t>(ws, pl.off_blocksums), P, p, st));
    CH_TRY(launch_sample(seed, P, at<uint64_t>(ws, pl.off_blocksums), n_A, pl.T, pl.q, idx, best,
                         p, st));
    CH_TRY(mark(ev, 4, st));
    // the split table of the draws (part of the exact pass); B's was written
    // while B was hashed, except for the uniform baseline, which does not
    // hash B
    if (bsplit) {
        if (pl.sampling == CHAMFER_UNIFORM) CH_TRY(launch_split_rows(B, n_B, d, bsplit, p, st));
        CH_TRY(launch_split_queries(A, idx, pl.T, d, at<uint16_t>(ws, pl.off_xsplit),
                                    at<float>(ws, pl.off_xn2), p, st));
    }
    if ((rc = nn_pass(pl, ws, A, idx, pl.T, B, n_B, best, nb2, p, st, bsplit != nullptr, true)))
        return rc;
    CH_TRY(mark(ev, 5, st));
    CH_TRY(launch_estimate_final(best, idx, D, pl.T, metric, p, eta_out, ax, st));
    CH_TRY(mark(ev, 6, st));
    return CHAMFER_OK;
}

int chamfer_estimate_noalloc(const float *A, const float *B, int64_t n_A, int64_t n_B,
                             int32_t d, int32_t metric, double eps, int64_t T, uint64_t seed,
                             double *eta_out, chamfer_aux *aux, const chamfer_opts *opts,
                             void *stream) {
    if (opts && opts->reduction != CHAMFER_REDUCE_NONE) return CHAMFER_EINVAL;
    Plan pl;
    int rc = make_plan(pl, n_A, n_B, d, metric, eps, T, opts, true);
    if (rc) return rc;
    if (pl.total > (size_t)CHAMFER_STATIC_SCRATCH_BYTES) return CHAMFER_ETOOLARGE;
    void *ws = nullptr;
    if ((rc = scratch_for_stream(static_cast<hipStream_t>(stream), &ws))) return rc;
    return chamfer_estimate(A, B, n_A, n_B, d, metric, eps, T, seed, eta_out, aux, opts, ws,
                            (size_t)CHAMFER_STATIC_SCRATCH_BYTES, stream);
}

int chamfer_hash_keys(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                      int32_t metric, double eps, uint64_t seed, uint64_t *keys_A_out,
                      uint64_t *keys_B_out, int32_t *e_top_out, const chamfer_opts *opts,
                      void *ws, size_t ws_bytes, void *stream) {
    Plan pl;
    int rc = make_plan(pl, n_A, n_B, d, metric, eps, 0, opts, true);
    if (rc) return rc;
    if ((A == nullptr && n_A > 0) || B == nullptr || pl.sampling != CHAMFER_IMPORTANCE)
        return CHAMFER_EINVAL;
    if ((rc = check_ws(pl, ws, ws_bytes))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = hash_prologue(pl, A, B, seed, ws, st))) return rc;
    DevParams *p = at<DevParams>(ws, pl.off_params);
    const uint32_t *lohi = at<uint32_t>(ws, pl.off_lohi);
    const int8_t *emb = at<int8_t>(ws, pl.off_embed);
    const float *zf = at<float>(ws, pl.off_zfrac);
    const uint64_t *mt = at<uint64_t>(ws, pl.off_mult);
    if (keys_A_out)
        CH_TRY(launch_hash(2, A, n_A, B, n_B, d, metric, pl.L, pl.ke, lohi, emb, zf, mt, nullptr,
                           pl.log2cap, keys_A_out, nullptr, nullptr, nullptr, nullptr, p, 1, 0,
                           st));
    if (keys_B_out)
        CH_TRY(launch_hash(2, B, n_B, B, n_B, d, metric, pl.L, pl.ke, lohi, emb, zf, mt, nullptr,
                           pl.log2cap, keys_B_out, nullptr, nullptr, nullptr, nullptr, p, 1, 0,
                           st));
    if (e_top_out) {
        // e_top lives in the device parameter block.
        CH_TRY(hipMemcpyAsync(e_top_out, &p->e_top, sizeof(int32_t), hipMemcpyDeviceToDevice,
                              st));
    }
    return CHAMFER_OK;
}

int chamfer_estimate_symmetric(const float *A, const float *B, int64_t n_A, int64_t n_B,
                               int32_t d, int32_t metric, double eps, int64_t T, uint64_t seed,
                               double *eta_out, const chamfer_opts *opts, void *ws,
                               size_t ws_bytes, void *stream) {
    if (n_A < 1 || n_B < 1 || eta_out == nullptr) return CHAMFER_EINVAL;
    Plan ab, ba;
    int rc = make_plan(ab, n_A, n_B, d, metric, eps, T, opts, true);
    if (rc || (rc = make_plan(ba, n_B, n_A, d, metric, eps, T, opts, true))) return rc;
    if (ws == nullptr || ws_bytes < ab.total || ws_bytes < ba.total) return CHAMFER_EWORKSPACE;
    rc = chamfer_estimate(A, B, n_A, n_B, d, metric, eps, T, seed, eta_out + 1, nullptr, opts, ws,
                          ws_bytes, stream);
    if (rc) return rc;
    rc = chamfer_estimate(B, A, n_B, n_A, d, metric, eps, T, seed, eta_out + 2, nullptr, opts, ws,
                          ws_bytes, stream);
    if (rc) return rc;
    k_sum_pair<<<1, 64, 0, static_cast<hipStream_t>(stream)>>>(eta_out);
    return hipGetLastError() == hipSuccess ? CHAMFER_OK : CHAMFER_EHIP;
}

int chamfer_exact_symmetric(const float *A, const float *B, int64_t n_A, int64_t n_B, int32_t d,
                            int32_t metric, double *ch_out, const chamfer_opts *opts, void *ws,
                            size_t ws_bytes, void *stream) {
    if (n_A < 1 || n_B < 1 || ch_out == nullptr) return CHAMFER_EINVAL;
    Plan ab, ba;
    int rc = make_plan(ab, n_A, n_B, d, metric, 0.5, 0, opts, false);
    if (rc || (rc = make_plan(ba, n_B, n_A, d, metric, 0.5, 0, opts, false))) return rc;
    if (ws == nullptr || ws_bytes < ab.total || ws_bytes < ba.total) return CHAMFER_EWORKSPACE;
    rc = chamfer_exact(A, B, n_A, n_B, d, metric, ch_out + 1, nullptr, nullptr, opts, ws, ws_bytes,
                       stream);
    if (rc) return rc;
    rc = chamfer_exact(B, A, n_B, n_A, d, metric, ch_out + 2, nullptr, nullptr, opts, ws, ws_bytes,
                       stream);
    if (rc) return rc;
    k_sum_pair<<<1, 64, 0, static_cast<hipStream_t>(stream)>>>(ch_out);
    return hipGetLastError() == hipSuccess ? CHAMFER_OK : CHAMFER_EHIP;
}

int64_t chamfer_default_samples(int64_t n_A, double eps) {
    if (!(eps > 0.0 && eps < 1.0)) return -1;
    return default_samples(n_A, eps);
}

int32_t chamfer_default_scales(int64_t n_A, int64_t n_B, double eps) {
    if (!(eps > 0.0 && eps < 1.0)) return -1;
    return default_scales(n_A, n_B, eps);
}

int chamfer_embedding_matrix(uint64_t seed, int32_t d, int32_t embed_dim, int8_t *Z_host) {
    if (d < 1 || !valid_ke(embed_dim) || Z_host == nullptr) return CHAMFER_EINVAL;
    embedding_host(seed, d, embed_dim, Z_host);
    return CHAMFER_OK;
}

const char *chamfer_strerror(int status) {
    switch (status) {
        case CHAMFER_OK: return "ok";
        case CHAMFER_EINVAL: return "invalid argument";
        case CHAMFER_EWORKSPACE: return "workspace missing or too small";
        case CHAMFER_EHIP: return "HIP launch or runtime error";
        case CHAMFER_ENONFINITE: return "input contains NaN or Inf";
        case CHAMFER_ETOOLARGE:
            return "problem needs more workspace than the static scratch buffer holds";
        default: return "unknown status";
    }
}

}  // extern "C"
