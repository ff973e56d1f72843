// One-vs-many retrieval (the downstream experiment of the paper: the
// nearest point cloud to A under CH(A, B) + CH(B, A) in a collection):
//   1. est_i = eta(A, B_i) + eta(B_i, A) for every cloud: two estimator jobs
//      per cloud, run up to 256 at a time through the batched stage kernels (one
//      launch per stage for the whole batch);
//   2. the k smallest est_i (ties to the lower i);
//   3. the exact CH(A, B_i) + CH(B_i, A) of those k, ranked ascending (ties
//      to the lower i).
// Workspace: the batch descriptor, the jobs' (shared) embedding, the per-job eta
// and per-cloud estimates, then one estimator workspace per batch slot, each
// sized for the largest cloud in either direction and for the exact
// re-rank's plans (which run in full precision whatever opts.precision).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"

using namespace chamfer;

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t batch, embed, eta, est, per_job_ws, jobs, total;
    size_t off_embed, off_eta, off_est, off_jobs;
    int slots;  // jobs per batch
};

// Job workspaces of one batch stay within this many bytes (large clouds get
// fewer jobs per batch; small ones fill the whole descriptor).
constexpr size_t kSlotBudget = size_t(4) << 30;

int valid_offsets(const int64_t *offsets, int32_t m) {
    if (offsets == nullptr || m < 1 || offsets[0] != 0) return 0;
    for (int i = 0; i < m; ++i)
        if (offsets[i + 1] <= offsets[i]) return 0;  // every cloud non-empty
    return 1;
}

int layout(Layout &lo, int64_t n_A, const int64_t *offsets, int32_t m, int32_t d, int32_t metric,
           double eps, int64_t T, const chamfer_opts *opts) {
    if (n_A < 1 || d < 1 || d > 2048 || !valid_offsets(offsets, m)) return CHAMFER_EINVAL;
    chamfer_opts o{};
    if (opts) o = *opts;
    if (o.window > 1 || o.reps > 1 || o.sampling != CHAMFER_IMPORTANCE) return CHAMFER_EINVAL;
    const int ke = o.embed_dim ? o.embed_dim : 32;
    chamfer_opts ox = o;  // the re-rank is exact: full precision
    ox.precision = CHAMFER_FP32;
    size_t maxws = 0;
    for (int i = 0; i < m; ++i) {
        const int64_t nb = offsets[i + 1] - offsets[i];
        const size_t w[4] = {chamfer_workspace_bytes(n_A, nb, d, metric, eps, T, &o),
                             chamfer_workspace_bytes(nb, n_A, d, metric, eps, T, &o),
                             chamfer_workspace_bytes(n_A, nb, d, metric, 0.0, 0, &ox),
                             chamfer_workspace_bytes(nb, n_A, d, metric, 0.0, 0, &ox)};
        for (size_t x : w) {
            if (x == 0) return CHAMFER_EINVAL;
            maxws = std::max(maxws, x);
        }
    }
    std::memset(&lo, 0, sizeof(lo));
    lo.batch = up(sizeof(Batch));
    // every job has the same seed and d, hence one embedding matrix (l2)
    lo.embed = metric == CHAMFER_L2 ? up(embed_bytes(d, ke)) : 0;
    lo.eta = up((size_t)2 * m * sizeof(double));
    lo.est = up((size_t)4 * m * sizeof(double));  // estimates, then [3] per candidate
    lo.per_job_ws = up(maxws);
    lo.slots = (int)std::max<size_t>(1, std::min<size_t>(kBatchMax, kSlotBudget / lo.per_job_ws));
    lo.jobs = lo.per_job_ws * lo.slots;
    lo.off_embed = lo.batch;
    lo.off_eta = lo.off_embed + lo.embed;
    lo.off_est = lo.off_eta + lo.eta;
    lo.off_jobs = lo.off_est + lo.est;
    lo.total = lo.off_jobs + lo.jobs;
    return CHAMFER_OK;
}

// est[i] = eta[2i] + eta[2i + 1]
__global__ void k_pair_sums(const double *eta, int32_t m, double *est) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) est[i] = eta[2 * i] + eta[2 * i + 1];
}

// Two host staging buffers for the batch descriptor: batch
// j is written into buffer j % 2 once the copy of batch j - 2 out of it has
// completed (an event after each copy), so host preparation of one batch
// overlaps the device work of the previous one.
struct Staging {
    std::vector<char> buf[2];
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    hipStream_t st = nullptr;
    ~Staging() {
        if (used[0] || used[1]) (void)hipStreamSynchronize(st);  // copies read buf
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Side streams of the exact re-rank, created once per device and kept for
// the process (default priority, non-blocking); the mutex serialises the
// fork/join sequences of concurrent calls.
constexpr int kRerankStreams = 3;
struct SideStreams {
    std::mutex mu;
    int device = -1;
    hipStream_t s[kRerankStreams] = {};
    hipEvent_t fork = nullptr, join[kRerankStreams] = {};
    bool ready() {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return false;
        if (device == dev) return true;
        if (device >= 0) return false;  // one device per set (see side_streams)
        for (int j = 0; j < kRerankStreams; ++j)
            if (hipStreamCreateWithFlags(&s[j], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&join[j], hipEventDisableTiming) != hipSuccess)
                return false;
        if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return false;
        device = dev;
        return true;
    }
};

// The set of the current device.
SideStreams &side_streams() {
    static std::mutex mu;
    static std::map<int, SideStreams *> sets;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> hold(mu);
    SideStreams *&set = sets[dev];
    if (!set) set = new SideStreams();  // lives for the process
    return *set;
}

#define CH_TRY(expr)                                    \
    do {                                                \
        if ((expr) != hipSuccess) return CHAMFER_EHIP;  \
    } while (0)

}  // namespace

extern "C" {

size_t chamfer_retrieve_workspace_bytes(int64_t n_A, const int64_t *offsets, int32_t m,
                                        int32_t d, int32_t metric, double eps, int64_t T,
                                        const chamfer_opts *opts) {
    Layout lo;
    if (layout(lo, n_A, offsets, m, d, metric, eps, T, opts) != CHAMFER_OK) return 0;
    return lo.total;
}

int chamfer_retrieve(const float *A, int64_t n_A, const float *Bs, const int64_t *offsets,
                     int32_t m, int32_t d, int32_t metric, double eps, int64_t T, uint64_t seed,
                     int32_t k, const chamfer_opts *opts, double *est_out, int32_t *top_out,
                     double *top_ch_out, void *ws, size_t ws_bytes, void *stream) {
    Layout lo;
    int rc = layout(lo, n_A, offsets, m, d, metric, eps, T, opts);
    if (rc) return rc;
    if (A == nullptr || Bs == nullptr || k < 1 || k > m || top_out == nullptr ||
        top_ch_out == nullptr)
        return CHAMFER_EINVAL;
    if (ws == nullptr || ws_bytes < lo.total) return CHAMFER_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) return CHAMFER_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    Batch *bt_dev = reinterpret_cast<Batch *>(base);
    double *eta = reinterpret_cast<double *>(base + lo.off_eta);
    double *est = est_out ? est_out : reinterpret_cast<double *>(base + lo.off_est);
    double *sym = reinterpret_cast<double *>(base + lo.off_est) + m;  // [3] per candidate
    chamfer_opts o{};
    if (opts) o = *opts;
    chamfer_opts ox = o;
    ox.precision = CHAMFER_FP32;
    const int ke = metric == CHAMFER_L2 ? (o.embed_dim ? o.embed_dim : 32) : 0;
    const int prec = lowp_supported(d, metric, o.precision) ? o.precision : CHAMFER_FP32;

    // 1. estimates, kBatchMax jobs per batch (job 2i: A -> B_i, job 2i + 1:
    // B_i -> A)
    Staging stg;
    stg.st = st;
    std::vector<int8_t> emb;  // read by the copy below before the stream drains
    if (metric == CHAMFER_L2) {
        emb.resize(embed_bytes(d, ke));
        embedding_packed(seed, d, ke, emb.data());
        CH_TRY(hipMemcpyAsync(base + lo.off_embed, emb.data(), emb.size(), hipMemcpyHostToDevice,
                              st));
    }
    for (int b = 0; b < 2; ++b) {
        stg.buf[b].resize(lo.batch);  // the batch descriptor
        CH_TRY(hipEventCreateWithFlags(&stg.ev[b], hipEventDisableTiming));
    }
    const int njobs = 2 * m;
    for (int j0 = 0; j0 < njobs; j0 += lo.slots) {
        const int nb = std::min(lo.slots, njobs - j0);
        const int hb = (j0 / lo.slots) & 1;
        if (stg.used[hb]) CH_TRY(hipEventSynchronize(stg.ev[hb]));
        std::vector<char> &host = stg.buf[hb];
        Batch *bh = reinterpret_cast<Batch *>(host.data());
        std::memset(bh, 0, sizeof(Batch));
        for (int s = 0; s < nb; ++s) {
            const int j = j0 + s, i = j / 2;
            const float *B = Bs + (size_t)offsets[i] * d;
            const int64_t nB = offsets[i + 1] - offsets[i];
            const bool fwd = (j & 1) == 0;
            chamfer_aux aux{};
            rc = job_prepare(fwd ? A : B, fwd ? B : A, fwd ? n_A : nB, fwd ? nB : n_A, d, metric,
                             eps, T, seed, opts, base + lo.off_jobs + (size_t)s * lo.per_job_ws,
                             lo.per_job_ws, eta + j, aux,
                             reinterpret_cast<const int8_t *>(base + lo.off_embed), nullptr,
                             &bh->job[s]);
            if (rc) return rc;
        }
        job_share_nn(bh->job, nb);
        int64_t acc[kBsCount] = {};
        for (int s = 0; s < nb; ++s) {
            int64_t blocks[kBsCount];
            job_stage_blocks(bh->job[s], blocks);
            for (int q = 0; q < kBsCount; ++q) {
                bh->start[q][s] = (int32_t)acc[q];
                acc[q] += blocks[q];
                if (acc[q] > INT32_MAX) return CHAMFER_EINVAL;
            }
        }
        bh->njobs = nb;
        for (int q = 0; q < kBsCount; ++q) bh->start[q][nb] = (int32_t)acc[q];
        // the device descriptor is reused by every batch: stream order keeps
        // this copy (its used part) behind the previous batch's kernels
        CH_TRY(hipMemcpyAsync(bt_dev, host.data(), offsetof(Batch, job) + (size_t)nb * sizeof(Job),
                              hipMemcpyHostToDevice, st));
        CH_TRY(hipEventRecord(stg.ev[hb], st));
        stg.used[hb] = true;
        if ((rc = launch_estimate_batch(bt_dev, d, metric, ke, prec, st))) return rc;
    }
    k_pair_sums<<<(m + 255) / 256, 256, 0, st>>>(eta, m, est);
    CH_TRY(hipGetLastError());

    // 2. the k smallest estimates
    std::vector<double> h_est(m);
    CH_TRY(hipMemcpyAsync(h_est.data(), est, (size_t)m * sizeof(double), hipMemcpyDeviceToHost,
                          st));
    CH_TRY(hipStreamSynchronize(st));
    for (double &v : h_est)
        if (std::isnan(v)) v = INFINITY;  // a cloud with a non-finite coordinate ranks last
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::partial_sort(order.begin(), order.begin() + k, order.end(), [&](int x, int y) {
        return h_est[x] < h_est[y] || (h_est[x] == h_est[y] && x < y);
    });

    // 3. exact symmetric CH of the candidates, each into its own [3] slot:
    // the candidates are dealt to side streams (forked from and joined back
    // into the caller's stream), stream j using job workspace slot j, so the
    // small kernels of several candidates run at once; one copy back
    {
        SideStreams &side = side_streams();
        std::lock_guard<std::mutex> hold(side.mu);
        const int ns = std::min(kRerankStreams, lo.slots);
        if (!side.ready()) return CHAMFER_EHIP;
        CH_TRY(hipEventRecord(side.fork, st));
        for (int j = 0; j < ns; ++j) CH_TRY(hipStreamWaitEvent(side.s[j], side.fork, 0));
        for (int c = 0; c < k && rc == CHAMFER_OK; ++c) {
            const int i = order[c], j = c % ns;
            const float *B = Bs + (size_t)offsets[i] * d;
            const int64_t nB = offsets[i + 1] - offsets[i];
            rc = chamfer_exact_symmetric(A, B, n_A, nB, d, metric, sym + 3 * c, &ox,
                                         base + lo.off_jobs + (size_t)j * lo.per_job_ws,
                                         lo.per_job_ws, side.s[j]);
        }
        for (int j = 0; j < ns; ++j) {
            if (hipEventRecord(side.join[j], side.s[j]) != hipSuccess ||
                hipStreamWaitEvent(st, side.join[j], 0) != hipSuccess) {
                for (int q = 0; q < ns; ++q) (void)hipStreamSynchronize(side.s[q]);
                return CHAMFER_EHIP;
            }
        }
        if (rc) {
            (void)hipStreamSynchronize(st);
            return rc;
        }
    }
    std::vector<double> v((size_t)3 * k);
    CH_TRY(hipMemcpyAsync(v.data(), sym, v.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CH_TRY(hipStreamSynchronize(st));
    std::vector<std::pair<double, int>> ranked;
    for (int c = 0; c < k; ++c)
        ranked.emplace_back(std::isnan(v[3 * c]) ? INFINITY : v[3 * c], order[c]);
    std::sort(ranked.begin(), ranked.end());
    for (int c = 0; c < k; ++c) {
        top_out[c] = ranked[c].second;
        top_ch_out[c] = ranked[c].first;
    }
    return CHAMFER_OK;
}

}  // extern "C"
