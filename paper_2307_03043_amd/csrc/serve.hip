// Serving runtime: continuous batching of chamfer_estimate requests.
//
// A server owns one device arena (allocated once at creation) and a few
// batch lanes.  A lane runs one batch at a time on its own stream (default
// priority) and holds a device batch descriptor (the Job of every request:
// workspace regions, outputs, block counts), pinned staging for it, the
// requests' outputs and one instantiated HIP graph per request class
// (d, metric, k_e, effective precision).
//
// Requests are queued on the host.  progress() retires finished batches
// (their arena blocks and lanes are free at once) and, while a lane is free,
// forms the next batch: the first of the kLookahead + 1 oldest requests
// whose footprint (two point sets and the workspace of
// chamfer_workspace_bytes) fits the arena sets the class; when that is the
// oldest request, up to kServeBatchMax queued requests of the same class from the
// first kWindow that fit join it.  The members' inputs and the descriptor
// are copied in on the lane's stream, then the class graph is replayed:
// each stage of the estimator (calibration, shifts and tables, bucket
// insert, probe, weights, sampling, the exact pass, the final sum) is ONE
// persistent-grid launch over all members (batch_loop), so a batch of 60
// small requests costs the same 12 launches as one.  The graph is captured
// once per lane and class; its kernels read the lane's descriptor, whose
// contents change from batch to batch.  Every member's blocks are exactly
// the blocks of its direct launches, so a result is the same alone and in
// any batch.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace chamfer;

namespace {

constexpr size_t kArenaAlign = 256;
constexpr int kLookahead = 8;              // requests past the head that may set the class
constexpr int kWindow = 256;               // queued requests scanned to fill a batch
// Requests per served batch: fewer than a descriptor holds, so that under
// load a few lanes interleave batches instead of one batch holding most of
// the arena (measured: 64 serves a saturated stream ~20% faster than 256)
constexpr int kServeBatchMax = 64;
constexpr size_t kEmbedBudget = 4u << 20;  // embedding bytes per batch (l2)
constexpr int kMaxLanes = 16;
constexpr int kDefaultKe = 32;

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

size_t round_up(size_t x) { return (x + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
   public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

   private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;
};

// Requests of one class share a captured graph (same kernels, same
// dynamic LDS); the effective precision is FP32 where the low-precision
// pass does not apply.
struct ClassKey {
    int32_t d, metric, ke, precision;
    bool operator<(const ClassKey &o) const {
        return std::tie(d, metric, ke, precision) < std::tie(o.d, o.metric, o.ke, o.precision);
    }
    bool operator==(const ClassKey &o) const {
        return d == o.d && metric == o.metric && ke == o.ke && precision == o.precision;
    }
};

struct Pending {
    uint64_t id;
    chamfer_request req;
    double submit_s;
    size_t footprint, ws_bytes, embed_bytes;
    ClassKey key;
};

// Outputs of one request, written by the final stage.
struct Out {
    double eta;
    double D;
    uint64_t W;
    int32_t s;
    int32_t status;
};

struct Member {
    Pending job;
    size_t off;  // arena offset of A | B | workspace
};

// Lane device buffer: Batch | embeddings (kEmbedBudget) | Out[kBatchMax].
constexpr size_t kBatchBytes = (sizeof(Batch) + 255) / 256 * 256;
constexpr size_t kOutOff = kBatchBytes + kEmbedBudget;
constexpr size_t kLaneBytes = kOutOff + kBatchMax * sizeof(Out);

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    double admit_s = 0.0;
    std::vector<Member> members;
    char *dev = nullptr;      // device: Batch | embeddings | outputs
    char *host = nullptr;     // pinned: Batch | embeddings
    Out *out_host = nullptr;  // pinned copy of the outputs
    std::map<ClassKey, hipGraphExec_t> graphs;
};

}  // namespace

struct chamfer_server {
    char *arena_base = nullptr;
    Arena *arena = nullptr;
    std::vector<Lane> lanes;
    hipStream_t capture = nullptr;
    std::deque<Pending> queue;
    std::vector<chamfer_result> done;
    uint64_t next_id = 1;
    size_t peak_used = 0;
    int32_t in_flight = 0;
    int64_t batches = 0, batched = 0, graphs = 0, stalls = 0;
};

namespace {

size_t footprint_of(const chamfer_request &r, size_t *ws_bytes) {
    *ws_bytes = chamfer_workspace_bytes(r.n_A, r.n_B, r.d, r.metric, r.eps, r.T, &r.opts);
    if (*ws_bytes == 0) return 0;
    const size_t pa = round_up((size_t)r.n_A * r.d * sizeof(float));
    const size_t pb = round_up((size_t)r.n_B * r.d * sizeof(float));
    return pa + pb + round_up(*ws_bytes);
}

ClassKey class_of(const chamfer_request &r) {
    ClassKey k;
    k.d = r.d;
    k.metric = r.metric;
    k.ke = r.metric == CHAMFER_L2 ? (r.opts.embed_dim ? r.opts.embed_dim : kDefaultKe) : 0;
    k.precision = lowp_supported(r.d, r.metric, r.opts.precision) ? r.opts.precision
                                                                  : (int32_t)CHAMFER_FP32;
    return k;
}

chamfer_result result_of(const Pending &p, int status, double admit_s) {
    chamfer_result res{};
    res.id = p.id;
    res.status = status;
    res.submit_s = p.submit_s;
    res.admit_s = admit_s;
    res.done_s = now_s();
    res.footprint = p.footprint;
    return res;
}

// The class graph of a lane, captured and instantiated on first use.
hipGraphExec_t graph_for(chamfer_server *s, Lane &ln, const ClassKey &k) {
    auto it = ln.graphs.find(k);
    if (it != ln.graphs.end()) return it->second;
    if (hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return nullptr;
    const int rc = launch_estimate_batch(reinterpret_cast<const Batch *>(ln.dev), k.d, k.metric,
                                         k.ke, k.precision, s->capture);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->capture, &g);
    if (rc != CHAMFER_OK || e != hipSuccess || g == nullptr) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return nullptr;
    ln.graphs[k] = x;
    ++s->graphs;
    return x;
}

// Fail every member of a lane that could not be launched.
void fail_lane(chamfer_server *s, Lane &ln, int status) {
    (void)hipStreamSynchronize(ln.stream);
    for (auto &m : ln.members) {
        s->done.push_back(result_of(m.job, status, ln.admit_s));
        s->arena->release(m.off, m.job.footprint);
    }
    s->in_flight -= (int32_t)ln.members.size();
    ln.members.clear();
    ln.busy = false;
}

// Build the descriptor of the lane's members, copy inputs and descriptor
// in, replay the class graph and copy the outputs back.
int launch_lane(chamfer_server *s, Lane &ln, const ClassKey &key) {
    Batch *bh = reinterpret_cast<Batch *>(ln.host);
    int64_t acc[kBsCount] = {};
    size_t eoff = kBatchBytes;
    std::vector<Member> kept;
    kept.reserve(ln.members.size());
    for (auto &m : ln.members) {
        const chamfer_request &r = m.job.req;
        const int j = (int)kept.size();
        char *base = s->arena_base + m.off;
        const size_t pa = round_up((size_t)r.n_A * r.d * sizeof(float));
        const size_t pb = round_up((size_t)r.n_B * r.d * sizeof(float));
        float *A = reinterpret_cast<float *>(base);
        float *B = reinterpret_cast<float *>(base + pa);
        void *ws = base + pa + pb;
        Out *od = reinterpret_cast<Out *>(ln.dev + kOutOff) + j;
        chamfer_aux aux{};
        aux.D = &od->D;
        aux.W = &od->W;
        aux.s = &od->s;
        aux.status = &od->status;
        int rc = job_prepare(A, B, r.n_A, r.n_B, r.d, r.metric, r.eps, r.T, r.seed, &r.opts, ws,
                             m.job.ws_bytes, &od->eta, aux,
                             reinterpret_cast<const int8_t *>(ln.dev + eoff),
                             reinterpret_cast<int8_t *>(ln.host + eoff), &bh->job[j]);
        if (rc != CHAMFER_OK) {
            s->done.push_back(result_of(m.job, rc, ln.admit_s));
            s->arena->release(m.off, m.job.footprint);
            --s->in_flight;
            continue;
        }
        eoff += m.job.embed_bytes;
        kept.push_back(m);
    }
    ln.members.swap(kept);
    job_share_nn(bh->job, (int)ln.members.size());
    // block prefix of every stage; members past the int32 range are refused
    kept.clear();
    int n = 0;
    for (size_t i = 0; i < ln.members.size(); ++i) {
        int64_t blocks[kBsCount];
        job_stage_blocks(bh->job[i], blocks);
        bool fits = true;
        for (int st = 0; st < kBsCount; ++st) fits &= acc[st] + blocks[st] <= INT32_MAX;
        if (!fits) {
            const Member &m = ln.members[i];
            s->done.push_back(result_of(m.job, CHAMFER_EINVAL, ln.admit_s));
            s->arena->release(m.off, m.job.footprint);
            --s->in_flight;
            continue;
        }
        if ((int)i != n) {
            bh->job[n] = bh->job[i];
            Out *od = reinterpret_cast<Out *>(ln.dev + kOutOff) + n;  // outputs follow the job
            bh->job[n].eta = &od->eta;
            bh->job[n].aux.D = &od->D;
            bh->job[n].aux.W = &od->W;
            bh->job[n].aux.s = &od->s;
            bh->job[n].aux.status = &od->status;
        }
        for (int st = 0; st < kBsCount; ++st) {
            bh->start[st][n] = (int32_t)acc[st];
            acc[st] += blocks[st];
        }
        kept.push_back(ln.members[i]);
        ++n;
    }
    ln.members.swap(kept);
    if (n == 0) {
        ln.busy = false;
        return CHAMFER_OK;
    }
    bh->njobs = n;
    for (int st = 0; st < kBsCount; ++st) bh->start[st][n] = (int32_t)acc[st];

    hipGraphExec_t gx = graph_for(s, ln, key);
    if (gx == nullptr) return CHAMFER_EHIP;
    for (int j = 0; j < n; ++j) {
        const Job &J = bh->job[j];
        const chamfer_request &r = ln.members[j].job.req;
        if (hipMemcpyAsync(const_cast<float *>(J.A), r.A, (size_t)r.n_A * r.d * sizeof(float),
                           hipMemcpyHostToDevice, ln.stream) != hipSuccess ||
            hipMemcpyAsync(const_cast<float *>(J.B), r.B, (size_t)r.n_B * r.d * sizeof(float),
                           hipMemcpyHostToDevice, ln.stream) != hipSuccess)
            return CHAMFER_EHIP;
    }
    // the used part of the descriptor (header, block prefixes, n jobs), then
    // the batch's embeddings
    const size_t used = offsetof(Batch, job) + (size_t)n * sizeof(Job);
    if (hipMemcpyAsync(ln.dev, ln.host, used, hipMemcpyHostToDevice, ln.stream) != hipSuccess ||
        (eoff > kBatchBytes &&
         hipMemcpyAsync(ln.dev + kBatchBytes, ln.host + kBatchBytes, eoff - kBatchBytes,
                        hipMemcpyHostToDevice, ln.stream) != hipSuccess) ||
        hipGraphLaunch(gx, ln.stream) != hipSuccess ||
        hipMemcpyAsync(ln.out_host, ln.dev + kOutOff, n * sizeof(Out), hipMemcpyDeviceToHost,
                       ln.stream) != hipSuccess ||
        hipEventRecord(ln.done, ln.stream) != hipSuccess)
        return CHAMFER_EHIP;
    ++s->batches;
    s->batched += n;
    return CHAMFER_OK;
}

Lane *free_lane(chamfer_server *s) {
    for (auto &ln : s->lanes)
        if (!ln.busy) return &ln;
    return nullptr;
}

int admit(chamfer_server *s) {
    int admitted = 0;
    for (;;) {
        Lane *ln = free_lane(s);
        if (ln == nullptr || s->queue.empty()) return admitted;
        // the class: first request of the head window that fits
        const int look = (int)std::min<size_t>(s->queue.size(), kLookahead + 1);
        int first = -1;
        size_t off0 = 0;
        for (int qi = 0; qi < look; ++qi)
            if (s->arena->alloc(s->queue[qi].footprint, &off0)) {
                first = qi;
                break;
            }
        if (first < 0) {
            ++s->stalls;  // a lane is free but nothing at the head fits the arena
            return admitted;
        }
        const ClassKey key = s->queue[first].key;
        std::vector<int> taken{first};
        ln->members.clear();
        ln->members.push_back(Member{s->queue[first], off0});
        size_t embed = s->queue[first].embed_bytes;
        // fill from the wider window only when the oldest request is in, so a
        // large request at the head is not overtaken by a stream of small ones
        const int lim = (int)std::min<size_t>(s->queue.size(), first == 0 ? kWindow : look);
        for (int qi = first + 1; qi < lim && (int)ln->members.size() < kServeBatchMax; ++qi) {
            const Pending &pd = s->queue[qi];
            if (!(pd.key == key) || embed + pd.embed_bytes > kEmbedBudget) continue;
            size_t off;
            if (!s->arena->alloc(pd.footprint, &off)) continue;
            ln->members.push_back(Member{pd, off});
            embed += pd.embed_bytes;
            taken.push_back(qi);
        }
        for (auto it = taken.rbegin(); it != taken.rend(); ++it)
            s->queue.erase(s->queue.begin() + *it);
        if (s->arena->used() > s->peak_used) s->peak_used = s->arena->used();
        ln->busy = true;
        ln->admit_s = now_s();
        s->in_flight += (int32_t)ln->members.size();
        admitted += (int)ln->members.size();
        const int rc = launch_lane(s, *ln, key);
        if (rc != CHAMFER_OK) fail_lane(s, *ln, rc);
    }
}

int poll(chamfer_server *s) {
    int n = 0;
    for (auto &ln : s->lanes) {
        if (!ln.busy) continue;
        const hipError_t q = hipEventQuery(ln.done);
        if (q == hipErrorNotReady) continue;
        for (size_t j = 0; j < ln.members.size(); ++j) {
            const Member &m = ln.members[j];
            const Out &o = ln.out_host[j];
            chamfer_result res = result_of(m.job, q == hipSuccess ? o.status : CHAMFER_EHIP,
                                           ln.admit_s);
            res.eta = o.eta;
            res.D = o.D;
            res.W = o.W;
            res.s = o.s;
            s->done.push_back(res);
            s->arena->release(m.off, m.job.footprint);
            ++n;
        }
        s->in_flight -= (int32_t)ln.members.size();
        ln.members.clear();
        ln.busy = false;
    }
    return n;
}

}  // namespace

extern "C" {

int chamfer_server_create(size_t arena_bytes, int32_t lanes, chamfer_server **out) {
    if (out == nullptr || lanes < 1 || lanes > kMaxLanes || arena_bytes < kArenaAlign)
        return CHAMFER_EINVAL;
    *out = nullptr;
    auto *s = new chamfer_server();
    if (hipMalloc(&s->arena_base, arena_bytes) != hipSuccess) {
        delete s;
        return CHAMFER_EHIP;
    }
    s->arena = new Arena(arena_bytes);
    s->lanes.resize(lanes);
    if (hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking) != hipSuccess) {
        chamfer_server_destroy(s);
        return CHAMFER_EHIP;
    }
    for (auto &ln : s->lanes) {
        if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&ln.dev), kLaneBytes) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&ln.host), kOutOff, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&ln.out_host), kBatchMax * sizeof(Out),
                          hipHostMallocDefault) != hipSuccess) {
            chamfer_server_destroy(s);
            return CHAMFER_EHIP;
        }
    }
    *out = s;
    return CHAMFER_OK;
}

int chamfer_server_warm(chamfer_server *s, int32_t d, int32_t metric, int32_t embed_dim,
                        int32_t precision) {
    if (s == nullptr || d < 1 || d > 2048 || (metric != CHAMFER_L1 && metric != CHAMFER_L2) ||
        (embed_dim != 0 && embed_dim != 8 && embed_dim != 16 && embed_dim != 32 &&
         embed_dim != 64) ||
        precision < CHAMFER_FP32 || precision > CHAMFER_FP8)
        return CHAMFER_EINVAL;
    chamfer_request r{};
    r.d = d;
    r.metric = metric;
    r.opts.embed_dim = embed_dim;
    r.opts.precision = precision;
    const ClassKey key = class_of(r);
    for (auto &ln : s->lanes)
        if (graph_for(s, ln, key) == nullptr) return CHAMFER_EHIP;
    return CHAMFER_OK;
}

int chamfer_server_submit(chamfer_server *s, const chamfer_request *req, uint64_t *id_out) {
    if (s == nullptr || req == nullptr) return CHAMFER_EINVAL;
    if ((req->n_A > 0 && req->A == nullptr) || req->B == nullptr) return CHAMFER_EINVAL;
    if (req->d > 2048) return CHAMFER_EINVAL;  // widest class the batched stages take
    if (req->opts.window > 1 || req->opts.reps > 1 || req->opts.sampling != CHAMFER_IMPORTANCE)
        return CHAMFER_EINVAL;  // one structure, W = 1, importance sampling
    Pending pd{};
    pd.req = *req;
    pd.footprint = footprint_of(pd.req, &pd.ws_bytes);
    if (pd.footprint == 0) return CHAMFER_EINVAL;
    if (pd.footprint > s->arena->size()) return CHAMFER_EWORKSPACE;  // can never be admitted
    pd.key = class_of(pd.req);
    pd.embed_bytes = pd.key.metric == CHAMFER_L2 ? round_up(embed_bytes(pd.key.d, pd.key.ke)) : 0;
    pd.id = s->next_id++;
    pd.submit_s = now_s();
    if (id_out) *id_out = pd.id;
    if (req->n_A == 0) {
        // CH of an empty A is 0: finished at once, nothing to run
        s->done.push_back(result_of(pd, CHAMFER_OK, pd.submit_s));
        return CHAMFER_OK;
    }
    s->queue.push_back(pd);
    return CHAMFER_OK;
}

int chamfer_server_progress(chamfer_server *s) {
    if (s == nullptr) return CHAMFER_EINVAL;
    int total = 0;
    for (;;) {
        const int done = poll(s);
        const int adm = admit(s);
        total += done;
        if (done == 0 && adm == 0) return total;
    }
}

int chamfer_server_results(chamfer_server *s, chamfer_result *out, int32_t max) {
    if (s == nullptr || (out == nullptr && max > 0)) return CHAMFER_EINVAL;
    const int n = (int)std::min<size_t>(s->done.size(), (size_t)std::max(0, max));
    for (int i = 0; i < n; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + n);
    return n;
}

int chamfer_server_stats(const chamfer_server *s, chamfer_server_stat *st) {
    if (s == nullptr || st == nullptr) return CHAMFER_EINVAL;
    st->queued = (int64_t)s->queue.size();
    st->in_flight = s->in_flight;
    int busy = 0;
    for (auto &ln : s->lanes) busy += ln.busy ? 1 : 0;
    st->lanes_busy = busy;
    st->arena_bytes = s->arena->size();
    st->arena_used = s->arena->used();
    st->arena_peak = s->peak_used;
    st->batches = s->batches;
    st->batched = s->batched;
    st->graphs = s->graphs;
    st->stalls = s->stalls;
    return CHAMFER_OK;
}

int chamfer_server_destroy(chamfer_server *s) {
    if (s == nullptr) return CHAMFER_EINVAL;
    for (auto &ln : s->lanes) {
        if (ln.stream) (void)hipStreamSynchronize(ln.stream);
        for (auto &g : ln.graphs) (void)hipGraphExecDestroy(g.second);
        if (ln.done) (void)hipEventDestroy(ln.done);
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
        if (ln.dev) (void)hipFree(ln.dev);
        if (ln.host) (void)hipHostFree(ln.host);
        if (ln.out_host) (void)hipHostFree(ln.out_host);
    }
    if (s->capture) (void)hipStreamDestroy(s->capture);
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s->arena;
    delete s;
    return CHAMFER_OK;
}

}  // extern "C"
