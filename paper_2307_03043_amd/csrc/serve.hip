// Serving runtime: continuous batching of chamfer_estimate requests.
//
// A server owns one device arena (allocated once at creation) and a fixed
// number of slots, each with its own stream (default priority) and a small
// pinned result block.  Requests are queued on the host; progress() admits
// queued requests whenever a slot is free and the arena can hold the
// request's footprint (its two point sets, the workspace of
// chamfer_workspace_bytes and the outputs), copies the inputs in on the
// slot's stream, enqueues the whole estimate there, and polls completion
// events.  Requests admitted while others run overlap on the device; a
// completion frees its slot and arena block at once, so the next request
// can be admitted in the same progress() call.  Admission is FIFO with a
// bounded look-ahead: when the head of the queue does not fit, up to
// kLookahead later requests that do fit may go first.  Results depend only
// on the request (all kernels are deterministic), so a request's result is
// the same alone and in any mix.
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "internal.h"

namespace {

constexpr size_t kArenaAlign = 256;
constexpr int kLookahead = 8;

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

struct Pending {
    uint64_t id;
    chamfer_request req;
    double submit_s;
    size_t footprint, ws_bytes;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    Pending job{};
    size_t off = 0;
    double admit_s = 0.0;
    // pinned: eta, status, W, s, D
    struct Out {
        double eta;
        double D;
        int32_t status;
        int32_t s;
        uint64_t W;
    } *out = nullptr;
};

}  // namespace

struct chamfer_server {
    char *arena_base = nullptr;
    Arena *arena = nullptr;
    std::vector<Slot> slots;
    std::deque<Pending> queue;
    std::vector<chamfer_result> done;
    uint64_t next_id = 1;
    size_t peak_used = 0;
};

namespace {

size_t footprint_of(const chamfer_request &r, size_t *ws_bytes) {
    const chamfer_opts *o = &r.opts;
    *ws_bytes = chamfer_workspace_bytes(r.n_A, r.n_B, r.d, r.metric, r.eps, r.T, o);
    if (*ws_bytes == 0) return 0;
    const size_t pa = round_up((size_t)r.n_A * r.d * sizeof(float));
    const size_t pb = round_up((size_t)r.n_B * r.d * sizeof(float));
    return pa + pb + round_up(*ws_bytes) + round_up(sizeof(Slot::Out));
}

int launch_job(chamfer_server *s, Slot &sl) {
    const chamfer_request &r = sl.job.req;
    char *base = s->arena_base + sl.off;
    const size_t pa = round_up((size_t)r.n_A * r.d * sizeof(float));
    const size_t pb = round_up((size_t)r.n_B * r.d * sizeof(float));
    float *A = reinterpret_cast<float *>(base);
    float *B = reinterpret_cast<float *>(base + pa);
    char *ws = base + pa + pb;
    Slot::Out *dout = reinterpret_cast<Slot::Out *>(ws + round_up(sl.job.ws_bytes));
    hipStream_t st = sl.stream;
    if (r.n_A > 0 &&
        hipMemcpyAsync(A, r.A, (size_t)r.n_A * r.d * sizeof(float), hipMemcpyHostToDevice, st) !=
            hipSuccess)
        return CHAMFER_EHIP;
    if (hipMemcpyAsync(B, r.B, (size_t)r.n_B * r.d * sizeof(float), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return CHAMFER_EHIP;
    chamfer_aux aux{};
    aux.D = &dout->D;
    aux.status = &dout->status;
    aux.s = &dout->s;
    aux.W = &dout->W;
    int rc = chamfer_estimate(A, B, r.n_A, r.n_B, r.d, r.metric, r.eps, r.T, r.seed, &dout->eta,
                              &aux, &r.opts, ws, sl.job.ws_bytes, st);
    if (rc) return rc;
    if (hipMemcpyAsync(sl.out, dout, sizeof(Slot::Out), hipMemcpyDeviceToHost, st) != hipSuccess)
        return CHAMFER_EHIP;
    if (hipEventRecord(sl.done, st) != hipSuccess) return CHAMFER_EHIP;
    return CHAMFER_OK;
}

// Admit queued requests into free slots while the arena has room.
int admit(chamfer_server *s) {
    int admitted = 0;
    for (;;) {
        int free_slot = -1;
        for (size_t i = 0; i < s->slots.size(); ++i)
            if (!s->slots[i].busy) {
                free_slot = (int)i;
                break;
            }
        if (free_slot < 0 || s->queue.empty()) return admitted;
        bool placed = false;
        const int look = (int)std::min<size_t>(s->queue.size(), kLookahead + 1);
        for (int qi = 0; qi < look && !placed; ++qi) {
            Pending &pd = s->queue[qi];
            size_t off;
            if (!s->arena->alloc(pd.footprint, &off)) continue;
            Slot &sl = s->slots[free_slot];
            sl.job = pd;
            sl.off = off;
            sl.busy = true;
            sl.admit_s = now_s();
            s->queue.erase(s->queue.begin() + qi);
            if (s->arena->used() > s->peak_used) s->peak_used = s->arena->used();
            const int rc = launch_job(s, sl);
            if (rc != CHAMFER_OK) {
                // report the failure as this request's result and free at once
                chamfer_result res{};
                res.id = sl.job.id;
                res.status = rc;
                res.submit_s = sl.job.submit_s;
                res.admit_s = res.done_s = sl.admit_s;
                res.footprint = sl.job.footprint;
                s->done.push_back(res);
                (void)hipStreamSynchronize(sl.stream);
                s->arena->release(sl.off, sl.job.footprint);
                sl.busy = false;
            }
            placed = true;
            ++admitted;
        }
        if (!placed) return admitted;  // nothing in the window fits right now
    }
}

int poll(chamfer_server *s) {
    int n = 0;
    for (auto &sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        chamfer_result res{};
        res.id = sl.job.id;
        res.status = q == hipSuccess ? sl.out->status : CHAMFER_EHIP;
        res.eta = sl.out->eta;
        res.D = sl.out->D;
        res.W = sl.out->W;
        res.s = sl.out->s;
        res.submit_s = sl.job.submit_s;
        res.admit_s = sl.admit_s;
        res.done_s = now_s();
        res.footprint = sl.job.footprint;
        s->done.push_back(res);
        s->arena->release(sl.off, sl.job.footprint);
        sl.busy = false;
        ++n;
    }
    return n;
}

}  // namespace

extern "C" {

int chamfer_server_create(size_t arena_bytes, int32_t slots, chamfer_server **out) {
    if (out == nullptr || slots < 1 || slots > 256 || arena_bytes < kArenaAlign)
        return CHAMFER_EINVAL;
    *out = nullptr;
    auto *s = new chamfer_server();
    if (hipMalloc(&s->arena_base, arena_bytes) != hipSuccess) {
        delete s;
        return CHAMFER_EHIP;
    }
    s->arena = new Arena(arena_bytes);
    s->slots.resize(slots);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&sl.out), sizeof(Slot::Out),
                          hipHostMallocDefault) != hipSuccess) {
            chamfer_server_destroy(s);
            return CHAMFER_EHIP;
        }
    }
    *out = s;
    return CHAMFER_OK;
}

int chamfer_server_submit(chamfer_server *s, const chamfer_request *req, uint64_t *id_out) {
    if (s == nullptr || req == nullptr) return CHAMFER_EINVAL;
    Pending pd{};
    pd.req = *req;
    if ((req->n_A > 0 && req->A == nullptr) || req->B == nullptr) return CHAMFER_EINVAL;
    pd.footprint = footprint_of(pd.req, &pd.ws_bytes);
    if (pd.footprint == 0) return CHAMFER_EINVAL;
    if (pd.footprint > s->arena->size()) return CHAMFER_EWORKSPACE;  // can never be admitted
    pd.id = s->next_id++;
    pd.submit_s = now_s();
    s->queue.push_back(pd);
    if (id_out) *id_out = pd.id;
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
    int busy = 0;
    for (auto &sl : s->slots) busy += sl.busy ? 1 : 0;
    st->in_flight = busy;
    st->arena_bytes = s->arena->size();
    st->arena_used = s->arena->used();
    st->arena_peak = s->peak_used;
    return CHAMFER_OK;
}

int chamfer_server_destroy(chamfer_server *s) {
    if (s == nullptr) return CHAMFER_EINVAL;
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.out) (void)hipHostFree(sl.out);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s->arena;
    delete s;
    return CHAMFER_OK;
}

}  // extern "C"
