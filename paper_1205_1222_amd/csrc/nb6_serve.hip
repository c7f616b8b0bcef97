// nb6_serve.hip -- the serving queue behind nb6_submit / nb6_poll.
//
// Requests (one regular-force block of one cluster each) are admitted in
// arrival order while their device scratch fits an arena of the context's
// HBM budget and no request of the same cluster is in flight.  A scheduler
// thread fuses every admitted request into one batch:
//   prepare      predict each request's cluster to its block time and clear
//                its neighbour counts (one launch for the batch),
//   force        one persistent launch per coordinate mode: wavefronts take
//                (request, i-group, j-slice) items from an atomic counter,
//   finalize     one launch over every active particle of the batch (sums,
//                sorted lists, ordered rebuild of overflowed lists),
// on one of kSlots streams, so up to kSlots batches run at once and requests
// that arrive meanwhile form the next batch.  A batch holds at most about
// kBatchWork pair interactions (a larger request runs alone), and each
// persistent grid is sized to its work (a wave per item, at most what the chip
// holds at the kernel's occupancy), so short batches start beside long ones
// as their waves retire.  Requests with host arrays cross PCIe through the
// slot's pinned staging (one copy each way per request), so no copy waits
// on the host.  A host completion thread watches each batch's end-of-work
// event (spinning on it while batches are in flight), places the host
// requests' outputs in the callers' arrays, then stamps the batch's requests
// and frees their memory and clusters.
//
// A request's plan (make_plan: the rule of a plain call on the same context)
// and its summation order depend only on the request, so its results are
// bit-identical alone, in any mix, and to the plain call.
#include "nb6_arena.h"
#include "nb6_context.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>

namespace nb6 {

namespace {

constexpr int kSlots = 4;          // batches in flight
constexpr int kMaxBatch = 512;     // requests per batch
constexpr double kBatchWork = 2.5e8;  // pair interactions per batch (~0.2 ms)
constexpr size_t kAlign = 256;

constexpr size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int serve_class(const Plan& p) {
    return p.jl_shift > 0 ? SERVE_LANES : p.ipl == 2 ? SERVE_TWO_I : SERVE_ONE_I;
}

// Work items of a request in its class's persistent launch: one per
// (i-group, slice), or for the lanes class one per (four i-groups, slice),
// which a workgroup takes whole.
long long serve_items(int groups, const Plan& p) {
    const long long units = serve_class(p) == SERVE_LANES ? (groups + 3) / 4 : groups;
    return units * p.nslices;
}

// What a batch uploads ahead of its descriptors, zeroed on the host: the
// persistent kernels' work-item counters (one per coordinate mode and
// i-per-lane class) and the requests' status words.  Header and descriptors
// go up in one copy.
struct BatchHeader {
    unsigned long long counters[NMODES * SERVE_CLASSES];
    unsigned status[kMaxBatch];
};
constexpr size_t kHeaderBytes = align_up(sizeof(BatchHeader));

// The serving arena: one device allocation of the HBM budget, carved by
// OffsetArena (first fit, coalescing on free).
class Arena {
  public:
    int init(nb6_ctx* c, size_t bytes) {
        const size_t size = bytes / kAlign * kAlign;
        if (size == 0) return fail(c, NB6_ERR_ARG, "serving budget is zero");
        if (hipMalloc(&base_, size) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            return fail(c, NB6_ERR_NOMEM, "serving arena of %zu bytes", size);
        }
        off_.reset(size);
        return NB6_OK;
    }
    void release() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
        off_.reset(0);
    }
    size_t size() const { return off_.size(); }
    size_t used() const { return off_.used(); }
    bool alloc(size_t bytes, size_t* off) { return off_.alloc(bytes, off); }
    void free(size_t off, size_t bytes) { off_.free(off, bytes); }
    char* base() const { return static_cast<char*>(base_); }

  private:
    void* base_ = nullptr;
    OffsetArena off_;
};

struct ServeReq {
    uint64_t ticket = 0;
    nb6_request rq{};
    int mi = 0;
    int km = 0;             // the force kernel's mode: kernel_mode(mi, plan)
    Plan plan{};
    size_t bytes = 0, off = 0;
    ClusterState* cl = nullptr;
    int64_t n_submit = 0;   // cluster size the request was checked and sized against
    int status = NB6_PENDING;
    int batch_size = 0;
    size_t stage = 0;       // HOST requests: offset of its region in the slot's pinned staging
    double t_submit = 0, t_admit = 0, t_done = 0;
    // scratch carved from the arena
    double* part = nullptr;
    int32_t* cnt = nullptr;   // [ni]
    int32_t* lst = nullptr;
    int32_t* d_idx = nullptr;
    double* d_h2 = nullptr;
    double* d_dtr = nullptr;
    double* d_acc = nullptr;
    double* d_jerk = nullptr;
    int32_t* d_nnb = nullptr;
    int32_t* d_list = nullptr;
};

// Arena bytes of a request, and (when base != null) its buffers.
size_t carve(ServeReq* r, char* base) {
    const size_t ni = (size_t)r->rq.n_i, cap = (size_t)r->rq.cap, caps = cap + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t ni64 = (ni + 63) / 64 * 64;  // partials are kept by 64-particle block
    r->part = (double*)take(ni64 * r->plan.nslices * NPART * sizeof(double));
    r->cnt = (int32_t*)take(ni * sizeof(int32_t));
    r->lst = (int32_t*)take(ni * caps * sizeof(int32_t));
    if (r->rq.mem_kind == NB6_MEM_HOST) {
        r->d_idx = (int32_t*)take(ni * sizeof(int32_t));
        r->d_h2 = (double*)take(ni * sizeof(double));
        r->d_dtr = (double*)take(ni * sizeof(double));
        r->d_acc = (double*)take(3 * ni * sizeof(double));
        r->d_jerk = (double*)take(3 * ni * sizeof(double));
        r->d_nnb = (int32_t*)take(ni * sizeof(int32_t));
        r->d_list = (int32_t*)take(std::max<size_t>(1, ni * cap) * sizeof(int32_t));
    } else {
        r->d_idx = const_cast<int32_t*>(r->rq.idx_i);
        r->d_h2 = const_cast<double*>(r->rq.h2_i);
        r->d_dtr = const_cast<double*>(r->rq.dtr_i);
        r->d_acc = r->rq.acc;
        r->d_jerk = r->rq.jerk;
        r->d_nnb = r->rq.nnb;
        r->d_list = r->rq.list;
    }
    return off;
}

// Bytes from a HOST request's first device input to the end of its inputs,
// and from its first output to the end of its outputs: carve() lays each
// group out contiguously, so each crosses PCIe in one copy through the slot's
// pinned staging, with the same layout there.
size_t in_span(const ServeReq* r) {
    return (size_t)((const char*)(r->d_dtr + r->rq.n_i) - (const char*)r->d_idx);
}
size_t out_span(const ServeReq* r) {
    const size_t ni = (size_t)r->rq.n_i, cap = (size_t)r->rq.cap;
    return (size_t)((const char*)(r->d_list + std::max<size_t>(1, ni * cap)) -
                    (const char*)r->d_acc);
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;           // recorded after the batch's last work
    char* host_blob = nullptr;           // pinned: BatchHeader, then kMaxBatch ReqDesc
    char* dev_blob = nullptr;            // its device copy
    char* stage = nullptr;               // pinned staging of the HOST requests' arrays
    size_t stage_cap = 0;
    bool busy = false;                   // holds a batch
    bool launched = false;               // its work is enqueued; `done` is pending
    std::vector<ServeReq*> reqs;

    BatchHeader* host_hdr() const { return reinterpret_cast<BatchHeader*>(host_blob); }
    BatchHeader* dev_hdr() const { return reinterpret_cast<BatchHeader*>(dev_blob); }
    ReqDesc* host_desc() const { return reinterpret_cast<ReqDesc*>(host_blob + kHeaderBytes); }
    ReqDesc* dev_desc() const { return reinterpret_cast<ReqDesc*>(dev_blob + kHeaderBytes); }
};
constexpr size_t kBlobBytes = kHeaderBytes + kMaxBatch * sizeof(ReqDesc);

}  // namespace

class Engine {
  public:
    explicit Engine(nb6_ctx* c) : c_(c), t0_(std::chrono::steady_clock::now()) {}

    int start() {
        HIP_TRY(c_, hipSetDevice(c_->device));
        for (int m = 0; m < NMODES; ++m)
            for (int k = 0; k < SERVE_CLASSES; ++k) {
                HIP_TRY(c_, serve_regf_blocks_per_cu(m, k, &blocks_per_cu_[m][k]));
                blocks_per_cu_[m][k] = std::max(1, blocks_per_cu_[m][k]);
            }
        if (int rc = arena_.init(c_, (size_t)c_->hbm_budget)) return rc;
        for (Slot& s : slots_) {
            HIP_TRY(c_, hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
            HIP_TRY(c_, hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
            HIP_TRY(c_, hipHostMalloc((void**)&s.host_blob, kBlobBytes));
            HIP_TRY(c_, hipMalloc((void**)&s.dev_blob, kBlobBytes));
        }
        sched_ = std::thread([this] { sched_loop(); });
        done_ = std::thread([this] { done_loop(); });
        return NB6_OK;
    }

    void shutdown() {
        {
            std::unique_lock<std::mutex> lk(mu_);
            stop_ = true;
            for (ServeReq* r : pending_) {
                r->status = NB6_ERR_STATE;
                r->t_done = now();
                r->cl->queued.fetch_sub(1);
            }
            pending_.clear();
            cv_sched_.notify_all();
            cv_polled_.notify_all();
        }
        if (sched_.joinable()) sched_.join();
        {
            std::unique_lock<std::mutex> lk(mu_);  // batches still on the GPU
            if (done_.joinable())
                cv_sched_.wait(lk, [&] {
                    for (const Slot& s : slots_)
                        if (s.busy) return false;
                    return true;
                });
            stop_done_ = true;
            cv_done_.notify_all();
        }
        if (done_.joinable()) done_.join();
        (void)hipSetDevice(c_->device);
        for (Slot& s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.host_blob) (void)hipHostFree(s.host_blob);
            if (s.stage) (void)hipHostFree(s.stage);
            if (s.dev_blob) (void)hipFree(s.dev_blob);
            s = Slot();
        }
        arena_.release();
        for (auto& kv : tickets_) delete kv.second;
        tickets_.clear();
    }

    int submit(const nb6_request* rq, uint64_t* ticket) {
        std::unique_ptr<ServeReq> r(new ServeReq());
        r->rq = *rq;
        const int64_t ni = rq->n_i;
        r->mi = mode_index(rq->dx_mode);
        if (r->mi < 0) return fail(c_, NB6_ERR_ARG, "bad dx_mode %d", rq->dx_mode);
        if (ni <= 0 || ni > INT32_MAX / 2) return fail(c_, NB6_ERR_ARG, "n_i = %lld", (long long)ni);
        if (rq->cap < 0 || rq->cap > NB6_MAX_CAP)
            return fail(c_, NB6_ERR_ARG, "cap = %d outside [0, %d]", rq->cap, NB6_MAX_CAP);
        if (rq->mem_kind != NB6_MEM_HOST && rq->mem_kind != NB6_MEM_DEVICE)
            return fail(c_, NB6_ERR_ARG, "bad mem_kind %d", rq->mem_kind);
        if (!rq->idx_i || !rq->h2_i || !rq->dtr_i || !rq->acc || !rq->jerk || !rq->nnb ||
            (rq->cap > 0 && !rq->list))
            return fail(c_, NB6_ERR_ARG, "null argument");
        if (!std::isfinite(rq->t_block)) return fail(c_, NB6_ERR_ARG, "non-finite t_block");
        {
            std::lock_guard<std::mutex> lk(c_->cluster_mu);
            if (rq->cluster < 0 || rq->cluster >= kMaxClusters || !c_->clusters[rq->cluster] ||
                c_->clusters[rq->cluster]->n == 0)
                return fail(c_, NB6_ERR_STATE, "cluster %d is not loaded", rq->cluster);
            r->cl = c_->clusters[rq->cluster];
            if (rq->mem_kind == NB6_MEM_HOST) {
                for (int64_t q = 0; q < ni; ++q) {
                    if (rq->idx_i[q] < 0 || rq->idx_i[q] >= r->cl->n)
                        return fail(c_, NB6_ERR_ARG, "idx_i[%lld] out of range", (long long)q);
                    const float h2f = (float)rq->h2_i[q];
                    if (!(h2f >= 1.17549435e-38f) || !(h2f <= 3.40282347e38f))
                        return fail(c_, NB6_ERR_ARG, "h2_i[%lld] is not a positive normal float",
                                    (long long)q);
                    if (!valid_dtr(rq->dtr_i[q]))
                        return fail(c_, NB6_ERR_ARG, "dtr_i[%lld] is not a finite value >= 0",
                                    (long long)q);
                }
            }
            // the record stream of this mode is allocated once, here; requests
            // in flight on the cluster use other modes' streams
            if (!r->cl->rec[r->mi].p) {
                if (int rc = ensure(c_, r->cl->rec[r->mi], (size_t)r->cl->n * rec_size(r->mi)))
                    return rc;
            }
            if (!r->cl->tmax.p) {
                if (int rc = ensure(c_, r->cl->tmax, (size_t)vtiles(r->cl->n) * sizeof(float)))
                    return rc;
            }
            if (r->mi == MODE_LOC) {  // the float-float i-side and the tile centres
                if (!r->cl->order_valid)
                    return fail(c_, NB6_ERR_STATE, "cluster %d has no spatial order", rq->cluster);
                int rc = NB6_OK;
                if ((!r->cl->rec[MODE_FF].p &&
                     (rc = ensure(c_, r->cl->rec[MODE_FF], (size_t)r->cl->n * sizeof(RecFF)))) ||
                    (!r->cl->org.p &&
                     (rc = ensure(c_, r->cl->org, (size_t)vtiles(r->cl->n) * sizeof(TileOrg)))))
                    return rc;
            }
            r->plan = make_plan(c_, r->cl->n, ni);
            // a small block runs on the float-float records (the plain call's rule)
            r->km = kernel_mode(r->mi, r->plan);
            r->n_submit = r->cl->n;
            // held until the request finishes: the cluster keeps its size and
            // buffers meanwhile
            r->cl->queued.fetch_add(1);
        }
        r->bytes = carve(r.get(), nullptr);
        std::unique_lock<std::mutex> lk(mu_);
        if (r->bytes > arena_.size()) {
            r->cl->queued.fetch_sub(1);
            return fail(c_, NB6_ERR_ADMISSION,
                        "request needs %zu bytes of scratch; the serving budget is %zu",
                        r->bytes, arena_.size());
        }
        r->ticket = next_ticket_++;
        r->t_submit = now();
        *ticket = r->ticket;
        tickets_[r->ticket] = r.get();
        pending_.push_back(r.release());
        blocked_ = false;
        cv_sched_.notify_all();
        return NB6_OK;
    }

    // A cluster became free outside the queue (a plain call ended).
    void kick() {
        std::lock_guard<std::mutex> lk(mu_);
        blocked_ = false;
        cv_sched_.notify_all();
    }

    int poll(uint64_t ticket, int wait, nb6_ticket_info* info) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = tickets_.find(ticket);
        if (it == tickets_.end())
            return fail(c_, NB6_ERR_UNKNOWN_TICKET, "unknown ticket %llu",
                        (unsigned long long)ticket);
        ServeReq* r = it->second;
        if (r->status == NB6_PENDING) {
            if (!wait) return NB6_PENDING;
            cv_polled_.wait(lk, [&] { return r->status != NB6_PENDING; });
        }
        if (info) {
            info->status = r->status;
            info->slices = r->plan.nslices;
            info->batch_size = r->batch_size;
            info->submit_us = r->t_submit;
            info->admit_us = r->t_admit;
            info->done_us = r->t_done;
        }
        const int st = r->status;
        tickets_.erase(it);
        delete r;
        return st;
    }

  private:
    double now() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0_)
            .count();
    }

    int free_slot() const {
        for (int i = 0; i < kSlots; ++i)
            if (!slots_[i].busy) return i;
        return -1;
    }

    // Called with mu_ held; takes no other lock and makes no HIP call (the
    // completion thread runs it while the scheduler may be enqueueing).
    void finish(ServeReq* r, int status, double t) {
        // A batch that failed may have marked records current that it never
        // wrote: its clusters predict again on their next use.
        if (status < 0 && status != NB6_ERR_DEVICE_INPUT)
            r->cl->pred_valid = 0;
        r->status = status;
        r->t_done = t;
        arena_.free(r->off, r->bytes);
        r->cl->owner.store(0);
        r->cl->queued.fetch_sub(1);
    }

    // The buffers a request was sized against are still those of its
    // cluster (a resize is refused while it is queued; this is the check
    // that no descriptor is built from anything else).
    static bool cluster_intact(const ServeReq* r) {
        const ClusterState* cl = r->cl;
        return cl->n == r->n_submit && cl->state && cl->rec[r->mi].p && cl->tmax.p &&
               (r->mi != MODE_LOC || (cl->org.p && cl->perm.p && cl->inv.p &&
                                      cl->rec[MODE_FF].p && cl->order_valid));
    }

    void sched_loop() {
        (void)hipSetDevice(c_->device);
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            // A blocked queue is retried on every submission, completion and
            // cluster release, and at least every 2 ms.
            cv_sched_.wait_for(lk, std::chrono::milliseconds(2), [&] {
                return stop_ || (!pending_.empty() && !blocked_ && free_slot() >= 0);
            });
            if (stop_) break;
            blocked_ = false;
            if (pending_.empty() || free_slot() < 0) continue;
            const int si = free_slot();
            Slot& sl = slots_[si];
            std::vector<ServeReq*> batch;
            double work = 0.0;
            for (auto it = pending_.begin();
                 it != pending_.end() && (int)batch.size() < kMaxBatch;) {
                ServeReq* r = *it;
                const double w = (double)r->rq.n_i * (double)r->cl->n;
                if (!batch.empty() && work + w > kBatchWork) break;
                int free_owner = 0;  // one request per cluster, no plain call on it
                if (!r->cl->owner.compare_exchange_strong(free_owner, 1)) {
                    ++it;
                    continue;
                }
                if (!cluster_intact(r)) {  // never launched: fails on its own
                    it = pending_.erase(it);
                    r->status = NB6_ERR_STATE;
                    r->t_done = now();
                    r->cl->owner.store(0);
                    r->cl->queued.fetch_sub(1);
                    cv_polled_.notify_all();
                    continue;
                }
                size_t off;
                if (!arena_.alloc(r->bytes, &off)) {  // arrival order for memory
                    r->cl->owner.store(0);
                    break;
                }
                work += w;
                r->off = off;
                carve(r, arena_.base() + off);
                r->t_admit = now();
                batch.push_back(r);
                it = pending_.erase(it);
            }
            if (batch.empty()) {
                blocked_ = true;  // until a batch finishes
                continue;
            }
            for (ServeReq* r : batch) r->batch_size = (int)batch.size();
            sl.busy = true;
            sl.reqs = batch;
            lk.unlock();
            const int rc = launch(sl);
            if (rc != NB6_OK) (void)hipStreamSynchronize(sl.stream);  // work enqueued so far
            lk.lock();
            if (rc != NB6_OK) {
                const double t = now();
                for (ServeReq* r : sl.reqs) finish(r, rc, t);
                sl.reqs.clear();
                sl.busy = false;
                cv_polled_.notify_all();
                continue;
            }
            sl.launched = true;
            cv_done_.notify_all();
        }
    }

    // Completion: while any batch is in flight, query the slots' end events
    // in a loop (the lock is dropped around the queries); when none is, sleep
    // until the scheduler launches one.  A spinning waiter sees the end of a
    // batch within a few microseconds, where a stream callback takes tens.
    void done_loop() {
        (void)hipSetDevice(c_->device);
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_done_.wait(lk, [&] { return stop_done_ || any_launched(); });
            if (!any_launched()) {
                if (stop_done_) break;
                continue;
            }
            Slot* cand[kSlots];
            int nc = 0;
            for (Slot& s : slots_)
                if (s.launched) cand[nc++] = &s;
            lk.unlock();
            Slot* ready = nullptr;
            hipError_t err = hipSuccess;
            for (;;) {
                for (int i = 0; i < nc && !ready; ++i) {
                    const hipError_t e = hipEventQuery(cand[i]->done);
                    if (e != hipErrorNotReady) {
                        ready = cand[i];
                        err = e;
                    }
                }
                if (ready) break;
                std::this_thread::yield();
                if (nc < kSlots) break;  // look for slots launched meanwhile
            }
            // the HOST requests' outputs, from the pinned staging into the
            // callers' arrays (the slot stays busy until complete(), so
            // neither its staging nor its requests change meanwhile)
            if (ready && err == hipSuccess) copy_out(*ready);
            lk.lock();
            if (ready) {
                ready->launched = false;
                complete(*ready, err);
            }
        }
    }

    static void copy_out(const Slot& sl) {
        for (const ServeReq* r : sl.reqs) {
            if (r->rq.mem_kind != NB6_MEM_HOST) continue;
            const size_t ni = (size_t)r->rq.n_i, cap = (size_t)r->rq.cap;
            const char* base = sl.stage + r->stage + in_span(r);
            auto at = [&](const void* dev) {
                return base + ((const char*)dev - (const char*)r->d_acc);
            };
            std::memcpy(r->rq.acc, at(r->d_acc), 3 * ni * sizeof(double));
            std::memcpy(r->rq.jerk, at(r->d_jerk), 3 * ni * sizeof(double));
            std::memcpy(r->rq.nnb, at(r->d_nnb), ni * sizeof(int32_t));
            if (cap == 0) continue;
            // the first min(nnb, cap) entries of each row, as a plain call's
            const int32_t* nnb = reinterpret_cast<const int32_t*>(at(r->d_nnb));
            const int32_t* rows = reinterpret_cast<const int32_t*>(at(r->d_list));
            for_rows((int)ni, (int64_t)(ni * cap), [&](int q0, int q1) {
                for (int q = q0; q < q1; ++q) {
                    const size_t k = (size_t)std::min<int64_t>(std::max(nnb[q], 0), (int64_t)cap);
                    std::memcpy(r->rq.list + (size_t)q * cap, rows + (size_t)q * cap,
                                k * sizeof(int32_t));
                }
            });
        }
    }

    bool any_launched() const {
        for (const Slot& s : slots_)
            if (s.launched) return true;
        return false;
    }

    // Called with mu_ held, after the batch's stream work has ended.
    void complete(Slot& sl, hipError_t err) {
        const double t = now();
        const unsigned* status = sl.host_hdr()->status;
        for (size_t b = 0; b < sl.reqs.size(); ++b) {
            int st = NB6_OK;
            if (err != hipSuccess)
                st = NB6_ERR_HIP;
            else if (status[b] & (ST_BAD_INDEX | ST_BAD_H2 | ST_NONFINITE | ST_BAD_DTR))
                st = NB6_ERR_DEVICE_INPUT;
            else if (status[b] & ST_OVERFLOW)
                st = NB6_WARN_NB_OVERFLOW;
            finish(sl.reqs[b], st, t);
        }
        sl.reqs.clear();
        sl.busy = false;
        blocked_ = false;
        cv_sched_.notify_all();
        cv_polled_.notify_all();
    }

    // Enqueue the work of one batch on its slot's stream.  Runs on the
    // scheduler thread, so errors are returned as codes only (the context's
    // error text belongs to the caller's thread).
    int launch(Slot& sl) {
        HIP_TRY(nullptr, hipSetDevice(c_->device));
        hipStream_t st = sl.stream;
        std::vector<ServeReq*>& reqs = sl.reqs;
        // one persistent launch per (mode, work-partition class) present
        auto launch_class = [](const ServeReq* r) {
            return r->km * SERVE_CLASSES + serve_class(r->plan);
        };
        std::stable_sort(reqs.begin(), reqs.end(), [&](const ServeReq* a, const ServeReq* b) {
            return launch_class(a) < launch_class(b);
        });
        const int nreq = (int)reqs.size();
        // pinned staging of the HOST requests: inputs then outputs of each
        size_t stage_bytes = 0;
        for (ServeReq* r : reqs) {
            if (r->rq.mem_kind != NB6_MEM_HOST) continue;
            r->stage = stage_bytes;
            stage_bytes += align_up(in_span(r) + out_span(r));
        }
        if (stage_bytes > sl.stage_cap) {  // the slot is idle: its old staging is free
            const size_t want = std::max(stage_bytes, 2 * sl.stage_cap);
            if (sl.stage) HIP_TRY(nullptr, hipHostFree(sl.stage));
            sl.stage = nullptr;
            sl.stage_cap = 0;
            HIP_TRY(nullptr, hipHostMalloc((void**)&sl.stage, want));
            sl.stage_cap = want;
        }
        long long blk0 = 0, item_in_mode = 0;
        int64_t chunk_need = 0;
        int prev_class = -1;
        for (int b = 0; b < nreq; ++b) {
            ServeReq* r = reqs[b];
            ClusterState* cl = r->cl;
            const int ni = (int)r->rq.n_i;
            if (r->rq.mem_kind == NB6_MEM_HOST) {
                char* in = sl.stage + r->stage;
                auto at = [&](const void* dev) { return in + ((const char*)dev - (const char*)r->d_idx); };
                std::memcpy(at(r->d_idx), r->rq.idx_i, ni * sizeof(int32_t));
                std::memcpy(at(r->d_h2), r->rq.h2_i, ni * sizeof(double));
                std::memcpy(at(r->d_dtr), r->rq.dtr_i, ni * sizeof(double));
                HIP_TRY(nullptr, hipMemcpyAsync(r->d_idx, in, in_span(r), hipMemcpyHostToDevice, st));
            }
            if (launch_class(r) != prev_class) {
                item_in_mode = 0;
                prev_class = launch_class(r);
            }
            if (cl->last_plain) HIP_TRY(nullptr, hipStreamWaitEvent(st, cl->last_plain, 0));
            ReqDesc& d = sl.host_desc()[b];
            std::memset(&d, 0, sizeof d);
            const int bit = mode_bit(r->mi);
            // the queue owns the cluster while the request is in flight
            d.do_predict = !((cl->pred_valid & bit) && cl->t_pred == r->rq.t_block);
            if (d.do_predict) {
                cl->pred_valid = (cl->t_pred == r->rq.t_block ? cl->pred_valid : 0) | bit;
                cl->t_pred = r->rq.t_block;
            }
            unsigned* status = sl.dev_hdr()->status + b;
            d.pred.n = cl->n;
            d.pred.st = cl->state;
            d.pred.tb = r->rq.t_block;
            d.pred.ff = r->mi == MODE_FF ? (RecFF*)cl->rec[MODE_FF].p : nullptr;
            d.pred.f64 = r->mi == MODE_F64 ? (RecF64*)cl->rec[MODE_F64].p : nullptr;
            d.pred.f32 = r->mi == MODE_F32 ? (RecF32*)cl->rec[MODE_F32].p : nullptr;
            if (r->mi == MODE_LOC) {  // the local stream and its float-float i-side
                d.pred.ff = (RecFF*)cl->rec[MODE_FF].p;
                d.pred.loc = (RecLoc*)cl->rec[MODE_LOC].p;
                d.pred.org = (TileOrg*)cl->org.p;
                d.pred.perm = (const int32_t*)cl->perm.p;
            }
            d.pred.tmax = (float*)cl->tmax.p;
            d.pred.status = status;
            const Plan& p = r->plan;
            d.rg.rec = cl->rec[r->km].p;
            d.rg.n = (int)cl->n;
            d.rg.idx = r->d_idx; d.rg.h2 = r->d_h2; d.rg.dtr = r->d_dtr;
            d.rg.ni = ni;
            d.rg.slice_len = p.slice_len;
            d.rg.nslices = p.nslices;
            d.rg.jl_shift = p.jl_shift;
            d.rg.tmax = (const float*)cl->tmax.p;
            if (r->km == MODE_LOC) {
                d.rg.org = (const TileOrg*)cl->org.p;
                d.rg.ivw = cl->rec[MODE_FF].p;
            }
            d.rg.part = r->part; d.rg.cnt = r->cnt; d.rg.lst = r->lst;
            d.rg.caps = r->rq.cap + 1;
            d.rg.status = status;
            d.fin.part = r->part; d.fin.cnt = r->cnt; d.fin.lst = r->lst;
            d.fin.nslices = p.nslices; d.fin.ni = ni; d.fin.caps = r->rq.cap + 1;
            d.fin.n = (int)cl->n; d.fin.idx = r->d_idx; d.fin.h2 = r->d_h2;
            d.fin.acc = r->d_acc; d.fin.jerk = r->d_jerk; d.fin.nnb = r->d_nnb;
            d.fin.list = r->d_list; d.fin.cap = r->rq.cap; d.fin.status = status;
            d.fin.rec = d.rg.rec; d.fin.dtr = r->d_dtr; d.fin.mode = r->km;
            d.fin.org = d.rg.org; d.fin.ivw = d.rg.ivw;
            d.fin.inv = r->km == MODE_LOC ? (const int32_t*)cl->inv.p : nullptr;
            d.mode = r->km;
            const int gsize = regf_group_size(p.ipl, p.jl_shift);
            d.groups = (ni + gsize - 1) / gsize;
            d.item0 = item_in_mode;
            d.blk0 = blk0;
            item_in_mode += serve_items(d.groups, p);
            blk0 += final_blocks(ni, NPART);
            chunk_need = std::max<int64_t>(chunk_need, std::max<int64_t>(cl->n, ni));
        }
        std::memset(sl.host_hdr(), 0, sizeof(BatchHeader));
        HIP_TRY(nullptr, hipMemcpyAsync(sl.dev_blob, sl.host_blob,
                                   kHeaderBytes + nreq * sizeof(ReqDesc),
                                   hipMemcpyHostToDevice, st));
        unsigned long long* counters = sl.dev_hdr()->counters;
        BatchArgs all{};
        all.reqs = sl.dev_desc();
        all.nreq = nreq;
        all.nblk_total = blk0;
        HIP_TRY(nullptr, launch_serve_prepare(
                        all, (int)((chunk_need + PREPARE_CHUNK - 1) / PREPARE_CHUNK), st));
        // one persistent force launch per class present: a wave (lanes class:
        // a workgroup) per work item up to the number the chip holds at the
        // kernel's occupancy
        for (int b = 0; b < nreq;) {
            int e = b;
            long long items = 0;
            const int cls = launch_class(reqs[b]);
            while (e < nreq && launch_class(reqs[e]) == cls) {
                items += serve_items(sl.host_desc()[e].groups, reqs[e]->plan);
                ++e;
            }
            const int mi = reqs[b]->km, k = serve_class(reqs[b]->plan);
            const long long fit = (long long)c_->num_cu * blocks_per_cu_[mi][k];
            const int blocks =
                (int)std::min<long long>(fit, k == SERVE_LANES ? items : (items + 3) / 4);
            BatchArgs g{};
            g.reqs = sl.dev_desc() + b;
            g.nreq = e - b;
            g.nitems = items;
            g.counter = counters + cls;
            HIP_TRY(nullptr, launch_serve_regf(mi, k, g, blocks, st));
            b = e;
        }
        HIP_TRY(nullptr, launch_serve_finalize(all, st));
        for (ServeReq* r : reqs) {  // outputs into the staging; copy_out() places them
            if (r->rq.mem_kind != NB6_MEM_HOST) continue;
            HIP_TRY(nullptr, hipMemcpyAsync(sl.stage + r->stage + in_span(r), r->d_acc,
                                       out_span(r), hipMemcpyDeviceToHost, st));
        }
        HIP_TRY(nullptr, hipMemcpyAsync(sl.host_hdr()->status, sl.dev_hdr()->status,
                                   nreq * sizeof(unsigned), hipMemcpyDeviceToHost, st));
        for (ServeReq* r : reqs) {  // plain calls on these clusters wait for this
            if (!r->cl->last_served)
                HIP_TRY(nullptr, hipEventCreateWithFlags(&r->cl->last_served, hipEventDisableTiming));
            HIP_TRY(nullptr, hipEventRecord(r->cl->last_served, st));
        }
        HIP_TRY(nullptr, hipEventRecord(sl.done, st));
        return NB6_OK;
    }

    nb6_ctx* c_;
    std::chrono::steady_clock::time_point t0_;
    std::mutex mu_;
    std::condition_variable cv_sched_, cv_polled_;
    std::deque<ServeReq*> pending_;
    std::unordered_map<uint64_t, ServeReq*> tickets_;
    Slot slots_[kSlots];
    int blocks_per_cu_[NMODES][SERVE_CLASSES] = {};  // resident workgroups per CU, per launch
    Arena arena_;
    uint64_t next_ticket_ = 1;
    bool stop_ = false;
    bool stop_done_ = false;
    bool blocked_ = false;
    std::condition_variable cv_done_;
    std::thread sched_, done_;
};

void engine_kick(nb6_ctx* c) {
    if (c->engine) c->engine->kick();
}

void engine_shutdown(nb6_ctx* c) {
    if (!c->engine) return;
    c->engine->shutdown();
    delete c->engine;
    c->engine = nullptr;
}

}  // namespace nb6

using namespace nb6;

extern "C" {

int nb6_submit(nb6_ctx* c, const nb6_request* req, uint64_t* ticket) {
    if (!c || !req || !ticket) return NB6_ERR_ARG;
    if (!c->engine) {
        std::unique_ptr<Engine> e(new Engine(c));
        if (int rc = e->start()) {
            e->shutdown();
            return rc;
        }
        c->engine = e.release();
    }
    return c->engine->submit(req, ticket);
}

int nb6_poll(nb6_ctx* c, uint64_t ticket, int wait, nb6_ticket_info* info) {
    if (!c) return NB6_ERR_ARG;
    if (!c->engine) return fail(c, NB6_ERR_UNKNOWN_TICKET, "no request was ever submitted");
    return c->engine->poll(ticket, wait, info);
}

}  // extern "C"
