// nb6_api.hip -- the C ABI of include/nb6.h: contexts, cluster state,
// argument checking, work partitioning and kernel launches.
#include "nb6_context.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

using namespace nb6;

namespace nb6 {

int fail(nb6_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

// Grow a device buffer to at least `bytes`.  Growing waits for the device,
// because earlier stream-ordered work may still use the old allocation.
int ensure(nb6_ctx* c, DevBuf& b, size_t bytes) {
    if (bytes <= b.cap) return NB6_OK;
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    HIP_TRY(c, hipDeviceSynchronize());
    if (b.p) {
        HIP_TRY(c, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return fail(c, NB6_ERR_NOMEM, "device allocation of %zu bytes failed", bytes);
        }
        want = bytes;
    }
    b.cap = want;
    return NB6_OK;
}

void release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

int ensure_pinned(nb6_ctx* c, PinBuf& b, size_t bytes) {
    if (bytes <= b.cap) return NB6_OK;
    const size_t want = std::max(bytes, b.cap + b.cap / 2);
    if (b.p) HIP_TRY(c, hipHostFree(b.p));
    b.p = nullptr;
    b.cap = 0;
    if (hipHostMalloc((void**)&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(c, NB6_ERR_NOMEM, "pinned host allocation of %zu bytes failed", want);
    }
    b.cap = want;
    return NB6_OK;
}

static_assert(kPlanTile == VTILE, "slice lengths must be whole candidate-bound tiles");

Plan make_plan(const nb6_ctx* c, int64_t n, int64_t ni, int ipl) {
    return plan_rule(PlanInputs{c->num_cu, c->ipl_hint, c->jl_hint, c->slice_hint}, n, ni, ipl);
}

}  // namespace nb6

namespace {

// Scratch of nb6_regular_force_noalloc: one fixed array per GPU in the code
// object, held from the library's first use on that GPU until the process
// ends.  Host code never passes its name as an address (in host code the
// name is a host-side stand-in): the array's device address on each GPU is
// taken once, with that GPU current, by hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[NB6_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
int scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return NB6_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return NB6_ERR_HIP;
        }
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return NB6_OK;
}

bool finite_all(const double* p, int64_t n) {
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(p[k])) return false;
    return true;
}

// Event pair around one launch when timing is on (kind: 0 predict, 1 force,
// 2 finalize).
struct TimedLaunch {
    nb6_ctx* c;
    int kind;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    // kind < 0: not timed
    TimedLaunch(nb6_ctx* c_, int k, hipStream_t s) : c(c_), kind(k), st(s) {
        if (!c->timing || kind < 0) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, st);
    }
    void done() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        c->timed.push_back({kind, a, b});
        a = b = nullptr;
    }
};

// Ownership of a cluster for the duration of one plain call.  The call's
// stream first waits for the serving queue's last work on the cluster; at
// release, the call's own stream work is recorded for the queue to wait on.
class PlainClaim {
  public:
    PlainClaim() = default;
    PlainClaim(const PlainClaim&) = delete;
    PlainClaim& operator=(const PlainClaim&) = delete;
    // NB6_OK or NB6_ERR_STATE (a serving request is in flight on it).
    int claim(nb6_ctx* c, ClusterState* cl, hipStream_t st) {
        c_ = c;
        int expect = 0;
        if (!cl->owner.compare_exchange_strong(expect, -1))
            return fail(c, NB6_ERR_STATE, "cluster is in use by the serving queue");
        cl_ = cl;
        st_ = st;
        if (cl->last_served && hipStreamWaitEvent(st, cl->last_served, 0) != hipSuccess) {
            release();
            return fail(c, NB6_ERR_HIP, "hipStreamWaitEvent failed");
        }
        return NB6_OK;
    }
    ~PlainClaim() { release(); }

  private:
    void release() {
        if (!cl_) return;
        if (!cl_->last_plain)
            (void)hipEventCreateWithFlags(&cl_->last_plain, hipEventDisableTiming);
        if (cl_->last_plain) (void)hipEventRecord(cl_->last_plain, st_);
        cl_->owner.store(0);
        cl_ = nullptr;
        engine_kick(c_);
    }
    nb6_ctx* c_ = nullptr;
    ClusterState* cl_ = nullptr;
    hipStream_t st_ = nullptr;
};

// The cluster, if loaded.
int get_cluster(nb6_ctx* c, int cluster, ClusterState** out) {
    if (cluster < 0 || cluster >= kMaxClusters || !c->clusters[cluster] ||
        c->clusters[cluster]->n == 0)
        return fail(c, NB6_ERR_STATE, "cluster %d is not loaded", cluster);
    *out = c->clusters[cluster];
    return NB6_OK;
}

}  // namespace

extern "C" {

int nb6_create(nb6_ctx** out, const nb6_options* opt) {
    if (!out) return NB6_ERR_ARG;
    *out = nullptr;
    nb6_ctx* c = new nb6_ctx();
    if (opt) {
        c->device = opt->device;
        c->slice_hint = opt->slice_hint;
        c->hbm_budget = opt->hbm_budget;
        c->timing = (opt->flags & NB6_OPT_TIMING) != 0;
        c->iorder = (opt->flags & NB6_OPT_CALLER_ORDER) == 0;
        c->ipl_hint = opt->ipl_hint;
        c->jl_hint = opt->jl_hint;
        if (c->ipl_hint < 0 || c->ipl_hint > 2 || c->jl_hint < 0 || c->jl_hint > 64 ||
            (c->jl_hint & (c->jl_hint - 1)) != 0 || (c->jl_hint > 1 && c->ipl_hint == 2)) {
            delete c;
            return NB6_ERR_ARG;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || c->device < 0 || c->device >= ndev) {
        delete c;
        return NB6_ERR_ARG;
    }
    if (hipSetDevice(c->device) != hipSuccess) {
        delete c;
        return NB6_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    if (hipMalloc(&c->status, 4 * sizeof(unsigned)) != hipSuccess) {
        delete c;
        return NB6_ERR_NOMEM;
    }
    void* scr = nullptr;  // the no-allocation scratch's address on this GPU
    if (launch_zero_u32(c->status, 4, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess || scratch_address(c->device, &scr) != NB6_OK) {
        (void)hipFree(c->status);
        delete c;
        return NB6_ERR_HIP;
    }
    if (c->hbm_budget <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) c->hbm_budget = (int64_t)(fr / 4);
    }
    c->clusters.assign(kMaxClusters, nullptr);
    *out = c;
    return NB6_OK;
}

int nb6_destroy(nb6_ctx* c) {
    if (!c) return NB6_OK;
    engine_shutdown(c);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (ClusterState* cl : c->clusters) {
        if (!cl) continue;
        if (cl->state) (void)hipFree(cl->state);
        for (auto& r : cl->rec) release(r);
        for (DevBuf* b : {&cl->tmax, &cl->org, &cl->perm, &cl->inv, &cl->nbl, &cl->nbc})
            release(*b);
        if (cl->last_plain) (void)hipEventDestroy(cl->last_plain);
        if (cl->last_served) (void)hipEventDestroy(cl->last_served);
        delete cl;
    }
    for (DevBuf* b : {&c->part, &c->cnt, &c->lst, &c->io, &c->out_list, &c->order_tmp, &c->iord,
                       &c->iord_tmp})
        release(*b);
    if (c->pin.p) (void)hipHostFree(c->pin.p);
    for (auto& b : c->ld) release(b);
    if (c->status) (void)hipFree(c->status);
    for (auto& t : c->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    delete c;
    return NB6_OK;
}

int nb6_kernel_times(nb6_ctx* c, double* ms, int64_t* counts) {
    if (!c || !ms || !counts) return NB6_ERR_ARG;
    if (!c->timing) return fail(c, NB6_ERR_STATE, "context created without NB6_OPT_TIMING");
    HIP_TRY(c, hipSetDevice(c->device));
    for (int k = 0; k < 4; ++k) { ms[k] = 0.0; counts[k] = 0; }
    int rc = NB6_OK;
    for (auto& t : c->timed) {
        float e = 0.0f;
        if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&e, t.a, t.b) != hipSuccess)
            rc = fail(c, NB6_ERR_HIP, "event timing failed");
        ms[t.kind] += e;
        counts[t.kind] += 1;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    c->timed.clear();
    return rc;
}

const char* nb6_last_error(const nb6_ctx* c) { return c ? c->err.c_str() : "no context"; }

int nb6_last_slices(const nb6_ctx* c) { return c ? c->last_plan.nslices : 0; }

int nb6_last_plan(const nb6_ctx* c, int out[4]) {
    if (!c || !out) return NB6_ERR_ARG;
    out[0] = c->last_plan.ipl;
    out[1] = 1 << c->last_plan.jl_shift;
    out[2] = c->last_plan.nslices;
    out[3] = c->last_plan.slice_len;
    return NB6_OK;
}

// Spatial order of the cluster's particles (the local-coordinate stream's
// record order) from its stored positions, on stream st.
static int build_order(nb6_ctx* c, ClusterState* cl, hipStream_t st) {
    const size_t n = (size_t)cl->n;
    int rc;
    if ((rc = ensure(c, cl->perm, n * sizeof(int32_t))) ||
        (rc = ensure(c, cl->inv, n * sizeof(int32_t))) ||
        (rc = ensure(c, c->order_tmp, order_scratch_bytes(cl->n))))
        return rc;
    HIP_TRY(c, launch_order(cl->state, cl->n, c->order_tmp.p, c->order_tmp.cap,
                            (int32_t*)cl->perm.p, (int32_t*)cl->inv.p, st));
    cl->order_valid = true;
    cl->updated_since_order = 0;
    return NB6_OK;
}

int nb6_load_particles(nb6_ctx* c, int cluster, int64_t n, const double* m, const double* x,
                       const double* v, const double* a, const double* jerk, const double* t,
                       const int32_t* idx, int mem_kind, void* stream) {
    if (!c) return NB6_ERR_ARG;
    c->err.clear();
    if (cluster < 0 || cluster >= kMaxClusters)
        return fail(c, NB6_ERR_ARG, "cluster %d out of range [0, %d)", cluster, kMaxClusters);
    if (n <= 0 || n > INT32_MAX) return fail(c, NB6_ERR_ARG, "n = %lld out of range", (long long)n);
    if (!m || !x || !v || !a || !jerk || !t) return fail(c, NB6_ERR_ARG, "null state array");
    if (mem_kind != NB6_MEM_HOST && mem_kind != NB6_MEM_DEVICE)
        return fail(c, NB6_ERR_ARG, "bad mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    std::lock_guard<std::mutex> lk(c->cluster_mu);
    ClusterState*& cl = c->clusters[cluster];
    if (!cl) cl = new ClusterState();
    PlainClaim claim;
    if (int rc = claim.claim(c, cl, st)) return rc;

    if (mem_kind == NB6_MEM_HOST) {
        if (!finite_all(m, n) || !finite_all(t, n) || !finite_all(x, 3 * n) ||
            !finite_all(v, 3 * n) || !finite_all(a, 3 * n) || !finite_all(jerk, 3 * n))
            return fail(c, NB6_ERR_ARG, "non-finite value in the particle state");
    }
    if (!idx) {  // full load
        if (cl->n != n && cl->queued.load() > 0)
            return fail(c, NB6_ERR_STATE,
                        "cluster %d has serving requests queued; it cannot be resized", cluster);
        if (cl->n != n) {
            HIP_TRY(c, hipDeviceSynchronize());
            if (cl->state) HIP_TRY(c, hipFree(cl->state));
            cl->state = nullptr;
            cl->n = 0;
            // the predicted records and stored lists are sized by n:
            // reallocated on next use
            for (DevBuf& b : cl->rec) release(b);
            for (DevBuf* b : {&cl->tmax, &cl->org, &cl->perm, &cl->inv, &cl->nbl, &cl->nbc})
                release(*b);
            cl->lcap = 0;
            cl->order_valid = false;
            if (hipMalloc(&cl->state, (size_t)n * sizeof(StateRec)) != hipSuccess) {
                (void)hipGetLastError();
                cl->state = nullptr;
                return fail(c, NB6_ERR_NOMEM, "cluster state of %lld particles", (long long)n);
            }
            cl->n = n;
        }
    } else {
        if (!cl || cl->n == 0) return fail(c, NB6_ERR_STATE, "cluster %d is not loaded", cluster);
        if (n > cl->n) return fail(c, NB6_ERR_ARG, "subset of %lld > cluster size", (long long)n);
    }
    // both forms pack the structure-of-arrays input into the state records
    ScatterArgs sa{};
    sa.n = n;
    sa.limit = cl->n;
    sa.status = c->status;
    sa.dst = cl->state;
    if (mem_kind == NB6_MEM_HOST) {
        if (idx)
            for (int64_t k = 0; k < n; ++k)
                if (idx[k] < 0 || idx[k] >= cl->n)
                    return fail(c, NB6_ERR_ARG, "idx[%lld] = %d out of range", (long long)k,
                                idx[k]);
        const size_t sz[7] = {n * sizeof(int32_t), n * sizeof(double), n * sizeof(double),
                              3 * n * sizeof(double), 3 * n * sizeof(double),
                              3 * n * sizeof(double), 3 * n * sizeof(double)};
        const void* src[7] = {idx, m, t, x, v, a, jerk};
        const void* dst[7] = {};
        Stage lay;
        size_t off[7] = {};
        for (int k = idx ? 0 : 1; k < 7; ++k) off[k] = lay.add(sz[k]);
        if (lay.end <= kStageLoadMax) {
            // a block's subset update: the arrays go up in one copy through
            // the pinned buffer (one call, one DMA, instead of seven)
            int rc;
            if ((rc = ensure(c, c->io, lay.end)) || (rc = ensure_pinned(c, c->pin, lay.end)))
                return rc;
            for (int k = idx ? 0 : 1; k < 7; ++k) {
                std::memcpy(c->pin.p + off[k], src[k], sz[k]);
                dst[k] = (const char*)c->io.p + off[k];
            }
            HIP_TRY(c, hipMemcpyAsync(c->io.p, c->pin.p, lay.end, hipMemcpyHostToDevice, st));
        } else {
            // a large load: the runtime pipelines pageable copies by itself
            for (int k = idx ? 0 : 1; k < 7; ++k) {
                int rc = ensure(c, c->ld[k], sz[k]);
                if (rc) return rc;
                HIP_TRY(c, hipMemcpyAsync(c->ld[k].p, src[k], sz[k], hipMemcpyHostToDevice, st));
                dst[k] = c->ld[k].p;
            }
        }
        sa.idx = idx ? (const int32_t*)dst[0] : nullptr;
        sa.m = (const double*)dst[1];
        sa.t = (const double*)dst[2];
        sa.x = (const double*)dst[3];
        sa.v = (const double*)dst[4];
        sa.a = (const double*)dst[5];
        sa.jk = (const double*)dst[6];
    } else {
        sa.idx = idx; sa.m = m; sa.t = t; sa.x = x; sa.v = v; sa.a = a; sa.jk = jerk;
    }
    HIP_TRY(c, launch_scatter(sa, st));
    // a full load starts every stored neighbour list empty
    if (!idx && cl->nbc.p) HIP_TRY(c, launch_zero_u32((unsigned*)cl->nbc.p, (int)n, st));
    // the spatial order of the local-coordinate stream: rebuilt from the
    // stored state after a full load and once the subset updates since the
    // last build have touched as many particles as the cluster holds
    cl->updated_since_order = idx ? cl->updated_since_order + n : cl->n;
    if (!idx) cl->order_valid = false;
    if (!cl->order_valid || cl->updated_since_order >= cl->n) {
        if (int rc = build_order(c, cl, st)) return rc;
    }
    if (mem_kind == NB6_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(st));
    cl->pred_valid = 0;
    return NB6_OK;
}

int nb6_predict_j(nb6_ctx* c, int cluster, double t_block, int modes, void* stream) {
    if (!c) return NB6_ERR_ARG;
    c->err.clear();
    std::lock_guard<std::mutex> lk(c->cluster_mu);
    ClusterState* cl = nullptr;
    if (int rc = get_cluster(c, cluster, &cl)) return rc;
    PlainClaim claim;
    if (int rc = claim.claim(c, cl, (hipStream_t)stream)) return rc;
    if (modes == 0) modes = NB6_DX_ALL;
    if (modes & ~NB6_DX_ALL) return fail(c, NB6_ERR_ARG, "bad modes mask %d", modes);
    if (!std::isfinite(t_block)) return fail(c, NB6_ERR_ARG, "non-finite t_block");
    HIP_TRY(c, hipSetDevice(c->device));
    PredictArgs pa{};
    pa.n = cl->n;
    pa.st = cl->state;
    pa.tb = t_block;
    pa.status = c->status;
    const int bits[NMODES] = {NB6_DX_FF, NB6_DX_FP64, NB6_DX_FP32, NB6_DX_LOCAL};
    const bool loc = (modes & NB6_DX_LOCAL) != 0;
    for (int mi = 0; mi < NMODES; ++mi) {
        if (!(modes & bits[mi]) && !(loc && mi == MODE_FF)) continue;
        int rc = ensure(c, cl->rec[mi], (size_t)cl->n * rec_size(mi));
        if (rc) return rc;
    }
    if (int rc = ensure(c, cl->tmax, (size_t)vtiles(cl->n) * sizeof(float))) return rc;
    if (loc) {
        if (!cl->order_valid)
            return fail(c, NB6_ERR_STATE, "cluster %d has no spatial order", cluster);
        if (int rc = ensure(c, cl->org, (size_t)vtiles(cl->n) * sizeof(TileOrg))) return rc;
    }
    pa.tmax = (float*)cl->tmax.p;
    // the local mode's i-side is the float-float prediction by index, which
    // the index pass writes with its tiles' candidate bounds (a latency-bound
    // local-mode call runs the float-float kernel on them)
    pa.ff = (modes & NB6_DX_FF) || loc ? (RecFF*)cl->rec[MODE_FF].p : nullptr;
    pa.f64 = (modes & NB6_DX_FP64) ? (RecF64*)cl->rec[MODE_F64].p : nullptr;
    pa.f32 = (modes & NB6_DX_FP32) ? (RecF32*)cl->rec[MODE_F32].p : nullptr;
    TimedLaunch tl(c, 0, (hipStream_t)stream);
    if (pa.ff || pa.f64 || pa.f32) HIP_TRY(c, launch_predict(pa, (hipStream_t)stream));
    if (loc) {
        // the local stream by slot (the index pass above wrote its i-side)
        PredictArgs pl = pa;
        pl.f64 = nullptr;
        pl.f32 = nullptr;
        pl.ff = nullptr;
        pl.loc = (RecLoc*)cl->rec[MODE_LOC].p;
        pl.org = (TileOrg*)cl->org.p;
        pl.perm = (const int32_t*)cl->perm.p;
        HIP_TRY(c, launch_predict_loc(pl, (hipStream_t)stream));
    }
    tl.done();
    // records of other modes predicted to this same block time stay current
    cl->pred_valid = (cl->t_pred == t_block ? cl->pred_valid : 0) | modes;
    cl->t_pred = t_block;
    return NB6_OK;
}

// The lists of a HOST-mode call too big to stage with the other outputs:
// only the first min(nnb, cap) entries of each row cross PCIe.  The row
// offsets come from the counts already on the host; a kernel packs the rows
// into one array, one copy brings it into the pinned buffer, and host threads
// place each row in the caller's array (entries past a row's count are left
// as they were).
static int copy_lists_out(nb6_ctx* c, const int32_t* d_list, const int32_t* nnb, int ni,
                          int cap, int32_t* list, hipStream_t st) {
    Stage lay;
    const size_t o_off = lay.add(((size_t)ni + 1) * sizeof(int64_t));
    const std::vector<int64_t> off = row_offsets(nnb, ni, cap);
    const int64_t total = off[ni];
    const size_t o_pack = lay.add((size_t)total * sizeof(int32_t));
    if (int rc = ensure(c, c->io, lay.end)) return rc;
    if (int rc = ensure_pinned(c, c->pin, lay.end)) return rc;
    char* pin = c->pin.p;
    char* dev = (char*)c->io.p;
    std::memcpy(pin + o_off, off.data(), ((size_t)ni + 1) * sizeof(int64_t));
    HIP_TRY(c, hipMemcpyAsync(dev + o_off, pin + o_off, ((size_t)ni + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, st));
    HIP_TRY(c, launch_pack_rows(d_list, cap, (const int64_t*)(dev + o_off), ni,
                                (int32_t*)(dev + o_pack), st));
    HIP_TRY(c, hipMemcpyAsync(pin + o_pack, dev + o_pack, (size_t)total * sizeof(int32_t),
                              hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    unpack_rows_host(off, ni, cap, (const int32_t*)(pin + o_pack), list);
    return NB6_OK;
}

// Smallest one-lane-per-i block that a plain call runs in the i-order (it
// must also hold three quarters of its cluster).
constexpr int kIOrderMin = 8192;

// Device arrays of one force call: its inputs and outputs, and its scratch
// (slice partial sums, per-i counters that must be zero on entry, list rows).
struct ForceIO {
    const int32_t* idx;
    const double* h2;
    const double* dtr;
    double* acc;
    double* jerk;
    double* pot;  // null: no potential
    int32_t* nnb;
    int32_t* list;
};
// An i-order of the call: iord[work position] = active position, and the
// force kernel's i-side in work order (index, radius, dtr, i-record).
struct IOrder {
    const int32_t* iord;
    const int32_t* idx;
    const double* h2;
    const double* dtr;
    const void* irec;
};
struct ForceScratch {
    double* part;
    int32_t* cnt;
    int32_t* lst;
    IOrder io;  // all null: the caller's order
};

// Bytes of a force call's scratch for plan p: the partials of every
// 64-particle block and slice, then the counters, then the list rows, each
// starting on a 256-byte boundary (the layout of the no-allocation array).
static size_t force_scratch_layout(const Plan& p, int ni, int npart, int caps, size_t off[3]) {
    const size_t ni64 = ((size_t)ni + 63) / 64 * 64;
    Stage lay;
    off[0] = lay.add((size_t)p.nslices * npart * ni64 * sizeof(double));
    off[1] = lay.add((size_t)ni * sizeof(int32_t));
    off[2] = lay.add((size_t)ni * caps * sizeof(int32_t));
    return lay.end;
}

// The two launches of a force call, force kernel then finalize, on st (event
// timing when `timed` and the context has it on).
static int launch_force_call(nb6_ctx* c, const ClusterState* cl, int mi, int ni, int cap,
                             const Plan& p, const ForceIO& io, const ForceScratch& fs,
                             hipStream_t st, bool timed) {
    mi = kernel_mode(mi, p);  // a latency-bound local-mode call: float-float
    RegfArgs ra{};
    ra.rec = cl->rec[mi].p;
    ra.n = (int)cl->n;
    const bool ord = fs.io.iord != nullptr;
    ra.idx = ord ? fs.io.idx : io.idx;
    ra.h2 = ord ? fs.io.h2 : io.h2;
    ra.dtr = ord ? fs.io.dtr : io.dtr;
    ra.irec = ord ? fs.io.irec : nullptr;
    ra.ni = ni;
    ra.slice_len = p.slice_len;
    ra.nslices = p.nslices;
    ra.jl_shift = p.jl_shift;
    ra.tmax = (const float*)cl->tmax.p;
    if (mi == MODE_LOC) {
        ra.org = (const TileOrg*)cl->org.p;
        ra.ivw = cl->rec[MODE_FF].p;
    }
    ra.part = fs.part;
    ra.cnt = fs.cnt;
    ra.lst = fs.lst;
    ra.caps = cap + 1;  // room for the i-particle itself
    ra.status = c->status;
    {
        TimedLaunch tl(c, timed ? 1 : -1, st);
        HIP_TRY(c, launch_regf(mi, p.ipl, p.wpb, io.pot != nullptr, ra, st));
        tl.done();
    }
    FinalArgs fa{};
    fa.part = ra.part;
    fa.cnt = ra.cnt;
    fa.lst = ra.lst;
    fa.nslices = p.nslices;
    fa.ni = ni;
    fa.caps = ra.caps;
    fa.n = (int)cl->n;
    fa.idx = io.idx;
    fa.h2 = io.h2;
    fa.acc = io.acc;
    fa.jerk = io.jerk;
    fa.pot = io.pot;
    fa.nnb = io.nnb;
    fa.list = io.list;
    fa.cap = cap;
    fa.status = c->status;
    fa.rec = ra.rec;
    fa.dtr = io.dtr;
    fa.mode = mi;
    fa.org = ra.org;
    fa.inv = mi == MODE_LOC ? (const int32_t*)cl->inv.p : nullptr;
    fa.ivw = ra.ivw;
    fa.iord = fs.io.iord;
    {
        TimedLaunch tl(c, timed ? 2 : -1, st);
        HIP_TRY(c, launch_finalize(fa, st));
        tl.done();
    }
    return NB6_OK;
}

int nb6_regular_force(nb6_ctx* c, int cluster, int64_t n_i, const int32_t* idx_i,
                      const double* h2_i, const double* dtr_i, int dx_mode, double* acc,
                      double* jerk, double* pot, int32_t* nnb, int32_t* list, int32_t cap,
                      int mem_kind, void* stream) {
    if (!c) return NB6_ERR_ARG;
    c->err.clear();
    std::lock_guard<std::mutex> lk(c->cluster_mu);
    ClusterState* cl = nullptr;
    if (int rc = get_cluster(c, cluster, &cl)) return rc;
    PlainClaim claim;
    if (int rc = claim.claim(c, cl, (hipStream_t)stream)) return rc;
    const int mi = mode_index(dx_mode);
    if (mi < 0) return fail(c, NB6_ERR_ARG, "bad dx_mode %d", dx_mode);
    if (!(cl->pred_valid & dx_mode))
        return fail(c, NB6_ERR_STATE, "cluster %d has no current prediction for dx_mode %d",
                    cluster, dx_mode);
    if (n_i < 0 || n_i > INT32_MAX / 2) return fail(c, NB6_ERR_ARG, "n_i = %lld", (long long)n_i);
    static_assert(MAX_CAPS - 1 == NB6_MAX_CAP, "list capacity limits disagree");
    if (cap < 0 || cap > MAX_CAPS - 1)
        return fail(c, NB6_ERR_ARG, "cap = %d outside [0, %d]", cap, MAX_CAPS - 1);
    if (mem_kind != NB6_MEM_HOST && mem_kind != NB6_MEM_DEVICE)
        return fail(c, NB6_ERR_ARG, "bad mem_kind %d", mem_kind);
    if (n_i == 0) return NB6_OK;
    if (!idx_i || !h2_i || !dtr_i || !acc || !jerk || !nnb || (cap > 0 && !list))
        return fail(c, NB6_ERR_ARG, "null argument");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = cl->n;
    const int ni = (int)n_i;

    const int32_t* d_idx = idx_i;
    const double* d_h2 = h2_i;
    const double* d_dtr = dtr_i;
    double* d_acc = acc;
    double* d_jerk = jerk;
    double* d_pot = pot;
    int32_t* d_nnb = nnb;
    int32_t* d_list = list;
    struct {
        Stage lay;
        size_t idx, h2, dtr, in_end, acc, jerk, pot, nnb, list, out_end, status;
        bool list_staged;
    } hs{};
    if (mem_kind == NB6_MEM_HOST) {
        for (int q = 0; q < ni; ++q) {
            if (idx_i[q] < 0 || idx_i[q] >= n)
                return fail(c, NB6_ERR_ARG, "idx_i[%d] = %d out of range", q, idx_i[q]);
            const float h2f = (float)h2_i[q];
            if (!(h2f >= FLT_MIN) || !(h2f <= FLT_MAX))
                return fail(c, NB6_ERR_ARG, "h2_i[%d] = %g is not a positive normal float", q,
                            h2_i[q]);
            if (!valid_dtr(dtr_i[q]))
                return fail(c, NB6_ERR_ARG, "dtr_i[%d] = %g is not a finite value >= 0", q,
                            dtr_i[q]);
        }
        // inputs go up in one copy from the pinned buffer; the outputs (and
        // lists up to kStageListMax bytes) come back in one copy into it
        const size_t list_bytes = (size_t)ni * cap * sizeof(int32_t);
        hs.list_staged = cap > 0 && list_bytes <= kStageListMax;
        hs.idx = hs.lay.add(ni * sizeof(int32_t));
        hs.h2 = hs.lay.add(ni * sizeof(double));
        hs.dtr = hs.lay.add(ni * sizeof(double));
        hs.in_end = hs.lay.end;
        hs.acc = hs.lay.add(3 * ni * sizeof(double));
        hs.jerk = hs.lay.add(3 * ni * sizeof(double));
        hs.pot = pot ? hs.lay.add(ni * sizeof(double)) : 0;
        hs.nnb = hs.lay.add(ni * sizeof(int32_t));
        hs.list = hs.list_staged ? hs.lay.add(list_bytes) : 0;
        hs.out_end = hs.lay.end;
        hs.status = hs.lay.add(4 * sizeof(unsigned));
        int rc;
        if ((rc = ensure(c, c->io, hs.lay.end)) || (rc = ensure_pinned(c, c->pin, hs.lay.end)) ||
            (cap > 0 && !hs.list_staged && (rc = ensure(c, c->out_list, list_bytes))))
            return rc;
        char* pin = c->pin.p;
        char* dev = (char*)c->io.p;
        std::memcpy(pin + hs.idx, idx_i, ni * sizeof(int32_t));
        std::memcpy(pin + hs.h2, h2_i, ni * sizeof(double));
        std::memcpy(pin + hs.dtr, dtr_i, ni * sizeof(double));
        HIP_TRY(c, hipMemcpyAsync(dev, pin, hs.in_end, hipMemcpyHostToDevice, st));
        d_idx = (const int32_t*)(dev + hs.idx);
        d_h2 = (const double*)(dev + hs.h2);
        d_dtr = (const double*)(dev + hs.dtr);
        d_acc = (double*)(dev + hs.acc);
        d_jerk = (double*)(dev + hs.jerk);
        d_nnb = (int32_t*)(dev + hs.nnb);
        d_list = hs.list_staged ? (int32_t*)(dev + hs.list) : (int32_t*)c->out_list.p;
        if (pot) d_pot = (double*)(dev + hs.pot);
    }

    const Plan p = make_plan(c, n, ni);
    const int npart = pot ? NPART_POT : NPART;
    const int caps = cap + 1;  // room for the i-particle itself
    int rc;
    const size_t ni64 = ((size_t)ni + 63) / 64 * 64;  // partials by 64-particle block
    const size_t cnt_cap_before = c->cnt.cap;  // a reallocation changes the capacity
    if ((rc = ensure(c, c->part, (size_t)p.nslices * npart * ni64 * sizeof(double))) ||
        (rc = ensure(c, c->cnt, (size_t)ni * sizeof(int32_t))) ||
        (rc = ensure(c, c->lst, (size_t)ni * caps * sizeof(int32_t))))
        return rc;
    int32_t* d_cnt = (int32_t*)c->cnt.p;  // [ni] counts: zero between calls
    if (c->cnt_dirty || c->cnt.cap != cnt_cap_before) {
        HIP_TRY(c, launch_zero_u32((unsigned*)d_cnt, (int)(c->cnt.cap / sizeof(int32_t)), st));
        c->cnt_dirty = false;
    }

    // A block of one lane per i that holds most of its cluster runs in the
    // cluster's spatial order of its particles (the i-order): a wavefront's
    // i then lie close together, so its lanes take the candidate branch for
    // nearly the same j, and the branch is taken far less often.  Measured
    // in one process against the caller's order: C3 all active, force
    // kernel 2.2 % faster, call 1.3 % (the finalize's scattered stores and
    // the counting sort take the rest); half of C3 active, no change; 8192
    // and 16384 of it, 4-6 % slower (their i are too sparse to share
    // candidates, and the candidate work bunches in few work items).  The
    // bits of every result are the same either way.
    // The force kernel reads its i-side in work order, staged contiguously:
    // read through the i-order directly, each work item's 64 lanes would
    // touch 64 scattered lines per array, every slice over again.
    IOrder ord{};
    if (c->iorder && p.jl_shift == 0 && ni >= kIOrderMin && 4 * (int64_t)ni >= 3 * n &&
        cl->order_valid && cl->inv.p) {
        const int irec_mode = mi == MODE_LOC ? MODE_FF : mi;  // the mode's i-records
        const size_t rb = rec_size(irec_mode);
        Stage lay;
        const size_t o_iord = lay.add((size_t)ni * sizeof(int32_t));
        const size_t o_idx = lay.add((size_t)ni * sizeof(int32_t));
        const size_t o_h2 = lay.add((size_t)ni * sizeof(double));
        const size_t o_dtr = lay.add((size_t)ni * sizeof(double));
        const size_t o_rec = lay.add((size_t)ni * rb);
        if ((rc = ensure(c, c->iord, lay.end)) ||
            (rc = ensure(c, c->iord_tmp, iorder_scratch_bytes(ni, n))))
            return rc;
        char* b = (char*)c->iord.p;
        int32_t* iord = (int32_t*)(b + o_iord);
        HIP_TRY(c, launch_iorder(d_idx, ni, (const int32_t*)cl->inv.p, n, c->iord_tmp.p,
                                 c->iord_tmp.cap, iord, st));
        HIP_TRY(c, launch_istage(iord, ni, d_idx, d_h2, d_dtr, n, cl->rec[irec_mode].p, (int)rb,
                                 (int32_t*)(b + o_idx), (double*)(b + o_h2),
                                 (double*)(b + o_dtr), b + o_rec, st));
        ord = IOrder{iord, (const int32_t*)(b + o_idx), (const double*)(b + o_h2),
                     (const double*)(b + o_dtr), b + o_rec};
    }

    // the finalize resets the counts; until it is launched they are dirty
    c->cnt_dirty = true;
    const ForceIO io{d_idx, d_h2, d_dtr, d_acc, d_jerk, pot ? d_pot : nullptr, d_nnb, d_list};
    const ForceScratch fs{(double*)c->part.p, d_cnt, (int32_t*)c->lst.p, ord};
    if (int rc2 = launch_force_call(c, cl, mi, ni, cap, p, io, fs, st, true)) return rc2;
    c->cnt_dirty = false;
    c->last_plan = p;

    if (mem_kind == NB6_MEM_DEVICE) return NB6_OK;

    char* pin = c->pin.p;
    HIP_TRY(c, hipMemcpyAsync(pin + hs.in_end, (char*)c->io.p + hs.in_end, hs.out_end - hs.in_end,
                              hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(pin + hs.status, c->status, 4 * sizeof(unsigned),
                              hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    HIP_TRY(c, launch_zero_u32(c->status, 4, st));
    std::memcpy(acc, pin + hs.acc, 3 * ni * sizeof(double));
    std::memcpy(jerk, pin + hs.jerk, 3 * ni * sizeof(double));
    std::memcpy(nnb, pin + hs.nnb, ni * sizeof(int32_t));
    if (pot) std::memcpy(pot, pin + hs.pot, ni * sizeof(double));
    if (hs.list_staged) std::memcpy(list, pin + hs.list, (size_t)ni * cap * sizeof(int32_t));
    unsigned status[4];
    std::memcpy(status, pin + hs.status, sizeof status);
    if (cap > 0 && !hs.list_staged) {
        if (int rc = copy_lists_out(c, d_list, nnb, ni, cap, list, st)) return rc;
    }
    if (status[0] & (ST_BAD_INDEX | ST_BAD_H2 | ST_NONFINITE | ST_BAD_DTR))
        return fail(c, NB6_ERR_DEVICE_INPUT, "GPU validation flagged 0x%x", status[0]);
    for (int q = 0; q < ni; ++q)
        if (nnb[q] > cap) return NB6_WARN_NB_OVERFLOW;
    return NB6_OK;
}

int nb6_regular_force_noalloc(nb6_ctx* c, int cluster, int64_t n_i, const int32_t* idx_i,
                              const double* h2_i, const double* dtr_i, int dx_mode,
                              double* acc, double* jerk, double* pot, int32_t* nnb,
                              int32_t* list, int32_t cap, void* stream) {
    if (!c) return NB6_ERR_ARG;
    c->err.clear();
    std::lock_guard<std::mutex> lk(c->cluster_mu);
    ClusterState* cl = nullptr;
    if (int rc = get_cluster(c, cluster, &cl)) return rc;
    PlainClaim claim;
    if (int rc = claim.claim(c, cl, (hipStream_t)stream)) return rc;
    const int mi = mode_index(dx_mode);
    if (mi < 0) return fail(c, NB6_ERR_ARG, "bad dx_mode %d", dx_mode);
    if (!(cl->pred_valid & dx_mode))
        return fail(c, NB6_ERR_STATE, "cluster %d has no current prediction for dx_mode %d",
                    cluster, dx_mode);
    if (n_i < 0 || n_i > INT32_MAX / 2) return fail(c, NB6_ERR_ARG, "n_i = %lld", (long long)n_i);
    if (cap < 0 || cap > MAX_CAPS - 1)
        return fail(c, NB6_ERR_ARG, "cap = %d outside [0, %d]", cap, MAX_CAPS - 1);
    if (n_i == 0) return NB6_OK;
    if (!idx_i || !h2_i || !dtr_i || !acc || !jerk || !nnb || (cap > 0 && !list))
        return fail(c, NB6_ERR_ARG, "null argument");
    HIP_TRY(c, hipSetDevice(c->device));
    void* base = nullptr;
    if (scratch_address(c->device, &base) != NB6_OK)
        return fail(c, NB6_ERR_HIP, "no address for the scratch array on device %d", c->device);
    hipStream_t st = (hipStream_t)stream;
    const int ni = (int)n_i;
    const int npart = pot ? NPART_POT : NPART;
    const size_t limit = NB6_NOALLOC_SCRATCH_BYTES;
    // the plain call's plan when its scratch fits; otherwise the most
    // j-slices whose partials fit beside the counters and the list rows
    Plan p = make_plan(c, cl->n, ni);
    size_t off[3];
    size_t need = force_scratch_layout(p, ni, npart, cap + 1, off);
    if (need > limit) {
        Plan none = p;
        none.nslices = 0;
        const size_t fixed = force_scratch_layout(none, ni, npart, cap + 1, off);
        const size_t per_slice = (((size_t)ni + 63) / 64 * 64) * npart * sizeof(double);
        int64_t s = fixed + 256 < limit ? (int64_t)((limit - fixed - 256) / per_slice) : 0;
        if (s >= 8) s = s / 8 * 8;
        if (s >= 1) {
            p = plan_rule(PlanInputs{c->num_cu, c->ipl_hint, c->jl_hint, (int)s}, cl->n, ni, 0);
            need = force_scratch_layout(p, ni, npart, cap + 1, off);
        }
        if (s < 1 || need > limit)
            return fail(c, NB6_ERR_ARG,
                        "the call needs %zu bytes of scratch (%zu with one j-slice); the "
                        "no-allocation array holds %zu", need, fixed + per_slice, limit);
    }
    char* b = static_cast<char*>(base);
    // no i-order here: its sort would need scratch of its own (the results
    // are the same bits without it)
    const ForceScratch fs{(double*)(b + off[0]), (int32_t*)(b + off[1]), (int32_t*)(b + off[2]),
                          IOrder{}};
    // the counters start at zero: cleared by a kernel (no memset node, so a
    // captured graph may hold the call)
    HIP_TRY(c, launch_zero_u32((unsigned*)fs.cnt, ni, st));
    const ForceIO io{idx_i, h2_i, dtr_i, acc, jerk, pot, nnb, list};
    if (int rc = launch_force_call(c, cl, mi, ni, cap, p, io, fs, st, false)) return rc;
    c->last_plan = p;
    return NB6_OK;
}

int nb6_get_predicted(nb6_ctx* c, int cluster, int dx_mode, double* x, double* v,
                      int mem_kind, void* stream) {
    if (!c) return NB6_ERR_ARG;
    c->err.clear();
    std::lock_guard<std::mutex> lk(c->cluster_mu);
    ClusterState* cl = nullptr;
    if (int rc = get_cluster(c, cluster, &cl)) return rc;
    PlainClaim claim;
    if (int rc = claim.claim(c, cl, (hipStream_t)stream)) return rc;
    const int mi = mode_index(dx_mode);
    if (mi < 0) return fail(c, NB6_ERR_ARG, "bad dx_mode %d", dx_mode);
    if (!(cl->pred_valid & dx_mode))
        return fail(c, NB6_ERR_STATE, "no current prediction for dx_mode %d", dx_mode);
    if (!x || !v) return fail(c, NB6_ERR_ARG, "null output");
    if (mem_kind != NB6_MEM_HOST && mem_kind != NB6_MEM_DEVICE)
        return fail(c, NB6_ERR_ARG, "bad mem_kind %d", mem_kind);
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = cl->n;
    double* dx = x;
    double* dv = v;
    if (mem_kind == NB6_MEM_HOST) {  // a diagnostic read: through device scratch
        Stage lay;
        const size_t o_v = (lay.add(3 * n * sizeof(double)), lay.add(3 * n * sizeof(double)));
        if (int rc = ensure(c, c->io, lay.end)) return rc;
        dx = (double*)c->io.p;
        dv = (double*)((char*)c->io.p + o_v);
    }
    // the local stream's positions are those of the float-float prediction
    // written with it (the records hold tile offsets)
    const int um = mi == MODE_LOC ? MODE_FF : mi;
    HIP_TRY(c, launch_unpack(um, cl->rec[um].p, n, dx, dv, st));
    if (mem_kind == NB6_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(x, dx, 3 * n * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipMemcpyAsync(v, dv, 3 * n * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
    }
    return NB6_OK;
}

// Stored lists of a cluster exist (counts zeroed) and rows hold >= cap entries.
static int ensure_lists(nb6_ctx* c, ClusterState* cl, int cap, hipStream_t st) {
    const int64_t n = cl->n;
    if (!cl->nbc.p) {
        if (int rc = ensure(c, cl->nbc, (size_t)n * sizeof(int32_t))) return rc;
        HIP_TRY(c, launch_zero_u32((unsigned*)cl->nbc.p, (int)n, st));
    }
    if (cap <= cl->lcap) return NB6_OK;
    DevBuf grown;
    if (int rc = ensure(c, grown, (size_t)n * cap * sizeof(int32_t))) return rc;
    if (cl->lcap > 0) {
        HIP_TRY(c, launch_copy_rows((const int32_t*)cl->nbl.p, cl->lcap, (int32_t*)grown.p, cap,
                                    (const int32_t*)cl->nbc.p, n, st));
        HIP_TRY(c, hipStreamSynchronize(st));  // the old rows are freed next
    }
    release(cl->nbl);
    cl->nbl = grown;
    cl->lcap = cap;
    return NB6_OK;
}

int nb6_set_lists(nb6_ctx* c, int cluster, int64_t n_i, const int32_t* idx_i,
                  const int32_t* nnb_i, const int32_t* list, int32_t cap, int mem_kind,
                  void* stream) {
    if (!c) return NB6_ERR_ARG;
    c->err.clear();
    std::lock_guard<std::mutex> lk(c->cluster_mu);
    ClusterState* cl = nullptr;
    if (int rc = get_cluster(c, cluster, &cl)) return rc;
    PlainClaim claim;
    if (int rc = claim.claim(c, cl, (hipStream_t)stream)) return rc;
    static_assert(MAX_LIST_CAP == NB6_MAX_LIST_CAP, "stored-list limits disagree");
    if (n_i < 0 || n_i > cl->n) return fail(c, NB6_ERR_ARG, "n_i = %lld", (long long)n_i);
    if (cap < 1 || cap > MAX_LIST_CAP)
        return fail(c, NB6_ERR_ARG, "cap = %d outside [1, %d]", cap, MAX_LIST_CAP);
    if (mem_kind != NB6_MEM_HOST && mem_kind != NB6_MEM_DEVICE)
        return fail(c, NB6_ERR_ARG, "bad mem_kind %d", mem_kind);
    if (n_i == 0) return NB6_OK;
    if (!idx_i || !nnb_i || !list) return fail(c, NB6_ERR_ARG, "null argument");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = cl->n;
    const int ni = (int)n_i;
    const int32_t* d_idx = idx_i;
    const int32_t* d_nnb = nnb_i;
    const int32_t* d_list = list;
    if (mem_kind == NB6_MEM_HOST) {
        std::vector<char> seen((size_t)n, 0);
        for (int k = 0; k < ni; ++k) {
            const int32_t p = idx_i[k];
            if (p < 0 || p >= n)
                return fail(c, NB6_ERR_ARG, "idx_i[%d] = %d out of range", k, p);
            if (seen[p]) return fail(c, NB6_ERR_ARG, "particle %d listed twice", p);
            seen[p] = 1;
            if (nnb_i[k] < 0 || nnb_i[k] > cap)
                return fail(c, NB6_ERR_ARG, "nnb_i[%d] = %d outside [0, %d]", k, nnb_i[k], cap);
            for (int e = 0; e < nnb_i[k]; ++e) {
                const int32_t j = list[(size_t)k * cap + e];
                if (j < 0 || j >= n)
                    return fail(c, NB6_ERR_ARG, "list entry (%d, %d) = %d out of range", k, e, j);
            }
        }
        // indices, counts and lists go up through the pinned buffer in one
        // copy: small lists as they are, larger ones packed to their rows'
        // used entries (a kernel then puts the rows back in place)
        const size_t list_bytes = (size_t)ni * cap * sizeof(int32_t);
        const bool staged = list_bytes <= kStageListMax;
        std::vector<int64_t> off;
        if (!staged) off = row_offsets(nnb_i, ni, cap);
        Stage lay;
        const size_t o_idx = lay.add(ni * sizeof(int32_t));
        const size_t o_nnb = lay.add(ni * sizeof(int32_t));
        const size_t o_off = staged ? 0 : lay.add(((size_t)ni + 1) * sizeof(int64_t));
        const size_t o_list =
            lay.add(staged ? list_bytes : (size_t)off[ni] * sizeof(int32_t));
        int rc;
        if ((rc = ensure(c, c->io, lay.end)) || (rc = ensure_pinned(c, c->pin, lay.end)) ||
            (!staged && (rc = ensure(c, c->out_list, list_bytes))))
            return rc;
        char* pin = c->pin.p;
        char* dev = (char*)c->io.p;
        std::memcpy(pin + o_idx, idx_i, ni * sizeof(int32_t));
        std::memcpy(pin + o_nnb, nnb_i, ni * sizeof(int32_t));
        if (staged) {
            std::memcpy(pin + o_list, list, list_bytes);
        } else {
            std::memcpy(pin + o_off, off.data(), ((size_t)ni + 1) * sizeof(int64_t));
            pack_rows_host(off, ni, cap, list, (int32_t*)(pin + o_list));
        }
        HIP_TRY(c, hipMemcpyAsync(dev, pin, lay.end, hipMemcpyHostToDevice, st));
        if (!staged)
            HIP_TRY(c, launch_unpack_rows((const int32_t*)(dev + o_list),
                                          (const int64_t*)(dev + o_off), ni,
                                          (int32_t*)c->out_list.p, cap, st));
        d_idx = (const int32_t*)(dev + o_idx);
        d_nnb = (const int32_t*)(dev + o_nnb);
        d_list = staged ? (const int32_t*)(dev + o_list) : (const int32_t*)c->out_list.p;
    }
    if (int rc = ensure_lists(c, cl, cap, st)) return rc;
    SetListArgs sa{};
    sa.n = n;
    sa.idx = d_idx;
    sa.ni = ni;
    sa.nnb = d_nnb;
    sa.list = d_list;
    sa.cap = cap;
    sa.nbl = (int32_t*)cl->nbl.p;
    sa.nbc = (int32_t*)cl->nbc.p;
    sa.lcap = cl->lcap;
    sa.status = c->status;
    HIP_TRY(c, launch_set_lists(sa, st));
    if (mem_kind == NB6_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(st));
    return NB6_OK;
}

int nb6_irregular_force(nb6_ctx* c, int cluster, double t_block, int64_t n_i,
                        const int32_t* idx_i, double* acc, double* jerk, double* pot,
                        int mem_kind, void* stream) {
    if (!c) return NB6_ERR_ARG;
    c->err.clear();
    std::lock_guard<std::mutex> lk(c->cluster_mu);
    ClusterState* cl = nullptr;
    if (int rc = get_cluster(c, cluster, &cl)) return rc;
    PlainClaim claim;
    if (int rc = claim.claim(c, cl, (hipStream_t)stream)) return rc;
    if (!std::isfinite(t_block)) return fail(c, NB6_ERR_ARG, "non-finite t_block");
    if (n_i < 0 || n_i > INT32_MAX / 4) return fail(c, NB6_ERR_ARG, "n_i = %lld", (long long)n_i);
    if (mem_kind != NB6_MEM_HOST && mem_kind != NB6_MEM_DEVICE)
        return fail(c, NB6_ERR_ARG, "bad mem_kind %d", mem_kind);
    if (n_i == 0) return NB6_OK;
    if (!idx_i || !acc || !jerk) return fail(c, NB6_ERR_ARG, "null argument");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = cl->n;
    const int ni = (int)n_i;
    const int32_t* d_idx = idx_i;
    double* d_acc = acc;
    double* d_jerk = jerk;
    double* d_pot = pot;
    Stage lay;
    size_t o_idx = 0, o_acc = 0, o_jerk = 0, o_pot = 0, o_status = 0;
    if (mem_kind == NB6_MEM_HOST) {
        for (int q = 0; q < ni; ++q)
            if (idx_i[q] < 0 || idx_i[q] >= n)
                return fail(c, NB6_ERR_ARG, "idx_i[%d] = %d out of range", q, idx_i[q]);
        // the indices go up, and the outputs come back, through the pinned
        // buffer, one copy each way
        o_idx = lay.add(ni * sizeof(int32_t));
        o_acc = lay.add(3 * (size_t)ni * sizeof(double));
        o_jerk = lay.add(3 * (size_t)ni * sizeof(double));
        o_pot = pot ? lay.add(ni * sizeof(double)) : 0;
        o_status = lay.add(4 * sizeof(unsigned));
        int rc;
        if ((rc = ensure(c, c->io, lay.end)) || (rc = ensure_pinned(c, c->pin, lay.end)))
            return rc;
        char* dev = (char*)c->io.p;
        std::memcpy(c->pin.p + o_idx, idx_i, ni * sizeof(int32_t));
        HIP_TRY(c, hipMemcpyAsync(dev, c->pin.p, o_acc, hipMemcpyHostToDevice, st));
        d_idx = (const int32_t*)(dev + o_idx);
        d_acc = (double*)(dev + o_acc);
        d_jerk = (double*)(dev + o_jerk);
        if (pot) d_pot = (double*)(dev + o_pot);
    }
    if (int rc = ensure_lists(c, cl, 1, st)) return rc;  // no lists yet: all empty
    IrrArgs ia{};
    ia.n = n;
    ia.st = cl->state;
    ia.tb = t_block;
    ia.idx = d_idx;
    ia.ni = ni;
    ia.nbl = (const int32_t*)cl->nbl.p;
    ia.nbc = (const int32_t*)cl->nbc.p;
    ia.lcap = cl->lcap;
    ia.acc = d_acc;
    ia.jerk = d_jerk;
    ia.pot = pot ? d_pot : nullptr;
    ia.status = c->status;
    {
        TimedLaunch tl(c, 3, st);
        HIP_TRY(c, launch_irregular(ia, st));
        tl.done();
    }
    if (mem_kind == NB6_MEM_DEVICE) return NB6_OK;
    char* pin = c->pin.p;
    HIP_TRY(c, hipMemcpyAsync(pin + o_acc, (char*)c->io.p + o_acc, o_status - o_acc,
                              hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(pin + o_status, c->status, 4 * sizeof(unsigned),
                              hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    HIP_TRY(c, launch_zero_u32(c->status, 4, st));
    std::memcpy(acc, pin + o_acc, 3 * (size_t)ni * sizeof(double));
    std::memcpy(jerk, pin + o_jerk, 3 * (size_t)ni * sizeof(double));
    if (pot) std::memcpy(pot, pin + o_pot, ni * sizeof(double));
    unsigned status[4];
    std::memcpy(status, pin + o_status, sizeof status);
    if (status[0] & (ST_BAD_INDEX | ST_BAD_LIST))
        return fail(c, NB6_ERR_DEVICE_INPUT, "GPU validation flagged 0x%x", status[0]);
    return NB6_OK;
}

int nb6_regular_correct(nb6_ctx* c, const nb6_corr_block* b, const nb6_corr_params* par,
                        int mem_kind, void* stream) {
    if (!c) return NB6_ERR_ARG;
    c->err.clear();
    if (!b || !par) return fail(c, NB6_ERR_ARG, "null block or parameters");
    int e_min = 0, e_max = 0;
    if (!(par->eta > 0.0) || !(par->dt_min > 0.0) || !(par->dt_max >= par->dt_min) ||
        std::frexp(par->dt_min, &e_min) != 0.5 || std::frexp(par->dt_max, &e_max) != 0.5 ||
        !(par->f_lo > 0.0) || !(par->f_hi >= par->f_lo) || !std::isfinite(par->f_hi) ||
        !std::isfinite(par->eta))
        return fail(c, NB6_ERR_ARG, "bad corrector parameters");
    if (!std::isfinite(b->t)) return fail(c, NB6_ERR_ARG, "non-finite t");
    if (b->n_i < 0 || b->n_i > INT32_MAX) return fail(c, NB6_ERR_ARG, "n_i = %lld", (long long)b->n_i);
    if (mem_kind != NB6_MEM_HOST && mem_kind != NB6_MEM_DEVICE)
        return fail(c, NB6_ERR_ARG, "bad mem_kind %d", mem_kind);
    const int64_t n = b->n_i;
    if (n == 0) return NB6_OK;
    const double* vin[8] = {b->f_old, b->fd_old, b->f_new, b->fd_new,
                            b->g_old, b->gd_old, b->g_new, b->gd_new};
    double* vout[4] = {b->df, b->dfd, b->f2, b->f3};
    if (!b->t_old || !b->h_old || !b->nnb || !b->n_p || !b->dt_new || !b->h_new)
        return fail(c, NB6_ERR_ARG, "null array in the block");
    for (const double* p : vin) if (!p) return fail(c, NB6_ERR_ARG, "null array in the block");
    for (double* p : vout) if (!p) return fail(c, NB6_ERR_ARG, "null array in the block");
    std::lock_guard<std::mutex> lk(c->cluster_mu);
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    CorrArgs a{};
    a.n = n;
    a.t = b->t;
    a.eta = par->eta; a.dt_min = par->dt_min; a.dt_max = par->dt_max;
    a.f_lo = par->f_lo; a.f_hi = par->f_hi;
    a.status = c->status;
    const size_t v3 = 3 * (size_t)n * sizeof(double), s1 = (size_t)n * sizeof(double);
    if (mem_kind == NB6_MEM_HOST) {
        for (int64_t q = 0; q < n; ++q)
            if (!(b->t - b->t_old[q] > 0.0) || !std::isfinite(b->t_old[q]))
                return fail(c, NB6_ERR_ARG, "t_old[%lld] is not before t", (long long)q);
        // the inputs go up in one copy from the pinned buffer and the
        // outputs come back in one copy into it; the device mirror has the
        // same layout
        Stage lay;
        size_t o_vin[8], o_sin[3], o_vout[4], o_sout[2];
        for (auto& o : o_vin) o = lay.add(v3);
        for (auto& o : o_sin) o = lay.add(s1);
        const size_t o_nnb = lay.add((size_t)n * sizeof(int32_t));
        const size_t in_end = lay.end;
        for (auto& o : o_vout) o = lay.add(v3);
        for (auto& o : o_sout) o = lay.add(s1);
        if (int rc = ensure(c, c->io, lay.end)) return rc;
        if (int rc = ensure_pinned(c, c->pin, lay.end)) return rc;
        char* pin = c->pin.p;
        char* dev = (char*)c->io.p;
        const double* sin3[3] = {b->t_old, b->h_old, b->n_p};
        for (int k = 0; k < 8; ++k) std::memcpy(pin + o_vin[k], vin[k], v3);
        for (int k = 0; k < 3; ++k) std::memcpy(pin + o_sin[k], sin3[k], s1);
        std::memcpy(pin + o_nnb, b->nnb, (size_t)n * sizeof(int32_t));
        HIP_TRY(c, hipMemcpyAsync(dev, pin, in_end, hipMemcpyHostToDevice, st));
        auto dvec = [&](size_t o) { return (double*)(dev + o); };
        a.f_old = dvec(o_vin[0]); a.fd_old = dvec(o_vin[1]);
        a.f_new = dvec(o_vin[2]); a.fd_new = dvec(o_vin[3]);
        a.g_old = dvec(o_vin[4]); a.gd_old = dvec(o_vin[5]);
        a.g_new = dvec(o_vin[6]); a.gd_new = dvec(o_vin[7]);
        a.t_old = dvec(o_sin[0]); a.h_old = dvec(o_sin[1]); a.n_p = dvec(o_sin[2]);
        a.nnb = (const int32_t*)(dev + o_nnb);
        a.df = dvec(o_vout[0]); a.dfd = dvec(o_vout[1]);
        a.f2 = dvec(o_vout[2]); a.f3 = dvec(o_vout[3]);
        a.dt_new = dvec(o_sout[0]); a.h_new = dvec(o_sout[1]);
        HIP_TRY(c, launch_correct(a, st));
        HIP_TRY(c, hipMemcpyAsync(pin + in_end, dev + in_end, lay.end - in_end,
                                  hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        for (int k = 0; k < 4; ++k) std::memcpy(vout[k], pin + o_vout[k], v3);
        std::memcpy(b->dt_new, pin + o_sout[0], s1);
        std::memcpy(b->h_new, pin + o_sout[1], s1);
        return NB6_OK;
    }
    a.t_old = b->t_old;
    a.f_old = b->f_old; a.fd_old = b->fd_old; a.f_new = b->f_new; a.fd_new = b->fd_new;
    a.g_old = b->g_old; a.gd_old = b->gd_old; a.g_new = b->g_new; a.gd_new = b->gd_new;
    a.h_old = b->h_old; a.nnb = b->nnb; a.n_p = b->n_p;
    a.df = b->df; a.dfd = b->dfd; a.f2 = b->f2; a.f3 = b->f3;
    a.dt_new = b->dt_new; a.h_new = b->h_new;
    HIP_TRY(c, launch_correct(a, st));
    return NB6_OK;
}

int nb6_sync_status(nb6_ctx* c, void* stream) {
    if (!c) return NB6_ERR_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    unsigned status[4];
    HIP_TRY(c, hipMemcpyAsync(status, c->status, sizeof status, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    HIP_TRY(c, launch_zero_u32(c->status, 4, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (status[0] & ST_INPUT_ERRORS)
        return fail(c, NB6_ERR_DEVICE_INPUT, "GPU validation flagged 0x%x", status[0]);
    return NB6_OK;
}

}  // extern "C"
