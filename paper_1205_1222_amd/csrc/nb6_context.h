// nb6_context.h -- the context object behind the C ABI and the helpers its
// translation units share (nb6_api.hip: plain calls; nb6_serve.hip: the
// serving queue).
#pragma once

#include "../../include/nb6.h"
#include "nb6_internal.h"
#include "nb6_plan.h"
#include "nb6_rows.h"

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

namespace nb6 {

constexpr int kMaxClusters = 4096;

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

// Pinned host memory (hipHostMalloc).
struct PinBuf {
    char* p = nullptr;
    size_t cap = 0;
};

// Byte layout of the arrays one HOST-mode call stages: each array starts on a
// 256-byte boundary; the same offsets serve the pinned buffer and its device
// mirror.
struct Stage {
    size_t end = 0;
    size_t add(size_t bytes) {
        const size_t o = end;
        end = (end + bytes + 255) / 256 * 256;
        return o;
    }
};
// Lists of a HOST-mode call above this size are copied to the caller's array
// directly rather than through the pinned buffer (which would add a second
// host-side pass over them).
constexpr size_t kStageListMax = size_t(1) << 20;
// Host-array loads up to this size go up through the pinned buffer in one copy.
constexpr size_t kStageLoadMax = size_t(8) << 20;

struct ClusterState {
    int64_t n = 0;
    StateRec* state = nullptr; // [n] stored state, one record per particle
    DevBuf rec[NMODES];        // j-records by mode index (MODE_LOC: spatial order)
    DevBuf tmax;               // max vabs per tile of VTILE records (index order)
    DevBuf org;                // MODE_LOC tile centres [vtiles(n)]
    DevBuf perm, inv;          // spatial order: slot -> particle, particle -> slot
    bool order_valid = false;  // perm / inv hold the order of the current state
    int64_t updated_since_order = 0;  // particles of subset updates since then
    DevBuf nbl;                // stored neighbour lists [n][lcap] (irregular force)
    DevBuf nbc;                // entries of each stored list [n]
    int lcap = 0;
    int pred_valid = 0;        // NB6_DX_* bits whose records are current
    double t_pred = 0.0;
    // Owner of the cluster: 0 free, 1 a serving request in flight, -1 a plain
    // call in progress.  Claimed with compare-and-swap from 0.
    std::atomic<int> owner{0};
    // Serving requests submitted on this cluster and not yet finished.  A
    // full load that would resize the cluster (and so free the buffers those
    // requests were sized and will be launched with) is refused meanwhile.
    std::atomic<int> queued{0};
    // Last stream work of each side on this cluster; the other side's stream
    // waits for it before touching the cluster (created on first use).
    hipEvent_t last_plain = nullptr;
    hipEvent_t last_served = nullptr;
};

inline int mode_index(int dx_mode) {
    switch (dx_mode) {
        case NB6_DX_FF: return MODE_FF;
        case NB6_DX_FP64: return MODE_F64;
        case NB6_DX_FP32: return MODE_F32;
        case NB6_DX_LOCAL: return MODE_LOC;
        default: return -1;
    }
}

inline int mode_bit(int mi) {
    return mi == MODE_FF ? NB6_DX_FF : mi == MODE_F64 ? NB6_DX_FP64
         : mi == MODE_F32 ? NB6_DX_FP32 : NB6_DX_LOCAL;
}

// The force kernel's coordinate mode for a call in mode mi with plan p.  A
// local-mode call whose plan is latency-bound -- lanes per i (a small
// block), or j-slices shorter than 256 (a small call in a small cluster) --
// runs on the float-float records by particle index that the local
// prediction also writes (its i-side, with the per-tile candidate bounds in
// index order): such a work item spends its time on the chain of dependent
// loads, and the local form adds a tile-centre load and FP64 differences to
// it (measured on one box, force kernel, local against float-float: N = N_i =
// 1024, 16.3 against 12.6 us; N_i = 1024 of 16384, 40.8 against 29.2 us;
// from 256-j slices on the local form is the faster).  Plain and served calls
// take the same mode, so they give the same bits.
inline int kernel_mode(int mi, const Plan& p) {
    return (mi == MODE_LOC && (p.jl_shift > 0 || p.slice_len < 256)) ? MODE_FF : mi;
}

inline size_t rec_size(int mi) {
    return mi == MODE_FF ? sizeof(RecFF) : mi == MODE_F64 ? sizeof(RecF64)
         : mi == MODE_F32 ? sizeof(RecF32) : sizeof(RecLoc);
}

// Wave-level work partition of one force call.

class Engine;  // serving queue (nb6_serve.hip)

}  // namespace nb6

struct nb6_ctx {
    int device = 0;
    int num_cu = 256;
    int slice_hint = 0;
    int ipl_hint = 0;
    int jl_hint = 0;
    int64_t hbm_budget = 0;
    std::vector<nb6::ClusterState*> clusters;
    nb6::DevBuf part, cnt, lst;                       // force-kernel scratch
    bool cnt_dirty = true;  // cnt must be zeroed before the next force launch
    nb6::DevBuf io;                                   // HOST-mode staged inputs and outputs
    nb6::DevBuf out_list;                             // HOST-mode lists too big to stage
    nb6::PinBuf pin;                                  // pinned mirror of `io`
    nb6::DevBuf ld[7];                                // HOST-mode load staging
    nb6::DevBuf order_tmp;                            // spatial-order sort scratch
    nb6::DevBuf iord, iord_tmp;                       // a call's i-order and work-order i-side; sort scratch
    unsigned* status = nullptr;                       // device status word
    std::string err;
    nb6::Plan last_plan{0, 0, 0, 0, 0};
    bool timing = false;
    bool iorder = true;  // large plain calls run in the spatial i-order
    struct Timed { int kind; hipEvent_t a, b; };  // kind: 0 predict, 1 force, 2 finalize, 3 irregular
    std::vector<Timed> timed;                         // pending event pairs
    // Cluster states are shared with the serving queue's thread.
    std::mutex cluster_mu;
    nb6::Engine* engine = nullptr;
};

namespace nb6 {

int fail(nb6_ctx* c, int code, const char* fmt, ...);
int ensure(nb6_ctx* c, DevBuf& b, size_t bytes);
void release(DevBuf& b);
// Grow the pinned buffer to at least `bytes` (nothing may be pending on it).
int ensure_pinned(nb6_ctx* c, PinBuf& b, size_t bytes);
// ipl: 0 = the context's choice (its hint, else by n_i).
Plan make_plan(const nb6_ctx* c, int64_t n, int64_t ni, int ipl = 0);
// Shut the serving queue down (nb6_destroy).
void engine_shutdown(nb6_ctx* c);
// Tell the serving queue that a cluster was released by a plain call.
void engine_kick(nb6_ctx* c);


#define HIP_TRY(ctx, call)                                                          \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return ::nb6::fail((ctx), NB6_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

}  // namespace nb6
