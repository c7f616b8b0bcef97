// nb6_internal.h -- records, launch parameters and kernel launchers shared
// by the runtime (nb6_api.hip) and the kernels (nb6_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb6 {

// ---------------------------------------------------------------------------
// j-particle records written by the predictor and read by the force kernel.
// One record per particle, array-of-structures so that a wavefront reads a
// whole record with a few scalar loads (the record address is the same for
// every lane).
// ---------------------------------------------------------------------------
// vabs is an upper bound of |v| of the stored float velocity; the force
// kernel uses it to skip the velocity criterion for pairs that cannot be
// neighbours.
struct __attribute__((aligned(16))) RecFF {   // float-float coordinates, 48 B
    float xh, yh, zh, m;
    float xl, yl, zl, vabs;
    float vx, vy, vz, pad;
};
struct __attribute__((aligned(16))) RecF64 {  // double coordinates, 48 B
    double x, y, z;
    float vx, vy, vz, m;
    float vabs, pad;
};
struct __attribute__((aligned(16))) RecF32 {  // plain float coordinates, 32 B
    float x, y, z, m;
    float vx, vy, vz, vabs;
};
// Tile-local coordinates, 32 B.  These records follow the cluster's spatial
// order (slot k holds particle perm[k]); e is the FP32 rounding of the FP64
// difference between the predicted position and the centre of the record's
// tile of VTILE slots, p the particle's index in the cluster.
struct __attribute__((aligned(16))) RecLoc {
    float ex, ey, ez, m;
    float vx, vy, vz;
    int32_t p;
};
// Centre of one tile of VTILE local records: the FP64 midpoint of the
// bounding box of their predicted positions, and the largest vabs among them
// (the candidate bound of the force kernel).
struct __attribute__((aligned(16))) TileOrg {
    double x, y, z;
    float vmax, pad;
};

enum Mode { MODE_FF = 0, MODE_F64 = 1, MODE_F32 = 2, MODE_LOC = 3 };
constexpr int NMODES = 4;

// j-particles per tile of the force kernel: its FP32 partial sums are folded
// into FP64 once per tile, and the predictor records max |v| of every tile of
// VTILE consecutive particles (the bound of the candidate pre-test).
constexpr int VTILE = 32;
__host__ __device__ inline long long vtiles(long long n) { return (n + VTILE - 1) / VTILE; }

// Bits of the device status word.
enum StatusBits {
    ST_BAD_INDEX = 1, ST_BAD_H2 = 2, ST_NONFINITE = 4, ST_OVERFLOW = 8, ST_BAD_LIST = 16,
    ST_BAD_STEP = 32, ST_BAD_DTR = 64
};
// Bits that mark an input a call could not use (the caller's error).
constexpr unsigned ST_INPUT_ERRORS =
    ST_BAD_INDEX | ST_BAD_H2 | ST_NONFINITE | ST_BAD_LIST | ST_BAD_STEP | ST_BAD_DTR;

// The regular time-step of an active particle offsets the second end point
// of the velocity criterion forward in time (section 3.2), so it must be
// finite and >= 0: the candidate radius of the force kernels, which keeps the
// criterion off the common path, is a valid bound only then.
__host__ __device__ inline bool valid_dtr(double dtr) { return dtr >= 0.0 && dtr <= 1.79e308; }

// Cubic Taylor prediction of one coordinate in FP64 Horner form with explicit
// fused multiply-adds (section 3.3 step 3): h = dt/2, t3 = dt/3,
//   xp = x + dt (v + h (a + t3 jk)),   vp = v + dt (a + h jk).
// Every predictor of the library uses this one expression, so a particle
// predicted to the same time gets the same bits everywhere.
__device__ __forceinline__ void predict_coord(double dt, double h, double t3, double x,
                                              double v, double a, double jk, double& xp,
                                              double& vp) {
    xp = fma(dt, fma(h, fma(t3, jk, a), v), x);
    vp = fma(dt, fma(h, jk, a), v);
}

// Partial sums leave the force kernel as 6 FP64 components per (i, slice):
// acc xyz, jerk xyz; 7 when the potential is asked for (the sum of m / r over
// the non-neighbours last).
constexpr int NPART = 6;
constexpr int NPART_POT = 7;
// Largest per-i list capacity (cap + 1 slots: the i itself is found too).
constexpr int MAX_CAPS = 1024;
// Particles per finalize workgroup for the lists, one per wave (two per
// wave measured 2-3 us slower for blocks of 8 to 4096, the same from 16384
// on); the first np ceil(ni / 64) workgroups also reduce one component of the
// slice partials of 64 particles each.
constexpr int FINAL_PPB = 4;
__host__ __device__ inline long long final_list_blocks(long long ni) {
    return (ni + FINAL_PPB - 1) / FINAL_PPB;
}
__host__ __device__ inline long long final_blocks(long long ni, int np) {
    const long long sums = np * ((ni + 63) / 64);
    const long long lists = final_list_blocks(ni);
    return sums > lists ? sums : lists;
}

struct RegfArgs {
    const void*    rec;       // records of the cluster (mode dependent)
    int            n;         // number of j-particles
    const int32_t* idx;       // [ni] active indices
    const double*  h2;        // [ni]
    const double*  dtr;       // [ni]
    int            ni;
    int            slice_len; // j per slice (multiple of VTILE)
    int            nslices;
    int            jl_shift;  // log2 of the lanes that share one i (0: one lane per i)
    const float*   tmax;      // [vtiles(n)] max of vabs over each tile of VTILE j
    const TileOrg* org;       // MODE_LOC: [vtiles(n)] tile centres (else null)
    const void*    ivw;       // MODE_LOC: float-float records by particle (the i-side)
    double*        part;      // [ceil(ni/64)][nslices][NPART or NPART_POT][64]
    int32_t*       cnt;       // [ni] neighbours found, the i itself included (zero on
                              // entry; the finalize leaves it zero again)
    int32_t*       lst;       // [ni][caps] neighbours in the order found
    int            caps;      // per-i list capacity (cap + 1)
    unsigned*      status;    // device status word
    const void*    irec;      // [ni] or null: the i-records in work order (a call run in
                              // an i-order, whose idx, h2 and dtr are then in work
                              // order too); null: the records by particle index
};

struct FinalArgs {
    const double*  part;
    int32_t*       cnt;       // read, then reset to zero
    const int32_t* lst;
    int            nslices;
    int            ni;
    int            caps;
    int            n;
    const int32_t* idx;
    const double*  h2;
    double*        acc;       // [ni][3]
    double*        jerk;      // [ni][3]
    double*        pot;       // [ni] or null (then the partials have NPART components)
    int32_t*       nnb;       // [ni]
    int32_t*       list;      // [ni][cap]
    int            cap;
    unsigned*      status;
    // the ordered rescan of an overflowed list: the force call's records,
    // their coordinate mode (MODE_*) and the i's dtr; for MODE_LOC also the
    // tile centres, the slot of each particle and the float-float records
    const void*    rec;
    const double*  dtr;
    int            mode;
    const TileOrg* org;
    const int32_t* inv;
    const void*    ivw;
    const int32_t* iord;      // the force call's i-order (null: identity)
};

// ---------------------------------------------------------------------------
// Stored state of one particle: the corrected position, velocity,
// acceleration and jerk at its own time t, and its mass -- what the
// predictor works from (section 3.3 step 3).  One 128-byte record per
// particle, so that the gather of one particle (the irregular force reads
// its list's particles in arbitrary order) touches one cache line.
// ---------------------------------------------------------------------------
struct __attribute__((aligned(128))) StateRec {
    double x[3], v[3], a[3], jk[3];
    double m, t;
    double pad[2];
};
static_assert(sizeof(StateRec) == 128, "one cache line per particle");

struct PredictArgs {
    int64_t         n;
    const StateRec* st;  // [n]
    double          tb;
    RecFF*        ff;  // may be null
    RecF64*       f64; // may be null
    RecF32*       f32; // may be null
    float*        tmax; // [vtiles(n)] max vabs per tile (always written)
    unsigned*     status;
    // the local-coordinate stream (launch_predict_loc): slot k of `loc`
    // holds particle perm[k]; `ff` receives every particle's float-float
    // record
    RecLoc*        loc;
    TileOrg*       org;  // [vtiles(n)]
    const int32_t* perm;
};

struct ScatterArgs {
    int64_t        n;     // entries
    const int32_t* idx;   // [n] destination particle of each entry (null: entry e -> e)
    const double*  m;     // sources, [n] and [n][3]
    const double*  x;
    const double*  v;
    const double*  a;
    const double*  jk;
    const double*  t;
    StateRec*      dst;   // [limit] stored state
    int64_t        limit; // cluster size; entries with idx outside [0, limit) are skipped
    unsigned*      status;
};

// ---------------------------------------------------------------------------
// Irregular force over stored neighbour lists.
// ---------------------------------------------------------------------------
// Largest row of the stored neighbour lists.
constexpr int MAX_LIST_CAP = 8192;

struct IrrArgs {
    int64_t         n;        // cluster size
    const StateRec* st;       // [n] stored state
    double          tb;       // block time
    const int32_t* idx;       // [ni] active particles
    int            ni;
    const int32_t* nbl;       // [n][lcap] stored lists
    const int32_t* nbc;       // [n] entries of each stored list
    int            lcap;
    double*        acc;       // [ni][3]
    double*        jerk;      // [ni][3]
    double*        pot;       // [ni] or null
    unsigned*      status;
};

struct SetListArgs {
    int64_t        n;         // cluster size
    const int32_t* idx;       // [ni] particles whose lists are replaced
    int            ni;
    const int32_t* nnb;       // [ni] entries of each new list
    const int32_t* list;      // [ni][cap] the new lists
    int            cap;
    int32_t*       nbl;       // [n][lcap] storage
    int32_t*       nbc;       // [n]
    int            lcap;
    unsigned*      status;
};

hipError_t launch_irregular(const IrrArgs& a, hipStream_t s);
hipError_t launch_set_lists(const SetListArgs& a, hipStream_t s);
// Copy the first cnt[p] entries of every row p from rows of src_cap entries
// to rows of dst_cap entries (the stored lists grow).
hipError_t launch_copy_rows(const int32_t* src, int src_cap, int32_t* dst, int dst_cap,
                            const int32_t* cnt, int64_t n, hipStream_t s);
// Pack rows: entries [0, off[q+1] - off[q]) of row q of `list` (rows of cap
// entries) to out[off[q] ...], for q < n.
hipError_t launch_pack_rows(const int32_t* list, int cap, const int64_t* off, int64_t n,
                            int32_t* out, hipStream_t s);
// The inverse: packed[off[q] ...] to the first off[q+1] - off[q] entries of
// row q of `list`.
hipError_t launch_unpack_rows(const int32_t* packed, const int64_t* off, int64_t n,
                              int32_t* list, int cap, hipStream_t s);

// ---------------------------------------------------------------------------
// Regular corrector of a block (elementwise, FP64).
// ---------------------------------------------------------------------------
struct CorrArgs {
    int64_t        n;
    double         t;
    const double*  t_old;                       // [n]
    const double*  f_old; const double* fd_old; // [n][3]
    const double*  f_new; const double* fd_new;
    const double*  g_old; const double* gd_old;
    const double*  g_new; const double* gd_new;
    const double*  h_old;                       // [n]
    const int32_t* nnb;                         // [n]
    const double*  n_p;                         // [n]
    double eta, dt_min, dt_max, f_lo, f_hi;
    double* df; double* dfd; double* f2; double* f3;  // [n][3]
    double* dt_new; double* h_new;                     // [n]
    unsigned*      status;
};
hipError_t launch_correct(const CorrArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// Serving: one descriptor per request of a fused batch.
// ---------------------------------------------------------------------------
struct ReqDesc {
    RegfArgs     rg;          // force work of the request
    FinalArgs    fin;         // its reduction and lists
    PredictArgs  pred;        // prediction of its cluster (when do_predict)
    int          do_predict;
    int          mode;        // MODE_*
    int          groups;      // i-groups of regf_group_size(ipl, rg.jl_shift)
    long long    item0;       // first force work item within its launch
    long long    blk0;        // first finalize workgroup within the batch
};

struct BatchArgs {
    const ReqDesc*      reqs;      // device copy of the batch's descriptors
    int                 nreq;
    long long           nitems;    // force work items of this launch
    long long           nblk_total; // finalize workgroups of the batch
    unsigned long long* counter;   // work-item counter (zeroed before the launch)
};

// Work-partition classes of a served request, one persistent launch each:
// one i per lane, lanes sharing an i (jl_shift > 0), two i per lane.
enum { SERVE_ONE_I = 0, SERVE_LANES = 1, SERVE_TWO_I = 2, SERVE_CLASSES = 3 };
// Persistent fused force kernel over requests [reqs, reqs + nreq) of one
// mode and one class.
hipError_t launch_serve_regf(int mode, int cls, const BatchArgs& b, int blocks, hipStream_t s);
// Workgroups of that launch that fit one compute unit at once.
hipError_t serve_regf_blocks_per_cu(int mode, int cls, int* blocks);
hipError_t launch_serve_finalize(const BatchArgs& b, hipStream_t s);
// Predictions and count resets of every request of the batch, in one launch
// of (requests x chunks) blocks; a chunk covers PREPARE_CHUNK particles.
constexpr int PREPARE_CHUNK = 256;  // one particle per thread
hipError_t launch_serve_prepare(const BatchArgs& b, int chunks, hipStream_t s);

// Force kernel: ipl i-particles per lane (a.jl_shift == 0), or one i per
// 2^a.jl_shift lanes (ipl == 1).
hipError_t launch_regf(int mode, int ipl, int waves_per_block, bool pot, const RegfArgs& a,
                       hipStream_t s);
// i-particles of one work item (one wavefront) of the force kernel.
__host__ __device__ inline int regf_group_size(int ipl, int jl_shift) { return (64 * ipl) >> jl_shift; }
hipError_t launch_finalize(const FinalArgs& a, hipStream_t s);
hipError_t launch_predict(const PredictArgs& a, hipStream_t s);
// The local-coordinate stream: a.loc and a.org (and a.ff when set) from
// a.perm.
hipError_t launch_predict_loc(const PredictArgs& a, hipStream_t s);
// Spatial order of a cluster from its stored positions: perm[slot] =
// particle (Morton order, ties by index) and inv[particle] = slot.  scratch
// holds order_scratch_bytes(n) bytes.
size_t order_scratch_bytes(int64_t n);
hipError_t launch_order(const StateRec* st, int64_t n, void* scratch, size_t scratch_bytes,
                        int32_t* perm, int32_t* inv, hipStream_t s);
// i-order of an active block of ni positions: iord[k] = the active position
// of the k-th particle in the spatial order inv (positions of one slot, a
// repeated index, in either order; an index outside [0, n) sorts last).
// scratch holds iorder_scratch_bytes(ni, n) bytes.
size_t iorder_scratch_bytes(int64_t ni, int64_t n);
hipError_t launch_iorder(const int32_t* idx, int ni, const int32_t* inv, int64_t n,
                         void* scratch, size_t scratch_bytes, int32_t* iord, hipStream_t s);
// The force kernel's i-side in work order k = 0 .. ni-1 of an i-order:
// widx[k] = idx[iord[k]], wh2, wdtr likewise, and wrec[k] the rec_bytes-byte
// i-record (a multiple of 16) of particle widx[k] from irec (of particle 0
// for an index outside [0, n), which the force kernel flags).
hipError_t launch_istage(const int32_t* iord, int ni, const int32_t* idx, const double* h2,
                         const double* dtr, int64_t n, const void* irec, int rec_bytes,
                         int32_t* widx, double* wh2, double* wdtr, void* wrec, hipStream_t s);
hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s);
// Widen the j-records of one mode to double position and velocity arrays.
hipError_t launch_unpack(int mode, const void* rec, int64_t n, double* x, double* v,
                         hipStream_t s);
// Clear n words with a kernel (not a memset node, so it is safe under graph
// capture).
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s);

}  // namespace nb6
