// nb6_kernels.hip -- gfx950 kernels of the regular-force path.
//
//   predict_kernel    cubic Taylor prediction of every j-particle to the block
//                     time in FP64, writing the j-records the force kernel
//                     reads (section 3.3 step 3).
//   predict_loc_kernel the same for the local-coordinate stream: records in
//                     the cluster's spatial order, each tile of VTILE records
//                     with the FP64 centre of its predicted positions.
//   regf_kernel       regular force, jerk and neighbour appends for one
//                     (i-group, j-slice) pair (section 3.3 step 6 with the
//                     velocity criterion of section 3.2).
//   regf_lanes_kernel the same for small active blocks, with several lanes
//                     per i splitting the slice's j (at 16 or 32 lanes per
//                     i the workgroup's waves read the j-records from LDS).
//   finalize_kernel   fixed-order reduction of the j-slice partial sums and
//                     the sorted neighbour list of each i (the reduction and
//                     list-gathering kernels of section 3.4); the exact list
//                     of an i whose neighbours outnumber the list capacity
//                     (the first `cap` in ascending j) by an ordered rescan.
//
// Design:
//   * i-particles live in VGPRs, IPL of them per lane (or one per 2^k lanes
//     for small blocks).  A call on a large block that holds most of its
//     cluster passes its i-side in a spatial work order (the host side sorts
//     it), so the i of one wavefront lie close together; the partials, counts
//     and list rows are then by work position, and the finalize writes each
//     output at its active position.
//   * Every lane of a wavefront reads the same j-record, so records are
//     fetched with scalar loads into SGPRs and used directly as operands of
//     the vector instructions: no LDS traffic and no VGPRs spent on j.
//   * The neighbour test and the force use FP32; the coordinate difference
//     is formed from float-float, FP64 or FP32 coordinates, or (local mode)
//     as a record's FP32 offset from its tile's centre plus the FP32 rounding
//     of (centre - R_i), computed in FP64 once per tile: one FP32 add per
//     component, with the large coordinates cancelled in FP64.
//   * Force terms are summed in FP32 over tiles of TILE j-particles and each
//     tile sum is added into an FP64 accumulator (FP64 adds run at the full
//     vector rate on CDNA), so the rounding error is that of a TILE-term
//     FP32 sum and does not grow with N.
//   * The velocity criterion is evaluated only for candidate pairs inside a
//     conservative radius, behind a branch that a wavefront almost never
//     takes.
//   * A lane keeps the neighbours it finds for an i in a short run in its
//     own LDS column and moves a full run, and what is left at the end of
//     the work item, to the i's list with one atomic slot reservation (a
//     returning atomic per neighbour would stall the wavefront on every
//     one); the finalize kernel sorts each list.  A list that overflows its
//     capacity is rebuilt by an ordered scan, so the result is always the
//     first `cap` neighbours in ascending j.
//   * A call is two launches, force and finalize: the finalize leaves the
//     per-i counters at zero for the next call, and rescans overflowed lists
//     itself.
#include "nb6_internal.h"

#include <float.h>

// No implicit fused multiply-adds: the force kernel and the ordered rescan of
// an overflowed list must take bit-identical neighbour decisions, so every
// fma is explicit.
#pragma clang fp contract(off)

namespace nb6 {

constexpr int TILE = VTILE; // j per FP32 tile before the FP64 fold
constexpr int JG = 4;       // j-records loaded together
constexpr int RUN = 16;     // staged neighbours per lane (split among its i)
constexpr int WAVES = 4;    // most wavefronts in a force workgroup (256 threads)
// LDS of a force workgroup of wpb wavefronts: RUN entries per lane.
constexpr size_t run_lds_bytes(int wpb) { return (size_t)wpb * RUN * 64 * sizeof(int); }

// A lane's run of neighbours found for one list row, in LDS: entry e of
// lane l at run[64 e + l] (the wavefront's lanes interleaved, so the 64
// lanes' stores of one entry hit distinct banks).  The lane's row is
// row0 + (l >> shift); run, row0 and shift are wave-uniform, so n is the
// lane's only register.  flush() reserves n slots of the row with one atomic
// add on its counter and copies the run there; a neighbour found while the
// run is full takes a slot of its own.  Slots at or past the row capacity
// are dropped (the counter still counts them, and the finalize rebuilds such
// a list by its ordered rescan).  The row thus ends with the same entries as
// with one reservation per neighbour, in another order, which the
// finalize's sort removes.  Flushes happen between tiles of j (flush_half)
// and at the end of the work item.
template <int N>
struct Staged {
    int* run;
    int row0, shift;
    int n;

    // The lane id, opaque to the optimiser: what is derived from it stays on
    // the rare path that needs it instead of being kept live across the j
    // loop in registers.
    __device__ __forceinline__ static int lane() {
        int l = (int)__lane_id();
        __asm__ volatile("" : "+v"(l));
        return l;
    }
    __device__ __forceinline__ void flush(const RegfArgs& a) {
        if (n > 0) {
            const int l = lane();
            const int row = row0 + (l >> shift);
            const int base = atomicAdd(a.cnt + row, n);
            int* out = a.lst + (size_t)row * a.caps;
#pragma unroll 1
            for (int e = 0; e < n; ++e)
                if (base + e < a.caps) out[base + e] = run[64 * e + l];
            n = 0;
        }
    }
    __device__ __forceinline__ void flush_half(const RegfArgs& a) {
        if (n >= N / 2) flush(a);
    }
    // The flush of a wavefront whose 2^shift consecutive lanes share a row,
    // called by the whole wavefront: the lanes of a row add up their run
    // lengths (a scan over the row's lanes), its first lane reserves the
    // total with one atomic add, and each lane copies its run to the slots
    // after those of the row's lower lanes.  A row's lanes would otherwise
    // send their reservations to one counter, where they are served one by
    // one.
    __device__ __forceinline__ void flush_shared(const RegfArgs& a) {
        const int l = lane();
        const int w = 1 << shift;
        const int r = l & (w - 1);  // the lane's place among its row's lanes
        int incl = n;
        for (int d = 1; d < w; d <<= 1) {
            const int t = __shfl_up(incl, d, w);
            if (r >= d) incl += t;
        }
        const int total = __shfl(incl, w - 1, w);
        const int row = row0 + (l >> shift);
        int base = 0;
        if (r == 0 && total > 0) base = atomicAdd(a.cnt + row, total);
        base = __shfl(base, 0, w) + (incl - n);
        int* out = a.lst + (size_t)row * a.caps;
#pragma unroll 1
        for (int e = 0; e < n; ++e)
            if (base + e < a.caps) out[base + e] = run[64 * e + l];
        n = 0;
    }
    __device__ __forceinline__ void push(int j, const RegfArgs& a) {
        const int l = lane();
        if (n < N) {
            run[64 * n + l] = j;
            ++n;
        } else {
            const int row = row0 + (l >> shift);
            const int k = atomicAdd(a.cnt + row, 1);
            if (k < a.caps) a.lst[(size_t)row * a.caps + k] = j;
        }
    }
};

template <int MODE> struct RecOf;
template <> struct RecOf<MODE_FF>  { using T = RecFF; };
template <> struct RecOf<MODE_F64> { using T = RecF64; };
template <> struct RecOf<MODE_F32> { using T = RecF32; };
template <> struct RecOf<MODE_LOC> { using T = RecLoc; };

// The record an i-particle's own state is read from: its j-record, except in
// the local mode, whose i-side is the float-float prediction by particle
// index (hi + lo, exact in FP64).
template <int MODE> struct IRecOf { using T = typename RecOf<MODE>::T; };
template <> struct IRecOf<MODE_LOC> { using T = RecFF; };

// i-side coordinates.  In the local mode, c is (tile centre - R_i) rounded to
// FP32, formed in FP64 on entry to each tile of j (tile_enter).
template <int MODE> struct IPos;
template <> struct IPos<MODE_FF>  { float xh, yh, zh, xl, yl, zl; };
template <> struct IPos<MODE_F64> { double x, y, z; };
template <> struct IPos<MODE_F32> { float x, y, z; };
template <> struct IPos<MODE_LOC> { double x, y, z; float cx, cy, cz; };

// h2: squared neighbour radius; c: (h + dtr |v_i|) (1 + 2^-16), the i-part
// of the candidate radius.
struct IAux { float vx, vy, vz, vabs, h2, dtr, c; };

template <typename P>
__device__ __forceinline__ void take_vel(const P& r, IAux& v) {
    v.vx = r.vx; v.vy = r.vy; v.vz = r.vz; v.vabs = r.vabs;
}
__device__ __forceinline__ void get_ipos(const RecFF& r, IPos<MODE_FF>& p, IAux& v) {
    p.xh = r.xh; p.yh = r.yh; p.zh = r.zh;
    p.xl = r.xl; p.yl = r.yl; p.zl = r.zl;
    take_vel(r, v);
}
__device__ __forceinline__ void get_ipos(const RecF64& r, IPos<MODE_F64>& p, IAux& v) {
    p.x = r.x; p.y = r.y; p.z = r.z;
    take_vel(r, v);
}
__device__ __forceinline__ void get_ipos(const RecF32& r, IPos<MODE_F32>& p, IAux& v) {
    p.x = r.x; p.y = r.y; p.z = r.z;
    take_vel(r, v);
}
__device__ __forceinline__ void get_ipos(const RecFF& r, IPos<MODE_LOC>& p, IAux& v) {
    p.x = (double)r.xh + (double)r.xl;
    p.y = (double)r.yh + (double)r.yl;
    p.z = (double)r.zh + (double)r.zl;
    p.cx = p.cy = p.cz = 0.0f;
    take_vel(r, v);
}

// Entering a tile of j: the local mode forms (centre - R_i) in FP64 and
// rounds it once; the other modes need nothing per tile.
template <int MODE>
__device__ __forceinline__ void tile_enter(IPos<MODE>&, double, double, double) {}
template <>
__device__ __forceinline__ void tile_enter<MODE_LOC>(IPos<MODE_LOC>& p, double ox, double oy,
                                                     double oz) {
    p.cx = (float)(ox - p.x);
    p.cy = (float)(oy - p.y);
    p.cz = (float)(oz - p.z);
}

// R_j - R_i in FP32 from each coordinate representation.
__device__ __forceinline__ void coord_diff(const RecFF& j, const IPos<MODE_FF>& i, float d[3]) {
    d[0] = (j.xh - i.xh) + (j.xl - i.xl);
    d[1] = (j.yh - i.yh) + (j.yl - i.yl);
    d[2] = (j.zh - i.zh) + (j.zl - i.zl);
}
__device__ __forceinline__ void coord_diff(const RecF64& j, const IPos<MODE_F64>& i, float d[3]) {
    d[0] = (float)(j.x - i.x);
    d[1] = (float)(j.y - i.y);
    d[2] = (float)(j.z - i.z);
}
__device__ __forceinline__ void coord_diff(const RecF32& j, const IPos<MODE_F32>& i, float d[3]) {
    d[0] = j.x - i.x;
    d[1] = j.y - i.y;
    d[2] = j.z - i.z;
}
// (R_j - centre) + (centre - R_i): two FP32 quantities of the pair's own
// scale (the tile is compact), so one FP32 add per component.
__device__ __forceinline__ void coord_diff(const RecLoc& j, const IPos<MODE_LOC>& i, float d[3]) {
    d[0] = j.ex + i.cx;
    d[1] = j.ey + i.cy;
    d[2] = j.ez + i.cz;
}

// The cluster index of the j-particle a record holds: the record's position
// in the stream, except in the local mode (spatial order), whose record
// carries it.
template <typename R>
__device__ __forceinline__ int j_index(const R&, int slot) { return slot; }
__device__ __forceinline__ int j_index(const RecLoc& r, int) { return r.p; }

// |R|^2 in FP32.
__device__ __forceinline__ float dist2(float dx, float dy, float dz) {
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// The neighbour criterion of section 3.2 on FP32 differences:
// min(|R|^2, |R + dtr V|^2) < h^2.  Used verbatim by the force kernel (for
// candidates) and by the ordered rescan of an overflowed list, so both take
// the same decisions.
__device__ __forceinline__ bool velocity_criterion(float r2, float dx, float dy, float dz,
                                                   float dvx, float dvy, float dvz,
                                                   float dtr, float h2) {
    const float px = fmaf(dtr, dvx, dx);
    const float py = fmaf(dtr, dvy, dy);
    const float pz = fmaf(dtr, dvz, dz);
    const float p2 = dist2(px, py, pz);
    return fminf(r2, p2) < h2;
}

// Candidate bound (c_i + dtr_i w)^2 for an upper bound w of |v_j|.
__device__ __forceinline__ float sq_bound(const IAux& ia, float w) {
    const float b = fmaf(ia.dtr, w, ia.c);
    return b * b;
}

// The term of one (i, j) pair (section 3.3 step 6).  With u = 1/|R|,
// g = m_j u^3 and s = 3 (R.V) u^2:
//   sum[0..2] += g R                  (acceleration),
//   sum[3..5] += g (V - s R)          (its time derivative, the jerk),
//   sum[6]    += m_j u                (when NP == 7: the potential sum),
// unless j is a neighbour of i (section 3.2), which is then added to the
// lane's run for i's list row and contributes u = 0 instead.
//
// The criterion runs only for candidate pairs, |R|^2 < bnd2, where
// bnd2 = (c_i + dtr_i w)^2 for some w >= |v_j| (the caller's choice: v_j's
// own bound, or that of j's tile).  Since |R + dtr V| >= |R| - dtr (|v_i| +
// |v_j|), a pair outside that radius is no neighbour; the 2^-16 relative
// margin inside c_i covers the FP32 rounding of every quantity involved, so
// the decision is that of the criterion alone.  A wavefront takes the branch
// only when one of its lanes is near j.
template <int MODE, int NP, int N>
__device__ __forceinline__ void pair_term(const typename RecOf<MODE>::T& r, int slot,
                                          const IPos<MODE>& ip, const IAux& ia, float bnd2,
                                          float sum[NP], Staged<N>& stg,
                                          const RegfArgs& a) {
    float R[3];
    coord_diff(r, ip, R);
    const float V[3] = {r.vx - ia.vx, r.vy - ia.vy, r.vz - ia.vz};
    const float r2 = dist2(R[0], R[1], R[2]);
    float u = __builtin_amdgcn_rsqf(r2);
    const float rv = fmaf(R[2], V[2], fmaf(R[1], V[1], R[0] * V[0]));
    if (r2 < bnd2) {
        // Keeps the criterion behind the branch: without it the compiler may
        // compute it for every pair and merge the two tests (8 more vector
        // instructions per interaction).  Emits no instruction.
        __asm__ volatile("");
        if (velocity_criterion(r2, R[0], R[1], R[2], V[0], V[1], V[2], ia.dtr, ia.h2)) {
            stg.push(j_index(r, slot), a);
            u = 0.0f;
        }
    }
    const float u2 = u * u;
    const float mu = r.m * u;
    const float g = mu * u2;
    const float s = (3.0f * rv) * u2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sum[c] = fmaf(g, R[c], sum[c]);
        sum[3 + c] = fmaf(g, fmaf(-s, R[c], V[c]), sum[3 + c]);
    }
    if constexpr (NP == 7) sum[6] += mu;
}

// The j-records are not written while the force kernel runs, so they are
// read through the constant address space: a wave-uniform address then
// becomes a scalar load into SGPRs.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T*;

__device__ __forceinline__ RecFF load_rec(const_ptr<RecFF> p) {
    RecFF r;
    r.xh = p->xh; r.yh = p->yh; r.zh = p->zh; r.m = p->m;
    r.xl = p->xl; r.yl = p->yl; r.zl = p->zl; r.vabs = p->vabs;
    r.vx = p->vx; r.vy = p->vy; r.vz = p->vz; r.pad = 0.0f;
    return r;
}
__device__ __forceinline__ RecF64 load_rec(const_ptr<RecF64> p) {
    RecF64 r;
    r.x = p->x; r.y = p->y; r.z = p->z;
    r.vx = p->vx; r.vy = p->vy; r.vz = p->vz; r.m = p->m;
    r.vabs = p->vabs; r.pad = 0.0f;
    return r;
}
__device__ __forceinline__ RecF32 load_rec(const_ptr<RecF32> p) {
    RecF32 r;
    r.x = p->x; r.y = p->y; r.z = p->z; r.m = p->m;
    r.vx = p->vx; r.vy = p->vy; r.vz = p->vz; r.vabs = p->vabs;
    return r;
}
__device__ __forceinline__ RecLoc load_rec(const_ptr<RecLoc> p) {
    RecLoc r;
    r.ex = p->ex; r.ey = p->ey; r.ez = p->ez; r.m = p->m;
    r.vx = p->vx; r.vy = p->vy; r.vz = p->vz; r.p = p->p;
    return r;
}

// The candidate bound w of a tile of j (the largest vabs of its records),
// and, in the local mode, the tile's centre entered into the i-positions.
template <int MODE, int IPL>
__device__ __forceinline__ float enter_tile(const RegfArgs& a, int jt, IPos<MODE> ip[IPL]) {
    if constexpr (MODE == MODE_LOC) {
        const_ptr<TileOrg> o = (const_ptr<TileOrg>)(a.org) + jt / TILE;
        const double ox = o->x, oy = o->y, oz = o->z;
        const float w = o->vmax;
#pragma unroll
        for (int k = 0; k < IPL; ++k) tile_enter<MODE>(ip[k], ox, oy, oz);
        return w;
    } else {
        return ((const_ptr<float>)(a.tmax))[jt / TILE];
    }
}

// h2 as the float the kernels compare against, or -1 when it is not a
// positive normal float (then the i is invalid).
__device__ __forceinline__ float checked_h2(double h2) {
    const float f = (float)h2;
    return (f >= FLT_MIN && f <= FLT_MAX) ? f : -1.0f;
}

// Index of partial sum (q, s, c) in the block layout [q/64][s][c][q%64] of
// np components per (particle, slice).
__device__ __forceinline__ size_t part_index(int q, int s, int c, int nslices, int np) {
    return (((size_t)(q >> 6) * nslices + s) * np + c) * 64 + (q & 63);
}

// State of the i-particle at work position q for the force kernel: position,
// velocity, neighbour radius and the i-part of the candidate radius (from
// the i-records in work order when the call runs in an i-order, else from
// the records by particle index).  Returns the list row the lane appends to,
// q (row 0 for lanes without a valid i: those never append, since their h2
// is -1 and their candidate radius NaN).  A bad index or radius is flagged
// once, by the work items of slice 0.
template <int MODE>
__device__ __forceinline__ int load_i(const RegfArgs& a, const int q, const int s,
                                      IPos<MODE>& ip, IAux& ia) {
    using IRec = typename IRecOf<MODE>::T;
    bool live = q < a.ni;
    int pi = live ? a.idx[q] : 0;
    float h2f = live ? checked_h2(a.h2[q]) : -1.0f;
    const double dtr = live ? a.dtr[q] : 0.0;
    float dtf = (float)dtr;
    if (live) {
        unsigned bad = 0;
        if (pi < 0 || pi >= a.n) bad |= ST_BAD_INDEX;
        if (h2f < 0.0f) bad |= ST_BAD_H2;
        if (!valid_dtr(dtr)) bad |= ST_BAD_DTR;
        if (bad) {
            if (s == 0) atomicOr(a.status, bad);
            pi = 0;
            h2f = -1.0f;
            dtf = 0.0f;
            live = false;
        }
    }
    const IRec* rv = static_cast<const IRec*>(MODE == MODE_LOC ? a.ivw : a.rec);  // per lane
    get_ipos(live && a.irec ? static_cast<const IRec*>(a.irec)[q] : rv[pi], ip, ia);
    ia.h2 = h2f;
    ia.dtr = dtf;
    ia.c = (float)((sqrt((double)h2f) + (double)dtf * (double)ia.vabs) * (1.0 + 0x1p-16));
    return live ? q : 0;
}

// The wavefront's part of its workgroup's run storage (RUN entries per lane,
// wavefront after wavefront).
__device__ __forceinline__ int* run_wave(int* runs) {
    return runs + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * (RUN * 64);
}

// Force, jerk and neighbour appends of one (i-group, j-slice) work item:
// 64 * IPL active particles starting at group * 64 * IPL, against the
// j-particles of slice s.  runs: the wavefront's run storage (run_wave).
template <int MODE, int IPL, int NP>
__device__ __forceinline__ void regf_item(const RegfArgs& a, const int group, const int s,
                                          int* runs) {
    using Rec = typename RecOf<MODE>::T;
    const_ptr<Rec> rec = (const_ptr<Rec>)(a.rec);
    const int lane = threadIdx.x & 63;
    const int ibase = group * 64 * IPL;

    IPos<MODE> ip[IPL];
    IAux ia[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) (void)load_i<MODE>(a, ibase + k * 64 + lane, s, ip[k], ia[k]);
    // A lane's list row is its q = ibase + k * 64 + lane, recomputed from the
    // lane id where it is needed (lanes without a valid i never append).
    constexpr int N = RUN / IPL;
    Staged<N> stg[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        stg[k].run = runs + k * N * 64;
        stg[k].row0 = ibase + k * 64;
        stg[k].shift = 0;
        stg[k].n = 0;
    }

    const int j0 = s * a.slice_len;
    const int j1 = min(j0 + a.slice_len, a.n);

    double sum[IPL][NP];
#pragma unroll
    for (int k = 0; k < IPL; ++k)
#pragma unroll
        for (int c = 0; c < NP; ++c) sum[k][c] = 0.0;

    for (int jt = j0; jt < j1; jt += TILE) {  // j0 is a multiple of TILE
        const int je = min(jt + TILE, j1);
        float run[IPL][NP];
#pragma unroll
        for (int k = 0; k < IPL; ++k)
#pragma unroll
            for (int c = 0; c < NP; ++c) run[k][c] = 0.0f;
        // candidate bound of the tile: its largest |v_j| for every j
        const float vm = enter_tile<MODE, IPL>(a, jt, ip);
        float bnd2[IPL];
#pragma unroll
        for (int k = 0; k < IPL; ++k) bnd2[k] = sq_bound(ia[k], vm);

        // groups of G records: all their scalar loads are issued before the
        // first interaction of the group, so one load latency covers G j.
        // With two i per lane a group of 2 gives as many interactions per
        // load as 4 with one, and keeps the kernel within 128 VGPRs.
        constexpr int G = IPL == 2 ? 2 : JG;
        int j = jt;
        for (; j + G <= je; j += G) {
            Rec r[G];
#pragma unroll
            for (int g = 0; g < G; ++g) r[g] = load_rec(rec + j + g);
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int k = 0; k < IPL; ++k)
                    pair_term<MODE, NP, N>(r[g], j + g, ip[k], ia[k], bnd2[k], run[k],
                                           stg[k], a);
        }
        for (; j < je; ++j) {
            const Rec r = load_rec(rec + j);
#pragma unroll
            for (int k = 0; k < IPL; ++k)
                pair_term<MODE, NP, N>(r, j, ip[k], ia[k], bnd2[k], run[k], stg[k], a);
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k)
#pragma unroll
            for (int c = 0; c < NP; ++c) sum[k][c] += (double)run[k][c];
#pragma unroll
        for (int k = 0; k < IPL; ++k) stg[k].flush_half(a);
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) stg[k].flush(a);

    // partial sums by 64-particle block: part[q / 64][s][c][q % 64], so each
    // component of a wave's 64 particles is one contiguous 512-byte store
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int q = ibase + k * 64 + lane;
        if (q < a.ni) {
            double* p = a.part + part_index(q, s, 0, a.nslices, NP);
#pragma unroll
            for (int c = 0; c < NP; ++c) p[c * 64] = sum[k][c];
        }
    }
}

// Terms of G records j, j + jl, ... for a lane that reads its own records
// (the lanes-per-i kernel).  The candidate bound is each record's vabs; in
// the local mode it is that of the record's tile, whose centre the lane
// enters first (the tiles are loaded together, ahead of the terms).
template <int MODE, int NP, int G>
__device__ __forceinline__ void lane_terms(const RegfArgs& a, const typename RecOf<MODE>::T* r,
                                           int j, int jl, IPos<MODE>& ip, const IAux& ia,
                                           float run[NP], Staged<RUN>& stg) {
    if constexpr (MODE == MODE_LOC) {
        TileOrg o[G];
#pragma unroll
        for (int g = 0; g < G; ++g) o[g] = a.org[(j + g * jl) / TILE];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            tile_enter<MODE>(ip, o[g].x, o[g].y, o[g].z);
            pair_term<MODE, NP, RUN>(r[g], j + g * jl, ip, ia, sq_bound(ia, o[g].vmax), run, stg,
                                     a);
        }
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g)
            pair_term<MODE, NP, RUN>(r[g], j + g * jl, ip, ia, sq_bound(ia, r[g].vabs), run, stg,
                                     a);
    }
}

// The same work item when 2^jl_shift consecutive lanes share one i: the
// wavefront holds 64 >> jl_shift particles starting at group * (64 >>
// jl_shift), and lane k of an i's lanes takes the j-particles j0 + k,
// j0 + k + 2^jl_shift, ... of the slice.  The records are vector loads (the
// lanes read different j).  At the end, a butterfly over the i's lanes adds
// their FP64 sums; it gives the same bits in each of those lanes, and the
// first of them stores the partial.  Used when the active block is too small
// to give every lane its own i and still fill the chip.
template <int MODE, int NP>
__device__ __forceinline__ void regf_item_lanes(const RegfArgs& a, const int group, const int s,
                                                int* runs) {
    using Rec = typename RecOf<MODE>::T;
    const Rec* rec = static_cast<const Rec*>(a.rec);
    const int lane = threadIdx.x & 63;
    const int sh = a.jl_shift;
    const int jl = 1 << sh;
    const int jsub = lane & (jl - 1);
    const int q = group * (64 >> sh) + (lane >> sh);

    IPos<MODE> ip;
    IAux ia;
    (void)load_i<MODE>(a, q, s, ip, ia);
    Staged<RUN> stg;
    stg.run = runs;
    stg.row0 = group * (64 >> sh);
    stg.shift = sh;
    stg.n = 0;

    const int j0 = s * a.slice_len;
    const int j1 = min(j0 + a.slice_len, a.n);

    double sum[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) sum[c] = 0.0;

    for (int jt = j0; jt < j1; jt += TILE * jl) {
        const int je = min(jt + TILE * jl, j1);
        float run[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) run[c] = 0.0f;
        int j = jt + jsub;
        for (; j + (JG - 1) * jl < je; j += JG * jl) {
            Rec r[JG];
#pragma unroll
            for (int g = 0; g < JG; ++g) r[g] = rec[j + g * jl];
            lane_terms<MODE, NP, JG>(a, r, j, jl, ip, ia, run, stg);
        }
        for (; j < je; j += jl) {
            const Rec r[1] = {rec[j]};
            lane_terms<MODE, NP, 1>(a, r, j, jl, ip, ia, run, stg);
        }
#pragma unroll
        for (int c = 0; c < NP; ++c) sum[c] += (double)run[c];
        if (__any(stg.n >= RUN / 2)) stg.flush_shared(a);  // uniform
    }
    if (__any(stg.n > 0)) stg.flush_shared(a);  // uniform

    for (int d = 1; d < jl; d <<= 1)
#pragma unroll
        for (int c = 0; c < NP; ++c) sum[c] += __shfl_xor(sum[c], d);

    if (jsub == 0 && q < a.ni) {
        double* p = a.part + part_index(q, s, 0, a.nslices, NP);
#pragma unroll
        for (int c = 0; c < NP; ++c) p[c * 64] = sum[c];
    }
}

// j-records per chunk that a lanes workgroup stages through LDS: it divides
// the tile of 16, 32 or 64 lanes per i (TILE x 16 .. TILE x 64 j), so chunks
// nest in tiles (the smaller tiles of forced lane counts are one chunk each).
constexpr int LCHUNK = 256;
template <int MODE> constexpr size_t lanes_stage_bytes() { return LCHUNK * sizeof(typename RecOf<MODE>::T); }
// Staged when the workgroup has several waves and each wave reads each
// record in several lanes (at most 32 lanes per i): LDS serves such a read
// once for all its lanes.  At 64 lanes per i every lane reads a record of
// its own and the vector cache was the faster (C3, N = 131072: N_i = 8 .. 64
// took 12.3, 17.2, 18.6, 25.3 us per force kernel through it, 14.1, 21.4,
// 21.8, 28.0 through LDS; at 32 and 16 lanes N_i = 128 and 256 took 33.4
// and 55.2 us through it, 30.4 and 45.2 through LDS).
__host__ __device__ constexpr bool lanes_staged(int jl_shift, int wpb) {
    return wpb > 1 && jl_shift > 0 && jl_shift <= 5;
}

// regf_item_lanes for a workgroup of several waves (different i-groups, the
// same slice): the workgroup copies each chunk of the slice's j-records into
// LDS once, and every wave reads them there, where the plain form has each
// wave load the whole slice through the vector cache (a record per pair and
// lane, which the waves of small blocks mostly wait for).  Each lane visits
// the same j in the same order, folds its FP32 sums at the same tile ends
// and adds its i's lanes in the same butterfly, so the partials have the
// same bits.
// Waves without particles (live false) still copy chunks and meet every
// barrier; the chunk loop's bounds are uniform across the workgroup.
template <int MODE, int NP>
__device__ __forceinline__ void regf_item_lanes_lds(const RegfArgs& a, const int group, const int s,
                                                    int* runs, typename RecOf<MODE>::T* stage,
                                                    const bool live) {
    using Rec = typename RecOf<MODE>::T;
    constexpr int P = (int)(sizeof(Rec) / sizeof(uint4));  // 16-byte pieces per record
    static_assert(sizeof(Rec) % sizeof(uint4) == 0, "records are whole 16-byte pieces");
    const uint4* src = static_cast<const uint4*>(a.rec);
    uint4* dst = reinterpret_cast<uint4*>(stage);
    const int lane = threadIdx.x & 63;
    const int sh = a.jl_shift;
    const int jl = 1 << sh;
    const int jsub = lane & (jl - 1);
    const int q = group * (64 >> sh) + (lane >> sh);

    IPos<MODE> ip;
    IAux ia;
    if (live) (void)load_i<MODE>(a, q, s, ip, ia);
    Staged<RUN> stg;
    stg.run = runs;
    stg.row0 = group * (64 >> sh);
    stg.shift = sh;
    stg.n = 0;

    const int j0 = s * a.slice_len;
    const int j1 = min(j0 + a.slice_len, a.n);

    double sum[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) sum[c] = 0.0;

    for (int jt = j0; jt < j1; jt += TILE * jl) {
        const int te = min(jt + TILE * jl, j1);
        float run[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) run[c] = 0.0f;
        for (int jc = jt; jc < te; jc += LCHUNK) {
            const int ce = min(jc + LCHUNK, te);
            __syncthreads();  // every wave is done with the previous chunk
            for (int e = (int)threadIdx.x; e < (ce - jc) * P; e += (int)blockDim.x)
                dst[e] = src[(size_t)jc * P + e];
            __syncthreads();
            if (live) {  // uniform across the wave
                int j = jc + jsub;  // jc - jt is a multiple of jl
                for (; j + (JG - 1) * jl < ce; j += JG * jl) {
                    Rec r[JG];
#pragma unroll
                    for (int g = 0; g < JG; ++g) r[g] = stage[j + g * jl - jc];
                    lane_terms<MODE, NP, JG>(a, r, j, jl, ip, ia, run, stg);
                }
                for (; j < ce; j += jl) {
                    const Rec r[1] = {stage[j - jc]};
                    lane_terms<MODE, NP, 1>(a, r, j, jl, ip, ia, run, stg);
                }
            }
        }
        if (live) {
#pragma unroll
            for (int c = 0; c < NP; ++c) sum[c] += (double)run[c];
            if (__any(stg.n >= RUN / 2)) stg.flush_shared(a);  // uniform
        }
    }
    if (!live) return;
    if (__any(stg.n > 0)) stg.flush_shared(a);  // uniform

    for (int d = 1; d < jl; d <<= 1)
#pragma unroll
        for (int c = 0; c < NP; ++c) sum[c] += __shfl_xor(sum[c], d);

    if (jsub == 0 && q < a.ni) {
        double* p = a.part + part_index(q, s, 0, a.nslices, NP);
#pragma unroll
        for (int c = 0; c < NP; ++c) p[c * 64] = sum[c];
    }
}

// One launch of one request: a 1-D grid of nslices x gblocks workgroups,
// gblocks = i-groups / waves per block.  Workgroups are handed to the 8 XCDs
// in turn (workgroup id mod 8), so when nslices is a multiple of 8 the
// mapping below gives every slice to one XCD: each XCD's L2 then holds the
// j-records of its own slices only.  At least 4 waves per SIMD (<= 128
// VGPRs): below that the scalar-load latency of the j-records is no longer
// hidden.
template <int MODE, int IPL, int NP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(IPL == 1 ? 6 : 4)))
regf_kernel(RegfArgs a, int gblocks) {
    const int b = blockIdx.x;
    int s, gb;
    if ((a.nslices & 7) == 0) {
        const int xcd = b & 7, k = b >> 3;
        s = xcd + 8 * (k / gblocks);
        gb = k % gblocks;
    } else {
        s = b / gblocks;
        gb = b % gblocks;
    }
    const int wpb = blockDim.x >> 6;
    const int group = gb * wpb + (threadIdx.x >> 6);
    extern __shared__ int runs[];  // run_lds_bytes(wpb)
    if (group * 64 * IPL >= a.ni) return;  // uniform across the wave
    regf_item<MODE, IPL, NP>(a, group, s, run_wave(runs));
}

// The force kernel for lanes that share an i (a.jl_shift > 0), with the grid
// and XCD mapping of regf_kernel; a workgroup of several waves at 16 or 32
// lanes per i stages its slice's j-records through LDS.
template <int MODE, int NP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
regf_lanes_kernel(RegfArgs a, int gblocks) {
    const int b = blockIdx.x;
    int s, gb;
    if ((a.nslices & 7) == 0) {
        const int xcd = b & 7, k = b >> 3;
        s = xcd + 8 * (k / gblocks);
        gb = k % gblocks;
    } else {
        s = b / gblocks;
        gb = b % gblocks;
    }
    const int wpb = blockDim.x >> 6;
    const int group = gb * wpb + (threadIdx.x >> 6);
    // run_lds_bytes(wpb), then (several waves, not the local mode) the
    // stage of lanes_stage_bytes<MODE>()
    extern __shared__ int runs[];
    const bool live = group * (64 >> a.jl_shift) < a.ni;  // uniform across the wave
    if constexpr (MODE != MODE_LOC) {
        if (lanes_staged(a.jl_shift, wpb)) {  // uniform across the workgroup
            using Rec = typename RecOf<MODE>::T;
            Rec* stage = reinterpret_cast<Rec*>(runs + (size_t)wpb * RUN * 64);
            regf_item_lanes_lds<MODE, NP>(a, group, s, run_wave(runs), stage, live);
            return;
        }
    }
    if (!live) return;
    regf_item_lanes<MODE, NP>(a, group, s, run_wave(runs));
}

// ---------------------------------------------------------------------------
// Finalize: workgroup b of a request (4 waves) does
//   sums  -- for b < NP ceil(ni / 64), component b / ceil(ni / 64) of the
//            slice partials of particles 64 m .. 64 m + 63, m = b mod
//            ceil(ni / 64).  The four waves split each particle's partials
//            in runs of 8 slices and the run sums are combined in a fixed
//            order, so the result depends on the slicing only (lane t of a
//            wave reads particle 64 m + t: contiguous loads).
//   lists -- particles 4b .. 4b + 3, one per wave: the neighbour count, and
//            the counter reset to zero for the next call.  count <= caps:
//            every neighbour was stored, and an entry's output position is
//            its rank among the entries (they are distinct), less one past
//            the i itself.  count > caps: the list overflowed and the wave
//            rebuilds it by an ordered rescan of every j.
// A request therefore takes final_blocks(ni, NP) workgroups.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of the finalize kernels: the four waves' slice sums of one component,
// and later (the same bytes) one buffer of MAX_CAPS list entries per wave.
union FinalShared {
    double  sum[4][64];
    int32_t list[4][MAX_CAPS];
};

// Slice sums of component c of particles 64 blk .. 64 blk + 63, by the whole
// workgroup (NP partial components: acc, jerk and, for 7, the potential sum).
// Wave w adds the runs of 8 slices that start at 8 w, 8 w + 32, ... in slice
// order, and the four run sums are added in wave order: the result depends on
// the slicing only.  Four runs are loaded before the first of their adds.
template <int NP>
__device__ __forceinline__ void finalize_sums(const FinalArgs& a, const int blk, const int c,
                                              FinalShared& sh) {
    constexpr int RUNS = 4;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = blk * 64 + lane;
    // the i's own entries are loaded with the partials (one round of loads
    // for a small block); the active position first when the call ran in
    // the spatial order
    const bool mine = w == 0 && q < a.ni;
    const int o = mine && a.iord ? a.iord[q] : q;
    const int32_t self = mine ? a.idx[o] : 0;
    const double h2 = mine ? a.h2[o] : 0.0, dtr = mine ? a.dtr[o] : 0.0;
    double sum = 0.0;
    if (q < a.ni) {
        const double* p = a.part + part_index(q, 0, c, a.nslices, NP);
        for (int s0 = 8 * w; s0 < a.nslices; s0 += 32 * RUNS) {
            double v[RUNS][8];
#pragma unroll
            for (int r = 0; r < RUNS; ++r)
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int sl = s0 + 32 * r + u;
                    v[r][u] = sl < a.nslices ? p[(size_t)sl * NP * 64] : 0.0;
                }
#pragma unroll
            for (int r = 0; r < RUNS; ++r)
                if (s0 + 32 * r < a.nslices)
#pragma unroll
                    for (int u = 0; u < 8; ++u) sum += v[r][u];
        }
    }
    sh.sum[w][lane] = sum;
    __syncthreads();
    if (mine) {
        if (self < 0 || self >= a.n || checked_h2(h2) < 0.0f || !valid_dtr(dtr)) {
            const double nan = __builtin_nan("");
            if (c < 3) a.acc[3 * o + c] = nan;
            else if (c < 6) a.jerk[3 * o + c - 3] = nan;
            else a.pot[o] = nan;
        } else {
            const double t = ((sh.sum[0][lane] + sh.sum[1][lane]) + sh.sum[2][lane]) +
                             sh.sum[3][lane];
            if (c < 3) a.acc[3 * o + c] = t;
            else if (c < 6) a.jerk[3 * o + c - 3] = t;
            else a.pot[o] = -t;  // the potential is minus the sum of m / r
        }
    }
    __syncthreads();  // the LDS is reused for lists
}

// Ordered rescan of particle q (wave-uniform, valid), whose neighbours
// outnumber its list capacity: every j in ascending order under the force
// kernel's neighbour test (the velocity criterion alone decides the same as
// the kernel's candidate bound followed by it), keeping the first cap.
// Four records per lane are in flight per step.
template <int MODE>
__device__ __forceinline__ void rescan_list(const FinalArgs& a, const int q, const int32_t self) {
    using Rec = typename RecOf<MODE>::T;
    using IRec = typename IRecOf<MODE>::T;
    const Rec* rec = static_cast<const Rec*>(a.rec);
    const int lane = threadIdx.x & 63;
    IPos<MODE> ip;
    IAux ia;
    get_ipos(static_cast<const IRec*>(MODE == MODE_LOC ? a.ivw : a.rec)[self], ip, ia);
    const float h2f = checked_h2(a.h2[q]);
    const float dtf = (float)a.dtr[q];
    int32_t* out = a.list + (size_t)q * a.cap;
    const unsigned long long below = (1ull << lane) - 1ull;
    int found = 0;  // wave-uniform
    for (int j0 = 0; j0 < a.n && found < a.cap; j0 += 4 * 64) {
        // the four records first (clamped indices: in bounds for every lane),
        // then the tests without short-circuit evaluation, so that the loads
        // are not moved into branches and issued one after another.  In the
        // local mode particle j sits in slot inv[j], and the test enters its
        // tile's centre as the force kernel does, so the bits are the same.
        Rec r[4];
        int slot[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = min(j0 + 64 * u + lane, a.n - 1);
            slot[u] = MODE == MODE_LOC ? a.inv[j] : j;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = rec[slot[u]];
        bool nb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = j0 + 64 * u + lane;
            if constexpr (MODE == MODE_LOC) {
                const TileOrg& o = a.org[slot[u] / TILE];
                tile_enter<MODE>(ip, o.x, o.y, o.z);
            }
            float d[3];
            coord_diff(r[u], ip, d);
            const bool hit = velocity_criterion(dist2(d[0], d[1], d[2]), d[0], d[1], d[2],
                                                r[u].vx - ia.vx, r[u].vy - ia.vy,
                                                r[u].vz - ia.vz, dtf, h2f);
            nb[u] = (j < a.n) & (j != self) & hit;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned long long m = __ballot(nb[u]);
            const int pos = found + __popcll(m & below);
            if (nb[u] && pos < a.cap) out[pos] = j0 + 64 * u + lane;
            found += __popcll(m);
        }
    }
}

// Sorted list of the i at active position q (wave-uniform; its found entries
// are in scratch row qs) from its `count` found entries; `first` holds entry
// `lane` when lane < min(count, caps).  sl: this wave's LDS buffer, for lists
// longer than one wavefront.
__device__ __forceinline__ void finalize_list(const FinalArgs& a, const int q, const int qs,
                                              const int32_t self, const int count,
                                              const int32_t first, int32_t* sl) {
    const int lane = threadIdx.x & 63;
    if (count > a.caps) {
        if (lane == 0) atomicOr(a.status, (unsigned)ST_OVERFLOW);
        switch (a.mode) {  // uniform
            case MODE_FF: rescan_list<MODE_FF>(a, q, self); break;
            case MODE_F64: rescan_list<MODE_F64>(a, q, self); break;
            case MODE_LOC: rescan_list<MODE_LOC>(a, q, self); break;
            default: rescan_list<MODE_F32>(a, q, self); break;
        }
        return;
    }
    int32_t* out = a.list + (size_t)q * a.cap;
    if (count <= 64) {
        // one entry per lane; ranks by reading every entry across the wave
        const int32_t v = lane < count ? first : INT32_MAX;
        int rank = 0;
        for (int k = 0; k < count; ++k) rank += __builtin_amdgcn_readlane(v, k) < v ? 1 : 0;
        const int pos = rank - (v > self ? 1 : 0);
        if (lane < count && v != self && pos < a.cap) out[pos] = v;
        return;
    }
    const int32_t* l = a.lst + (size_t)qs * a.caps;
    for (int e = lane; e < count; e += 64) sl[e] = l[e];
    wave_sync();
    for (int e = lane; e < count; e += 64) {
        const int32_t v = sl[e];
        if (v == self) continue;
        int rank = 0;
        for (int k = 0; k < count; ++k) rank += sl[k] < v ? 1 : 0;
        const int pos = rank - (v > self ? 1 : 0);
        if (pos >= 0 && pos < a.cap) out[pos] = v;
    }
    wave_sync();  // sl is rewritten for the next particle
}

// Workgroup blk of one request's finalize.
template <int NP>
__device__ __forceinline__ void finalize_block(const FinalArgs& a, const int blk,
                                               FinalShared& sh) {
    const int nb64 = (a.ni + 63) >> 6;
    if (blk < NP * nb64) finalize_sums<NP>(a, blk % nb64, blk / nb64, sh);  // uniform
    if (blk >= final_list_blocks(a.ni)) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int PPW = FINAL_PPB / 4;
    const int q0 = blk * FINAL_PPB + w * PPW;
    // every load of the wave's particles is issued before the first sort
    // (q0 + k: the work position, whose count and row the force kernel
    // filled; o: the active position, which the outputs are indexed by)
    int32_t self[PPW], count[PPW], first[PPW], o[PPW];
    bool live[PPW], ok[PPW];
#pragma unroll
    for (int k = 0; k < PPW; ++k) {
        const int q = q0 + k;
        live[k] = q < a.ni;
        o[k] = live[k] && a.iord ? a.iord[q] : q;
        self[k] = live[k] ? a.idx[o[k]] : -1;
        const float h2f = live[k] ? checked_h2(a.h2[o[k]]) : -1.0f;
        count[k] = live[k] ? a.cnt[q] : 0;
        first[k] = live[k] && lane < a.caps ? a.lst[(size_t)q * a.caps + lane] : 0;
        ok[k] = live[k] && self[k] >= 0 && self[k] < a.n && h2f >= 0.0f &&
                valid_dtr(a.dtr[o[k]]);
    }
    // the count is read: reset it for the next call, and store the number of
    // neighbours (the i itself is among the found; -1 marks an invalid i)
#pragma unroll
    for (int k = 0; k < PPW; ++k)
        if (live[k] && lane == 0) {
            a.cnt[q0 + k] = 0;
            a.nnb[o[k]] = ok[k] ? count[k] - 1 : -1;
        }
#pragma unroll
    for (int k = 0; k < PPW; ++k)
        if (ok[k]) finalize_list(a, o[k], q0 + k, self[k], count[k], first[k], sh.list[w]);
}

template <int NP>
__global__ void __launch_bounds__(256) finalize_kernel(FinalArgs a) {
    __shared__ FinalShared sh;
    finalize_block<NP>(a, blockIdx.x, sh);
}

// ---------------------------------------------------------------------------
// Serving: fused launches over the requests of a batch.  The descriptors are
// copied to the device before the launches and read with scalar loads.
// ---------------------------------------------------------------------------
// The copies below name every field (a struct copy out of the constant
// address space does not compile); the sizes pin the field lists, so a field
// added to an argument struct cannot be left out here unnoticed.
static_assert(sizeof(RegfArgs) == 128, "load_regf_args must copy every RegfArgs field");
static_assert(sizeof(FinalArgs) == 168, "load_final_args must copy every FinalArgs field");

__device__ __forceinline__ RegfArgs load_regf_args(const_ptr<ReqDesc> d) {
    RegfArgs a;
    a.rec = d->rg.rec; a.n = d->rg.n; a.idx = d->rg.idx; a.h2 = d->rg.h2; a.dtr = d->rg.dtr;
    a.ni = d->rg.ni; a.slice_len = d->rg.slice_len; a.nslices = d->rg.nslices;
    a.jl_shift = d->rg.jl_shift; a.tmax = d->rg.tmax; a.org = d->rg.org; a.ivw = d->rg.ivw;
    a.part = d->rg.part; a.cnt = d->rg.cnt; a.lst = d->rg.lst; a.caps = d->rg.caps;
    a.status = d->rg.status; a.irec = d->rg.irec;
    return a;
}
__device__ __forceinline__ FinalArgs load_final_args(const_ptr<ReqDesc> d) {
    FinalArgs f;
    f.part = d->fin.part; f.cnt = d->fin.cnt; f.lst = d->fin.lst; f.nslices = d->fin.nslices;
    f.ni = d->fin.ni; f.caps = d->fin.caps; f.n = d->fin.n; f.idx = d->fin.idx; f.h2 = d->fin.h2;
    f.acc = d->fin.acc; f.jerk = d->fin.jerk; f.pot = d->fin.pot; f.nnb = d->fin.nnb;
    f.list = d->fin.list;
    f.cap = d->fin.cap; f.status = d->fin.status;
    f.rec = d->fin.rec; f.dtr = d->fin.dtr; f.mode = d->fin.mode;
    f.org = d->fin.org; f.inv = d->fin.inv; f.ivw = d->fin.ivw; f.iord = d->fin.iord;
    return f;
}

__device__ __forceinline__ long long uniform_ll(long long v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Persistent: wavefront w of the launch takes work item (request, i-group,
// j-slice) w first, then, while the launch has fewer wavefronts W than
// items, items W + t for tickets t = 0, 1, ... drawn from the batch counter
// after each item.  A launch with a wavefront per item draws no ticket.  The
// lanes class does the same per workgroup, an item being four i-groups of a
// slice.  An item's result depends only on its request, so a request gives
// the same bits alone or in any batch.  Each work-partition class of request
// (SERVE_ONE_I, SERVE_LANES, SERVE_TWO_I) gets a launch of its own, so the
// one-i kernel keeps the registers, hence the occupancy, of the plain one.
template <int MODE, int CLASS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CLASS == SERVE_ONE_I ? 6 : 4)))
serve_regf_kernel(BatchArgs b) {
    __shared__ int runs[WAVES * RUN * 64];
    int* const wruns = run_wave(runs);
    const_ptr<ReqDesc> reqs = (const_ptr<ReqDesc>)(b.reqs);
    if constexpr (CLASS == SERVE_LANES) {
        // A work item per workgroup: WAVES consecutive i-groups of one
        // slice, wave w taking the w-th, so that at 16 or 32 lanes per i the waves share the slice's
        // j-records through LDS as the plain call's workgroups do (the same
        // bits either way).  The item and the exit are uniform across the
        // workgroup, and every wave meets every barrier.
        using Rec = typename RecOf<MODE>::T;
        __shared__ Rec stage[LCHUNK];
        __shared__ long long next;
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        long long item = blockIdx.x;
        while (item < b.nitems) {
            int lo = 0, hi = b.nreq - 1;  // last request with item0 <= item
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (reqs[mid].item0 <= item) lo = mid; else hi = mid - 1;
            }
            const RegfArgs a = load_regf_args(reqs + lo);
            const long long local = item - reqs[lo].item0;
            const int groups = reqs[lo].groups;
            const int gblocks = (groups + WAVES - 1) / WAVES;
            const int g = (int)(local % gblocks) * WAVES + w, s = (int)(local / gblocks);
            const bool live = g < groups;  // uniform across the wave
            bool staged = false;
            if constexpr (MODE != MODE_LOC) {
                if (lanes_staged(a.jl_shift, WAVES)) {
                    regf_item_lanes_lds<MODE, NPART>(a, g, s, wruns, stage, live);
                    staged = true;
                }
            }
            if (!staged && live) regf_item_lanes<MODE, NPART>(a, g, s, wruns);
            if ((long long)gridDim.x >= b.nitems) break;  // no item beyond the first
            __syncthreads();  // every wave has read `next`
            if (threadIdx.x == 0) next = (long long)gridDim.x + (long long)atomicAdd(b.counter, 1ull);
            __syncthreads();
            item = next;
        }
        return;
    }
    const int wpb = blockDim.x >> 6;
    const long long waves = (long long)gridDim.x * wpb;
    long long item = (long long)blockIdx.x * wpb +
                     __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    while (item < b.nitems) {
        int lo = 0, hi = b.nreq - 1;  // last request with item0 <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (reqs[mid].item0 <= item) lo = mid; else hi = mid - 1;
        }
        const RegfArgs a = load_regf_args(reqs + lo);
        const long long local = item - reqs[lo].item0;
        const int groups = reqs[lo].groups;
        const int g = (int)(local % groups), s = (int)(local / groups);
        if (CLASS == SERVE_TWO_I)
            regf_item<MODE, 2, NPART>(a, g, s, wruns);
        else
            regf_item<MODE, 1, NPART>(a, g, s, wruns);
        if (waves >= b.nitems) break;  // uniform: no item beyond the first
        unsigned long long got = 0;
        if ((threadIdx.x & 63) == 0) got = atomicAdd(b.counter, 1ull);
        item = waves + uniform_ll((long long)got);
    }
}

__global__ void __launch_bounds__(256) serve_finalize_kernel(BatchArgs b) {
    __shared__ FinalShared sh;
    const_ptr<ReqDesc> reqs = (const_ptr<ReqDesc>)(b.reqs);
    const long long gb = blockIdx.x;  // finalize workgroup within the batch
    if (gb >= b.nblk_total) return;
    int lo = 0, hi = b.nreq - 1;      // last request with blk0 <= gb
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (reqs[mid].blk0 <= gb) lo = mid; else hi = mid - 1;
    }
    const FinalArgs f = load_final_args(reqs + lo);
    finalize_block<NPART>(f, (int)(gb - reqs[lo].blk0), sh);
}


// Block (r, chunk): predict chunk of request r's cluster (when flagged) and
// clear the same chunk of its n_i neighbour counts.
__device__ __forceinline__ float predict_one(const PredictArgs& a, int64_t k);
__device__ __forceinline__ void store_tile_max(const PredictArgs& a, int64_t k, float v);
__device__ __forceinline__ void predict_loc_slot(const PredictArgs& a, int64_t k);

__global__ void __launch_bounds__(256) serve_prepare_kernel(BatchArgs b) {
    const ReqDesc* d = b.reqs + blockIdx.x;
    const int ni = d->rg.ni;
    const int64_t base = (int64_t)blockIdx.y * PREPARE_CHUNK;
    for (int64_t e = base + threadIdx.x; e < base + PREPARE_CHUNK; e += blockDim.x) {
        if (e < ni) d->rg.cnt[e] = 0;
        if (d->do_predict) {  // uniform across the workgroup
            // the records by index (in the local mode: the float-float ones,
            // its i-side) with their tiles' candidate bounds ...
            const float v = e < d->pred.n ? predict_one(d->pred, e) : 0.0f;
            store_tile_max(d->pred, e, v);
            if (d->pred.loc) {  // ... and the local stream by slot
                PredictArgs q = d->pred;
                q.ff = nullptr;
                predict_loc_slot(q, e);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Prediction of every j-particle to the block time (FP64 Horner form of the
// cubic Taylor series), and the j-records of each requested mode.
// ---------------------------------------------------------------------------
// Prediction of particle k to a.tb (FP64; non-finite results are flagged in
// the status word): position xp, velocity vp, the FP32 velocity vf and mass
// m of its records, and vabs, an upper bound of |vf| (rounded up by 2^-20).
struct Predicted {
    double xp[3], vp[3];
    float vf[3], m, vabs;
};
__device__ __forceinline__ Predicted predict_particle(const PredictArgs& a, const int64_t k) {
    const StateRec& s = a.st[k];
    const double dt = a.tb - s.t;
    const double h = 0.5 * dt, t3 = dt * (1.0 / 3.0);
    Predicted P;
    bool finite = isfinite(dt);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        predict_coord(dt, h, t3, s.x[c], s.v[c], s.a[c], s.jk[c], P.xp[c], P.vp[c]);
        finite = finite && isfinite(P.xp[c]) && isfinite(P.vp[c]);
    }
    if (!finite) atomicOr(a.status, (unsigned)ST_NONFINITE);
    P.m = (float)s.m;
#pragma unroll
    for (int c = 0; c < 3; ++c) P.vf[c] = (float)P.vp[c];
    P.vabs = (float)(sqrt((double)P.vf[0] * P.vf[0] + (double)P.vf[1] * P.vf[1] +
                          (double)P.vf[2] * P.vf[2]) * (1.0 + 0x1p-20));
    return P;
}

__device__ __forceinline__ RecF64 f64_record(const Predicted& P) {
    RecF64 r;
    r.x = P.xp[0]; r.y = P.xp[1]; r.z = P.xp[2];
    r.vx = P.vf[0]; r.vy = P.vf[1]; r.vz = P.vf[2]; r.m = P.m;
    r.vabs = P.vabs; r.pad = 0.0f;
    return r;
}

__device__ __forceinline__ RecFF ff_record(const Predicted& P) {
    RecFF r;
    r.xh = (float)P.xp[0]; r.xl = (float)(P.xp[0] - (double)r.xh);
    r.yh = (float)P.xp[1]; r.yl = (float)(P.xp[1] - (double)r.yh);
    r.zh = (float)P.xp[2]; r.zl = (float)(P.xp[2] - (double)r.zh);
    r.m = P.m; r.vabs = P.vabs;
    r.vx = P.vf[0]; r.vy = P.vf[1]; r.vz = P.vf[2]; r.pad = 0.0f;
    return r;
}

// Predicts particle k, writes its record of each requested mode in index
// order, and returns its vabs.
__device__ __forceinline__ float predict_one(const PredictArgs& a, const int64_t k) {
    const Predicted P = predict_particle(a, k);
    if (a.ff) a.ff[k] = ff_record(P);
    if (a.f64) a.f64[k] = f64_record(P);
    if (a.f32) {
        RecF32 r;
        r.x = (float)P.xp[0]; r.y = (float)P.xp[1]; r.z = (float)P.xp[2]; r.m = P.m;
        r.vx = P.vf[0]; r.vy = P.vf[1]; r.vz = P.vf[2]; r.vabs = P.vabs;
        a.f32[k] = r;
    }
    return P.vabs;
}

// Largest vabs of the VTILE consecutive particles k0 .. k0 + VTILE - 1 held by
// lanes that are VTILE-aligned within the wavefront (v = 0 for particles past
// the end), stored by the first of those lanes.
__device__ __forceinline__ void store_tile_max(const PredictArgs& a, const int64_t k, float v) {
#pragma unroll
    for (int d = VTILE / 2; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, VTILE));
    if (k < a.n && (k % VTILE) == 0) a.tmax[k / VTILE] = v;
}

__global__ void __launch_bounds__(256) predict_kernel(PredictArgs a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float v = k < a.n ? predict_one(a, k) : 0.0f;
    store_tile_max(a, k, v);
}

// Slot k of the local-coordinate stream, by every lane of a VTILE-aligned
// group of lanes holding slots k0 .. k0 + VTILE - 1 (lanes past the end take
// part with empty values): predicts particle perm[k] (and writes its
// float-float record by particle index when a.ff is set; the library writes
// those in an index pass, with their tiles' candidate bounds); then the
// tile's centre -- the midpoint of the bounding box of its predicted
// positions, in FP64 -- and largest vabs go to org[k0 / VTILE], and the
// slot's record holds the FP32 rounding of the offset from that centre.
__device__ __forceinline__ void predict_loc_slot(const PredictArgs& a, const int64_t k) {
    const bool live = k < a.n;
    Predicted P{};
    int p = 0;
    if (live) {
        p = a.perm[k];
        P = predict_particle(a, p);
        if (a.ff) a.ff[p] = ff_record(P);
    }
    double lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c] = live ? P.xp[c] : __builtin_inf();
        hi[c] = live ? P.xp[c] : -__builtin_inf();
    }
    float vmax = live ? P.vabs : 0.0f;
#pragma unroll
    for (int d = VTILE / 2; d > 0; d >>= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], __shfl_xor(lo[c], d, VTILE));
            hi[c] = fmax(hi[c], __shfl_xor(hi[c], d, VTILE));
        }
        vmax = fmaxf(vmax, __shfl_xor(vmax, d, VTILE));
    }
    double o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) o[c] = 0.5 * (lo[c] + hi[c]);
    if (!live) return;
    RecLoc r;
    r.ex = (float)(P.xp[0] - o[0]);
    r.ey = (float)(P.xp[1] - o[1]);
    r.ez = (float)(P.xp[2] - o[2]);
    r.m = P.m;
    r.vx = P.vf[0]; r.vy = P.vf[1]; r.vz = P.vf[2];
    r.p = p;
    a.loc[k] = r;
    if ((k % VTILE) == 0) {
        TileOrg t;
        t.x = o[0]; t.y = o[1]; t.z = o[2];
        t.vmax = vmax; t.pad = 0.0f;
        a.org[k / VTILE] = t;
    }
}

__global__ void __launch_bounds__(256) predict_loc_kernel(PredictArgs a) {
    predict_loc_slot(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Load or subset update of the stored state: entry e (structure-of-arrays
// sources) becomes the record of particle idx[e], or of particle e for a full
// load.  An index outside the cluster is skipped and flagged in the status
// word.
__global__ void __launch_bounds__(256) scatter_kernel(ScatterArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    const int64_t k = a.idx ? a.idx[e] : e;
    if (k < 0 || k >= a.limit) {
        atomicOr(a.status, (unsigned)ST_BAD_INDEX);
        return;
    }
    StateRec r;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        r.x[c] = a.x[3 * e + c];
        r.v[c] = a.v[3 * e + c];
        r.a[c] = a.a[3 * e + c];
        r.jk[c] = a.jk[3 * e + c];
    }
    r.m = a.m[e];
    r.t = a.t[e];
    r.pad[0] = r.pad[1] = 0.0;
    a.dst[k] = r;
}

__device__ __forceinline__ void unpack_one(const RecFF& r, double* x, double* v) {
    x[0] = (double)r.xh + (double)r.xl;
    x[1] = (double)r.yh + (double)r.yl;
    x[2] = (double)r.zh + (double)r.zl;
    v[0] = r.vx; v[1] = r.vy; v[2] = r.vz;
}
__device__ __forceinline__ void unpack_one(const RecF64& r, double* x, double* v) {
    x[0] = r.x; x[1] = r.y; x[2] = r.z;
    v[0] = r.vx; v[1] = r.vy; v[2] = r.vz;
}
__device__ __forceinline__ void unpack_one(const RecF32& r, double* x, double* v) {
    x[0] = r.x; x[1] = r.y; x[2] = r.z;
    v[0] = r.vx; v[1] = r.vy; v[2] = r.vz;
}

template <typename Rec>
__global__ void __launch_bounds__(256) unpack_kernel(const Rec* rec, int64_t n, double* x,
                                                     double* v) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    unpack_one(rec[k], x + 3 * k, v + 3 * k);
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0u;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int MODE, int IPL, int NP>
static hipError_t launch_regf_t(int wpb, const RegfArgs& a, hipStream_t st) {
    if (a.jl_shift < 0 || a.jl_shift > 6 || (a.jl_shift > 0 && IPL != 1))
        return hipErrorInvalidValue;
    const int gsize = regf_group_size(IPL, a.jl_shift);
    const int groups = (a.ni + gsize - 1) / gsize;
    const int gblocks = (groups + wpb - 1) / wpb;
    const long long blocks = (long long)gblocks * a.nslices;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (a.jl_shift > 0) {
        const size_t stage =
            MODE != MODE_LOC && lanes_staged(a.jl_shift, wpb) ? lanes_stage_bytes<MODE>() : 0;
        hipLaunchKernelGGL((regf_lanes_kernel<MODE, NP>), dim3((unsigned)blocks), dim3(64 * wpb),
                           run_lds_bytes(wpb) + stage, st, a, gblocks);
    }
    else
        hipLaunchKernelGGL((regf_kernel<MODE, IPL, NP>), dim3((unsigned)blocks), dim3(64 * wpb),
                           run_lds_bytes(wpb), st, a, gblocks);
    return hipGetLastError();
}

hipError_t launch_regf(int mode, int ipl, int wpb, bool pot, const RegfArgs& a,
                       hipStream_t s) {
    if (wpb < 1 || wpb > 4) return hipErrorInvalidValue;
    switch ((mode * 4 + ipl) * 2 + (pot ? 1 : 0)) {
#define NB6_REGF_CASE(M, I)                                                                   \
        case (M * 4 + I) * 2: return launch_regf_t<M, I, NPART>(wpb, a, s);                  \
        case (M * 4 + I) * 2 + 1: return launch_regf_t<M, I, NPART_POT>(wpb, a, s);
        NB6_REGF_CASE(MODE_FF, 1)
        NB6_REGF_CASE(MODE_FF, 2)
        NB6_REGF_CASE(MODE_F64, 1)
        NB6_REGF_CASE(MODE_F64, 2)
        NB6_REGF_CASE(MODE_F32, 1)
        NB6_REGF_CASE(MODE_F32, 2)
        NB6_REGF_CASE(MODE_LOC, 1)
        NB6_REGF_CASE(MODE_LOC, 2)
#undef NB6_REGF_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
    if (a.ni <= 0) return hipSuccess;
    if (a.caps > MAX_CAPS) return hipErrorInvalidValue;
    const dim3 grid((unsigned)final_blocks(a.ni, a.pot ? NPART_POT : NPART)), block(256);
    if (a.pot)
        hipLaunchKernelGGL(finalize_kernel<NPART_POT>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(finalize_kernel<NPART>, grid, block, 0, s, a);
    return hipGetLastError();
}


hipError_t launch_predict(const PredictArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.n + 255) / 256));
    hipLaunchKernelGGL(predict_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_predict_loc(const PredictArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    if (!a.loc || !a.org || !a.perm) return hipErrorInvalidValue;
    dim3 grid((unsigned)((a.n + 255) / 256));
    hipLaunchKernelGGL(predict_loc_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.n + 255) / 256));
    hipLaunchKernelGGL(scatter_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_unpack(int mode, const void* rec, int64_t n, double* x, double* v,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256));
    switch (mode) {
        case MODE_FF:
            hipLaunchKernelGGL(unpack_kernel<RecFF>, grid, dim3(256), 0, s, (const RecFF*)rec, n, x, v);
            break;
        case MODE_F64:
            hipLaunchKernelGGL(unpack_kernel<RecF64>, grid, dim3(256), 0, s, (const RecF64*)rec, n, x, v);
            break;
        case MODE_F32:
            hipLaunchKernelGGL(unpack_kernel<RecF32>, grid, dim3(256), 0, s, (const RecF32*)rec, n, x, v);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE>
static const void* serve_regf_fn_mode(int cls) {
    switch (cls) {
        case SERVE_ONE_I: return (const void*)serve_regf_kernel<MODE, SERVE_ONE_I>;
        case SERVE_LANES: return (const void*)serve_regf_kernel<MODE, SERVE_LANES>;
        case SERVE_TWO_I: return (const void*)serve_regf_kernel<MODE, SERVE_TWO_I>;
        default: return nullptr;
    }
}

static const void* serve_regf_fn(int mode, int cls) {
    switch (mode) {
        case MODE_FF: return serve_regf_fn_mode<MODE_FF>(cls);
        case MODE_F64: return serve_regf_fn_mode<MODE_F64>(cls);
        case MODE_F32: return serve_regf_fn_mode<MODE_F32>(cls);
        case MODE_LOC: return serve_regf_fn_mode<MODE_LOC>(cls);
        default: return nullptr;
    }
}

hipError_t serve_regf_blocks_per_cu(int mode, int cls, int* blocks) {
    const void* fn = serve_regf_fn(mode, cls);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, 256, 0);
}

hipError_t launch_serve_regf(int mode, int cls, const BatchArgs& b, int blocks,
                             hipStream_t s) {
    if (b.nitems <= 0) return hipSuccess;
    const void* fn = serve_regf_fn(mode, cls);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {const_cast<BatchArgs*>(&b)};
    return hipLaunchKernel(fn, dim3(blocks), dim3(256), args, 0, s);
}

hipError_t launch_serve_finalize(const BatchArgs& b, hipStream_t s) {
    if (b.nblk_total <= 0) return hipSuccess;
    const dim3 grid((unsigned)b.nblk_total), block(256);
    hipLaunchKernelGGL(serve_finalize_kernel, grid, block, 0, s, b);
    return hipGetLastError();
}


hipError_t launch_serve_prepare(const BatchArgs& b, int chunks, hipStream_t s) {
    if (b.nreq <= 0 || chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(serve_prepare_kernel, dim3(b.nreq, chunks), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace nb6
