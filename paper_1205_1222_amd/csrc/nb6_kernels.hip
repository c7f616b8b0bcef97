// nb6_kernels.hip -- gfx950 kernels of the regular-force path.
//
//   predict_kernel   cubic Taylor prediction of every j-particle to the block
//                    time in FP64, writing the j-records the force kernel
//                    reads (section 3.3 step 3).
//   regf_kernel      regular force, jerk and neighbour appends for one
//                    (i-group, j-slice) pair (section 3.3 step 6 with the
//                    velocity criterion of section 3.2).
//   finalize_*       fixed-order reduction of the j-slice partial sums and
//                    gathering of the per-slice neighbour lists into one
//                    ascending list per i (the reduction and list-gathering
//                    kernels of section 3.4).
//
// Design (see the repository's design notes for the derivation):
//   * i-particles live in VGPRs, IPL of them per lane.
//   * Every lane of a wavefront reads the same j-record, so the record is
//     fetched with scalar loads into SGPRs and used directly as an operand
//     of the vector instructions: no LDS traffic and no VGPRs spent on j.
//   * The neighbour test and the force use FP32; the coordinate difference
//     is formed from float-float, FP64 or FP32 coordinates.
//   * Force terms are summed in FP32 over tiles of TILE j-particles and each
//     tile sum is added into an FP64 accumulator (FP64 adds run at the full
//     vector rate on CDNA), so the rounding error is that of a TILE-term
//     FP32 sum and does not grow with N.
//   * A neighbour is appended to the lane's own list for this slice; slices
//     are visited in ascending j, so the gathered list is already sorted.
#include "nb6_internal.h"

#include <float.h>

namespace nb6 {

constexpr int TILE = 32;    // j per FP32 tile before the FP64 fold

template <int MODE> struct RecOf;
template <> struct RecOf<MODE_FF>  { using T = RecFF; };
template <> struct RecOf<MODE_F64> { using T = RecF64; };
template <> struct RecOf<MODE_F32> { using T = RecF32; };

template <int MODE> struct IPos;
template <> struct IPos<MODE_FF>  { float xh, yh, zh, xl, yl, zl; };
template <> struct IPos<MODE_F64> { double x, y, z; };
template <> struct IPos<MODE_F32> { float x, y, z; };

struct IAux { float vx, vy, vz, h2, dtr; };

__device__ __forceinline__ void get_ipos(const RecFF& r, IPos<MODE_FF>& p, IAux& v) {
    p.xh = r.xh; p.yh = r.yh; p.zh = r.zh;
    p.xl = r.xl; p.yl = r.yl; p.zl = r.zl;
    v.vx = r.vx; v.vy = r.vy; v.vz = r.vz;
}
__device__ __forceinline__ void get_ipos(const RecF64& r, IPos<MODE_F64>& p, IAux& v) {
    p.x = r.x; p.y = r.y; p.z = r.z;
    v.vx = r.vx; v.vy = r.vy; v.vz = r.vz;
}
__device__ __forceinline__ void get_ipos(const RecF32& r, IPos<MODE_F32>& p, IAux& v) {
    p.x = r.x; p.y = r.y; p.z = r.z;
    v.vx = r.vx; v.vy = r.vy; v.vz = r.vz;
}

// R_j - R_i in FP32 from each coordinate representation.
__device__ __forceinline__ void coord_diff(const RecFF& j, const IPos<MODE_FF>& i,
                                           float& dx, float& dy, float& dz) {
    dx = (j.xh - i.xh) + (j.xl - i.xl);
    dy = (j.yh - i.yh) + (j.yl - i.yl);
    dz = (j.zh - i.zh) + (j.zl - i.zl);
}
__device__ __forceinline__ void coord_diff(const RecF64& j, const IPos<MODE_F64>& i,
                                           float& dx, float& dy, float& dz) {
    dx = (float)(j.x - i.x);
    dy = (float)(j.y - i.y);
    dz = (float)(j.z - i.z);
}
__device__ __forceinline__ void coord_diff(const RecF32& j, const IPos<MODE_F32>& i,
                                           float& dx, float& dy, float& dz) {
    dx = j.x - i.x;
    dy = j.y - i.y;
    dz = j.z - i.z;
}

// One i-j interaction.  run[0..2] += m r^-3 R, run[3..5] += m r^-3 (V + alpha R)
// with alpha = -3 (R.V)/r^2, unless j is a neighbour of i, in which case j is
// appended to the lane's list instead.
template <int MODE>
__device__ __forceinline__ void interact(const typename RecOf<MODE>::T& r, int j,
                                         const IPos<MODE>& ip, const IAux& ia,
                                         float run[6], int& count,
                                         int32_t* __restrict__ lb, int caps) {
    float dx, dy, dz;
    coord_diff(r, ip, dx, dy, dz);
    const float dvx = r.vx - ia.vx;
    const float dvy = r.vy - ia.vy;
    const float dvz = r.vz - ia.vz;
    const float px = fmaf(ia.dtr, dvx, dx);
    const float py = fmaf(ia.dtr, dvy, dy);
    const float pz = fmaf(ia.dtr, dvz, dz);
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float p2 = fmaf(pz, pz, fmaf(py, py, px * px));
    const float rv = fmaf(dz, dvz, fmaf(dy, dvy, dx * dvx));
    float rinv = __builtin_amdgcn_rsqf(r2);
    const bool nb = fminf(r2, p2) < ia.h2;
    if (nb) {
        if (count < caps) lb[count] = j;
        ++count;
    }
    rinv = nb ? 0.0f : rinv;
    const float rinv2 = rinv * rinv;
    const float mr3 = (r.m * rinv) * rinv2;
    const float alpha = (-3.0f * rv) * rinv2;
    run[0] = fmaf(mr3, dx, run[0]);
    run[1] = fmaf(mr3, dy, run[1]);
    run[2] = fmaf(mr3, dz, run[2]);
    run[3] = fmaf(mr3, fmaf(alpha, dx, dvx), run[3]);
    run[4] = fmaf(mr3, fmaf(alpha, dy, dvy), run[4]);
    run[5] = fmaf(mr3, fmaf(alpha, dz, dvz), run[5]);
}

// The j-records are not written while the force kernel runs, so they are
// read through the constant address space: a wave-uniform address then
// becomes a scalar load into SGPRs.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T*;

__device__ __forceinline__ RecFF load_rec(const_ptr<RecFF> p) {
    RecFF r;
    r.xh = p->xh; r.yh = p->yh; r.zh = p->zh; r.m = p->m;
    r.xl = p->xl; r.yl = p->yl; r.zl = p->zl; r.pad0 = 0.0f;
    r.vx = p->vx; r.vy = p->vy; r.vz = p->vz; r.pad1 = 0.0f;
    return r;
}
__device__ __forceinline__ RecF64 load_rec(const_ptr<RecF64> p) {
    RecF64 r;
    r.x = p->x; r.y = p->y; r.z = p->z;
    r.vx = p->vx; r.vy = p->vy; r.vz = p->vz; r.m = p->m; r.pad = 0.0;
    return r;
}
__device__ __forceinline__ RecF32 load_rec(const_ptr<RecF32> p) {
    RecF32 r;
    r.x = p->x; r.y = p->y; r.z = p->z; r.m = p->m;
    r.vx = p->vx; r.vy = p->vy; r.vz = p->vz; r.pad = 0.0f;
    return r;
}

template <int MODE, int IPL>
__global__ void __launch_bounds__(256) regf_kernel(RegfArgs a) {
    using Rec = typename RecOf<MODE>::T;
    const_ptr<Rec> rec = (const_ptr<Rec>)(a.rec);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int group = blockIdx.x * wpb + wave;
    const int s = blockIdx.y;
    const int ibase = group * 64 * IPL;
    if (ibase >= a.ni) return;  // uniform across the wave

    IPos<MODE> ip[IPL];
    IAux ia[IPL];
    int q[IPL];
    bool live[IPL];
    int32_t* lb[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        q[k] = ibase + k * 64 + lane;
        live[k] = q[k] < a.ni;
        int pi = live[k] ? a.idx[q[k]] : 0;
        float h2f = live[k] ? (float)a.h2[q[k]] : -1.0f;
        float dtf = live[k] ? (float)a.dtr[q[k]] : 0.0f;
        if (live[k]) {
            unsigned bad = 0;
            if (pi < 0 || pi >= a.n) bad |= ST_BAD_INDEX;
            if (!(h2f >= FLT_MIN) || !(h2f <= FLT_MAX)) bad |= ST_BAD_H2;
            if (bad) {
                if (s == 0) atomicOr(a.status, bad);
                pi = 0;
                h2f = -1.0f;   // never a neighbour: this lane appends nothing
                live[k] = false;
            }
        }
        const Rec* rv = static_cast<const Rec*>(a.rec);  // per-lane address
        get_ipos(rv[pi], ip[k], ia[k]);
        ia[k].h2 = h2f;
        ia[k].dtr = dtf;
        lb[k] = a.lst + ((size_t)s * a.ni + (live[k] ? q[k] : 0)) * (size_t)a.caps;
    }

    const int j0 = s * a.slice_len;
    const int j1 = min(j0 + a.slice_len, a.n);

    double sum[IPL][6];
    int count[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        count[k] = 0;
#pragma unroll
        for (int c = 0; c < 6; ++c) sum[k][c] = 0.0;
    }

    for (int jt = j0; jt < j1; jt += TILE) {
        const int je = min(jt + TILE, j1);
        float run[IPL][6];
#pragma unroll
        for (int k = 0; k < IPL; ++k)
#pragma unroll
            for (int c = 0; c < 6; ++c) run[k][c] = 0.0f;

#pragma unroll 4
        for (int j = jt; j < je; ++j) {
            const Rec r = load_rec(rec + j);
#pragma unroll
            for (int k = 0; k < IPL; ++k)
                interact<MODE>(r, j, ip[k], ia[k], run[k], count[k], lb[k], a.caps);
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k)
#pragma unroll
            for (int c = 0; c < 6; ++c) sum[k][c] += (double)run[k][c];
    }

#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        if (q[k] < a.ni) {
            double* p = a.part + (size_t)s * NPART * a.ni + q[k];
#pragma unroll
            for (int c = 0; c < NPART; ++c) p[(size_t)c * a.ni] = sum[k][c];
            a.cnt[(size_t)s * a.ni + q[k]] = live[k] ? count[k] : 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Finalize: one thread per i (few slices; partial loads are coalesced).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool bad_i(const FinalArgs& a, int q, int32_t self) {
    float h2f = (float)a.h2[q];
    return self < 0 || self >= a.n || !(h2f >= FLT_MIN) || !(h2f <= FLT_MAX);
}

__device__ __forceinline__ void write_bad(const FinalArgs& a, int q) {
    const double nan = __builtin_nan("");
    for (int c = 0; c < 3; ++c) { a.acc[3 * q + c] = nan; a.jerk[3 * q + c] = nan; }
    a.nnb[q] = -1;
}

__global__ void __launch_bounds__(256) finalize_thread_kernel(FinalArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.ni) return;
    const int32_t self = a.idx[q];
    if (bad_i(a, q, self)) { write_bad(a, q); return; }

    double sum[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sum[c] = 0.0;
    int64_t total = 0;
    int out = 0;
    for (int s = 0; s < a.nslices; ++s) {
        const double* p = a.part + (size_t)s * NPART * a.ni + q;
#pragma unroll
        for (int c = 0; c < NPART; ++c) sum[c] += p[(size_t)c * a.ni];
        const int c_s = a.cnt[(size_t)s * a.ni + q];
        total += c_s;
        const int st = min(c_s, a.caps);
        const int32_t* l = a.lst + ((size_t)s * a.ni + q) * (size_t)a.caps;
        for (int e = 0; e < st && out < a.cap; ++e) {
            const int32_t j = l[e];
            if (j == self) continue;
            a.list[(size_t)q * a.cap + out] = j;
            ++out;
        }
    }
    a.acc[3 * q + 0] = sum[0];
    a.acc[3 * q + 1] = sum[1];
    a.acc[3 * q + 2] = sum[2];
    a.jerk[3 * q + 0] = sum[3];
    a.jerk[3 * q + 1] = sum[4];
    a.jerk[3 * q + 2] = sum[5];
    const int32_t nn = (int32_t)(total - 1);  // the i-particle itself
    a.nnb[q] = nn;
    if (nn > a.cap) atomicOr(a.status, (unsigned)ST_OVERFLOW);
}

// ---------------------------------------------------------------------------
// Finalize: one wavefront per i (many slices, few i).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) finalize_wave_kernel(FinalArgs a) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= a.ni) return;
    const int32_t self = a.idx[q];
    if (bad_i(a, q, self)) {
        if (lane == 0) write_bad(a, q);
        return;
    }

    double sum[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sum[c] = 0.0;
    for (int s = lane; s < a.nslices; s += 64) {
        const double* p = a.part + (size_t)s * NPART * a.ni + q;
#pragma unroll
        for (int c = 0; c < NPART; ++c) sum[c] += p[(size_t)c * a.ni];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) sum[c] += __shfl_xor(sum[c], off);

    int64_t total = 0;
    int running = 0;  // stored entries of all earlier slices
    for (int s0 = 0; s0 < a.nslices; s0 += 64) {
        const int s = s0 + lane;
        const int c_s = (s < a.nslices) ? a.cnt[(size_t)s * a.ni + q] : 0;
        total += c_s;
        const int st = min(c_s, a.caps);
        int incl = st;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        const int excl = running + incl - st;
        running += __shfl(incl, 63);
        unsigned long long mask = __ballot(st > 0 && excl <= a.cap);
        while (mask) {
            const int l = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            const int sl = s0 + l;
            const int ne = __shfl(st, l);
            const int base = __shfl(excl, l);
            const int32_t* lst = a.lst + ((size_t)sl * a.ni + q) * (size_t)a.caps;
            for (int e = lane; e < ne; e += 64) {
                const int32_t j = lst[e];
                if (j == self) continue;
                const int pos = base + e - (j > self ? 1 : 0);
                if (pos >= 0 && pos < a.cap) a.list[(size_t)q * a.cap + pos] = j;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off);

    if (lane == 0) {
        a.acc[3 * q + 0] = sum[0];
        a.acc[3 * q + 1] = sum[1];
        a.acc[3 * q + 2] = sum[2];
        a.jerk[3 * q + 0] = sum[3];
        a.jerk[3 * q + 1] = sum[4];
        a.jerk[3 * q + 2] = sum[5];
        const int32_t nn = (int32_t)(total - 1);
        a.nnb[q] = nn;
        if (nn > a.cap) atomicOr(a.status, (unsigned)ST_OVERFLOW);
    }
}

// ---------------------------------------------------------------------------
// Prediction of every j-particle to the block time (FP64 Horner form of the
// cubic Taylor series), and the j-records of each requested mode.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) predict_kernel(PredictArgs a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const double dt = a.tb - a.t[k];
    const double h = 0.5 * dt, t3 = dt * (1.0 / 3.0);
    double xp[3], vp[3];
    bool finite = isfinite(dt);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double x = a.x[3 * k + c], v = a.v[3 * k + c];
        const double acc = a.a[3 * k + c], jk = a.jk[3 * k + c];
        xp[c] = x + dt * (v + h * (acc + t3 * jk));
        vp[c] = v + dt * (acc + h * jk);
        finite = finite && isfinite(xp[c]) && isfinite(vp[c]);
    }
    const float m = (float)a.m[k];
    if (!finite) atomicOr(a.status, (unsigned)ST_NONFINITE);
    if (a.ff) {
        RecFF r;
        r.xh = (float)xp[0]; r.xl = (float)(xp[0] - (double)r.xh);
        r.yh = (float)xp[1]; r.yl = (float)(xp[1] - (double)r.yh);
        r.zh = (float)xp[2]; r.zl = (float)(xp[2] - (double)r.zh);
        r.m = m; r.pad0 = 0.0f;
        r.vx = (float)vp[0]; r.vy = (float)vp[1]; r.vz = (float)vp[2]; r.pad1 = 0.0f;
        a.ff[k] = r;
    }
    if (a.f64) {
        RecF64 r;
        r.x = xp[0]; r.y = xp[1]; r.z = xp[2];
        r.vx = (float)vp[0]; r.vy = (float)vp[1]; r.vz = (float)vp[2]; r.m = m;
        r.pad = 0.0;
        a.f64[k] = r;
    }
    if (a.f32) {
        RecF32 r;
        r.x = (float)xp[0]; r.y = (float)xp[1]; r.z = (float)xp[2]; r.m = m;
        r.vx = (float)vp[0]; r.vy = (float)vp[1]; r.vz = (float)vp[2]; r.pad = 0.0f;
        a.f32[k] = r;
    }
}

// Subset update of the stored state: entry e goes to particle idx[e].  An
// index outside the cluster is skipped and flagged in the status word.
__global__ void __launch_bounds__(256) scatter_kernel(ScatterArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    const int64_t k = a.idx[e];
    if (k < 0 || k >= a.limit) {
        atomicOr(a.status, (unsigned)ST_BAD_INDEX);
        return;
    }
    a.dm[k] = a.m[e];
    a.dt[k] = a.t[e];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a.dx[3 * k + c] = a.x[3 * e + c];
        a.dv[3 * k + c] = a.v[3 * e + c];
        a.da[3 * k + c] = a.a[3 * e + c];
        a.djk[3 * k + c] = a.jk[3 * e + c];
    }
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
template <int MODE, int IPL>
static hipError_t launch_regf_t(int wpb, const RegfArgs& a, hipStream_t st) {
    const int groups = (a.ni + 64 * IPL - 1) / (64 * IPL);
    dim3 grid((groups + wpb - 1) / wpb, a.nslices);
    dim3 block(64 * wpb);
    hipLaunchKernelGGL((regf_kernel<MODE, IPL>), grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_regf(int mode, int ipl, int wpb, const RegfArgs& a, hipStream_t s) {
    if (wpb < 1 || wpb > 4) return hipErrorInvalidValue;
    switch (mode * 4 + ipl) {
        case MODE_FF * 4 + 1:  return launch_regf_t<MODE_FF, 1>(wpb, a, s);
        case MODE_FF * 4 + 2:  return launch_regf_t<MODE_FF, 2>(wpb, a, s);
        case MODE_F64 * 4 + 1: return launch_regf_t<MODE_F64, 1>(wpb, a, s);
        case MODE_F64 * 4 + 2: return launch_regf_t<MODE_F64, 2>(wpb, a, s);
        case MODE_F32 * 4 + 1: return launch_regf_t<MODE_F32, 1>(wpb, a, s);
        case MODE_F32 * 4 + 2: return launch_regf_t<MODE_F32, 2>(wpb, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
    if (a.ni <= 0) return hipSuccess;
    if (a.nslices <= 16) {
        dim3 grid((a.ni + 255) / 256);
        hipLaunchKernelGGL(finalize_thread_kernel, grid, dim3(256), 0, s, a);
    } else {
        dim3 grid((a.ni + 3) / 4);
        hipLaunchKernelGGL(finalize_wave_kernel, grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_predict(const PredictArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.n + 255) / 256));
    hipLaunchKernelGGL(predict_kernel, grid, dim3(256), 0, s, a);
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

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace nb6
