// nb6_irr.hip -- gfx950 kernels of the irregular force (section 3.3 step 4)
// over the neighbour lists the library stores per particle (the
// irregular-force library of section 3.5 keeps each particle's list between
// regular steps and predicts the particles it needs itself).
//
//   irregular_kernel   one wavefront per active particle i: the lanes take
//                      the entries of i's list in turn, predict each j from
//                      the stored FP64 state to the block time, add its
//                      terms in FP64, and a butterfly over the wavefront
//                      gives the sums.
//   set_lists_kernel   one wavefront per replaced list: copy, validate.
//   copy_rows_kernel   re-lay the stored lists when their rows grow.
//   pack_rows_kernel   pack the used part of each list row into one array,
//   unpack_rows_kernel and back (host-array calls move only that over PCIe).
//
// The work per pair is one gather of a 128-byte state record and ~60
// FP64 operations, so the kernel is bound by the latency and bandwidth of
// the gathers, not by arithmetic: it computes in FP64 throughout (FP64 runs
// at the FP32 fma rate on this chip), which makes its result independent of
// how the lists were ordered up to FP64 rounding and keeps the difference
// between old-list and new-list forces of one particle exact to that level.
#include "nb6_internal.h"

// Every fma is explicit, as in the other kernels.
#pragma clang fp contract(off)

namespace nb6 {

// Predicted position and velocity of particle k at time tb.
// Predicted position and velocity of particle k at time tb, and its mass.
__device__ __forceinline__ double predict_particle(const IrrArgs& a, const int64_t k,
                                                   double xp[3], double vp[3]) {
    const StateRec s = a.st[k];  // one 128-byte record
    const double dt = a.tb - s.t;
    const double h = 0.5 * dt, t3 = dt * (1.0 / 3.0);
#pragma unroll
    for (int c = 0; c < 3; ++c) predict_coord(dt, h, t3, s.x[c], s.v[c], s.a[c], s.jk[c], xp[c], vp[c]);
    return s.m;
}

__global__ void __launch_bounds__(256) irregular_kernel(IrrArgs a) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);  // one wavefront per active i
    if (q >= a.ni) return;                               // uniform across the wave
    const int32_t i = a.idx[q];
    if (i < 0 || i >= a.n) {
        if (lane == 0) {
            atomicOr(a.status, (unsigned)ST_BAD_INDEX);
            const double nan = __builtin_nan("");
            for (int c = 0; c < 3; ++c) a.acc[3 * q + c] = a.jerk[3 * q + c] = nan;
            if (a.pot) a.pot[q] = nan;
        }
        return;
    }
    // the first row entry of each lane is loaded before the count is known
    // (the row holds lcap entries), so the count, the row and the i record
    // arrive in one memory round trip
    const int32_t* row = a.nbl + (size_t)i * a.lcap;
    const int32_t first = lane < a.lcap ? row[lane] : 0;
    const int cnt = a.nbc[i];
    double xi[3], vi[3];
    (void)predict_particle(a, i, xi, vi);

    double s[7];  // acc, jerk, sum of m / r
#pragma unroll
    for (int c = 0; c < 7; ++c) s[c] = 0.0;
    bool bad = false;
    for (int e = lane; e < cnt; e += 64) {
        const int32_t j = e < 64 ? first : row[e];
        if (j == i) continue;  // no self-term
        if (j < 0 || j >= a.n) {
            bad = true;
            continue;
        }
        double xj[3], vj[3];
        const double mj = predict_particle(a, j, xj, vj);
        const double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
        const double dvx = vj[0] - vi[0], dvy = vj[1] - vi[1], dvz = vj[2] - vi[2];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double rv = fma(dz, dvz, fma(dy, dvy, dx * dvx));
        const double rinv = 1.0 / sqrt(r2);
        const double rinv2 = rinv * rinv;
        const double mr = mj * rinv;
        const double mr3 = mr * rinv2;
        s[6] += mr;
        const double alpha = (-3.0 * rv) * rinv2;
        s[0] = fma(mr3, dx, s[0]);
        s[1] = fma(mr3, dy, s[1]);
        s[2] = fma(mr3, dz, s[2]);
        s[3] = fma(mr3, fma(alpha, dx, dvx), s[3]);
        s[4] = fma(mr3, fma(alpha, dy, dvy), s[4]);
        s[5] = fma(mr3, fma(alpha, dz, dvz), s[5]);
    }
    // butterfly over the wavefront: every lane ends with the same bits
    for (int d = 32; d > 0; d >>= 1)
#pragma unroll
        for (int c = 0; c < 7; ++c) s[c] += __shfl_xor(s[c], d);
    const bool any_bad = __ballot(bad) != 0;
    if (lane == 0) {
        if (any_bad) atomicOr(a.status, (unsigned)ST_BAD_LIST);
        for (int c = 0; c < 3; ++c) {
            a.acc[3 * q + c] = s[c];
            a.jerk[3 * q + c] = s[3 + c];
        }
        if (a.pot) a.pot[q] = -s[6];
    }
}

__global__ void __launch_bounds__(256) set_lists_kernel(SetListArgs a) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);  // one wavefront per list
    if (k >= a.ni) return;
    const int32_t p = a.idx[k];
    if (p < 0 || p >= a.n) {
        if (lane == 0) atomicOr(a.status, (unsigned)ST_BAD_INDEX);
        return;
    }
    const int cnt = a.nnb[k];
    const bool bad_count = cnt < 0 || cnt > a.cap;
    const int c = bad_count ? 0 : cnt;
    bool bad = false;
    for (int e = lane; e < c; e += 64) {
        const int32_t v = a.list[(size_t)k * a.cap + e];
        bad = bad || v < 0 || v >= a.n;
        a.nbl[(size_t)p * a.lcap + e] = v;
    }
    const bool any_bad = bad_count || __ballot(bad) != 0;
    if (lane == 0) {
        a.nbc[p] = any_bad ? 0 : c;  // an invalid list is stored empty
        if (any_bad) atomicOr(a.status, (unsigned)ST_BAD_LIST);
    }
}

__global__ void __launch_bounds__(256) copy_rows_kernel(const int32_t* src, int src_cap,
                                                       int32_t* dst, int dst_cap,
                                                       const int32_t* cnt, int64_t n) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = g / src_cap;
    const int e = (int)(g % src_cap);
    if (p >= n) return;
    if (e < cnt[p]) dst[p * dst_cap + e] = src[p * src_cap + e];
}

// One wavefront per row.
__global__ void __launch_bounds__(256) pack_rows_kernel(const int32_t* list, int cap,
                                                       const int64_t* off, int64_t n,
                                                       int32_t* out) {
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= n) return;
    const int64_t o = off[q];
    const int cnt = (int)(off[q + 1] - o);
    const int32_t* row = list + q * cap;
    for (int e = threadIdx.x & 63; e < cnt; e += 64) out[o + e] = row[e];
}

__global__ void __launch_bounds__(256) unpack_rows_kernel(const int32_t* packed,
                                                         const int64_t* off, int64_t n,
                                                         int32_t* list, int cap) {
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= n) return;
    const int64_t o = off[q];
    const int cnt = (int)(off[q + 1] - o);
    int32_t* row = list + q * cap;
    for (int e = threadIdx.x & 63; e < cnt; e += 64) row[e] = packed[o + e];
}

hipError_t launch_irregular(const IrrArgs& a, hipStream_t s) {
    if (a.ni <= 0) return hipSuccess;
    hipLaunchKernelGGL(irregular_kernel, dim3((unsigned)((a.ni + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_set_lists(const SetListArgs& a, hipStream_t s) {
    if (a.ni <= 0) return hipSuccess;
    if (a.cap > a.lcap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(set_lists_kernel, dim3((unsigned)((a.ni + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy_rows(const int32_t* src, int src_cap, int32_t* dst, int dst_cap,
                            const int32_t* cnt, int64_t n, hipStream_t s) {
    if (n <= 0 || src_cap <= 0) return hipSuccess;
    if (dst_cap < src_cap) return hipErrorInvalidValue;
    const int64_t total = n * src_cap;
    hipLaunchKernelGGL(copy_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       src, src_cap, dst, dst_cap, cnt, n);
    return hipGetLastError();
}

hipError_t launch_pack_rows(const int32_t* list, int cap, const int64_t* off, int64_t n,
                            int32_t* out, hipStream_t s) {
    if (n <= 0 || cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_rows_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, list, cap,
                       off, n, out);
    return hipGetLastError();
}

hipError_t launch_unpack_rows(const int32_t* packed, const int64_t* off, int64_t n,
                              int32_t* list, int cap, hipStream_t s) {
    if (n <= 0 || cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(unpack_rows_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, packed,
                       off, n, list, cap);
    return hipGetLastError();
}

}  // namespace nb6
