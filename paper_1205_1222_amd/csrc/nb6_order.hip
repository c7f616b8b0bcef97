// nb6_order.hip -- spatial order of a cluster's particles.
//
// The local-coordinate j-stream (NB6_DX_LOCAL) stores every particle's
// position as an FP32 offset from the FP64 centre of its tile of VTILE
// records, and the force kernel forms R_ij as that offset plus the FP32
// rounding of (tile centre - x_i).  The rounding error of a pair is then
// about 2^-24 (|R_ij| + tile extent), so the tiles must be compact: the
// records follow the particles' Morton order (a Z-order curve through a grid
// of 2^16 cells per axis over the cluster's bounding box), not their index
// order.
//
//   bbox kernels    bounding box of the stored positions (non-finite values
//                   skipped) on order-preserving 64-bit words, in two passes;
//   key_kernel      Morton key of every particle (48 bits) and its index;
//   rocPRIM radix sort of (key, index) pairs: perm[slot] = particle, stable,
//                   so equal keys keep ascending index;
//   invert_kernel   inv[particle] = slot.
//
// The order is a function of the stored state it is built from; which state
// that is (the runtime rebuilds it after a full load and after a cluster's
// worth of subset updates) is decided on the host.
//
// launch_iorder: the i-order of an active block, its positions sorted by
// their particles' slots in that order (a counting sort over the n slots:
// counts, an exclusive scan, placement), so that the i-particles of one
// wavefront of the force kernel lie close together and take the candidate
// branch for nearly the same j.  Every i-particle's result is independent of
// where in the launch it is computed, so the i-order changes no bits.
#include "nb6_internal.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

namespace nb6 {

namespace {

constexpr int kKeyBits = 16;  // grid cells per axis: 2^16
constexpr int kBoxBlocks = 256;  // workgroups of the first bounding-box pass
// Scratch head: the box (6 words, padded to 8), then kBoxBlocks partial boxes,
// rounded up to 256 bytes (the keys and the sort's storage follow).
constexpr size_t kHead = ((8 + 6 * kBoxBlocks) * sizeof(unsigned long long) + 255) / 256 * 256;

// Monotone map of a double onto unsigned 64-bit integers: a < b iff
// ord(a) < ord(b) for finite a, b.
__device__ __forceinline__ unsigned long long ord(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord(unsigned long long u) {
    return __longlong_as_double((long long)((u >> 63) ? (u & 0x7fffffffffffffffull) : ~u));
}

// Spread the low 16 bits of v to every third bit.
__device__ __forceinline__ unsigned long long spread3(unsigned long long v) {
    v &= 0xffffull;
    v = (v | (v << 16)) & 0x0000ff0000ffull;
    v = (v | (v << 8)) & 0x00f00f00f00full;
    v = (v | (v << 4)) & 0x0c30c30c30c3ull;
    v = (v | (v << 2)) & 0x249249249249ull;
    return v;
}

// First pass: workgroup b writes the minima and maxima of the finite
// coordinates of its share of the particles, as ord() words, to part[b][6].
__global__ void __launch_bounds__(256) bbox_part_kernel(const StateRec* st, int64_t n,
                                                        unsigned long long* part) {
    __shared__ unsigned long long sh[4][6];
    unsigned long long lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0ull, 0ull, 0ull};
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = st[k].x[c];
            if (isfinite(v)) {
                const unsigned long long o = ord(v);
                lo[c] = min(lo[c], o);
                hi[c] = max(hi[c], o);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        for (int d = 32; d > 0; d >>= 1) {
            lo[c] = min(lo[c], (unsigned long long)__shfl_xor((long long)lo[c], d));
            hi[c] = max(hi[c], (unsigned long long)__shfl_xor((long long)hi[c], d));
        }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sh[w][c] = lo[c];
            sh[w][3 + c] = hi[c];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int c = threadIdx.x;
        unsigned long long v = sh[0][c];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
            v = c < 3 ? min(v, sh[k][c]) : max(v, sh[k][c]);
        part[6 * blockIdx.x + c] = v;
    }
}

// Second pass, one workgroup: box[0..2] = minima, box[3..5] = maxima over the
// nparts partial boxes.
__global__ void __launch_bounds__(256) bbox_final_kernel(const unsigned long long* part,
                                                         int nparts, unsigned long long* box) {
    __shared__ unsigned long long sh[4][6];
    unsigned long long v[6] = {~0ull, ~0ull, ~0ull, 0ull, 0ull, 0ull};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
        for (int c = 0; c < 6; ++c)
            v[c] = c < 3 ? min(v[c], part[6 * b + c]) : max(v[c], part[6 * b + c]);
#pragma unroll
    for (int c = 0; c < 6; ++c)
        for (int d = 32; d > 0; d >>= 1) {
            const unsigned long long o = (unsigned long long)__shfl_xor((long long)v[c], d);
            v[c] = c < 3 ? min(v[c], o) : max(v[c], o);
        }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) sh[w][c] = v[c];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int c = threadIdx.x;
        unsigned long long r = sh[0][c];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
            r = c < 3 ? min(r, sh[k][c]) : max(r, sh[k][c]);
        box[c] = r;
    }
}

// Morton key of particle k on a grid of 2^16 cubic cells spanning the
// largest extent of the box; a non-finite coordinate maps to cell 0.
__global__ void __launch_bounds__(256) key_kernel(const StateRec* st, int64_t n,
                                                  const unsigned long long* box,
                                                  unsigned long long* key) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double lo[3], ext = 0.0;
    bool any = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        any = any && box[c] != ~0ull;
        lo[c] = unord(box[c]);
        ext = fmax(ext, unord(box[3 + c]) - lo[c]);
    }
    const double cells = (double)((1 << kKeyBits) - 1);
    const double scale = (any && ext > 0.0) ? cells / ext : 0.0;
    unsigned long long out = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double v = st[k].x[c];
        double q = isfinite(v) ? (v - lo[c]) * scale : 0.0;
        q = fmin(fmax(q, 0.0), cells);
        out |= spread3((unsigned long long)q) << c;
    }
    key[k] = out;
}

__global__ void __launch_bounds__(256) invert_kernel(const int32_t* perm, int64_t n,
                                                     int32_t* inv) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) inv[perm[k]] = (int32_t)k;
}

// Slot of active position q's particle in the cluster's spatial order (n
// for an index out of range, which the force kernel flags).
__device__ __forceinline__ int slot_of(const int32_t* idx, int q, const int32_t* inv,
                                       int64_t n) {
    const int32_t p = idx[q];
    return (p >= 0 && p < n) ? inv[p] : (int)n;
}

// Counting sort of the active positions by slot: count per slot, ...
__global__ void __launch_bounds__(256) slot_count_kernel(const int32_t* idx, int ni,
                                                         const int32_t* inv, int64_t n,
                                                         int* count) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < ni) atomicAdd(count + slot_of(idx, q, inv, n), 1);
}

// ... then, after the exclusive scan of the counts, place each position at
// its slot's next free place.  Positions that share a slot (a repeated
// index) land in either order.
__global__ void __launch_bounds__(256) slot_place_kernel(const int32_t* idx, int ni,
                                                         const int32_t* inv, int64_t n,
                                                         int* next, int32_t* iord) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < ni) iord[atomicAdd(next + slot_of(idx, q, inv, n), 1)] = q;
}

// One work position k of an i-order: its index, radius, dtr and i-record.
__global__ void __launch_bounds__(256) istage_kernel(const int32_t* iord, int ni,
                                                     const int32_t* idx, const double* h2,
                                                     const double* dtr, int64_t n,
                                                     const uint4* irec, int words,
                                                     int32_t* widx, double* wh2, double* wdtr,
                                                     uint4* wrec) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ni) return;
    const int q = iord[k];
    const int32_t p = idx[q];
    widx[k] = p;
    wh2[k] = h2[q];
    wdtr[k] = dtr[q];
    const uint4* src = irec + (size_t)((p >= 0 && p < n) ? p : 0) * words;
    uint4* dst = wrec + (size_t)k * words;
    for (int w = 0; w < words; ++w) dst[w] = src[w];
}

}  // namespace

hipError_t launch_istage(const int32_t* iord, int ni, const int32_t* idx, const double* h2,
                         const double* dtr, int64_t n, const void* irec, int rec_bytes,
                         int32_t* widx, double* wh2, double* wdtr, void* wrec, hipStream_t s) {
    if (ni <= 0) return hipSuccess;
    if (rec_bytes <= 0 || rec_bytes % 16 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(istage_kernel, dim3((unsigned)((ni + 255) / 256)), dim3(256), 0, s, iord,
                       ni, idx, h2, dtr, n, static_cast<const uint4*>(irec), rec_bytes / 16,
                       widx, wh2, wdtr, static_cast<uint4*>(wrec));
    return hipGetLastError();
}

size_t iorder_scratch_bytes(int64_t ni, int64_t n) {
    (void)ni;
    size_t tmp = 0;
    (void)rocprim::exclusive_scan(nullptr, tmp, (const int*)nullptr, (int*)nullptr, 0,
                                  (size_t)n + 1, rocprim::plus<int>());
    const size_t cbytes = ((size_t)(n + 1) * sizeof(int) + 255) / 256 * 256;
    return 2 * cbytes + tmp;
}

hipError_t launch_iorder(const int32_t* idx, int ni, const int32_t* inv, int64_t n,
                         void* scratch, size_t scratch_bytes, int32_t* iord, hipStream_t s) {
    if (ni <= 0) return hipSuccess;
    if (n <= 0 || n >= 0x7fffffffLL) return hipErrorInvalidValue;
    char* p = static_cast<char*>(scratch);
    const size_t cbytes = ((size_t)(n + 1) * sizeof(int) + 255) / 256 * 256;
    int* count = reinterpret_cast<int*>(p);
    int* next = reinterpret_cast<int*>(p + cbytes);
    void* tmp = p + 2 * cbytes;
    size_t tmp_bytes = 0;
    hipError_t e = rocprim::exclusive_scan(nullptr, tmp_bytes, count, next, 0, (size_t)n + 1,
                                           rocprim::plus<int>(), s);
    if (e != hipSuccess) return e;
    if (2 * cbytes + tmp_bytes > scratch_bytes) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((ni + 255) / 256)), block(256);
    if ((e = launch_zero_u32(reinterpret_cast<unsigned*>(count), (int)(n + 1), s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(slot_count_kernel, grid, block, 0, s, idx, ni, inv, n, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = rocprim::exclusive_scan(tmp, tmp_bytes, count, next, 0, (size_t)n + 1,
                                rocprim::plus<int>(), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(slot_place_kernel, grid, block, 0, s, idx, ni, inv, n, next, iord);
    return hipGetLastError();
}

size_t order_scratch_bytes(int64_t n) {
    size_t tmp = 0;
    (void)rocprim::radix_sort_pairs(nullptr, tmp, (const unsigned long long*)nullptr,
                                    (unsigned long long*)nullptr,
                                    rocprim::counting_iterator<int32_t>(0), (int32_t*)nullptr,
                                    (unsigned)n, 0, 3 * kKeyBits);
    const size_t kbytes = ((size_t)n * sizeof(unsigned long long) + 255) / 256 * 256;
    return kHead + 2 * kbytes + tmp;
}

hipError_t launch_order(const StateRec* st, int64_t n, void* scratch, size_t scratch_bytes,
                        int32_t* perm, int32_t* inv, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > 0x7fffffffLL) return hipErrorInvalidValue;
    char* p = static_cast<char*>(scratch);
    unsigned long long* box = reinterpret_cast<unsigned long long*>(p);
    unsigned long long* part = box + 8;
    const size_t kbytes = ((size_t)n * sizeof(unsigned long long) + 255) / 256 * 256;
    unsigned long long* key_in = reinterpret_cast<unsigned long long*>(p + kHead);
    unsigned long long* key_out = reinterpret_cast<unsigned long long*>(p + kHead + kbytes);
    void* tmp = p + kHead + 2 * kbytes;
    size_t tmp_bytes = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, tmp_bytes, key_in, key_out,
                                             rocprim::counting_iterator<int32_t>(0), perm,
                                             (unsigned)n, 0, 3 * kKeyBits, s);
    if (e != hipSuccess) return e;
    if (kHead + 2 * kbytes + tmp_bytes > scratch_bytes) return hipErrorInvalidValue;

    const int blocks = (int)std::min<int64_t>((n + 255) / 256, kBoxBlocks);
    hipLaunchKernelGGL(bbox_part_kernel, dim3(blocks), dim3(256), 0, s, st, n, part);
    hipLaunchKernelGGL(bbox_final_kernel, dim3(1), dim3(256), 0, s,
                       (const unsigned long long*)part, blocks, box);
    hipLaunchKernelGGL(key_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, st, n,
                       (const unsigned long long*)box, key_in);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = rocprim::radix_sort_pairs(tmp, tmp_bytes, key_in, key_out,
                                  rocprim::counting_iterator<int32_t>(0), perm, (unsigned)n, 0,
                                  3 * kKeyBits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(invert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const int32_t*)perm, n, inv);
    return hipGetLastError();
}

}  // namespace nb6
