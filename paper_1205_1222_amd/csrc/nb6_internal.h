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
struct __attribute__((aligned(16))) RecFF {   // float-float coordinates, 48 B
    float xh, yh, zh, m;
    float xl, yl, zl, pad0;
    float vx, vy, vz, pad1;
};
struct __attribute__((aligned(16))) RecF64 {  // double coordinates, 48 B
    double x, y, z;
    float vx, vy, vz, m;
    double pad;
};
struct __attribute__((aligned(16))) RecF32 {  // plain float coordinates, 32 B
    float x, y, z, m;
    float vx, vy, vz, pad;
};

enum Mode { MODE_FF = 0, MODE_F64 = 1, MODE_F32 = 2 };

// Bits of the device status word.
enum StatusBits { ST_BAD_INDEX = 1, ST_BAD_H2 = 2, ST_NONFINITE = 4, ST_OVERFLOW = 8 };

// Partial sums leave the force kernel as 6 FP64 components per (slice, i):
// acc xyz, jerk xyz.
constexpr int NPART = 6;

struct RegfArgs {
    const void*    rec;       // records of the cluster (mode dependent)
    int            n;         // number of j-particles
    const int32_t* idx;       // [ni] active indices
    const double*  h2;        // [ni]
    const double*  dtr;       // [ni]
    int            ni;
    int            slice_len; // j per slice (multiple of 4)
    int            nslices;
    double*        part;      // [nslices][NPART][ni]
    int32_t*       cnt;       // [nslices][ni] neighbours found (true count)
    int32_t*       lst;       // [nslices][ni][caps]
    int            caps;      // per-(i, slice) list capacity
    unsigned*      status;    // device status word
};

struct FinalArgs {
    const double*  part;
    const int32_t* cnt;
    const int32_t* lst;
    int            nslices;
    int            ni;
    int            caps;
    int            n;
    const int32_t* idx;
    const double*  h2;
    double*        acc;       // [ni][3]
    double*        jerk;      // [ni][3]
    int32_t*       nnb;       // [ni]
    int32_t*       list;      // [ni][cap]
    int            cap;
    unsigned*      status;
};

struct PredictArgs {
    int64_t       n;
    const double* m;
    const double* x;   // [n][3]
    const double* v;
    const double* a;
    const double* jk;
    const double* t;
    double        tb;
    RecFF*        ff;  // may be null
    RecF64*       f64; // may be null
    RecF32*       f32; // may be null
    unsigned*     status;
};

struct ScatterArgs {
    int64_t        n;     // entries
    const int32_t* idx;   // [n] destination particle of each entry
    const double*  m;     // sources, [n] and [n][3]
    const double*  x;
    const double*  v;
    const double*  a;
    const double*  jk;
    const double*  t;
    double* dm; double* dx; double* dv; double* da; double* djk; double* dt;
    int64_t        limit; // cluster size; entries with idx outside [0, limit) are skipped
    unsigned*      status;
};

// i-particles per lane of the force kernel.
hipError_t launch_regf(int mode, int ipl, int waves_per_block, const RegfArgs& a,
                       hipStream_t s);
hipError_t launch_finalize(const FinalArgs& a, hipStream_t s);
hipError_t launch_predict(const PredictArgs& a, hipStream_t s);
hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s);
// Widen the j-records of one mode to double position and velocity arrays.
hipError_t launch_unpack(int mode, const void* rec, int64_t n, double* x, double* v,
                         hipStream_t s);
// Clear n words with a kernel (not a memset node, so it is safe under graph
// capture).
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s);

}  // namespace nb6
