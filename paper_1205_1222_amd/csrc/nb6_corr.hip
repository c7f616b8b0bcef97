// nb6_corr.hip -- the regular corrector of a block (section 3.3 step 7),
// elementwise over the particles that reached their regular time:
//   * the regular force change over the step with the neighbour set held
//     fixed: the raw change plus the change of the irregular force at the new
//     time from the old to the new list (section 3.6);
//   * the second and third derivatives of the regular force from the cubic
//     Hermite interpolation over the step (the fourth-order Hermite scheme of
//     Makino & Aarseth 1992, cited in section 2 for the neighbour-change
//     corrections);
//   * the next regular step: the standard step criterion on the new-time
//     derivatives, taken down to a power of two that divides the block time
//     (block steps), at most twice the last step, within [dt_min, dt_max];
//   * the new neighbour radius of equation (1), with its factor limited to
//     [f_lo, f_hi] and the upper limit for an empty list.
// One thread per particle, FP64, every operation in the order the formulas
// state them.
#include "nb6_internal.h"

#pragma clang fp contract(off)

namespace nb6 {

__device__ __forceinline__ double norm3(const double x[3]) {
    return sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
}

__global__ void __launch_bounds__(256) correct_kernel(CorrArgs a) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n) return;
    const double h = a.t - a.t_old[q];
    if (!(h > 0.0) || !isfinite(h)) {
        atomicOr(a.status, (unsigned)ST_BAD_STEP);
        const double nan = __builtin_nan("");
        for (int c = 0; c < 3; ++c)
            a.df[3 * q + c] = a.dfd[3 * q + c] = a.f2[3 * q + c] = a.f3[3 * q + c] = nan;
        a.dt_new[q] = a.h_new[q] = nan;
        return;
    }
    double F2[3], F3[3], fn[3], fdn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t k = 3 * q + c;
        const double dF = (a.f_new[k] - a.f_old[k]) + (a.g_new[k] - a.g_old[k]);
        const double dFd = (a.fd_new[k] - a.fd_old[k]) + (a.gd_new[k] - a.gd_old[k]);
        const double f2_old = (6.0 * dF - h * (6.0 * a.fd_old[k] + 2.0 * dFd)) / (h * h);
        F3[c] = (-12.0 * dF + 6.0 * h * (2.0 * a.fd_old[k] + dFd)) / (h * h * h);
        F2[c] = f2_old + h * F3[c];
        fn[c] = a.f_new[k];
        fdn[c] = a.fd_new[k];
        a.df[k] = dF;
        a.dfd[k] = dFd;
        a.f2[k] = F2[c];
        a.f3[k] = F3[c];
    }
    const double f = norm3(fn), fd = norm3(fdn), f2 = norm3(F2), f3 = norm3(F3);
    // a vanishing denominator (or 0/0) leaves the step to the other limits
    const double est = sqrt(a.eta * (f * f2 + fd * fd) / (fd * f3 + f2 * f2));
    const double lim = fmin(fmin(est, 2.0 * h), a.dt_max);
    double d = a.dt_max;  // powers of two from dt_max down to dt_min (bounded loop)
    while (d > a.dt_min && (d > lim || fmod(a.t, d) != 0.0)) d *= 0.5;
    a.dt_new[q] = d;
    double g = a.f_hi;
    if (a.nnb[q] > 0) g = fmin(fmax(cbrt(a.n_p[q] / (double)a.nnb[q]), a.f_lo), a.f_hi);
    a.h_new[q] = a.h_old[q] * g;
}

hipError_t launch_correct(const CorrArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(correct_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace nb6
