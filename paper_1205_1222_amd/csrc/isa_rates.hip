// isa_rates.hip -- issue rate of the vector instructions the force kernel is
// made of, on the GPU it runs on (lane-operations per second).
//
// Each thread runs ITER iterations of 8 independent instances of one
// instruction on its own registers and stores one value per thread into a
// buffer of one value per thread.  The rates, divided by the CU count and
// clock, give the per-instruction issue cost the force kernel's roofline is
// built from.  Built by paper_1205_1222_amd/build.py; run by
// `python bench.py --isa-rates`.
#include <hip/hip_runtime.h>
#include <cstdio>

#define ITER 4096
#define BODY8(INS) INS(a0) INS(a1) INS(a2) INS(a3) INS(a4) INS(a5) INS(a6) INS(a7)

#define KERNEL(NAME, T, INS)                                                   \
__global__ void __launch_bounds__(256) NAME(T* out, T seed, int n) {          \
  int tid = blockIdx.x * blockDim.x + threadIdx.x;                            \
  T a0 = seed + tid, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4,      \
    a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;                                   \
  T b = seed * 0.5f;                                                          \
  for (int it = 0; it < ITER; ++it) { BODY8(INS) }                            \
  if (tid < n) out[tid] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;              \
}

#define FMAC(x) asm volatile("v_fmac_f32 %0, %1, %1" : "+v"(x) : "v"(b));
#define ADD(x) asm volatile("v_add_f32 %0, %0, %1" : "+v"(x) : "v"(b));
#define MUL(x) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x) : "v"(b));
#define SUBS(x) asm volatile("v_sub_f32 %0, %1, %0" : "+v"(x) : "s"(b));
#define MIN(x) asm volatile("v_min_f32 %0, %0, %1" : "+v"(x) : "v"(b));
#define CND(x) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(x) : "v"(b));
#define CMP(x) asm volatile("v_cmp_lt_f32 vcc, %0, %1" : : "v"(x), "v"(b) : "vcc");
#define RSQ(x) asm volatile("v_rsq_f32 %0, %0" : "+v"(x));
#define FMA3(x) asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(x) : "v"(b));
#define ADD64(x) asm volatile("v_add_f64 %0, %0, %1" : "+v"(x) : "v"(b));
#define FMA64(x) asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(x) : "v"(b));
#define CVT(x) asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(f) : "v"(x)); x = x + 0.0;

KERNEL(k_fmac, float, FMAC)
KERNEL(k_fma, float, FMA3)
KERNEL(k_add, float, ADD)
KERNEL(k_mul, float, MUL)
KERNEL(k_subs, float, SUBS)
KERNEL(k_min, float, MIN)
KERNEL(k_cnd, float, CND)
KERNEL(k_cmp, float, CMP)
KERNEL(k_rsq, float, RSQ)
KERNEL(k_add64, double, ADD64)
KERNEL(k_fma64, double, FMA64)

// Mixes: FMAs beside instructions of another kind, on
// separate registers.  If the other kind runs beside the FMAs rather than in
// their issue slots, a mix iteration takes the time of its FMAs alone.
#define MIXKERNEL(NAME, BODY)                                                  \
__global__ void __launch_bounds__(256) NAME(float* out, float seed, int n) {  \
  int tid = blockIdx.x * blockDim.x + threadIdx.x;                            \
  float a0 = seed + tid, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4,  \
    a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;                                   \
  float b = seed * 0.5f;                                                      \
  for (int it = 0; it < ITER; ++it) { BODY }                                  \
  if (tid < n) out[tid] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;              \
}
MIXKERNEL(k_fma4, FMA3(a0) FMA3(a1) FMA3(a2) FMA3(a3) FMA3(a4) FMA3(a5) FMA3(a6) FMA3(a7))
MIXKERNEL(k_fma4_rsq1, FMA3(a0) FMA3(a1) FMA3(a2) FMA3(a3) RSQ(a4) FMA3(a5) FMA3(a6) FMA3(a7)
                       FMA3(a0) FMA3(a1) FMA3(a2) FMA3(a3) RSQ(a6))
MIXKERNEL(k_fma4_cmp1, FMA3(a0) FMA3(a1) FMA3(a2) FMA3(a3) CMP(a4) FMA3(a5) FMA3(a6) FMA3(a7)
                       FMA3(a0) FMA3(a1) FMA3(a2) FMA3(a3) CMP(a6))
MIXKERNEL(k_fma4_add4, FMA3(a0) FMA3(a1) FMA3(a2) FMA3(a3) ADD(a4) ADD(a5) ADD(a6) ADD(a7))

__global__ void __launch_bounds__(256) k_cvt(float* out, double seed, int n) {
  int tid = blockIdx.x * blockDim.x + threadIdx.x;
  double a0 = seed + tid, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5,
         a6 = a0 + 6, a7 = a0 + 7;
  float f0 = 0, f1 = 0, f2 = 0, f3 = 0, f4 = 0, f5 = 0, f6 = 0, f7 = 0;
  for (int it = 0; it < ITER; ++it) {
#define C(x, f) asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(f) : "v"(x));
    C(a0, f0) C(a1, f1) C(a2, f2) C(a3, f3) C(a4, f4) C(a5, f5) C(a6, f6) C(a7, f7)
  }
  if (tid < n) out[tid] = f0 + f1 + f2 + f3 + f4 + f5 + f6 + f7;
}

// Time of one launch of a mix kernel, in FMA-issue slots per FMA it holds
// (1.00: the other instructions cost nothing beside the FMAs).
void run_mix(const char* name, void (*kern)(float*, float, int), int fmas, int others,
             void* out, int blocks, double fma_rate) {
  hipEvent_t e0, e1;
  hipEventCreate(&e0); hipEventCreate(&e1);
  const int n = blocks * 256;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, 0, (float*)out, 1.0f, n);
  hipDeviceSynchronize();
  hipEventRecord(e0);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, 0, (float*)out, 1.0f, n);
  hipEventRecord(e1);
  hipEventSynchronize(e1);
  float ms = 0; hipEventElapsedTime(&ms, e0, e1);
  const double fma_ops = (double)n * ITER * fmas;
  const double slots = ms * 1e-3 * fma_rate;  // FMA lane-op slots the launch took
  printf("%-12s %8.3f ms  %d fma + %d other per iteration: %.2f FMA slots per FMA, "
         "%.2f per other instruction\n", name, ms, fmas, others, slots / fma_ops,
         others ? (slots - fma_ops) / ((double)n * ITER * others) : 0.0);
}

template <typename K, typename T>
void run(const char* name, K kern, T seed, void* out, int blocks) {
  hipEvent_t e0, e1;
  hipEventCreate(&e0); hipEventCreate(&e1);
  const int n = blocks * 256;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, 0, (decltype(seed)*)out, seed, n);
  hipDeviceSynchronize();
  hipEventRecord(e0);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, 0, (decltype(seed)*)out, seed, n);
  hipEventRecord(e1);
  hipEventSynchronize(e1);
  float ms = 0; hipEventElapsedTime(&ms, e0, e1);
  double ops = (double)n * ITER * 8;
  printf("%-12s %8.3f ms  %7.2f T lane-op/s  %6.2f per CU per clock at 2.4 GHz\n", name, ms,
         ops / (ms * 1e-3) / 1e12, ops / (ms * 1e-3) / (256 * 2.4e9));
}

int main() {
  const int blocks = 256 * 32;  // 8192 blocks x 256 threads
  void* out;
  if (hipMalloc(&out, (size_t)blocks * 256 * 8) != hipSuccess) { printf("alloc\n"); return 1; }
  run("fmac", k_fmac, 1.0f, out, blocks);
  run("fma", k_fma, 1.0f, out, blocks);
  run("add", k_add, 1.0f, out, blocks);
  run("mul", k_mul, 1.0f, out, blocks);
  run("sub_sgpr", k_subs, 1.0f, out, blocks);
  run("min", k_min, 1.0f, out, blocks);
  run("cndmask", k_cnd, 1.0f, out, blocks);
  run("cmp", k_cmp, 1.0f, out, blocks);
  run("rsq", k_rsq, 1.0f, out, blocks);
  run("add_f64", k_add64, 1.0, out, blocks);
  run("fma_f64", k_fma64, 1.0, out, blocks);
  {
    hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
    const int n = blocks * 256;
    hipLaunchKernelGGL(k_cvt, dim3(blocks), dim3(256), 0, 0, (float*)out, 1.0, n);
    hipDeviceSynchronize();
    hipEventRecord(e0);
    hipLaunchKernelGGL(k_cvt, dim3(blocks), dim3(256), 0, 0, (float*)out, 1.0, n);
    hipEventRecord(e1); hipEventSynchronize(e1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    double ops = (double)n * ITER * 8;
    printf("%-12s %8.3f ms  %7.2f T lane-op/s  %6.2f per CU per clock at 2.4 GHz\n", "cvt_f32_f64",
           ms, ops / (ms * 1e-3) / 1e12, ops / (ms * 1e-3) / (256 * 2.4e9));
  }
  {
    // the FMA-only reference rate for the mixes, from the same kind of launch
    hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
    const int n = blocks * 256;
    hipLaunchKernelGGL(k_fma4, dim3(blocks), dim3(256), 0, 0, (float*)out, 1.0f, n);
    hipDeviceSynchronize();
    hipEventRecord(e0);
    hipLaunchKernelGGL(k_fma4, dim3(blocks), dim3(256), 0, 0, (float*)out, 1.0f, n);
    hipEventRecord(e1); hipEventSynchronize(e1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    const double rate = (double)n * ITER * 8 / (ms * 1e-3);
    run_mix("fma+rsq", k_fma4_rsq1, 11, 2, out, blocks, rate);
    run_mix("fma+cmp", k_fma4_cmp1, 11, 2, out, blocks, rate);
    run_mix("fma+add", k_fma4_add4, 4, 4, out, blocks, rate);
  }
  if (hipDeviceSynchronize() != hipSuccess) { printf("error\n"); return 1; }
  hipFree(out);
  return 0;
}
