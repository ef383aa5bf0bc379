// opbench.hip -- throughput of the gfx950 VALU instruction classes the Metropolis update
// uses, measured on the GPU: each lane runs 8 independent chains of one instruction, enough
// waves are resident to hide latency, and the rate is lanes * chains * iterations / time.
// The ratio to v_add_f32 gives each class's issue cost in full-rate lane slots, the unit of
// the engine's VALU roofline. ALU-only inline assembly (no memory operand) pins the exact
// instruction.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int CH = 8;  // independent chains per lane

#define OPBENCH_KERNEL(NAME, TYPE, INIT, BODY)                                   \
    __global__ __launch_bounds__(256) void NAME(uint32_t *sink, int iters)        \
    {                                                                             \
        TYPE x[CH];                                                               \
        const uint32_t t = threadIdx.x + blockIdx.x * 256u;                       \
        _Pragma("unroll") for (int c = 0; c < CH; ++c) x[c] = INIT;               \
        const uint32_t yb = t * 0x9E3779B9u + 1u;                                 \
        const float yf = 1.0f + 1e-7f * (float)(t & 7);                           \
        const double yd = 1.0 + 1e-12 * (double)(t & 7);                         \
        (void)yb; (void)yf; (void)yd;                                             \
        for (int i = 0; i < iters; ++i) {                                         \
            _Pragma("unroll") for (int c = 0; c < CH; ++c) { BODY; }              \
        }                                                                         \
        uint32_t h = 0;                                                           \
        _Pragma("unroll") for (int c = 0; c < CH; ++c) h ^= (uint32_t)x[c];       \
        if (h == 0x12345678u) sink[t] = h;                                        \
    }

OPBENCH_KERNEL(k_add_f32, float, 1.0f + c, asm volatile("v_add_f32 %0, %0, %1" : "+v"(x[c]) : "v"(yf)))
OPBENCH_KERNEL(k_fma_f32, float, 1.0f + c, asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(x[c]) : "v"(yf)))
OPBENCH_KERNEL(k_mul_f32, float, 1.0f + c, asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x[c]) : "v"(yf)))
OPBENCH_KERNEL(k_sub_f32, float, 1.0f + c, asm volatile("v_sub_f32 %0, %0, %1" : "+v"(x[c]) : "v"(yf)))
OPBENCH_KERNEL(k_cndmask_b32, uint32_t, t + c,
               uint64_t m = 0x5555555555555555ull; asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(x[c]) : "v"(yb), "s"(m)))
OPBENCH_KERNEL(k_cmp_lt_f32, float, 1.0f + c,
               uint64_t m; asm volatile("v_cmp_lt_f32_e64 %0, %1, %2" : "=s"(m) : "v"(x[c]), "v"(yf)))
OPBENCH_KERNEL(k_alignbit_b32, uint32_t, t + c, asm volatile("v_alignbit_b32 %0, %1, %0, 9" : "+v"(x[c]) : "v"(yb)))
OPBENCH_KERNEL(k_xor_b32, uint32_t, t + c, asm volatile("v_xor_b32 %0, %0, %1" : "+v"(x[c]) : "v"(yb)))
OPBENCH_KERNEL(k_bitop3_b32, uint32_t, t + c, asm volatile("v_bitop3_b32 %0, %0, %1, %0 bitop3:0x96" : "+v"(x[c]) : "v"(yb)))
OPBENCH_KERNEL(k_add_u32, uint32_t, t + c, asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[c]) : "v"(yb)))
OPBENCH_KERNEL(k_mul_hi_u32, uint32_t, t + c, asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[c]) : "v"(yb)))
OPBENCH_KERNEL(k_mul_lo_u32, uint32_t, t + c, asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[c]) : "v"(yb)))
OPBENCH_KERNEL(k_mad_u64_u32, uint64_t, t + c,
               uint64_t sc; asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(x[c]), "=s"(sc) : "v"(yb), "v"(yb + 1u)))
OPBENCH_KERNEL(k_cvt_f32_u32, uint32_t, t + c, asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(x[c])))
OPBENCH_KERNEL(k_exp_f32, float, 0.5f + c, asm volatile("v_exp_f32 %0, %0" : "+v"(x[c])))
OPBENCH_KERNEL(k_sin_f32, float, 0.1f * c, asm volatile("v_sin_f32 %0, %0" : "+v"(x[c])))
OPBENCH_KERNEL(k_cos_f32, float, 0.1f * c, asm volatile("v_cos_f32 %0, %0" : "+v"(x[c])))
OPBENCH_KERNEL(k_sqrt_f32, float, 2.0f + c, asm volatile("v_sqrt_f32 %0, %0" : "+v"(x[c])))
OPBENCH_KERNEL(k_fma_f64, double, 1.0 + c, asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(x[c]) : "v"(yd)))
OPBENCH_KERNEL(k_add_f64, double, 1.0 + c, asm volatile("v_add_f64 %0, %0, %1" : "+v"(x[c]) : "v"(yd)))

struct Op {
    const char *name;
    void (*fn)(uint32_t *, int);
};

const Op k_ops[] = {
    {"v_add_f32", k_add_f32},         {"v_fma_f32", k_fma_f32},         {"v_mul_f32", k_mul_f32},
    {"v_sub_f32", k_sub_f32},         {"v_cndmask_b32", k_cndmask_b32}, {"v_cmp_lt_f32", k_cmp_lt_f32},
    {"v_alignbit_b32", k_alignbit_b32}, {"v_xor_b32", k_xor_b32},
    {"v_bitop3_b32", k_bitop3_b32},   {"v_add_u32", k_add_u32},         {"v_mul_hi_u32", k_mul_hi_u32},
    {"v_mul_lo_u32", k_mul_lo_u32},   {"v_mad_u64_u32", k_mad_u64_u32}, {"v_cvt_f32_u32", k_cvt_f32_u32},
    {"v_exp_f32", k_exp_f32},         {"v_sin_f32", k_sin_f32},         {"v_cos_f32", k_cos_f32},
    {"v_sqrt_f32", k_sqrt_f32},       {"v_fma_f64", k_fma_f64},         {"v_add_f64", k_add_f64},
};

}  // namespace

extern "C" {

int mmc_opbench_count(void) { return (int)(sizeof(k_ops) / sizeof(k_ops[0])); }

const char *mmc_opbench_name(int i) { return (i >= 0 && i < mmc_opbench_count()) ? k_ops[i].name : nullptr; }

// Instructions per second (wave-level instructions x 64 lanes) of op i; *ms = kernel time.
// Returns 0 on success, -1 on a bad index, -3 on a HIP error.
int mmc_opbench_run(int i, int iters, double *lane_ops_per_s, double *ms)
{
    if (i < 0 || i >= mmc_opbench_count() || iters < 1) return -1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -3;
    const int blocks = cus * 8;  // 8 x 256 threads = 32 waves per CU
    uint32_t *sink = nullptr;
    if (hipMalloc(&sink, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) return -3;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(k_ops[i].fn, dim3(blocks), dim3(256), 0, 0, sink, 1);  // warm-up
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL(k_ops[i].fn, dim3(blocks), dim3(256), 0, 0, sink, iters);
    (void)hipEventRecord(b, 0);
    hipError_t e = hipEventSynchronize(b);
    float t = 0;
    (void)hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(sink);
    if (e != hipSuccess) return -3;
    *ms = t;
    *lane_ops_per_s = (double)blocks * 256.0 * CH * (double)iters / (t * 1e-3);
    return 0;
}

}  // extern "C"
