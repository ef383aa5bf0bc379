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

// The algorithmic VALU instructions of two FP32 Metropolis updates (81.5 each: Philox4x32-10
// with its wave-uniform half on the scalar unit, three uniforms, the proposal, the local
// field, the energy change and test, the new-spin select and the fused measurement, one fma
// of which falls on odd sites only), in the order an update issues them, on independent
// register chains: no memory traffic and no dependency beyond each chain's own, so the rate
// is the ALU ceiling of the update's instruction mix, whatever the classes' overlap.
__global__ __launch_bounds__(256) void k_update_mix(uint32_t *sink, int iters)
{
    // shader-clock cycles and constant-rate wall-clock ticks of the loop (per workgroup)
    const uint64_t c0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    const uint32_t t = threadIdx.x + blockIdx.x * 256u;
    const uint32_t yb = t * 0x9E3779B9u + 1u;
    const float yf = 1.0f + 1e-7f * (float)(t & 7);
    uint64_t m[4];
    uint32_t b[4], al[2], cm[3];
    float sb[4], fm[4], mu[2], ad[4], tr[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        m[c] = t + c;
        b[c] = t ^ (c * 77u);
        sb[c] = 1.0f + c;
        fm[c] = 0.5f + c;
        ad[c] = 2.0f + c;
        tr[c] = 0.25f + 0.1f * c;
    }
    al[0] = t; al[1] = t + 9u; cm[0] = t; cm[1] = t + 3u; cm[2] = t + 5u; mu[0] = 1.5f; mu[1] = 2.5f;
    // 64-bit product-accumulate as the compiler writes it (carry to a dead scalar pair); the
    // empty asm keeps each one in place
    auto mad = [&](uint64_t &x) {
        x = (uint64_t)yb * (uint32_t)(x >> 32) + x;
        asm volatile("" : "+v"(x));
    };
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            // Philox: 18 64-bit products, 15 three-way and 4 two-way xors
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                mad(m[(2 * r) & 3]);
                asm volatile("v_bitop3_b32 %0, %0, %1, %0 bitop3:0x96" : "+v"(b[r & 3]) : "v"(yb));
                mad(m[(2 * r + 1) & 3]);
                if (r < 6) asm volatile("v_bitop3_b32 %0, %0, %1, %0 bitop3:0x96" : "+v"(b[(r + 2) & 3]) : "v"(yb));
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(b[c]) : "v"(yb));
            // three uniforms (alignbit + subtract) and z = 2u - 1
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                asm volatile("v_alignbit_b32 %0, %1, %0, 9" : "+v"(al[c & 1]) : "v"(yb));
                asm volatile("v_sub_f32 %0, %0, %1" : "+v"(sb[c]) : "v"(yf));
            }
            asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(fm[0]) : "v"(yf));
            // proposal: fma, sqrt, sin, cos, two products
            asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(fm[1]) : "v"(yf));
            asm volatile("v_sqrt_f32 %0, %0" : "+v"(tr[0]));
            asm volatile("v_sin_f32 %0, %0" : "+v"(tr[1]));
            asm volatile("v_cos_f32 %0, %0" : "+v"(tr[2]));
            asm volatile("v_mul_f32 %0, %0, %1" : "+v"(mu[0]) : "v"(yf));
            asm volatile("v_mul_f32 %0, %0, %1" : "+v"(mu[1]) : "v"(yf));
            // local field: 15 additions
#pragma unroll
            for (int c = 0; c < 15; ++c) asm volatile("v_add_f32 %0, %0, %1" : "+v"(ad[c & 3]) : "v"(yf));
            // energy change and test: 3 subtractions, product, 2 fma, product, exp2, compare
#pragma unroll
            for (int c = 0; c < 3; ++c) asm volatile("v_sub_f32 %0, %0, %1" : "+v"(sb[3 - c]) : "v"(yf));
            asm volatile("v_mul_f32 %0, %0, %1" : "+v"(mu[0]) : "v"(yf));
            asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(fm[2]) : "v"(yf));
            asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(fm[3]) : "v"(yf));
            asm volatile("v_mul_f32 %0, %0, %1" : "+v"(mu[1]) : "v"(yf));
            asm volatile("v_exp_f32 %0, %0" : "+v"(tr[3]));
            // compare and the new-spin select on its mask (as the compiler writes them)
            const bool acc = tr[3] < yf;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                uint32_t v = acc ? cm[c] : yb;
                asm volatile("" : "+v"(v));
                cm[c] = v;
            }
            // measurement: 3 additions, and 3 fma on the odd one of the two updates
#pragma unroll
            for (int c = 0; c < 3; ++c) asm volatile("v_add_f32 %0, %0, %1" : "+v"(ad[(c + 1) & 3]) : "v"(yf));
            if (u == 1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(fm[c]) : "v"(yf));
            }
        }
    }
    uint32_t h = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) h ^= (uint32_t)m[c] ^ b[c] ^ (uint32_t)sb[c] ^ (uint32_t)fm[c] ^ (uint32_t)ad[c] ^ (uint32_t)tr[c];
    h ^= al[0] ^ al[1] ^ cm[0] ^ cm[1] ^ cm[2] ^ (uint32_t)mu[0] ^ (uint32_t)mu[1];
    if (h == 0x12345678u && threadIdx.x >= 4) sink[t] = h;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
        uint64_t *clk = reinterpret_cast<uint64_t *>(sink + blockIdx.x * 256u);
        clk[0] = c1 - c0;
        clk[1] = r1 - r0;
    }
}

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
    {"update_mix", k_update_mix},
};

// Streaming kernels over n 16-byte elements, grid-stride, each thread moving U elements per
// step (all loads issued before the stores, TB elements apart, so that a wave keeps U loads in
// flight): KIND 0 copies src to dst, 1 only reads src (xor-folding what it reads, stored only
// if it hits a value that never occurs), 2 only writes dst. NT: nontemporal loads and stores
// (streamed past the caches' normal allocation). Every index is checked against n.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int U, int TB, int KIND, bool NT>
__global__ __launch_bounds__(TB) void k_stream16(const uint4 *__restrict__ src4, uint4 *__restrict__ dst4, size_t n)
{
    const u32x4 *src = reinterpret_cast<const u32x4 *>(src4);
    u32x4 *dst = reinterpret_cast<u32x4 *>(dst4);
    const size_t step = (size_t)gridDim.x * TB * U;
    uint32_t fold = 0;
    for (size_t base = (size_t)blockIdx.x * TB * U + threadIdx.x; base < n; base += step) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + (size_t)u * TB;
            if (KIND != 2 && i < n) v[u] = NT ? __builtin_nontemporal_load(src + i) : src[i];
            else v[u] = u32x4{(uint32_t)i, 1u, 2u, 3u};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + (size_t)u * TB;
            if (i < n) {
                if (KIND == 1) {
                    fold ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
                } else if (NT) {
                    __builtin_nontemporal_store(v[u], dst + i);
                } else {
                    dst[i] = v[u];
                }
            }
        }
    }
    if (KIND == 1 && fold == 0x9E3779B9u && n > 0) dst[0] = u32x4{fold, 0u, 0u, 0u};
}

template <int U, int TB, int KIND, bool NT>
void launch_stream(int blocks, hipStream_t s, const uint4 *src, uint4 *dst, size_t n)
{
    hipLaunchKernelGGL((k_stream16<U, TB, KIND, NT>), dim3(blocks), dim3(TB), 0, s, src, dst, n);
}

template <int TB, int KIND, bool NT>
bool launch_u(int unroll, int blocks, hipStream_t s, const uint4 *src, uint4 *dst, size_t n)
{
    switch (unroll) {
    case 1: launch_stream<1, TB, KIND, NT>(blocks, s, src, dst, n); return true;
    case 2: launch_stream<2, TB, KIND, NT>(blocks, s, src, dst, n); return true;
    case 4: launch_stream<4, TB, KIND, NT>(blocks, s, src, dst, n); return true;
    case 8: launch_stream<8, TB, KIND, NT>(blocks, s, src, dst, n); return true;
    default: return false;
    }
}

template <int KIND, bool NT>
bool launch_tb(int threads, int unroll, int blocks, hipStream_t s, const uint4 *src, uint4 *dst, size_t n)
{
    if (threads == 256) return launch_u<256, KIND, NT>(unroll, blocks, s, src, dst, n);
    if (threads == 1024) return launch_u<1024, KIND, NT>(unroll, blocks, s, src, dst, n);
    return false;
}

bool launch_any(int kind, int nt, int threads, int unroll, int blocks, hipStream_t s, const uint4 *src, uint4 *dst,
                size_t n)
{
    switch (kind * 2 + (nt ? 1 : 0)) {
    case 0: return launch_tb<0, false>(threads, unroll, blocks, s, src, dst, n);
    case 1: return launch_tb<0, true>(threads, unroll, blocks, s, src, dst, n);
    case 2: return launch_tb<1, false>(threads, unroll, blocks, s, src, dst, n);
    case 3: return launch_tb<1, true>(threads, unroll, blocks, s, src, dst, n);
    case 4: return launch_tb<2, false>(threads, unroll, blocks, s, src, dst, n);
    case 5: return launch_tb<2, true>(threads, unroll, blocks, s, src, dst, n);
    default: return false;
    }
}

}  // namespace

extern "C" {

// Time of one streaming pass over `bytes` (a multiple of 16) averaged over reps launches after
// one warm-up, on the null stream: kind 0 copies src to dst (disjoint device buffers), 1 reads
// src, 2 writes dst; nt = 1 for nontemporal accesses; blocks_per_cu x CUs workgroups of
// `threads` (256 or 1024) threads, unroll 1, 2, 4 or 8 elements per thread and step.
// Returns 0, -1 on bad arguments, -3 on a HIP error.
int mmc_opbench_stream(const void *src, void *dst, size_t bytes, int reps, int kind, int nt, int threads,
                       int blocks_per_cu, int unroll, double *ms)
{
    if (!src || !dst || !ms || bytes == 0 || bytes % 16 || reps < 1 || blocks_per_cu < 1 || blocks_per_cu > 64 ||
        kind < 0 || kind > 2 || (threads != 256 && threads != 1024) ||
        (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8))
        return -1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -3;
    const size_t n = bytes / 16;
    const int blocks = cus * blocks_per_cu;
    const uint4 *s = static_cast<const uint4 *>(src);
    uint4 *d = static_cast<uint4 *>(dst);
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -3;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -3;
    }
    launch_any(kind, nt, threads, unroll, blocks, 0, s, d, n);  // warm-up
    (void)hipEventRecord(a, 0);
    for (int r = 0; r < reps; ++r) launch_any(kind, nt, threads, unroll, blocks, 0, s, d, n);
    (void)hipEventRecord(b, 0);
    hipError_t e = hipEventSynchronize(b);
    float t = 0;
    (void)hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess || hipGetLastError() != hipSuccess) return -3;
    *ms = t / reps;
    return 0;
}

// The plain 256-thread copy (kind 0, no nontemporal hints): the calibration kernel of the
// byte counters.
int mmc_opbench_copy(const void *src, void *dst, size_t bytes, int reps, int blocks_per_cu, int unroll, double *ms)
{
    return mmc_opbench_stream(src, dst, bytes, reps, 0, 0, 256, blocks_per_cu, unroll, ms);
}

// The update mix alone at full occupancy for iters iterations (two updates per lane each),
// after one warm-up launch: updates per second, kernel time (HIP events) and the mean shader
// clock of the run in MHz (s_memtime cycles over s_memrealtime ticks of each workgroup, the
// latter at the device's wall-clock rate). Returns 0, -1 on bad arguments, -3 on a HIP error.
int mmc_opbench_update_mix(int iters, double *updates_per_s, double *ms, double *clock_mhz)
{
    if (iters < 1 || !updates_per_s || !ms || !clock_mhz) return -1;
    int dev = 0, cus = 0, wall_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
        return -3;
    const int blocks = cus * 8;
    uint32_t *sink = nullptr;
    if (hipMalloc(&sink, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) return -3;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_update_mix, dim3(blocks), dim3(256), 0, 0, sink, 1);  // warm-up
        (void)hipEventRecord(a, 0);
        hipLaunchKernelGGL(k_update_mix, dim3(blocks), dim3(256), 0, 0, sink, iters);
        (void)hipEventRecord(b, 0);
        e = hipEventSynchronize(b);
    }
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    double cyc = 0, ticks = 0;
    if (e == hipSuccess) {
        uint64_t *h = new uint64_t[(size_t)blocks * 128];
        e = hipMemcpy(h, sink, (size_t)blocks * 256 * sizeof(uint32_t), hipMemcpyDeviceToHost);
        for (int i = 0; i < blocks && e == hipSuccess; ++i) {
            cyc += (double)h[(size_t)i * 128];
            ticks += (double)h[(size_t)i * 128 + 1];
        }
        delete[] h;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(sink);
    if (e != hipSuccess || t <= 0 || ticks <= 0) return -3;
    *ms = t;
    *updates_per_s = (double)blocks * 256.0 * 2.0 * (double)iters / (t * 1e-3);
    *clock_mhz = cyc / (ticks / ((double)wall_khz * 1e3)) / 1e6;
    return 0;
}

int mmc_opbench_count(void) { return (int)(sizeof(k_ops) / sizeof(k_ops[0])); }

const char *mmc_opbench_name(int i) { return (i >= 0 && i < mmc_opbench_count()) ? k_ops[i].name : nullptr; }

// Instructions per second (wave-level instructions x 64 lanes) of op i -- for "update_mix",
// updates per second; *ms = kernel time.
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
    // the update mix: two updates per lane and iteration; a single class: CH instructions
    const double per_iter = k_ops[i].fn == k_update_mix ? 2.0 : (double)CH;
    *lane_ops_per_s = (double)blocks * 256.0 * per_iter * (double)iters / (t * 1e-3);
    return 0;
}

}  // extern "C"
