// engine.hpp -- internal interface between the host runtime (runtime.cpp) and the HIP
// kernels (kernels.hip) of the multipath Metropolis engine. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mmc {

// Per-path accumulators in device memory (16 doubles = 128 bytes, one cache line).
// Sums run over measured sweeps; final_* is the state after the last sweep run.
struct PathAcc {
    double sum_e, sum_e2, sum_m, sum_m2, sum_m4;
    double final_e, final_m[3];
    unsigned long long n_accept;
    double pad[6];
};
static_assert(sizeof(PathAcc) == 128, "PathAcc layout");

enum { TAG_INIT = 0, TAG_MET = 1 };
enum { INIT_SPHERE = 0, INIT_ANGLES = 1, INIT_ORDERED = 2, INIT_MIXED = 3 };
enum { PROPOSAL_SPHERE = 0, PROPOSAL_ANGLES = 1 };

// One instance as the kernels see it.
struct InstDev {
    int L;               // side (even, >= 2)
    int n_paths;
    int n_therm, n_meas; // sweeps: measured when k >= n_therm
    int trace_sweeps;    // trace rows for k < trace_sweeps
    int init;            // INIT_*
    int proposal;        // PROPOSAL_* (ANGLES: plain FP64 engine only)
    int renorm_every;    // FP32 only; <= 0: never
    uint32_t ctr3;       // Philox counter word 3 without the tag: instance_id << 8
    uint32_t key0, key1; // Philox key = seed
    double beta, J;
    void *spins;         // resident state [n_paths][2 colours][3][N/2] (T), or nullptr
    PathAcc *acc;        // [n_paths]
    double *trace;       // [n_paths][trace_sweeps][4] or nullptr
    // 2-D Ising model: accept iff the word is below ithr[(a + 4) / 2] or bit (a + 4) / 2 of iall
    // is set, for a = s h in {-4, -2, 0, 2, 4}
    uint32_t ithr[5];
    uint32_t iall;
};

// One work item of a batch: paths [path0, path0 + paths_per_item) of instance inst.
struct BatchItem {
    int inst;
    int path0;
};

struct BatchDev {
    const InstDev *inst;     // [n_inst]
    const int *variant;      // [n_inst] batch variant of each instance (the shared device-memory kernel)
    const BatchItem *items;  // [n_items] of one launch, largest first
    int n_items;
    unsigned int *head;      // work-queue head (zeroed before each launch)
    char *slots;             // HBM spin slots, slot_bytes per resident workgroup
    size_t slot_bytes;
    int n_slots;
};

// A compiled kernel variant for single-instance (resident) runs.
struct Variant {
    const char *name;
    int fp64;        // 0: FP32, 1: FP64
    int L;           // compile-time side, 0 = any even L
    int lds;         // 1: spins in LDS, 0: in device memory, 2: colour 0 in LDS, colour 1 in device memory,
                     // 3: colour 0's x and y components in LDS, the rest in device memory,
                     // 4: in device memory, swept through a ring of z-planes in LDS,
                     // 5: in device memory, colour 0 swept through a ring of z-planes in LDS,
                     // 6: as 4, two sweeps per pass
    int block;       // threads per workgroup
    int lanes;       // threads per path (block % lanes == 0)
    size_t lds_bytes;                 // dynamic LDS per workgroup
    // launch over all paths: sweeps [k0, k1); fresh = initialise first
    hipError_t (*launch)(const InstDev &in, int k0, int k1, int fresh, hipStream_t s);
    const void *kernel;  // the __global__ function (resident variants)
    int window;          // sweeps per pass of the z-pipelined window variants, 0 otherwise
    // batch variants: the variant's persistent kernel over a queue of items
    hipError_t (*launch_batch)(const BatchDev &b, int grid, size_t lds, hipStream_t s);
};

// Variants usable by resident runs, and by the batch kernel (fixed block size).
const Variant *variants(int *count);
const Variant *ising_variants(int *count);  // 2-D Ising model (spins in LDS)
size_t ising_variant_lds_bytes(int L);
size_t ising_spin_bytes(int L);  // bytes of one path's state in device memory
int ising_row_stride(int L);     // bytes per row: [colour][y][row stride], byte j = x >> 1
const Variant *batch_variants(int fp64, int *count);  // index = BatchDev::variant value
size_t variant_lds_bytes(const Variant &v, int L);             // dynamic LDS at side L
// The persistent kernel of one batch variant, with lds bytes of dynamic LDS per workgroup.
hipError_t launch_batch(const BatchDev &b, int fp64, int variant, int grid, size_t lds, hipStream_t s);
int batch_blocks_per_cu(int fp64, int variant, size_t lds);  // resident workgroups per CU; 0 if unknown
int batch_paths_per_item(int fp64, int variant);
size_t batch_slot_bytes(int fp64, int variant, int L);  // HBM slot bytes needed (0 for LDS)

// The fused batch kernel (one launch for a batch mixing lattice sides, FP32): the member that
// runs a batch variant's paths identically, or -1; per member its dynamic LDS, spin-slot bytes
// per workgroup and paths per item; resident workgroups per CU at a given LDS size.
int fused_member(int fp64, const char *batch_variant);
size_t fused_lds_bytes(int member);
size_t fused_slot_bytes(int member);
int fused_paths_per_item(int member);
int fused_blocks_per_cu(size_t lds);
int fused_block();  // threads per workgroup of the fused kernel
const char *fused_member_name(int member);  // the batch variant a member runs like
int fused_member_like(int fp64, int L, int place);  // a member of that side and placement, or -1
hipError_t launch_fused(const BatchDev &b, int grid, size_t lds, hipStream_t s);

hipError_t prepare_kernels(int max_lds);  // once per process, before the first launch

// Plain FP64 engine: one launch per half-sweep, one thread per site.
hipError_t plain_init(const InstDev &in, hipStream_t s);
hipError_t plain_half(const InstDev &in, const int *k_dev, int colour, hipStream_t s);
hipError_t plain_measure(const InstDev &in, int *k_dev, int k_last, hipStream_t s);

// The proposal step alone: xyz[3t..3t+2] = unit vector of words w[2t], w[2t+1] (device arrays).
hipError_t proposal_vectors(int fp64, int angles, const uint32_t *w, long long n, double *xyz, hipStream_t s);

// Sets the calling thread's C-ABI error (mmc_last_error / mmc_last_status); returns code.
int report_error(int code, const char *msg);

// Small helpers (kernel-based; no hipMemset inside captured graphs).
hipError_t fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t fill_nan(double *p, size_t n, hipStream_t s);
hipError_t set_int(int *p, int v, hipStream_t s);

}  // namespace mmc
