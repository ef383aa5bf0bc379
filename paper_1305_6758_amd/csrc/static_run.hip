// static_run.hip -- mmc_batch_run_static: the batch run for callers that cannot allocate.
//
// The same persistent LDS batch kernels as mmc_batch_run (one per variant in use, workgroups
// taking (instance, path group) items from a device queue), with every piece of device memory
// they need beyond the caller's output -- the instance table, the work lists, the queue heads
// and the per-path FP64 accumulators -- in one file-scope device array, `scratch`, of
// MMC_STATIC_SCRATCH_BYTES. Only instances whose whole lattice fits in a workgroup's LDS are
// accepted (no device-memory spin slots). The host side allocates no device memory and no
// host heap: its tables live on the stack and reach the scratch array as kernel arguments.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>

#include <mutex>

#include "../../include/mmc.h"
#include "engine.hpp"

// The device memory of mmc_batch_run_static, one copy per GPU, held until the process ends.
static __device__ __align__(256) char scratch[MMC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_INST = MMC_STATIC_MAX_INSTANCES;
constexpr int MAX_PATHS = MMC_STATIC_MAX_PATHS;
constexpr int MAX_LAUNCH = 16;
constexpr int MAX_DEV = 64;

// One run of consecutive items of a launch: the items of one instance.
struct Run {
    int inst, item_begin, n_items, paths_per_item;
};

// The tables the host fills on its stack: the instances as the kernels see them, each one's
// variant, its first path in the output, and the launches' runs of items.
struct HostTables {
    mmc::InstDev d[MAX_INST];
    int var[MAX_INST];
    int path_off[MAX_INST + 1];
    Run runs[MAX_INST];
};

// Scratch layout (byte offsets from the array's device address): the host tables, then the
// queue heads, the work lists and the per-path accumulators.
struct Layout {
    static constexpr size_t inst = offsetof(HostTables, d);
    static constexpr size_t var = offsetof(HostTables, var);
    static constexpr size_t path_off = offsetof(HostTables, path_off);
    static constexpr size_t runs = offsetof(HostTables, runs);
    static constexpr size_t head = (sizeof(HostTables) + 255) / 256 * 256;                      // 64 B per launch
    static constexpr size_t items = head + 64 * MAX_LAUNCH;                                     // BatchItem[MAX_PATHS]
    static constexpr size_t acc = (items + sizeof(mmc::BatchItem) * MAX_PATHS + 255) / 256 * 256;  // PathAcc[MAX_PATHS]
    static constexpr size_t end = acc + sizeof(mmc::PathAcc) * MAX_PATHS;
};
static_assert(Layout::end <= MMC_STATIC_SCRATCH_BYTES, "scratch layout exceeds the static array");

// Host-to-device copy through kernel arguments (captured at launch, so the host tables may
// live on the stack): CHUNK bytes per launch.
constexpr int CHUNK = 2048;
struct Bytes {
    unsigned char b[CHUNK];
};

__global__ __launch_bounds__(256) void k_static_upload(Bytes src, int n, char *dst)
{
    for (int i = threadIdx.x; i < n; i += 256) dst[i] = (char)src.b[i];
}

hipError_t upload(char *dst, const void *src, size_t n, hipStream_t s)
{
    const unsigned char *p = static_cast<const unsigned char *>(src);
    for (size_t o = 0; o < n; o += CHUNK) {
        Bytes b;
        const int k = (int)(n - o < (size_t)CHUNK ? n - o : (size_t)CHUNK);
        for (int i = 0; i < k; ++i) b.b[i] = p[o + i];
        hipLaunchKernelGGL(k_static_upload, dim3(1), dim3(256), 0, s, b, k, dst + o);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Work list of one launch: item i lies in the run r with item_begin <= i < item_begin + n_items.
__global__ __launch_bounds__(256) void k_static_items(const Run *runs, int run0, int n_runs, int n_items,
                                                      mmc::BatchItem *items)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n_items; i += gridDim.x * 256) {
        int lo = run0, hi = run0 + n_runs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (runs[mid].item_begin <= i) lo = mid;
            else hi = mid - 1;
        }
        const Run r = runs[lo];
        items[i] = mmc::BatchItem{r.inst, (i - r.item_begin) * r.paths_per_item};
    }
}

// Per-path results from the accumulators (means over the measured sweeps, NaN without any).
__global__ __launch_bounds__(256) void k_static_results(const mmc::InstDev *inst, const int *path_off, int n_inst,
                                                        const mmc::PathAcc *acc, int n_total, mmc_path_result *out)
{
    for (int g = blockIdx.x * 256 + threadIdx.x; g < n_total; g += gridDim.x * 256) {
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (path_off[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const mmc::PathAcc a = acc[g];
        const int n_meas = inst[lo].n_meas;
        mmc_path_result r;
        if (n_meas > 0) {
            const double nm = (double)n_meas;
            r.e_mean = a.sum_e / nm;
            r.e2_mean = a.sum_e2 / nm;
            r.absm_mean = a.sum_m / nm;
            r.m2_mean = a.sum_m2 / nm;
            r.m4_mean = a.sum_m4 / nm;
        } else {
            r.e_mean = r.e2_mean = r.absm_mean = r.m2_mean = r.m4_mean = __builtin_nan("");
        }
        r.final_m[0] = a.final_m[0];
        r.final_m[1] = a.final_m[1];
        r.final_m[2] = a.final_m[2];
        r.final_e = a.final_e;
        r.n_accept = a.n_accept;
        out[g] = r;
    }
}

std::mutex g_mu;
char *g_scratch[MAX_DEV];  // device address of `scratch` on each device (null: not looked up yet)

int err(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int err(int code, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return mmc::report_error(code, buf);
}

// The default LDS batch variant of side L (the one mmc_batch_create starts from: the first LDS
// variant compiled for L, else the first generic one), or -1 when none fits.
int default_lds_variant(int fp64, int L, int max_lds)
{
    int n;
    const mmc::Variant *vs = mmc::batch_variants(fp64, &n);
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < n; ++i) {
            const mmc::Variant &v = vs[i];
            if (v.lds != 1 || v.L != (pass ? 0 : L)) continue;
            if (mmc::variant_lds_bytes(v, L) <= (size_t)max_lds) return i;
        }
    return -1;
}

}  // namespace

extern "C" int mmc_batch_run_static(const mmc_instance *inst, int n_inst, uint64_t seed, const mmc_config *cfg,
                                    mmc_path_result *out, void *hip_stream)
{
    if (!inst || !out) return err(MMC_EINVAL, "null instances or output");
    if (n_inst < 1 || n_inst > MAX_INST)
        return err(MMC_EINVAL, "n_inst = %d: the static batch takes 1 .. %d instances", n_inst, MAX_INST);
    mmc_config c0{};
    if (cfg) c0 = *cfg;
    if (c0.precision != MMC_FP32 && c0.precision != MMC_FP64) return err(MMC_EINVAL, "precision out of range");
    if (c0.model != MMC_MODEL_HEISENBERG3D || c0.proposal != MMC_PROPOSAL_SPHERE)
        return err(MMC_EUNSUPPORTED, "the static batch runs the Heisenberg model with the sphere proposal");
    if (c0.placement != MMC_PLACE_AUTO && c0.placement != MMC_PLACE_LDS)
        return err(MMC_EUNSUPPORTED, "the static batch keeps every lattice in LDS (placement AUTO or LDS)");
    if (c0.init < MMC_INIT_SPHERE || c0.init > MMC_INIT_MIXED) return err(MMC_EINVAL, "init out of range");
    const int fp64 = c0.precision == MMC_FP64;

    int dev = 0, n_cu = 0, max_lds = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) return err(MMC_EHIP, "no HIP device");
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return err(MMC_EHIP, "device attributes");
    char *base = nullptr;
    {
        // once per device, with that device current: the device address of its copy of scratch
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch[dev]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return err(MMC_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            if (mmc::prepare_kernels(max_lds) != hipSuccess) return err(MMC_EHIP, "kernel set-up failed");
            g_scratch[dev] = static_cast<char *>(p);
        }
        base = g_scratch[dev];
    }

    HostTables h;  // (stack)
    long long total = 0;
    for (int i = 0; i < n_inst; ++i) {
        const mmc_instance &x = inst[i];
        if (x.L < 2 || (x.L & 1) || (long long)x.L * x.L * x.L > (1LL << 30))
            return err(MMC_EINVAL, "instance %d: L = %d must be even, >= 2, L^3 <= 2^30", i, x.L);
        if (!(x.T > 0) || !isfinite(x.J) || x.n_paths < 1 || x.n_therm < 0 || x.n_meas < 0 ||
            (long long)x.n_therm + x.n_meas >= (1LL << 31))
            return err(MMC_EINVAL, "instance %d: need T > 0, finite J, n_paths >= 1, n_therm, n_meas >= 0", i);
        const int v = default_lds_variant(fp64, x.L, max_lds);
        if (v < 0)
            return err(MMC_EUNSUPPORTED, "instance %d: L = %d does not fit in LDS (the static batch has no device-memory spins)",
                       i, x.L);
        h.var[i] = v;
        h.path_off[i] = (int)total;
        total += x.n_paths;
        if (total > MAX_PATHS)
            return err(MMC_EINVAL, "%lld paths exceed the static batch's %d (scratch of %zu bytes)", total, MAX_PATHS,
                       (size_t)MMC_STATIC_SCRATCH_BYTES);
        mmc::InstDev &d = h.d[i];
        d = mmc::InstDev{};
        d.L = x.L;
        d.n_paths = x.n_paths;
        d.n_therm = x.n_therm;
        d.n_meas = x.n_meas;
        d.trace_sweeps = 0;
        d.init = c0.init;
        d.proposal = MMC_PROPOSAL_SPHERE;
        d.renorm_every = c0.renorm_every == 0 ? 64 : (c0.renorm_every < 0 ? 0 : c0.renorm_every);
        d.ctr3 = (uint32_t)i << 8;  // instance word = index, as in mmc_batch_create
        d.key0 = (uint32_t)seed;
        d.key1 = (uint32_t)(seed >> 32);
        d.beta = isinf(x.T) ? 0.0 : 1.0 / x.T;
        d.J = x.J;
        d.spins = nullptr;
        d.acc = reinterpret_cast<mmc::PathAcc *>(base + Layout::acc) + h.path_off[i];
        d.trace = nullptr;
    }
    h.path_off[n_inst] = (int)total;

    // one launch per variant in use; its items instance by instance, longest instances first
    int order[MAX_INST];
    for (int i = 0; i < n_inst; ++i) order[i] = i;
    auto cost = [&](int i) { return (double)inst[i].L * inst[i].L * inst[i].L * ((double)inst[i].n_therm + inst[i].n_meas); };
    for (int i = 1; i < n_inst; ++i)
        for (int j = i; j > 0 && cost(order[j]) > cost(order[j - 1]); --j) {
            const int t = order[j];
            order[j] = order[j - 1];
            order[j - 1] = t;
        }
    int lv[MAX_LAUNCH], lrun0[MAX_LAUNCH], lruns[MAX_LAUNCH], litems[MAX_LAUNCH], litem0[MAX_LAUNCH];
    int n_launch = 0, n_runs = 0, n_items = 0;
    for (int a = 0; a < n_inst; ++a) {
        const int v = h.var[order[a]];
        bool seen = false;
        for (int l = 0; l < n_launch; ++l) seen |= lv[l] == v;
        if (seen) continue;
        if (n_launch == MAX_LAUNCH) return err(MMC_EUNSUPPORTED, "more than %d kernel variants in one static batch", MAX_LAUNCH);
        const int l = n_launch++;
        lv[l] = v;
        lrun0[l] = n_runs;
        litem0[l] = n_items;
        int items = 0;
        for (int b = a; b < n_inst; ++b) {
            const int i = order[b];
            if (h.var[i] != v) continue;
            const int ppi = mmc::batch_paths_per_item(fp64, v);
            const int k = (inst[i].n_paths + ppi - 1) / ppi;
            h.runs[n_runs++] = Run{i, items, k, ppi};
            items += k;
        }
        lruns[l] = n_runs - lrun0[l];
        litems[l] = items;
        n_items += items;
    }

    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = upload(base + Layout::inst, h.d, sizeof(mmc::InstDev) * n_inst, s);
    if (e == hipSuccess) e = upload(base + Layout::var, h.var, sizeof(int) * n_inst, s);
    if (e == hipSuccess) e = upload(base + Layout::path_off, h.path_off, sizeof(int) * (n_inst + 1), s);
    if (e == hipSuccess) e = upload(base + Layout::runs, h.runs, sizeof(Run) * n_runs, s);
    if (e == hipSuccess) e = mmc::fill_zero(base + Layout::head, 64 * MAX_LAUNCH, s);
    int n;
    const mmc::Variant *vs = mmc::batch_variants(fp64, &n);
    for (int l = 0; l < n_launch && e == hipSuccess; ++l) {
        mmc::BatchItem *items = reinterpret_cast<mmc::BatchItem *>(base + Layout::items) + litem0[l];
        const int grid = (litems[l] + 255) / 256 < 1024 ? (litems[l] + 255) / 256 : 1024;
        hipLaunchKernelGGL(k_static_items, dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<const Run *>(base + Layout::runs), lrun0[l], lruns[l], litems[l], items);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        size_t lds = 0;
        for (int r = 0; r < lruns[l]; ++r) {
            const size_t b = mmc::variant_lds_bytes(vs[lv[l]], inst[h.runs[lrun0[l] + r].inst].L);
            lds = b > lds ? b : lds;
        }
        int per_cu = mmc::batch_blocks_per_cu(fp64, lv[l], lds);
        if (per_cu < 1) per_cu = 1;
        const int slots = per_cu * n_cu < litems[l] ? per_cu * n_cu : litems[l];
        mmc::BatchDev b;
        b.inst = reinterpret_cast<const mmc::InstDev *>(base + Layout::inst);
        b.variant = reinterpret_cast<const int *>(base + Layout::var);
        b.items = items;
        b.n_items = litems[l];
        b.head = reinterpret_cast<unsigned int *>(base + Layout::head + 64 * l);
        b.slots = nullptr;  // LDS variants never touch a spin slot
        b.slot_bytes = 0;
        b.n_slots = slots;
        e = mmc::launch_batch(b, fp64, lv[l], slots, lds, s);
    }
    if (e == hipSuccess) {
        const int grid = (int)((total + 255) / 256 < 1024 ? (total + 255) / 256 : 1024);
        hipLaunchKernelGGL(k_static_results, dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<const mmc::InstDev *>(base + Layout::inst),
                           reinterpret_cast<const int *>(base + Layout::path_off), n_inst,
                           reinterpret_cast<const mmc::PathAcc *>(base + Layout::acc), (int)total, out);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return err(MMC_EHIP, "static batch: %s", hipGetErrorString(e));
    return MMC_OK;
}
