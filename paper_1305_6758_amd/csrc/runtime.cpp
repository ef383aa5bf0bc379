// runtime.cpp -- host runtime of the multipath Metropolis engine: the C ABI of include/mmc.h.
// Owns validation, planning (variant choice and the tuner), device memory, hipGraph capture,
// timing, result readout, checkpoints and the batch work list.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mmc.h"
#include "engine.hpp"

namespace mmc {
// Host statistics of n path results of a lattice of N sites (stats.cpp).
int stats_of(const mmc_path_result *res, int n, double N, double T, mmc_stats_t *out);
}  // namespace mmc

namespace {

thread_local std::string g_last_error;
thread_local int g_last_status = MMC_OK;

// Diagnostics on stderr when the environment variable MMC_LOG is a positive number.
int log_level()
{
    static int level = -1;
    if (level < 0) {
        const char *e = getenv("MMC_LOG");
        level = e ? atoi(e) : 0;
        if (level < 0) level = 0;
    }
    return level;
}

void mmc_log(const char *fmt, ...)
{
    if (log_level() <= 0) return;
    va_list ap;
    va_start(ap, fmt);
    fprintf(stderr, "[mmc] ");
    vfprintf(stderr, fmt, ap);
    fprintf(stderr, "\n");
    va_end(ap);
}

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    g_last_status = code;
    return code;
}

}  // namespace

namespace mmc {
// The thread-local error of the C ABI, for the library's other translation units.
int report_error(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace mmc

namespace {

#define HIP_TRY(call)                                                                                     \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return fail(MMC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Instance {
    int L = 0;
    double T = 0, J = 0;
    int n_paths = 0, n_therm = 0, n_meas = 0;
    // plan
    int variant = -1;  // index into mmc::variants() (single) or mmc::batch_variants() (batch)
    bool plain = false;
    bool pinned = false;  // batch: variant fixed by mmc_set_variant, not tuned
    int member = -1;      // batch run by the fused kernel: the variant's member in it
    // device views (offsets into the workspace)
    size_t off_spins = 0, off_acc = 0, off_trace = 0;
};

struct GraphKey {
    int k0, k1, fresh;
    bool operator<(const GraphKey &o) const
    {
        return k0 != o.k0 ? k0 < o.k0 : (k1 != o.k1 ? k1 < o.k1 : fresh < o.fresh);
    }
};

}  // namespace

struct mmc_ctx {
    bool batch = false;
    mmc_config cfg{};
    uint64_t seed = 0;
    int fp64 = 0;
    std::vector<Instance> inst;
    // device
    int device = 0;
    hipStream_t stream = nullptr;       // the context's own stream (default priority)
    hipStream_t user_stream = nullptr;  // caller's stream to order against (may be null)
    bool bound_user_stream = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    bool ready = false;  // memory and plan in place
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_in = nullptr, ev_out = nullptr;
    // batch: a stream and a join event per graph branch after the first (default priority), so
    // the captured graph runs the variants' persistent kernels side by side
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;
    double last_ms = 0;
    int sweeps_done = 0;
    std::map<GraphKey, hipGraphExec_t> graphs;
    // single-instance extras
    size_t off_kdev = 0;
    // batch
    // one persistent launch per batch variant in use (or one fused launch), largest items
    // first, each with its own work list, queue head (64 bytes apart), resident workgroups,
    // LDS size and spin slots (the launches run side by side)
    struct Launch {
        bool fused = false;  // the fused kernel (the whole batch)
        int variant = 0;  // a variant of the launch's kernel (the first; the shared
                          // device-memory kernel serves several)
        std::string name;
        std::vector<mmc::BatchItem> items;
        size_t off_items = 0, lds = 0;
        int n_slots = 0;                       // resident workgroups (the grid)
        double updates = 0;                    // Metropolis attempts of its items
        size_t off_slots = 0, slot_bytes = 0;  // device-memory and split variants: this launch's spin slots
    };
    std::vector<Launch> launches;
    size_t off_inst = 0, off_var = 0, off_head = 0, off_slots = 0;
    size_t slot_area = 0;  // bytes of all launches' slots (the launches run side by side)
    bool fused_refused = false;  // batch_launch FUSED asked for, but a variant has no member
    int n_cu = 0;
    bool tuned = false;
};

size_t spin_bytes_of(const mmc_ctx *c, int L)
{
    if (c->cfg.model == MMC_MODEL_ISING2D) return mmc::ising_spin_bytes(L);  // padded byte rows
    return 3 * (size_t)L * L * L * (c->fp64 ? 8 : 4);
}

// Kernel variants of a single-instance context's model.
const mmc::Variant *single_table(const mmc_ctx *c, int *n)
{
    return c->cfg.model == MMC_MODEL_ISING2D ? mmc::ising_variants(n) : mmc::variants(n);
}

namespace {

bool valid_instance(int L, double T, double J, int n_paths, int n_therm, int n_meas, std::string &why)
{
    char b[256];
    if (L < 2 || (L & 1)) {
        snprintf(b, sizeof b, "L = %d: need an even L >= 2 (checkerboard on a periodic lattice)", L);
        why = b;
        return false;
    }
    if ((long long)L * L * L > (1LL << 30)) {
        why = "L too large";
        return false;
    }
    if (!(T > 0)) {
        why = "T must be > 0 (T = inf allowed)";
        return false;
    }
    if (!isfinite(J)) {
        why = "J must be finite";
        return false;
    }
    if (n_paths < 1 || n_therm < 0 || n_meas < 0 || (long long)n_therm + n_meas >= (1LL << 31)) {
        why = "need n_paths >= 1, n_therm >= 0, n_meas >= 0";
        return false;
    }
    return true;
}

mmc::InstDev inst_dev(const mmc_ctx *c, const Instance &in, uint32_t instance_id)
{
    mmc::InstDev d{};
    d.L = in.L;
    d.n_paths = in.n_paths;
    d.n_therm = in.n_therm;
    d.n_meas = in.n_meas;
    d.trace_sweeps = c->batch ? 0 : c->cfg.trace_sweeps;
    d.init = c->cfg.init;
    d.proposal = c->cfg.proposal;
    d.renorm_every = c->cfg.renorm_every == 0 ? 64 : (c->cfg.renorm_every < 0 ? 0 : c->cfg.renorm_every);
    d.ctr3 = instance_id << 8;
    d.key0 = (uint32_t)c->seed;
    d.key1 = (uint32_t)(c->seed >> 32);
    d.beta = isinf(in.T) ? 0.0 : 1.0 / in.T;
    d.J = in.J;
    d.spins = c->batch ? nullptr : c->ws + in.off_spins;
    d.acc = reinterpret_cast<mmc::PathAcc *>(c->ws + in.off_acc);
    d.trace = (!c->batch && c->cfg.trace_sweeps > 0) ? reinterpret_cast<double *>(c->ws + in.off_trace) : nullptr;
    if (c->cfg.model == MMC_MODEL_ISING2D) {
        // u = (w + 1/2) 2^-32 < p  <=>  w < ceil(p 2^32 - 1/2) for integer w (p 2^32 is exact
        // and the subtraction too, p < 2^20); p >= 1 - 2^-33 takes every word
        d.iall = 0;
        for (int i = 0; i < 5; ++i) {
            const double dE = 2.0 * in.J * (double)(2 * i - 4);
            const double p = exp(-d.beta * dE);
            const double t = ceil(p * 4294967296.0 - 0.5);
            if (t >= 4294967296.0) {
                d.iall |= 1u << i;
                d.ithr[i] = 0;
            } else {
                d.ithr[i] = (uint32_t)t;
            }
        }
    }
    return d;
}

int device_lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 64 * 1024;
    return v;
}

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string s = p.gcnArchName;
    const size_t colon = s.find(':');
    return colon == std::string::npos ? s : s.substr(0, colon);
}

// ---------------------------------------------------------------- tuning cache
std::mutex g_tune_mu;
std::map<std::string, std::string> g_tune_cache;
bool g_tune_loaded = false;

void tune_cache_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("MMC_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    fclose(f);
    // flat JSON object of string -> string
    size_t i = 0;
    auto next_str = [&](std::string &out) -> bool {
        size_t a = text.find('"', i);
        if (a == std::string::npos) return false;
        size_t b = text.find('"', a + 1);
        if (b == std::string::npos) return false;
        out = text.substr(a + 1, b - a - 1);
        i = b + 1;
        return true;
    };
    std::string k, v;
    while (next_str(k) && next_str(v)) g_tune_cache[k] = v;
}

void tune_cache_store()
{
    const char *path = getenv("MMC_TUNE_CACHE");
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto &kv : g_tune_cache)
        fprintf(f, "  \"%s\": \"%s\"%s\n", kv.first.c_str(), kv.second.c_str(), ++i < g_tune_cache.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

std::string tune_key(bool batch, int fp64, int L, int n_paths)
{
    int bucket = 0;
    while ((1 << (bucket + 1)) <= n_paths && bucket < 30) ++bucket;
    char b[128];
    snprintf(b, sizeof b, "%s|%s|%s|L%d|p2^%d", arch_name().c_str(), batch ? "batch" : "single", fp64 ? "f64" : "f32", L, bucket);
    return b;
}

// ---------------------------------------------------------------- candidates
// Variant::lds of the plane-ring variants (both colours, or colour 0 only, in the ring; one or
// two sweeps per pass): their spins live in device memory and stream through LDS, so they
// count as window placements, not LDS ones.
constexpr int LDS_RING = 4, LDS_HALF_RING = 5, LDS_RING2 = 6;
bool is_ring(const mmc::Variant &v) { return v.lds == LDS_RING || v.lds == LDS_HALF_RING || v.lds == LDS_RING2; }
bool lds_resident(const mmc::Variant &v) { return v.lds != 0 && !is_ring(v); }

bool variant_fits(const mmc::Variant &v, int fp64, int L, int lds_limit)
{
    if (v.fp64 != fp64) return false;
    if (v.L != 0 && v.L != L) return false;
    if ((v.lds || v.window) && mmc::variant_lds_bytes(v, L) > (size_t)lds_limit) return false;
    return true;
}

std::vector<int> single_candidates(const mmc_ctx *c, int L, bool keep_generic = false)
{
    int n;
    const mmc::Variant *vs = single_table(c, &n);
    const int lim = device_lds_limit();
    std::vector<int> out;
    if (c->cfg.model == MMC_MODEL_ISING2D) {
        // the variant compiled for this L, else the generic one if its LDS fits
        for (int i = 0; i < n; ++i)
            if (vs[i].L == L) out.push_back(i);
        if (out.empty() && mmc::ising_variant_lds_bytes(L) <= (size_t)lim)
            for (int i = 0; i < n; ++i)
                if (vs[i].L == 0) out.push_back(i);
        return out;
    }
    const int place = c->cfg.placement;
    for (int i = 0; i < n; ++i) {
        const mmc::Variant &v = vs[i];
        if (!variant_fits(v, c->fp64, L, lim)) continue;
        if (place == MMC_PLACE_LDS && !lds_resident(v)) continue;
        if (place == MMC_PLACE_HBM && (v.lds || v.window)) continue;
        if (place == MMC_PLACE_WINDOW && !v.window && !is_ring(v)) continue;
        if (c->cfg.block && v.block != c->cfg.block) continue;
        if (c->cfg.lanes_per_path && v.lanes != c->cfg.lanes_per_path) continue;
        out.push_back(i);
    }
    if (keep_generic) return out;
    // a generic variant only when no variant is compiled for this L
    bool have_exact = false;
    for (int i : out) have_exact |= vs[i].L == L;
    if (have_exact) out.erase(std::remove_if(out.begin(), out.end(), [&](int i) { return vs[i].L == 0; }), out.end());
    return out;
}

std::vector<int> batch_candidates(int fp64, int L, int placement, bool keep_generic = false)
{
    int n;
    const mmc::Variant *vs = mmc::batch_variants(fp64, &n);
    const size_t lds_budget = (size_t)device_lds_limit();
    std::vector<int> out;
    for (int i = 0; i < n; ++i) {
        const mmc::Variant &v = vs[i];
        if (v.L != 0 && v.L != L) continue;
        if (v.lds && mmc::variant_lds_bytes(v, L) > lds_budget) continue;
        if (placement == MMC_PLACE_LDS && !lds_resident(v)) continue;
        if (placement == MMC_PLACE_HBM && v.lds) continue;
        if (placement == MMC_PLACE_WINDOW && !is_ring(v)) continue;  // the batch window form
        out.push_back(i);
    }
    if (keep_generic) return out;
    bool have_exact = false;
    for (int i : out) have_exact |= vs[i].L == L;
    if (have_exact) out.erase(std::remove_if(out.begin(), out.end(), [&](int i) { return vs[i].L == 0; }), out.end());
    return out;
}

int ensure_device(mmc_ctx *c)
{
    if (c->stream) return MMC_OK;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(MMC_EHIP, "no HIP device available (%s)", hipGetErrorString(e));
    HIP_TRY(hipGetDevice(&c->device));
    HIP_TRY(mmc::prepare_kernels(device_lds_limit()));
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreate(&c->ev0));
    HIP_TRY(hipEventCreate(&c->ev1));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    return MMC_OK;
}

// ---------------------------------------------------------------- workspace layout
size_t layout_single(mmc_ctx *c)
{
    Instance &in = c->inst[0];
    size_t off = 0;
    in.off_spins = off;
    off = align_up(off + (size_t)in.n_paths * spin_bytes_of(c, in.L));
    in.off_acc = off;
    off = align_up(off + (size_t)in.n_paths * sizeof(mmc::PathAcc));
    in.off_trace = off;
    off = align_up(off + (size_t)in.n_paths * (size_t)std::max(c->cfg.trace_sweeps, 0) * 4 * sizeof(double));
    c->off_kdev = off;
    off = align_up(off + 4 * sizeof(int));
    return off;
}

size_t layout_batch(mmc_ctx *c)
{
    size_t off = 0;
    for (Instance &in : c->inst) {
        in.off_acc = off;
        off = align_up(off + (size_t)in.n_paths * sizeof(mmc::PathAcc));
    }
    c->off_inst = off;
    off = align_up(off + c->inst.size() * sizeof(mmc::InstDev));
    c->off_var = off;
    off = align_up(off + c->inst.size() * sizeof(int));
    for (auto &l : c->launches) {
        l.off_items = off;
        off = align_up(off + l.items.size() * sizeof(mmc::BatchItem));
    }
    c->off_head = off;
    off = align_up(off + 64 * std::max<size_t>(1, c->launches.size()));
    c->off_slots = off;
    off = align_up(off + c->slot_area);
    return off;
}

int ensure_memory(mmc_ctx *c)
{
    int rc = ensure_device(c);
    if (rc) return rc;
    if (c->ws) return MMC_OK;
    hipError_t e = hipMalloc(&c->ws, c->ws_bytes);
    if (e == hipErrorOutOfMemory) {
        c->ws = nullptr;
        (void)hipGetLastError();  // not sticky: clear it for the caller's next HIP call
        return fail(MMC_ENOMEM, "device memory: %zu bytes do not fit", c->ws_bytes);
    }
    if (e != hipSuccess) return fail(MMC_EHIP, "hipMalloc of %zu bytes: %s", c->ws_bytes, hipGetErrorString(e));
    c->own_ws = true;
    return MMC_OK;
}

void drop_graphs(mmc_ctx *c)
{
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

// Stream ordering against the caller's stream.
int begin_work(mmc_ctx *c)
{
    if (c->bound_user_stream) {
        HIP_TRY(hipEventRecord(c->ev_in, c->user_stream));
        HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_in, 0));
    }
    return MMC_OK;
}

int end_work(mmc_ctx *c)
{
    if (c->bound_user_stream) {
        HIP_TRY(hipEventRecord(c->ev_out, c->stream));
        HIP_TRY(hipStreamWaitEvent(c->user_stream, c->ev_out, 0));
    }
    return MMC_OK;
}

// ---------------------------------------------------------------- single-instance launches
// Enqueues sweeps [k0, k1) of the single instance (fresh: initial state first).
int enqueue_single(mmc_ctx *c, int k0, int k1, bool fresh, hipStream_t s)
{
    const Instance &in = c->inst[0];
    mmc::InstDev d = inst_dev(c, in, c->cfg.instance_id);
    if (fresh && d.trace) {
        hipError_t e = mmc::fill_nan(d.trace, (size_t)in.n_paths * c->cfg.trace_sweeps * 4, s);
        if (e != hipSuccess) return fail(MMC_EHIP, "trace fill: %s", hipGetErrorString(e));
    }
    if (in.plain) {
        int *kdev = reinterpret_cast<int *>(c->ws + c->off_kdev);
        hipError_t e;
        if (fresh && (e = mmc::plain_init(d, s)) != hipSuccess) return fail(MMC_EHIP, "plain init: %s", hipGetErrorString(e));
        if ((e = mmc::set_int(kdev, k0, s)) != hipSuccess) return fail(MMC_EHIP, "set k: %s", hipGetErrorString(e));
        if ((e = mmc::set_int(kdev + 1, 0, s)) != hipSuccess) return fail(MMC_EHIP, "set k: %s", hipGetErrorString(e));
        for (int k = k0; k < k1; ++k) {
            if ((e = mmc::plain_half(d, kdev, 0, s)) != hipSuccess) return fail(MMC_EHIP, "plain half: %s", hipGetErrorString(e));
            if ((e = mmc::plain_half(d, kdev, 1, s)) != hipSuccess) return fail(MMC_EHIP, "plain half: %s", hipGetErrorString(e));
            if ((e = mmc::plain_measure(d, kdev, k1 - 1, s)) != hipSuccess) return fail(MMC_EHIP, "plain measure: %s", hipGetErrorString(e));
        }
        return MMC_OK;
    }
    int n;
    const mmc::Variant *vs = single_table(c, &n);
    hipError_t e = vs[in.variant].launch(d, k0, k1, fresh ? 1 : 0, s);
    if (e != hipSuccess) return fail(MMC_EHIP, "launch %s: %s", vs[in.variant].name, hipGetErrorString(e));
    return MMC_OK;
}

// Captures (once) and launches the graph of sweeps [k0, k1); times it with events.
int run_graph(mmc_ctx *c, int k0, int k1, bool fresh)
{
    GraphKey key{k0, k1, fresh ? 1 : 0};
    auto it = c->graphs.find(key);
    hipGraphExec_t exec = nullptr;
    if (it != c->graphs.end()) {
        exec = it->second;
    } else {
        if (c->graphs.size() > 8) drop_graphs(c);
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        int rc = c->batch ? MMC_EUNSUPPORTED : enqueue_single(c, k0, k1, fresh, c->stream);
        hipError_t ec = hipStreamEndCapture(c->stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ec != hipSuccess) return fail(MMC_EHIP, "graph capture: %s", hipGetErrorString(ec));
        hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(MMC_EHIP, "graph instantiate: %s", hipGetErrorString(ei));
        c->graphs[key] = exec;
    }
    int rc = begin_work(c);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    HIP_TRY(hipGraphLaunch(exec, c->stream));
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    return end_work(c);
}

int finish(mmc_ctx *c)
{
    HIP_TRY(hipEventSynchronize(c->ev1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms = ms;
    return MMC_OK;
}

int total_sweeps(const Instance &in) { return in.n_therm + in.n_meas; }

// Times one candidate variant on the context's own buffers (results are discarded).
double time_single_candidate(mmc_ctx *c, int variant, int sweeps)
{
    Instance &in = c->inst[0];
    const int saved_variant = in.variant;
    in.variant = variant;
    mmc::InstDev d = inst_dev(c, in, c->cfg.instance_id);
    d.trace_sweeps = 0;
    d.trace = nullptr;
    int n;
    const mmc::Variant *vs = single_table(c, &n);
    double best = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
        if (hipEventRecord(c->ev0, c->stream) != hipSuccess) break;
        if (vs[variant].launch(d, 0, sweeps, 1, c->stream) != hipSuccess) {
            best = 1e30;
            break;
        }
        (void)hipEventRecord(c->ev1, c->stream);
        if (hipEventSynchronize(c->ev1) != hipSuccess) {
            best = 1e30;
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
        best = std::min(best, (double)ms);
    }
    in.variant = saved_variant;
    return best;
}

int plan_single(mmc_ctx *c)
{
    Instance &in = c->inst[0];
    if (c->cfg.placement == MMC_PLACE_PLAIN) {
        if (!c->fp64) return fail(MMC_EUNSUPPORTED, "the plain engine is FP64 only");
        in.plain = true;
        return MMC_OK;
    }
    std::vector<int> cand = single_candidates(c, in.L);
    if (cand.empty()) return fail(MMC_EUNSUPPORTED, "no kernel variant for L=%d with this configuration", in.L);
    in.variant = cand[0];
    int nv;
    mmc_log("plan L=%d paths=%d: %zu candidate(s), first %s", in.L, in.n_paths, cand.size(),
            single_table(c, &nv)[in.variant].name);
    return MMC_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *mmc_last_error(void) { return g_last_error.c_str(); }

int mmc_last_status(void) { return g_last_status; }

mmc_ctx *mmc_create_ex(int L, double T, double J, int n_paths, int n_therm, int n_meas, uint64_t seed,
                       const mmc_config *cfg)
{
    std::string why;
    if (!valid_instance(L, T, J, n_paths, n_therm, n_meas, why)) {
        fail(MMC_EINVAL, "%s", why.c_str());
        return nullptr;
    }
    mmc_config c0{};
    if (cfg) c0 = *cfg;
    if (c0.precision != MMC_FP32 && c0.precision != MMC_FP64) {
        fail(MMC_EINVAL, "precision must be MMC_FP32 or MMC_FP64");
        return nullptr;
    }
    if (c0.init < MMC_INIT_SPHERE || c0.init > MMC_INIT_MIXED || c0.placement < 0 || c0.placement > MMC_PLACE_WINDOW ||
        c0.proposal < MMC_PROPOSAL_SPHERE || c0.proposal > MMC_PROPOSAL_ANGLES ||
        c0.block < 0 || c0.lanes_per_path < 0 || c0.trace_sweeps < 0 || c0.instance_id >= (1u << 24)) {
        fail(MMC_EINVAL, "configuration out of range");
        return nullptr;
    }
    if (c0.model != MMC_MODEL_HEISENBERG3D && c0.model != MMC_MODEL_ISING2D) {
        fail(MMC_EINVAL, "model must be MMC_MODEL_HEISENBERG3D or MMC_MODEL_ISING2D");
        return nullptr;
    }
    if (c0.model == MMC_MODEL_ISING2D) {
        if (c0.placement != MMC_PLACE_AUTO && c0.placement != MMC_PLACE_LDS) {
            fail(MMC_EUNSUPPORTED, "the Ising model runs with its spins in LDS only");
            return nullptr;
        }
        if (c0.init == MMC_INIT_ANGLES || c0.proposal != MMC_PROPOSAL_SPHERE || c0.block || c0.lanes_per_path) {
            fail(MMC_EINVAL, "Ising: init must be SPHERE (random), ORDERED or MIXED; no proposal, block or lane choice");
            return nullptr;
        }
        c0.precision = MMC_FP32;  // integer spins; the statistics are FP64 either way
    }
    if (c0.trace_sweeps > n_therm + n_meas) c0.trace_sweeps = n_therm + n_meas;
    mmc_ctx *c = new mmc_ctx;
    c->cfg = c0;
    c->seed = seed;
    c->fp64 = c0.precision == MMC_FP64;
    Instance in;
    in.L = L;
    in.T = T;
    in.J = J;
    in.n_paths = n_paths;
    in.n_therm = n_therm;
    in.n_meas = n_meas;
    c->inst.push_back(in);
    c->ws_bytes = layout_single(c);
    if (c0.placement == MMC_PLACE_PLAIN && !c->fp64) {
        fail(MMC_EUNSUPPORTED, "the plain engine is FP64 only");
        delete c;
        return nullptr;
    }
    if (c0.proposal == MMC_PROPOSAL_ANGLES && c0.placement != MMC_PLACE_PLAIN) {
        fail(MMC_EUNSUPPORTED, "the both-angles proposal runs on the plain FP64 engine only");
        delete c;
        return nullptr;
    }
    return c;
}

mmc_ctx *mmc_create(int L, double T, double J, int n_paths, int n_therm, int n_meas, uint64_t seed)
{
    return mmc_create_ex(L, T, J, n_paths, n_therm, n_meas, seed, nullptr);
}

size_t mmc_workspace_bytes(const mmc_ctx *c) { return c ? c->ws_bytes : 0; }

int mmc_bind(mmc_ctx *c, void *dev_ptr, size_t bytes, void *hip_stream)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (c->ws) return fail(MMC_ESTATE, "memory already in place (bind before the first run)");
    if (!dev_ptr || bytes < c->ws_bytes) return fail(MMC_ENOMEM, "bound buffer of %zu bytes < %zu needed", bytes, c->ws_bytes);
    if ((uintptr_t)dev_ptr % ALIGN) return fail(MMC_EINVAL, "bound buffer must be %zu-byte aligned", ALIGN);
    int rc = ensure_device(c);
    if (rc) return rc;
    c->ws = reinterpret_cast<char *>(dev_ptr);
    c->own_ws = false;
    c->user_stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->bound_user_stream = true;
    return MMC_OK;
}

static int prepare(mmc_ctx *c)
{
    if (c->ready) return MMC_OK;
    int rc = ensure_memory(c);
    if (rc) return rc;
    if (c->batch) return MMC_OK;
    rc = plan_single(c);
    if (rc) return rc;
    c->ready = true;
    return MMC_OK;
}

int mmc_tune(mmc_ctx *c)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (c->batch) return MMC_OK;  // batch contexts are planned at creation
    int rc = prepare(c);
    if (rc) return rc;
    Instance &in = c->inst[0];
    if (in.plain || c->tuned) return MMC_OK;
    std::vector<int> cand = single_candidates(c, in.L);
    if (cand.size() <= 1) {
        c->tuned = true;
        return MMC_OK;
    }
    int n;
    const mmc::Variant *vs = single_table(c, &n);
    const std::string key = tune_key(false, c->fp64, in.L, in.n_paths);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end())
            for (int i : cand)
                if (it->second == vs[i].name) {
                    in.variant = i;
                    c->tuned = true;
                    return MMC_OK;
                }
    }
    if (c->sweeps_done) return fail(MMC_ESTATE, "tuning needs a context that has not run yet");
    // ~1 G updates per candidate (a few ms: shorter trials were swayed by clock ramps), in whole
    // passes of every window depth (1, 2, 3 sweeps): a short last pass would charge a window
    // variant a pipeline fill the long run does not pay
    const double per_sweep = (double)in.L * in.L * in.L * in.n_paths;
    const int sweeps = 6 * (int)ceil(std::min(64.0, std::max(2.0, 1e9 / per_sweep)) / 6.0);
    int best = cand[0];
    double best_ms = 1e30;
    // the candidates write the workspace: with caller memory bound, they wait for the work
    // already queued on the caller's stream, and the caller's later work waits for them
    int rc_order = begin_work(c);
    if (rc_order) return rc_order;
    for (int i : cand) {
        time_single_candidate(c, i, 1);  // warm-up (code load)
        const double ms = std::min(time_single_candidate(c, i, sweeps), time_single_candidate(c, i, sweeps));
        if (ms < best_ms) {
            best_ms = ms;
            best = i;
        }
    }
    rc_order = end_work(c);
    if (rc_order) return rc_order;
    if (best_ms >= 1e30) return fail(MMC_EHIP, "every tuning candidate failed to launch");
    in.variant = best;
    c->tuned = true;
    mmc_log("tuned L=%d paths=%d: %s (%.3f ms for %d sweeps)", in.L, in.n_paths, vs[best].name, best_ms, sweeps);
    drop_graphs(c);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = vs[best].name;
    tune_cache_store();
    return MMC_OK;
}

static void batch_plan(mmc_ctx *c);

int mmc_set_variant(mmc_ctx *c, const char *name)
{
    if (!c || !name) return fail(MMC_EINVAL, "null argument");
    if (c->sweeps_done) return fail(MMC_ESTATE, "the context has already run");
    if (c->batch) {
        // every instance whose L the named batch variant serves
        if (c->ws) return fail(MMC_ESTATE, "pin batch variants before mmc_bind and the first run");
        int nv;
        const mmc::Variant *vs = mmc::batch_variants(c->fp64, &nv);
        int hits = 0;
        for (Instance &in : c->inst)
            for (int v : batch_candidates(c->fp64, in.L, c->cfg.placement, true))
                if (strcmp(vs[v].name, name) == 0) {
                    in.variant = v;
                    in.pinned = true;
                    ++hits;
                }
        if (!hits) return fail(MMC_EINVAL, "batch variant '%s' fits no instance of this batch", name);
        drop_graphs(c);
        batch_plan(c);
        mmc_log("batch variant pinned: %s (%d instance(s))", name, hits);
        return MMC_OK;
    }
    int rc = prepare(c);
    if (rc) return rc;
    Instance &in = c->inst[0];
    if (in.plain) return fail(MMC_EUNSUPPORTED, "the plain engine has no kernel variants");
    int n;
    const mmc::Variant *vs = single_table(c, &n);
    for (int i : single_candidates(c, in.L, true))
        if (strcmp(vs[i].name, name) == 0) {
            in.variant = i;
            c->tuned = true;
            drop_graphs(c);
            mmc_log("variant pinned: %s", name);
            return MMC_OK;
        }
    return fail(MMC_EINVAL, "variant '%s' does not fit this context (L=%d)", name, in.L);
}

static int run_to(mmc_ctx *c, int k_end, bool wait)
{
    int rc = prepare(c);
    if (rc) return rc;
    if (!c->tuned && c->cfg.placement != MMC_PLACE_PLAIN && !(c->cfg.block && c->cfg.lanes_per_path)) {
        rc = mmc_tune(c);
        if (rc) return rc;
    }
    const int k0 = c->sweeps_done;
    if (k_end <= k0) return MMC_OK;
    rc = run_graph(c, k0, k_end, k0 == 0);
    if (rc) return rc;
    c->sweeps_done = k_end;
    return wait ? finish(c) : MMC_OK;
}

int mmc_run(mmc_ctx *c)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (c->batch) return mmc_batch_run(c);
    const Instance &in = c->inst[0];
    if (c->sweeps_done >= total_sweeps(in) && c->sweeps_done > 0) return fail(MMC_ESTATE, "all sweeps already run (mmc_reset to start over)");
    if (total_sweeps(in) == 0) return fail(MMC_EINVAL, "n_therm + n_meas = 0: nothing to run");
    return run_to(c, total_sweeps(in), !c->cfg.async);
}

int mmc_run_sweeps(mmc_ctx *c, int k)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (c->batch) return fail(MMC_EUNSUPPORTED, "mmc_run_sweeps is not available on a batch");
    const Instance &in = c->inst[0];
    if (k < 1 || c->sweeps_done + (long long)k > total_sweeps(in)) return fail(MMC_EINVAL, "k = %d out of range", k);
    return run_to(c, c->sweeps_done + k, !c->cfg.async);
}

int mmc_sync(mmc_ctx *c)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (!c->stream) return MMC_OK;
    return finish(c);
}

int mmc_reset(mmc_ctx *c)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
    c->sweeps_done = 0;
    return MMC_OK;
}

int mmc_sweeps_done(const mmc_ctx *c) { return c ? c->sweeps_done : MMC_EINVAL; }

static int read_acc(const mmc_ctx *c, const Instance &in, std::vector<mmc::PathAcc> &acc)
{
    acc.resize(in.n_paths);
    if (!c->ws) return fail(MMC_ESTATE, "nothing has run yet");
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(acc.data(), c->ws + in.off_acc, acc.size() * sizeof(mmc::PathAcc), hipMemcpyDeviceToHost));
    return MMC_OK;
}

static void acc_to_result(const mmc::PathAcc &a, int n_meas, mmc_path_result &r)
{
    const double nm = (double)n_meas;
    if (n_meas > 0) {
        r.e_mean = a.sum_e / nm;
        r.e2_mean = a.sum_e2 / nm;
        r.absm_mean = a.sum_m / nm;
        r.m2_mean = a.sum_m2 / nm;
        r.m4_mean = a.sum_m4 / nm;
    } else {
        r.e_mean = r.e2_mean = r.absm_mean = r.m2_mean = r.m4_mean = NAN;
    }
    r.final_e = a.final_e;
    r.final_m[0] = a.final_m[0];
    r.final_m[1] = a.final_m[1];
    r.final_m[2] = a.final_m[2];
    r.n_accept = a.n_accept;
}

static int results_of(const mmc_ctx *c, const Instance &in, int done, mmc_path_result *out, int n_out)
{
    if (!out || n_out < in.n_paths) return fail(MMC_EINVAL, "output holds %d results, need %d", n_out, in.n_paths);
    if (done == 0) return fail(MMC_ESTATE, "nothing has run yet");
    std::vector<mmc::PathAcc> acc;
    int rc = read_acc(c, in, acc);
    if (rc) return rc;
    // measured sweeps completed so far
    const int measured = std::max(0, done - in.n_therm);
    for (int p = 0; p < in.n_paths; ++p) acc_to_result(acc[p], measured, out[p]);
    return MMC_OK;
}

int mmc_results(const mmc_ctx *c, mmc_path_result *out, int n_out)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (c->batch) return fail(MMC_EINVAL, "use mmc_batch_results on a batch");
    return results_of(c, c->inst[0], c->sweeps_done, out, n_out);
}

int mmc_trace(const mmc_ctx *c, double *out, size_t n_out)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (c->batch) return fail(MMC_EUNSUPPORTED, "no trace on a batch");
    const Instance &in = c->inst[0];
    const size_t need = (size_t)in.n_paths * c->cfg.trace_sweeps * 4;
    if (c->cfg.trace_sweeps <= 0) return fail(MMC_ESTATE, "trace_sweeps = 0");
    if (!out || n_out < need) return fail(MMC_EINVAL, "trace output needs %zu doubles", need);
    if (!c->ws || c->sweeps_done == 0) return fail(MMC_ESTATE, "nothing has run yet");
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(out, c->ws + in.off_trace, need * sizeof(double), hipMemcpyDeviceToHost));
    return MMC_OK;
}

int mmc_spin_norm_deviation(const mmc_ctx *c, double *max_dev)
{
    if (!c || !max_dev) return fail(MMC_EINVAL, "null argument");
    if (c->batch) return fail(MMC_EUNSUPPORTED, "no resident spins on a batch");
    if (c->cfg.model != MMC_MODEL_HEISENBERG3D) return fail(MMC_EUNSUPPORTED, "Ising spins are +-1 by construction");
    if (!c->ws || c->sweeps_done == 0) return fail(MMC_ESTATE, "nothing has run yet");
    const Instance &in = c->inst[0];
    HIP_TRY(hipStreamSynchronize(c->stream));
    const size_t bytes = (size_t)in.n_paths * spin_bytes_of(c, in.L);
    std::vector<char> raw(bytes);
    HIP_TRY(hipMemcpy(raw.data(), c->ws + in.off_spins, bytes, hipMemcpyDeviceToHost));
    // [path][colour][component][N/2]: |S|^2 of site h of colour c gathers three words
    const size_t HALF = (size_t)in.L * in.L * in.L / 2;
    double worst = 0.0;
    for (size_t p = 0; p < (size_t)in.n_paths; ++p)
        for (size_t col = 0; col < 2; ++col)
            for (size_t h = 0; h < HALF; ++h) {
                double r2 = 0.0;
                for (size_t a = 0; a < 3; ++a) {
                    const size_t w = ((p * 2 + col) * 3 + a) * HALF + h;
                    const double v = c->fp64 ? reinterpret_cast<const double *>(raw.data())[w]
                                             : (double)reinterpret_cast<const float *>(raw.data())[w];
                    r2 += v * v;
                }
                const double d = fabs(sqrt(r2) - 1.0);
                if (!(d <= worst)) worst = d;  // a NaN spin makes the deviation NaN
            }
    *max_dev = worst;
    return MMC_OK;
}

int mmc_get_spins(const mmc_ctx *c, int path, double *xyz, size_t n_out)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (c->batch) return fail(MMC_EUNSUPPORTED, "no resident spins on a batch");
    const Instance &in = c->inst[0];
    const int L = in.L, HL = L / 2;
    const size_t N = (size_t)L * L * (c->cfg.model == MMC_MODEL_ISING2D ? 1 : L), HALF = N / 2;
    if (path < 0 || path >= in.n_paths) return fail(MMC_EINVAL, "path %d out of range", path);
    if (!xyz || n_out < 3 * N) return fail(MMC_EINVAL, "spin output needs %zu doubles", 3 * N);
    if (!c->ws || c->sweeps_done == 0) return fail(MMC_ESTATE, "nothing has run yet");
    HIP_TRY(hipStreamSynchronize(c->stream));
    const size_t bytes = spin_bytes_of(c, L);
    if (c->cfg.model == MMC_MODEL_ISING2D) {
        // [colour][y][row stride] bytes b = (s + 1)/2 at x >> 1; s goes to the z component of x + L y
        if (n_out < 3 * (size_t)L * L) return fail(MMC_EINVAL, "spin output needs %zu doubles", 3 * (size_t)L * L);
        const size_t RS = (size_t)mmc::ising_row_stride(L);
        std::vector<uint8_t> raw(bytes);
        HIP_TRY(hipMemcpy(raw.data(), c->ws + in.off_spins + (size_t)path * bytes, bytes, hipMemcpyDeviceToHost));
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const size_t i = (size_t)x + (size_t)L * y;
                const int colour = (x + y) & 1;
                xyz[3 * i + 0] = 0.0;
                xyz[3 * i + 1] = 0.0;
                xyz[3 * i + 2] = 2.0 * raw[(size_t)colour * L * RS + (size_t)y * RS + (x >> 1)] - 1.0;
            }
        return MMC_OK;
    }
    std::vector<char> raw(bytes);
    HIP_TRY(hipMemcpy(raw.data(), c->ws + in.off_spins + (size_t)path * bytes, bytes, hipMemcpyDeviceToHost));
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const size_t i = (size_t)x + (size_t)L * (y + (size_t)L * z);
                const int colour = (x + y + z) & 1;
                const size_t h = (size_t)(x >> 1) + (size_t)HL * (y + (size_t)L * z);
                for (int a = 0; a < 3; ++a) {
                    const size_t w = (size_t)colour * 3 * HALF + (size_t)a * HALF + h;
                    xyz[3 * i + a] = c->fp64 ? reinterpret_cast<const double *>(raw.data())[w]
                                             : (double)reinterpret_cast<const float *>(raw.data())[w];
                }
            }
    return MMC_OK;
}

int mmc_stats(const mmc_ctx *c, mmc_stats_t *out)
{
    if (!c || !out) return fail(MMC_EINVAL, "null argument");
    if (c->batch) return fail(MMC_EINVAL, "use mmc_batch_stats on a batch");
    const Instance &in = c->inst[0];
    std::vector<mmc_path_result> r(in.n_paths);
    int rc = mmc_results(c, r.data(), in.n_paths);
    if (rc) return rc;
    const double N = (double)in.L * in.L * (c->cfg.model == MMC_MODEL_ISING2D ? 1 : in.L);
    rc = mmc::stats_of(r.data(), in.n_paths, N, in.T, out);
    if (rc) return rc;
    double acc = 0;
    for (auto &x : r) acc += (double)x.n_accept;
    out->accept_rate = acc / ((double)in.n_paths * c->sweeps_done * N);
    return MMC_OK;
}

// ---------------------------------------------------------------- checkpoints
static const char k_magic[8] = {'M', 'M', 'C', 'C', 'K', 'P', 'T', '3'};

int mmc_save(const mmc_ctx *c, const char *file)
{
    if (!c || !file) return fail(MMC_EINVAL, "null argument");
    if (c->batch) return fail(MMC_EUNSUPPORTED, "checkpoints are not available on a batch");
    if (!c->ws || !c->ready) return fail(MMC_ESTATE, "nothing to save before the first run");
    const Instance &in = c->inst[0];
    HIP_TRY(hipStreamSynchronize(c->stream));
    const size_t sb = (size_t)in.n_paths * spin_bytes_of(c, in.L);
    const size_t ab = (size_t)in.n_paths * sizeof(mmc::PathAcc);
    const size_t tb = (size_t)in.n_paths * c->cfg.trace_sweeps * 4 * sizeof(double);
    std::vector<char> buf(sb + ab + tb);
    HIP_TRY(hipMemcpy(buf.data(), c->ws + in.off_spins, sb, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(buf.data() + sb, c->ws + in.off_acc, ab, hipMemcpyDeviceToHost));
    if (tb) HIP_TRY(hipMemcpy(buf.data() + sb + ab, c->ws + in.off_trace, tb, hipMemcpyDeviceToHost));
    int n;
    const mmc::Variant *vs = single_table(c, &n);
    char vname[64] = {0};
    snprintf(vname, sizeof vname, "%s", in.plain ? "plain" : vs[in.variant].name);
    FILE *f = fopen(file, "wb");
    if (!f) return fail(MMC_EIO, "cannot open %s for writing", file);
    bool ok = fwrite(k_magic, 1, 8, f) == 8;
    ok = ok && fwrite(&in.L, sizeof(int), 1, f) == 1 && fwrite(&in.T, sizeof(double), 1, f) == 1 &&
         fwrite(&in.J, sizeof(double), 1, f) == 1 && fwrite(&in.n_paths, sizeof(int), 1, f) == 1 &&
         fwrite(&in.n_therm, sizeof(int), 1, f) == 1 && fwrite(&in.n_meas, sizeof(int), 1, f) == 1 &&
         fwrite(&c->seed, sizeof(uint64_t), 1, f) == 1 && fwrite(&c->cfg, sizeof(mmc_config), 1, f) == 1 &&
         fwrite(&c->sweeps_done, sizeof(int), 1, f) == 1 && fwrite(vname, 1, 64, f) == 64;
    const uint64_t nbytes = buf.size();
    ok = ok && fwrite(&nbytes, sizeof nbytes, 1, f) == 1 && fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? MMC_OK : fail(MMC_EIO, "write to %s failed", file);
}

mmc_ctx *mmc_load(const char *file)
{
    if (!file) {
        fail(MMC_EINVAL, "null file name");
        return nullptr;
    }
    FILE *f = fopen(file, "rb");
    if (!f) {
        fail(MMC_EIO, "cannot open %s", file);
        return nullptr;
    }
    char magic[8];
    int L, n_paths, n_therm, n_meas, done;
    double T, J;
    uint64_t seed, nbytes;
    mmc_config cfg;
    char vname[64];
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, k_magic, 8) == 0;
    ok = ok && fread(&L, sizeof(int), 1, f) == 1 && fread(&T, sizeof(double), 1, f) == 1 &&
         fread(&J, sizeof(double), 1, f) == 1 && fread(&n_paths, sizeof(int), 1, f) == 1 &&
         fread(&n_therm, sizeof(int), 1, f) == 1 && fread(&n_meas, sizeof(int), 1, f) == 1 &&
         fread(&seed, sizeof(uint64_t), 1, f) == 1 && fread(&cfg, sizeof(mmc_config), 1, f) == 1 &&
         fread(&done, sizeof(int), 1, f) == 1 && fread(vname, 1, 64, f) == 64 && fread(&nbytes, sizeof nbytes, 1, f) == 1;
    if (!ok) {
        fclose(f);
        fail(MMC_EIO, "%s is not a checkpoint", file);
        return nullptr;
    }
    vname[63] = 0;
    // sweeps_done indexes the trace and divides the measured sums: it must be a sweep count
    // of this run
    if (done < 0 || (long long)done > (long long)n_therm + n_meas) {
        fclose(f);
        fail(MMC_EIO, "%s: sweep count %d outside 0..%lld", file, done, (long long)n_therm + n_meas);
        return nullptr;
    }
    mmc_ctx *c = mmc_create_ex(L, T, J, n_paths, n_therm, n_meas, seed, &cfg);
    if (!c) {
        fclose(f);
        return nullptr;
    }
    Instance &in = c->inst[0];
    const size_t sb = (size_t)n_paths * spin_bytes_of(c, L);
    const size_t ab = (size_t)n_paths * sizeof(mmc::PathAcc);
    const size_t tb = (size_t)n_paths * c->cfg.trace_sweeps * 4 * sizeof(double);
    std::vector<char> buf(sb + ab + tb);
    if (nbytes != buf.size() || fread(buf.data(), 1, buf.size(), f) != buf.size()) {
        fclose(f);
        mmc_destroy(c);
        fail(MMC_EIO, "%s: truncated or inconsistent checkpoint", file);
        return nullptr;
    }
    fclose(f);
    if (prepare(c) != MMC_OK) {
        mmc_destroy(c);
        return nullptr;
    }
    // same kernel variant as the saved run (bit-identical continuation needs nothing more,
    // but keeping it avoids a tuning run on a context that has state)
    if (!in.plain) {
        int n;
        const mmc::Variant *vs = single_table(c, &n);
        for (int i = 0; i < n; ++i)
            if (strcmp(vs[i].name, vname) == 0) in.variant = i;
    }
    c->tuned = true;
    if (hipMemcpy(c->ws + in.off_spins, buf.data(), sb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->ws + in.off_acc, buf.data() + sb, ab, hipMemcpyHostToDevice) != hipSuccess ||
        (tb && hipMemcpy(c->ws + in.off_trace, buf.data() + sb + ab, tb, hipMemcpyHostToDevice) != hipSuccess)) {
        mmc_destroy(c);
        fail(MMC_EHIP, "upload of checkpoint state failed");
        return nullptr;
    }
    c->sweeps_done = done;
    return c;
}

double mmc_last_timing_ms(const mmc_ctx *c) { return c ? c->last_ms : -1.0; }

int mmc_proposal_vectors(int precision, int proposal, const uint32_t *words, int64_t n, double *xyz)
{
    if (!words || !xyz || n < 1 || n > (1LL << 31)) return fail(MMC_EINVAL, "need words, xyz and 1 <= n <= 2^31");
    if ((precision != MMC_FP32 && precision != MMC_FP64) ||
        (proposal != MMC_PROPOSAL_SPHERE && proposal != MMC_PROPOSAL_ANGLES))
        return fail(MMC_EINVAL, "precision or proposal out of range");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(MMC_EHIP, "no HIP device available (%s)", hipGetErrorString(e));
    uint32_t *dw = nullptr;
    double *dx = nullptr;
    hipStream_t s = nullptr;
    const size_t wb = (size_t)n * 2 * sizeof(uint32_t), xb = (size_t)n * 3 * sizeof(double);
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&dw, wb);
    if (e == hipSuccess) e = hipMalloc(&dx, xb);
    if (e == hipSuccess) e = hipMemcpyAsync(dw, words, wb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = mmc::proposal_vectors(precision == MMC_FP64, proposal == MMC_PROPOSAL_ANGLES, dw, n, dx, s);
    if (e == hipSuccess) e = hipMemcpyAsync(xyz, dx, xb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (dw) (void)hipFree(dw);
    if (dx) (void)hipFree(dx);
    if (s) (void)hipStreamDestroy(s);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return fail(MMC_ENOMEM, "device memory for %lld proposals", (long long)n);
    }
    return e == hipSuccess ? MMC_OK : fail(MMC_EHIP, "proposal vectors: %s", hipGetErrorString(e));
}

int mmc_plan(const mmc_ctx *c, char *buf, size_t n)
{
    if (!c || !buf || n == 0) return fail(MMC_EINVAL, "null argument");
    std::string s;
    int nv;
    if (c->batch) {
        const mmc::Variant *vs = mmc::batch_variants(c->fp64, &nv);
        char b[200];
        snprintf(b, sizeof b, "batch launches=%zu", c->launches.size());
        s += b;
        for (const auto &l : c->launches) {
            snprintf(b, sizeof b, " [%s block=%d workgroups=%d items=%zu]", l.name.c_str(),
                     l.fused ? mmc::fused_block() : vs[l.variant].block, l.n_slots, l.items.size());
            s += b;
        }
        s += ";";
        for (size_t i = 0; i < c->inst.size(); ++i) {
            snprintf(b, sizeof b, " L%d:%s", c->inst[i].L, c->inst[i].variant >= 0 ? vs[c->inst[i].variant].name : "?");
            s += b;
        }
    } else {
        const Instance &in = c->inst[0];
        const mmc::Variant *vs = single_table(c, &nv);
        s = in.plain ? "plain-f64" : (in.variant >= 0 ? vs[in.variant].name : "unplanned");
    }
    snprintf(buf, n, "%s", s.c_str());
    return MMC_OK;
}

void mmc_destroy(mmc_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    for (hipEvent_t e : c->ev_join) (void)hipEventDestroy(e);
    for (hipStream_t a : c->aux) (void)hipStreamDestroy(a);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// ---------------------------------------------------------------- batch
// Work list (items of paths_per_item paths, largest first: longest-processing-time order),
// resident workgroups, HBM slot size and workspace layout of the batch's current variants.
static void batch_plan(mmc_ctx *c)
{
    struct Work {
        double cost;
        mmc::BatchItem item;
    };
    int nv;
    const mmc::Variant *vs = mmc::batch_variants(c->fp64, &nv);
    // one launch per kernel: each LDS variant has its own, the device-memory variants share one
    std::vector<const void *> kern;
    std::vector<std::vector<Work>> work;
    std::vector<size_t> lds, slot;
    std::vector<int> first;
    std::vector<std::string> names;
    for (size_t i = 0; i < c->inst.size(); ++i) {
        const Instance &in = c->inst[i];
        const int v = in.variant;
        size_t g = std::find(kern.begin(), kern.end(), vs[v].kernel) - kern.begin();
        if (g == kern.size()) {
            kern.push_back(vs[v].kernel);
            work.emplace_back();
            lds.push_back(0);
            slot.push_back(0);
            first.push_back(v);
            names.push_back("");
        }
        if (names[g].find(vs[v].name) == std::string::npos) names[g] += (names[g].empty() ? "" : "+") + std::string(vs[v].name);
        const int ppi = mmc::batch_paths_per_item(c->fp64, v);
        lds[g] = std::max(lds[g], mmc::variant_lds_bytes(vs[v], in.L));
        slot[g] = std::max(slot[g], mmc::batch_slot_bytes(c->fp64, v, in.L));
        for (int p = 0; p < in.n_paths; p += ppi) {
            const int np = std::min(ppi, in.n_paths - p);
            work[g].push_back({(double)in.L * in.L * in.L * (double)(in.n_therm + in.n_meas) * np, {(int)i, p}});
        }
    }
    c->launches.clear();
    c->fused_refused = false;
    // the fused kernel, when asked for and every variant has a member in it (a tuned variant
    // without a member is replaced by the member of the same side and placement, e.g. the
    // plane ring's 1024-lane form for its 768-lane one, else by any member of the same side:
    // every variant leaves the same spins and accept counts; pinned ones stay); AUTO runs
    // per-variant launches
    const int mode = c->cfg.batch_launch;
    bool members = true;
    std::vector<int> like(c->inst.size(), -1);
    for (size_t i = 0; i < c->inst.size(); ++i) {
        Instance &in = c->inst[i];
        in.member = mmc::fused_member(c->fp64, vs[in.variant].name);
        if (in.member < 0 && !in.pinned) {
            like[i] = mmc::fused_member_like(c->fp64, in.L, vs[in.variant].lds);
            for (int pl = 0; like[i] < 0 && pl <= LDS_RING2; ++pl) like[i] = mmc::fused_member_like(c->fp64, in.L, pl);
        }
        members = members && (in.member >= 0 || like[i] >= 0);
    }
    if (mode == MMC_BATCH_FUSED && !members) c->fused_refused = true;
    if (members && mode == MMC_BATCH_FUSED) {
        for (size_t i = 0; i < c->inst.size(); ++i) {
            if (like[i] < 0) continue;
            for (int v = 0; v < nv; ++v)
                if (strcmp(vs[v].name, mmc::fused_member_name(like[i])) == 0) c->inst[i].variant = v;
            c->inst[i].member = like[i];
        }
        names.clear();
        for (const Instance &in : c->inst)
            if (std::find(names.begin(), names.end(), std::string(vs[in.variant].name)) == names.end())
                names.push_back(vs[in.variant].name);
        std::vector<Work> all;
        mmc_ctx::Launch l;
        l.fused = true;
        l.variant = c->inst[0].variant;
        l.name = "fused:";
        for (size_t g = 0; g < names.size(); ++g) l.name += (g ? "+" : "") + names[g];
        size_t lds_max = 0, slot_max = 0;
        for (size_t i = 0; i < c->inst.size(); ++i) {
            const Instance &in = c->inst[i];
            const int ppi = mmc::fused_paths_per_item(in.member);
            lds_max = std::max(lds_max, mmc::fused_lds_bytes(in.member));
            slot_max = std::max(slot_max, mmc::fused_slot_bytes(in.member));
            for (int p = 0; p < in.n_paths; p += ppi) {
                const int np = std::min(ppi, in.n_paths - p);
                all.push_back({(double)in.L * in.L * in.L * (double)(in.n_therm + in.n_meas) * np, {(int)i, p}});
            }
        }
        std::stable_sort(all.begin(), all.end(), [](const Work &a, const Work &b) { return a.cost > b.cost; });
        for (auto &w : all) {
            l.items.push_back(w.item);
            l.updates += w.cost;
        }
        l.lds = lds_max;
        const int per_cu = std::max(1, mmc::fused_blocks_per_cu(l.lds));
        l.n_slots = std::min((int)std::min<size_t>(l.items.size(), 1u << 30), per_cu * std::max(1, c->n_cu));
        l.slot_bytes = align_up(slot_max);
        l.off_slots = 0;
        c->launches.push_back(std::move(l));
        c->slot_area = c->launches[0].slot_bytes * (size_t)c->launches[0].n_slots;
        c->ws_bytes = layout_batch(c);
        c->ready = false;
        return;
    }
    for (size_t g = 0; g < kern.size(); ++g) {
        std::stable_sort(work[g].begin(), work[g].end(), [](const Work &a, const Work &b) { return a.cost > b.cost; });
        mmc_ctx::Launch l;
        l.variant = first[g];
        l.name = names[g];
        for (auto &w : work[g]) {
            l.items.push_back(w.item);
            l.updates += w.cost;
        }
        l.lds = lds[g];
        int per_cu = mmc::batch_blocks_per_cu(c->fp64, first[g], l.lds);
        if (per_cu < 1) per_cu = 1;
        l.n_slots = std::min((int)std::min<size_t>(l.items.size(), 1u << 30), per_cu * std::max(1, c->n_cu));
        l.slot_bytes = align_up(slot[g]);
        c->launches.push_back(std::move(l));
    }
    // largest items first across the launches too
    std::stable_sort(c->launches.begin(), c->launches.end(), [&](const mmc_ctx::Launch &a, const mmc_ctx::Launch &b) {
        auto cost = [&](const mmc_ctx::Launch &l) {
            const Instance &in = c->inst[l.items[0].inst];
            return (double)in.L * in.L * in.L * (double)(in.n_therm + in.n_meas) * mmc::batch_paths_per_item(c->fp64, in.variant);
        };
        return cost(a) > cost(b);
    });
    c->slot_area = 0;
    for (auto &l : c->launches) {
        l.off_slots = c->slot_area;
        c->slot_area += (size_t)l.n_slots * l.slot_bytes;
    }
    c->ws_bytes = layout_batch(c);
    c->ready = false;
}

// Kernel time (ms, best of three graph launches) of batch variant var on a trial batch: one
// instance like proto with n_trial paths and `sweeps` measured sweeps, in a context of its own.
static double batch_time_candidate(const mmc_ctx *c, const Instance &proto, int var, int n_trial, int sweeps)
{
    mmc_ctx *t = new mmc_ctx;
    t->batch = true;
    t->cfg = c->cfg;
    t->cfg.async = 0;
    t->seed = c->seed;
    t->fp64 = c->fp64;
    t->n_cu = c->n_cu;
    Instance x = proto;
    x.n_paths = n_trial;
    x.n_therm = 0;
    x.n_meas = sweeps;
    x.variant = var;
    x.pinned = true;
    t->inst.push_back(x);
    double best = 1e30;
    if (ensure_device(t) == MMC_OK) {
        batch_plan(t);
        for (int rep = 0; rep < 3; ++rep) {
            if (mmc_batch_run(t) != MMC_OK) {
                best = 1e30;
                break;
            }
            best = std::min(best, t->last_ms);
        }
    }
    mmc_destroy(t);
    return best;
}

// The batch's autotuner: for each L among the instances that are not pinned, every batch
// variant that fits (placement, LDS budget; specific and generic site maps) runs a trial
// batch of about 1e9 updates at that L (best of three runs) and the fastest is taken for all
// of them. Choices are
// cached per (device, precision, L, path count) like the single-instance tuner's.
static int batch_tune(mmc_ctx *c)
{
    int nv;
    const mmc::Variant *vs = mmc::batch_variants(c->fp64, &nv);
    std::map<int, std::vector<int>> by_L;
    for (size_t i = 0; i < c->inst.size(); ++i)
        if (!c->inst[i].pinned) by_L[c->inst[i].L].push_back((int)i);
    bool changed = false;
    for (auto &kv : by_L) {
        const int L = kv.first;
        const std::vector<int> cand = batch_candidates(c->fp64, L, c->cfg.placement, true);
        if (cand.size() < 2) continue;
        long long paths = 0;
        for (int i : kv.second) paths += c->inst[i].n_paths;
        const std::string key = tune_key(true, c->fp64, L, (int)std::min<long long>(paths, 1 << 30));
        int best = -1;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_cache_load();
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end())
                for (int v : cand)
                    if (it->second == vs[v].name) best = v;
        }
        if (best < 0) {
            // one wave of items on every candidate's resident workgroups
            long long most = 1;
            for (int v : cand) {
                const int per_cu = std::max(1, mmc::batch_blocks_per_cu(c->fp64, v, mmc::variant_lds_bytes(vs[v], L)));
                most = std::max(most, (long long)mmc::batch_paths_per_item(c->fp64, v) * per_cu * c->n_cu);
            }
            const int n_trial = (int)std::min<long long>(paths, most);
            const double per_sweep = (double)L * L * L * n_trial;
            const int sweeps = 6 * (int)ceil(std::min(64.0, std::max(6.0, 1e9 / per_sweep)) / 6.0);
            double best_ms = 1e30;
            for (int v : cand) {
                const double ms = batch_time_candidate(c, c->inst[kv.second[0]], v, n_trial, sweeps);
                mmc_log("batch tuning L=%d (%d trial paths, %d sweeps): %s %.3f ms", L, n_trial, sweeps, vs[v].name, ms);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = v;
                }
            }
            if (best < 0) continue;  // no trial ran: keep the default
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = vs[best].name;
            tune_cache_store();
        }
        for (int i : kv.second) {
            changed |= c->inst[i].variant != best;
            c->inst[i].variant = best;
        }
    }
    if (changed) batch_plan(c);
    return MMC_OK;
}

mmc_ctx *mmc_batch_create(const mmc_instance *inst, int n_inst, uint64_t seed, const mmc_config *cfg)
{
    if (!inst || n_inst < 1 || n_inst >= (1 << 24)) {
        fail(MMC_EINVAL, "need 1 <= n_inst < 2^24 instances");
        return nullptr;
    }
    mmc_config c0{};
    if (cfg) c0 = *cfg;
    if (c0.precision != MMC_FP32 && c0.precision != MMC_FP64) {
        fail(MMC_EINVAL, "precision must be MMC_FP32 or MMC_FP64");
        return nullptr;
    }
    if (c0.placement == MMC_PLACE_PLAIN) {
        fail(MMC_EUNSUPPORTED, "the plain engine has no batch form");
        return nullptr;
    }
    if (c0.model != MMC_MODEL_HEISENBERG3D) {
        fail(MMC_EUNSUPPORTED, "batches run the Heisenberg model only");
        return nullptr;
    }
    if (c0.init < MMC_INIT_SPHERE || c0.init > MMC_INIT_MIXED || c0.proposal < MMC_PROPOSAL_SPHERE ||
        c0.proposal > MMC_PROPOSAL_ANGLES || c0.batch_launch < MMC_BATCH_AUTO || c0.batch_launch > MMC_BATCH_PER_VARIANT) {
        fail(MMC_EINVAL, "configuration out of range");
        return nullptr;
    }
    if (c0.proposal != MMC_PROPOSAL_SPHERE) {
        fail(MMC_EUNSUPPORTED, "the both-angles proposal runs on the plain FP64 engine only");
        return nullptr;
    }
    c0.trace_sweeps = 0;
    mmc_ctx *c = new mmc_ctx;
    c->batch = true;
    c->cfg = c0;
    c->seed = seed;
    c->fp64 = c0.precision == MMC_FP64;
    for (int i = 0; i < n_inst; ++i) {
        std::string why;
        const mmc_instance &x = inst[i];
        if (!valid_instance(x.L, x.T, x.J, x.n_paths, x.n_therm, x.n_meas, why)) {
            fail(MMC_EINVAL, "instance %d: %s", i, why.c_str());
            delete c;
            return nullptr;
        }
        Instance in;
        in.L = x.L;
        in.T = x.T;
        in.J = x.J;
        in.n_paths = x.n_paths;
        in.n_therm = x.n_therm;
        in.n_meas = x.n_meas;
        std::vector<int> cand = batch_candidates(c->fp64, x.L, c0.placement);
        if (cand.empty()) {
            fail(MMC_EUNSUPPORTED, "instance %d: no batch variant for L=%d", i, x.L);
            delete c;
            return nullptr;
        }
        // default: LDS when it fits (first LDS candidate), else the first device-memory one
        in.variant = cand[0];
        c->inst.push_back(in);
    }
    // occupancy decides the number of resident workgroups (and HBM spin slots)
    if (ensure_device(c) != MMC_OK) {
        delete c;
        return nullptr;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
        fail(MMC_EHIP, "hipGetDeviceProperties failed");
        mmc_destroy(c);
        return nullptr;
    }
    // each launch's resident workgroups come from the occupancy calculator (registers, LDS)
    c->n_cu = prop.multiProcessorCount;
    batch_plan(c);
    if (batch_tune(c) != MMC_OK) {
        mmc_destroy(c);
        return nullptr;
    }
    return c;
}

static int batch_upload(mmc_ctx *c)
{
    std::vector<mmc::InstDev> d;
    std::vector<int> var;
    const bool fused = !c->launches.empty() && c->launches[0].fused;
    for (size_t i = 0; i < c->inst.size(); ++i) {
        d.push_back(inst_dev(c, c->inst[i], (uint32_t)i));
        var.push_back(fused ? c->inst[i].member : c->inst[i].variant);
    }
    HIP_TRY(hipMemcpy(c->ws + c->off_inst, d.data(), d.size() * sizeof(mmc::InstDev), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->ws + c->off_var, var.data(), var.size() * sizeof(int), hipMemcpyHostToDevice));
    for (const auto &l : c->launches)
        HIP_TRY(hipMemcpy(c->ws + l.off_items, l.items.data(), l.items.size() * sizeof(mmc::BatchItem),
                          hipMemcpyHostToDevice));
    return MMC_OK;
}

// Parallel branches of a batch graph: one per launch, at most as many as the process has
// hardware queues (GPU_MAX_HW_QUEUES, HIP's default 4). With more branches than queues, some
// launches wait for a queue until another launch has ended; within the limit the largest
// launches get a branch each and the smallest run one after another on the last one, beside
// the others.
static int batch_branches(const mmc_ctx *c)
{
    int q = 4;
    if (const char *e = getenv("GPU_MAX_HW_QUEUES")) {
        const int v = atoi(e);
        if (v >= 1) q = v;
    }
    return std::max(1, std::min((int)c->launches.size(), q));
}

// The launches (largest items first): the first on the context's stream, the others on
// branches forked from it and joined back (batch_branches), so the kernels run side by side
// and compute-bound LDS work overlaps the memory-bound device-memory kernels. Where the LDS
// launches carry under a tenth of the updates they start after the device-memory kernel
// instead: side by side they would hold CU resources from the kernel on the critical path
// for longer than their share is worth. The kernels share no data but the read-only
// instance and variant tables, and each works its own queue to the end.

static int batch_enqueue(mmc_ctx *c, hipStream_t s)
{
    hipError_t e = mmc::fill_zero(c->ws + c->off_head, 64 * std::max<size_t>(1, c->launches.size()), s);
    if (e != hipSuccess) return fail(MMC_EHIP, "queue reset: %s", hipGetErrorString(e));
    int nv;
    const mmc::Variant *vs = mmc::batch_variants(c->fp64, &nv);
    double total = 0, in_lds = 0;
    for (const auto &l : c->launches) {
        total += l.updates;
        if (lds_resident(vs[l.variant])) in_lds += l.updates;
    }
    const bool after_memory = !lds_resident(vs[c->launches[0].variant]) && in_lds < 0.1 * total;
    const int nb = batch_branches(c);
    for (size_t k = 0; k < c->launches.size(); ++k) {
        const auto &l = c->launches[k];
        const int br = std::min((int)k, nb - 1);  // launches nb - 1 and later share the last branch
        hipStream_t sk = br ? c->aux[br - 1] : s;
        // fork point: before the first launch, or after it when the rest waits for it
        if (c->launches.size() > 1 && k == (after_memory ? 1 : 0)) HIP_TRY(hipEventRecord(c->ev_fork, s));
        if (br && (int)k == br) HIP_TRY(hipStreamWaitEvent(sk, c->ev_fork, 0));
        mmc::BatchDev b;
        b.inst = reinterpret_cast<const mmc::InstDev *>(c->ws + c->off_inst);
        b.variant = reinterpret_cast<const int *>(c->ws + c->off_var);
        b.items = reinterpret_cast<const mmc::BatchItem *>(c->ws + l.off_items);
        b.n_items = (int)l.items.size();
        b.head = reinterpret_cast<unsigned int *>(c->ws + c->off_head + 64 * k);
        b.slots = c->ws + c->off_slots + l.off_slots;  // all-LDS variants: slot_bytes 0, never touched
        b.slot_bytes = l.slot_bytes;
        b.n_slots = l.n_slots;
        e = l.fused ? mmc::launch_fused(b, l.n_slots, l.lds, sk) : mmc::launch_batch(b, c->fp64, l.variant, l.n_slots, l.lds, sk);
        if (e != hipSuccess) return fail(MMC_EHIP, "batch launch %s: %s", l.name.c_str(), hipGetErrorString(e));
    }
    for (int b = 1; b < nb; ++b) {
        HIP_TRY(hipEventRecord(c->ev_join[b - 1], c->aux[b - 1]));
        HIP_TRY(hipStreamWaitEvent(s, c->ev_join[b - 1], 0));
    }
    return MMC_OK;
}

int mmc_batch_run(mmc_ctx *c)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (!c->batch) return fail(MMC_EINVAL, "not a batch context");
    if (c->fused_refused)
        return fail(MMC_EUNSUPPORTED, "batch_launch FUSED: a variant of this batch has no member in the fused kernel");
    if (!c->ready) {
        int rc = ensure_memory(c);
        if (rc) return rc;
        rc = batch_upload(c);
        if (rc) return rc;
        if (!c->ev_fork) HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        while ((int)c->aux.size() + 1 < batch_branches(c)) {
            hipStream_t a = nullptr;
            hipEvent_t e = nullptr;
            HIP_TRY(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
            c->aux.push_back(a);
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            c->ev_join.push_back(e);
        }
        c->ready = true;
    }
    GraphKey key{0, 0, 1};
    hipGraphExec_t exec = nullptr;
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        exec = it->second;
    } else {
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        int rc = batch_enqueue(c, c->stream);
        hipError_t ec = hipStreamEndCapture(c->stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ec != hipSuccess) return fail(MMC_EHIP, "graph capture: %s", hipGetErrorString(ec));
        hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(MMC_EHIP, "graph instantiate: %s", hipGetErrorString(ei));
        c->graphs[key] = exec;
    }
    int rc = begin_work(c);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    HIP_TRY(hipGraphLaunch(exec, c->stream));
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    rc = end_work(c);
    if (rc) return rc;
    c->sweeps_done = 1;  // marks "ran"; every instance ran all of its sweeps
    return c->cfg.async ? MMC_OK : finish(c);
}

int mmc_batch_results(const mmc_ctx *c, int i, mmc_path_result *out, int n_out)
{
    if (!c) return fail(MMC_EINVAL, "null context");
    if (!c->batch) return fail(MMC_EINVAL, "not a batch context");
    if (i < 0 || i >= (int)c->inst.size()) return fail(MMC_EINVAL, "instance %d out of range", i);
    const Instance &in = c->inst[i];
    if (c->sweeps_done == 0) return fail(MMC_ESTATE, "nothing has run yet");
    return results_of(c, in, total_sweeps(in), out, n_out);
}

int mmc_batch_stats(const mmc_ctx *c, int i, mmc_stats_t *out)
{
    if (!c || !out) return fail(MMC_EINVAL, "null argument");
    if (!c->batch || i < 0 || i >= (int)c->inst.size()) return fail(MMC_EINVAL, "bad batch instance");
    const Instance &in = c->inst[i];
    std::vector<mmc_path_result> r(in.n_paths);
    int rc = mmc_batch_results(c, i, r.data(), in.n_paths);
    if (rc) return rc;
    rc = mmc_stats_from_results(r.data(), in.n_paths, in.L, in.T, out);
    if (rc) return rc;
    double acc = 0;
    for (auto &x : r) acc += (double)x.n_accept;
    out->accept_rate = acc / ((double)in.n_paths * total_sweeps(in) * (double)in.L * in.L * in.L);
    return MMC_OK;
}

}  // extern "C"
