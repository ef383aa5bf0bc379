// kernels.hip -- HIP kernels (gfx950) of the multipath Metropolis engine for the classical
// O(3) Heisenberg model (arXiv:1305.6758, Sec. 2).
//
// One simulation path is a periodic L^3 lattice of unit spins swept with single-spin
// Metropolis moves; paths are independent (Sec. 2: "embarrassingly parallel"), so a group
// of G lanes of one workgroup owns one path for all of its sweeps. Within a path the sweep
// is a checkerboard: every neighbour of an even site is odd, so all sites of one colour are
// updated at once, with a barrier between the two half-sweeps.
//
// Spin layout (LDS or device memory): [colour][component][N/2] for one path; the half-index
// of site (x, y, z) is h = (x >> 1) + (L/2)(y + L z), so consecutive lanes touch
// consecutive words (conflict-free LDS, coalesced global access).
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) on the counter
// (site id, sweep, path, tag | instance << 8), key = seed. Words 0 and 1 give the proposal,
// word 2 the acceptance uniform.
#include "engine.hpp"

#include <algorithm>
#include <type_traits>

namespace mmc {
namespace {

// ------------------------------------------------------------------ Philox4x32-10
constexpr uint32_t PHI_M0 = 0xD2511F53u, PHI_M1 = 0xCD9E8D57u;
constexpr uint32_t PHI_W0 = 0x9E3779B9u, PHI_W1 = 0xBB67AE85u;

struct Words { uint32_t w0, w1, w2, w3; };

// Ten rounds; each round takes the two 64-bit products apart and xors in the key, then the
// key moves along the Weyl sequence. With counter words 1-3 and the key wave-uniform, the
// compiler keeps their part of the first two rounds on the scalar unit.
__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)PHI_M0 * c0;
        const uint64_t p1 = (uint64_t)PHI_M1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += PHI_W0;
        k1 += PHI_W1;
    }
    return {c0, c1, c2, c3};
}

// ------------------------------------------------------------------ precision policies
template <typename T> struct Arith;

// FP32: uniforms with 23 random bits, ((w >> 8) | 1) 2^-24, exact in FP32 and never 0 or 1;
// transcendental unit for sqrt, sin, cos (argument in revolutions) and exp2.
template <> struct Arith<float> {
    static __device__ __forceinline__ float uni(uint32_t w) { return (float)((w >> 8) | 1u) * 0x1p-24f; }
    // 2u - 1 for the same u, exact: ((w >> 8) | 1) - 2^23 as a signed integer, times 2^-23.
    static __device__ __forceinline__ float sym(uint32_t w)
    {
        return (float)(((int32_t)(w ^ 0x80000000u) >> 8) | 1) * 0x1p-23f;
    }
    static __device__ __forceinline__ void sphere(uint32_t w0, uint32_t w1, float &x, float &y, float &z)
    {
        const float zz = sym(w0);
        const float r = __builtin_amdgcn_sqrtf(fmaf(-zz, zz, 1.0f));
        const float rev = uni(w1);  // phi / (2 pi)
        x = r * __builtin_amdgcn_cosf(rev);
        y = r * __builtin_amdgcn_sinf(rev);
        z = zz;
    }
    static __device__ __forceinline__ void angles(uint32_t w0, uint32_t w1, float &x, float &y, float &z)
    {
        const float th = 0.5f * uni(w0);  // theta / (2 pi), theta = pi u0
        const float ph = uni(w1);
        const float st = __builtin_amdgcn_sinf(th);
        x = st * __builtin_amdgcn_cosf(ph);
        y = st * __builtin_amdgcn_sinf(ph);
        z = __builtin_amdgcn_cosf(th);
    }
    // accept iff u < exp(beta J dot), dot = (S' - S) . h; q = beta J log2(e) precomputed.
    static __device__ __forceinline__ bool accept(uint32_t w2, float dot, float q)
    {
        return uni(w2) < __builtin_amdgcn_exp2f(q * dot);
    }
};

// FP64: uniforms (w + 1/2) 2^-32, IEEE arithmetic in the reference order (the file is
// compiled without contraction), library sin/cos/exp.
template <> struct Arith<double> {
    static __device__ __forceinline__ double uni(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }
    static __device__ __forceinline__ void sphere(uint32_t w0, uint32_t w1, double &x, double &y, double &z)
    {
        const double u0 = uni(w0), u1 = uni(w1);
        const double phi = 2.0 * 3.14159265358979323846 * u1;
        const double zz = 2.0 * u0 - 1.0;
        const double r = sqrt(1.0 - zz * zz);
        x = r * cos(phi);
        y = r * sin(phi);
        z = zz;
    }
    static __device__ __forceinline__ void angles(uint32_t w0, uint32_t w1, double &x, double &y, double &z)
    {
        const double u0 = uni(w0), u1 = uni(w1);
        const double phi = 2.0 * 3.14159265358979323846 * u1;
        const double th = 3.14159265358979323846 * u0;
        x = sin(th) * cos(phi);
        y = sin(th) * sin(phi);
        z = cos(th);
    }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

enum Map { COLZ = 0, FLAT = 1 };

// Everything a path group needs during its sweeps.
template <typename T>
struct GroupCtx {
    const InstDev *in;
    int path;
    bool active;       // path < n_paths
    int lane;          // 0 .. G-1
    T *sp;             // spins of this path while sweeping (LDS or device memory)
    double *shacc;     // 16 doubles in LDS: the path's PathAcc while sweeping
    T *red;            // LDS [waves of the group][4] measurement partials
};

// Site geometry of one update: half-index h, site id, and the six neighbour half-indices
// (in the other colour) in the order -x, +x, -y, +y, -z, +z.
struct Site {
    int h, id;
    int nb[6];
};

// Neighbour geometry of site (j, y, z) of colour c; x = 2j + p with p = (y + z + c) & 1.
__device__ __forceinline__ Site make_site(int L, int j, int y, int z, int c)
{
    const int HL = L >> 1, PLANE = HL * L;
    Site s;
    const int p = (y + z + c) & 1;
    const int x = 2 * j + p;
    s.h = j + HL * y + PLANE * z;
    s.id = x + L * (y + L * z);
    // x -> x-1: for p = 0 it is the other colour's word j-1 (wrapping to HL-1); for p = 1
    // it is word j. x -> x+1: for p = 0 word j; for p = 1 word j+1 (wrapping to 0).
    const int jm = (j == 0) ? HL - 1 : j - 1;
    const int jp = (j == HL - 1) ? 0 : j + 1;
    const int row = s.h - j;
    s.nb[0] = row + (p ? j : jm);
    s.nb[1] = row + (p ? jp : j);
    s.nb[2] = s.h + ((y == 0) ? (L - 1) * HL : -HL);
    s.nb[3] = s.h + ((y == L - 1) ? -(L - 1) * HL : HL);
    s.nb[4] = s.h + ((z == 0) ? (L - 1) * PLANE : -PLANE);
    s.nb[5] = s.h + ((z == L - 1) ? -(L - 1) * PLANE : PLANE);
    return s;
}

// One Metropolis attempt at site s of colour c, sweep k. Returns whether it was accepted
// and adds the new spin (and, for the odd colour, S . h) to the measurement partials.
template <typename T>
__device__ __forceinline__ bool update_site(const GroupCtx<T> &g, int HALF, int c, const Site &s, uint32_t k,
                                            T beta, T J, T q, T &pe, T &pmx, T &pmy, T &pmz)
{
    T *own = g.sp + (c ? 3 * HALF : 0);
    const T *oth = g.sp + (c ? 0 : 3 * HALF);
    const InstDev &in = *g.in;
    const Words w = philox4x32_10((uint32_t)s.id, k, (uint32_t)g.path, TAG_MET | in.ctr3, in.key0, in.key1);
    const T sx = own[s.h], sy = own[HALF + s.h], sz = own[2 * HALF + s.h];
    T hx, hy, hz;
    if constexpr (std::is_same<T, double>::value) {
        // h = ((((S_-x + S_+x) + S_-y) + S_+y) + S_-z) + S_+z, the reference order.
        hx = oth[s.nb[0]];
        hy = oth[HALF + s.nb[0]];
        hz = oth[2 * HALF + s.nb[0]];
#pragma unroll
        for (int n = 1; n < 6; ++n) {
            hx = hx + oth[s.nb[n]];
            hy = hy + oth[HALF + s.nb[n]];
            hz = hz + oth[2 * HALF + s.nb[n]];
        }
    } else {
        // FP32: pairwise tree (any order is a valid FP32 rounding of the same sum).
        T ax[6], ay[6], az[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            ax[n] = oth[s.nb[n]];
            ay[n] = oth[HALF + s.nb[n]];
            az[n] = oth[2 * HALF + s.nb[n]];
        }
        hx = ((ax[0] + ax[1]) + (ax[2] + ax[3])) + (ax[4] + ax[5]);
        hy = ((ay[0] + ay[1]) + (ay[2] + ay[3])) + (ay[4] + ay[5]);
        hz = ((az[0] + az[1]) + (az[2] + az[3])) + (az[4] + az[5]);
    }
    T nx, ny, nz;
    Arith<T>::sphere(w.w0, w.w1, nx, ny, nz);
    const T dx = nx - sx, dy = ny - sy, dz = nz - sz;
    bool acc;
    if constexpr (std::is_same<T, double>::value) {
        // dE = -J ((dx hx + dy hy) + dz hz); accept iff u < exp(-beta dE).
        const double dE = -J * ((dx * hx + dy * hy) + dz * hz);
        acc = Arith<double>::uni(w.w2) < exp(-beta * dE);
    } else {
        const float dot = fmaf(dz, hz, fmaf(dy, hy, dx * hx));
        acc = Arith<float>::accept(w.w2, dot, q);
    }
    T fx = sx, fy = sy, fz = sz;
    if (acc) {
        own[s.h] = nx;
        own[HALF + s.h] = ny;
        own[2 * HALF + s.h] = nz;
        fx = nx;
        fy = ny;
        fz = nz;
    }
    pmx += fx;
    pmy += fy;
    pmz += fz;
    if (c) {
        if constexpr (std::is_same<T, double>::value) pe = pe + ((fx * hx + fy * hy) + fz * hz);
        else pe = fmaf(fz, hz, fmaf(fy, hy, fmaf(fx, hx, pe)));
    }
    return acc;
}

// Calls f(Site) for every site of colour c owned by this lane.
//   COLZ: a lane owns whole columns (fixed x, y) and a stride of z: for G >= plane
//   (plane = L^2/2 sites of one colour), lane = column + plane * z0 and z = z0 + DZ t with
//   DZ = G / plane; for G < plane the lane owns columns lane + G t and every z.
//   FLAT: lane owns half-indices lane + G s (any L, ragged tail allowed).
template <int LC, int G, int MAP, typename F>
__device__ __forceinline__ void for_own_sites(int Lrt, int lane, int c, F &&f)
{
    const int L = LC ? LC : Lrt;
    const int HL = L >> 1, PLANE = HL * L, HALF = PLANE * L;
    if constexpr (MAP == COLZ) {
        if (G >= PLANE) {
            const int DZ = G / PLANE;
            if (lane >= DZ * PLANE) return;
            const int col = lane % PLANE, z0 = lane / PLANE;
            const int j = col % HL, y = col / HL;
            const int NZ = (L + DZ - 1) / DZ;
#pragma unroll 4
            for (int t = 0; t < NZ; ++t) {
                const int z = z0 + DZ * t;
                if (z < L) f(make_site(L, j, y, z, c));
            }
        } else {
            const int NCOL = (PLANE + G - 1) / G;
            for (int ct = 0; ct < NCOL; ++ct) {
                const int col = lane + G * ct;
                if (col >= PLANE) break;
                const int j = col % HL, y = col / HL;
#pragma unroll 4
                for (int z = 0; z < L; ++z) f(make_site(L, j, y, z, c));
            }
        }
    } else {
        const int SPL = (HALF + G - 1) / G;
#pragma unroll 4
        for (int s = 0; s < SPL; ++s) {
            const int h = lane + G * s;
            if (h < HALF) {
                const int col = h % PLANE, z = h / PLANE;
                f(make_site(L, col % HL, col / HL, z, c));
            }
        }
    }
}

// Initial state of Sec. 2.2 for this lane's sites (Philox counter (id, 0, path, TAG_INIT)).
// Out of line (runs once): inlined, it crashes the ROCm 7.2 optimizer (SimplifyCFG).
template <typename T, int LC, int G, int MAP>
__device__ __attribute__((noinline)) void init_own(const GroupCtx<T> &g)
{
    const InstDev &in = *g.in;
    const int L = LC ? LC : in.L;
    const int HALF = L * L * L / 2;
    for (int c = 0; c < 2; ++c) {
        T *own = g.sp + (c ? 3 * HALF : 0);
        for_own_sites<LC, G, MAP>(in.L, g.lane, c, [&](const Site &s) {
            T x, y, z;
            if (in.init == INIT_ORDERED) {
                x = T(0); y = T(0); z = T(1);
            } else {
                const Words w = philox4x32_10((uint32_t)s.id, 0u, (uint32_t)g.path, TAG_INIT | in.ctr3, in.key0, in.key1);
                if (in.init == INIT_ANGLES) Arith<T>::angles(w.w0, w.w1, x, y, z);
                else Arith<T>::sphere(w.w0, w.w1, x, y, z);
            }
            own[s.h] = x;
            own[HALF + s.h] = y;
            own[2 * HALF + s.h] = z;
        });
    }
}

// FP32 only: S <- S / |S| for this lane's sites.
template <typename T, int LC, int G, int MAP>
__device__ __attribute__((noinline)) void renorm_own(const GroupCtx<T> &g)
{
    const int L = LC ? LC : g.in->L;
    const int HALF = L * L * L / 2;
    for (int c = 0; c < 2; ++c) {
        T *own = g.sp + (c ? 3 * HALF : 0);
        for_own_sites<LC, G, MAP>(g.in->L, g.lane, c, [&](const Site &s) {
            const T x = own[s.h], y = own[HALF + s.h], z = own[2 * HALF + s.h];
            const T r = __builtin_amdgcn_rsqf(fmaf(z, z, fmaf(y, y, x * x)));
            own[s.h] = x * r;
            own[HALF + s.h] = y * r;
            own[2 * HALF + s.h] = z * r;
        });
    }
}

// Sweeps [k0, k1) of one path group. All groups of the workgroup call this together (same
// instance and sweep range), so __syncthreads() separates the half-sweeps of all of them.
// Idle groups (path >= n_paths) and idle lanes still take every barrier.
template <typename T, int LC, int G, int MAP>
__device__ void path_sweeps(const GroupCtx<T> &g, int k0, int k1, bool fresh)
{
    const InstDev &in = *g.in;
    const int L = LC ? LC : in.L;
    const int HALF = L * L * L / 2;
    const double Nd = 2.0 * (double)HALF;
    const T beta = (T)in.beta, J = (T)in.J;
    const T q = (T)(in.beta * in.J * 1.4426950408889634);  // beta J log2(e)
    const int wave = g.lane >> 6;
    const bool lead = g.active && g.lane == 0;
    unsigned long long n_acc = 0;  // this wave's accepted moves

    if (g.active && fresh) init_own<T, LC, G, MAP>(g);
    __syncthreads();

    for (int k = k0; k < k1; ++k) {
        if constexpr (std::is_same<T, float>::value) {
            if (in.renorm_every > 0 && k > 0 && k % in.renorm_every == 0) {
                if (g.active) renorm_own<T, LC, G, MAP>(g);
                __syncthreads();
            }
        }
        T pe = T(0), pmx = T(0), pmy = T(0), pmz = T(0);
        for (int c = 0; c < 2; ++c) {
            if (g.active) {
                for_own_sites<LC, G, MAP>(in.L, g.lane, c, [&](const Site &s) {
                    const bool a = update_site<T>(g, HALF, c, s, (uint32_t)k, beta, J, q, pe, pmx, pmy, pmz);
                    n_acc += (unsigned long long)__popcll(__ballot(a));
                });
            }
            if (c == 0) __syncthreads();
        }
        const bool meas = k >= in.n_therm || k < in.trace_sweeps || k == k1 - 1;
        if (meas) {
            pe = wave_sum(pe);
            pmx = wave_sum(pmx);
            pmy = wave_sum(pmy);
            pmz = wave_sum(pmz);
            if ((g.lane & 63) == 0) {
                g.red[4 * wave + 0] = pe;
                g.red[4 * wave + 1] = pmx;
                g.red[4 * wave + 2] = pmy;
                g.red[4 * wave + 3] = pmz;
            }
        }
        __syncthreads();
        if (meas && lead) {
            double se = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            for (int w = 0; w < G / 64; ++w) {
                se += (double)g.red[4 * w + 0];
                sx += (double)g.red[4 * w + 1];
                sy += (double)g.red[4 * w + 2];
                sz += (double)g.red[4 * w + 3];
            }
            // Every bond joins an even and an odd site: E = -J sum_odd S_i . h_i.
            const double e = -in.J * se / Nd;
            const double mx = sx / Nd, my = sy / Nd, mz = sz / Nd;
            if (k >= in.n_therm) {
                const double m = sqrt(mx * mx + my * my + mz * mz);
                g.shacc[0] += e;
                g.shacc[1] += e * e;
                g.shacc[2] += m;
                g.shacc[3] += m * m;
                g.shacc[4] += (m * m) * (m * m);
            }
            if (k < in.trace_sweeps) {
                double *tr = in.trace + ((size_t)g.path * in.trace_sweeps + k) * 4;
                tr[0] = e;
                tr[1] = mx;
                tr[2] = my;
                tr[3] = mz;
            }
            if (k == k1 - 1) {
                g.shacc[5] = e;
                g.shacc[6] = mx;
                g.shacc[7] = my;
                g.shacc[8] = mz;
            }
        }
    }
    if (g.active && (g.lane & 63) == 0)
        atomicAdd((unsigned long long *)&g.shacc[9], n_acc);
    __syncthreads();
}

// Loads the path's accumulators into LDS (zero on a fresh start).
__device__ __forceinline__ void load_acc(double *shacc, const PathAcc *acc, bool fresh, int lane, bool active)
{
    if (lane < 16) shacc[lane] = (active && !fresh) ? reinterpret_cast<const double *>(acc)[lane] : 0.0;
}

__device__ __forceinline__ void store_acc(const double *shacc, PathAcc *acc, int lane, bool active)
{
    if (active && lane < 16) reinterpret_cast<double *>(acc)[lane] = shacc[lane];
}

// Strided copy of one path's spins by the G lanes of its group (once per launch). Kept out
// of line: inlined into the sweep kernels it crashes the ROCm 7.2 optimizer (SimplifyCFG).
template <int G, typename T>
__device__ __attribute__((noinline)) void copy_spins(T *__restrict__ dst, const T *__restrict__ src, int n, int lane)
{
    for (int t = lane; t < n; t += G) dst[t] = src[t];
}

// LDS bytes of one workgroup: spins (LDS placement), accumulators, reduction slots.
template <typename T>
__host__ __device__ constexpr size_t lds_layout_bytes(int L, int B, int G, bool in_lds)
{
    return (in_lds ? (size_t)(B / G) * 3 * (size_t)L * L * L * sizeof(T) : 0) + (size_t)(B / G) * 128 +
           (size_t)(B / 64) * 4 * sizeof(T);
}

// Sets up the group views of one workgroup and runs sweeps [k0, k1) for paths
// path0 + group. gspins: the instance's resident spin array (or nullptr in a batch);
// slot: device memory for an HBM path when gspins is nullptr.
template <typename T, int LC, int G, int B, int MAP, bool IN_LDS>
__device__ void wg_run(const InstDev &in, int path0, int k0, int k1, bool fresh, char *smem, T *slot)
{
    constexpr int P = B / G;
    const int L = LC ? LC : in.L;
    const size_t NS = 3 * (size_t)L * L * L;  // spin words per path
    const int group = threadIdx.x / G;
    GroupCtx<T> g;
    g.in = &in;
    g.lane = threadIdx.x % G;
    g.path = path0 + group;
    g.active = g.path < in.n_paths;
    char *p = smem;
    T *lds_spins = reinterpret_cast<T *>(p);
    if (IN_LDS) p += P * NS * sizeof(T);
    g.shacc = reinterpret_cast<double *>(p) + 16 * group;
    p += P * 128;
    g.red = reinterpret_cast<T *>(p) + 4 * (group * (G / 64));
    T *gsp = in.spins ? reinterpret_cast<T *>(in.spins) + (size_t)g.path * NS : slot + (size_t)group * NS;
    g.sp = IN_LDS ? lds_spins + (size_t)group * NS : gsp;

    load_acc(g.shacc, in.acc + g.path, fresh, g.lane, g.active);
    if (IN_LDS && !fresh && g.active) copy_spins<G>(g.sp, gsp, (int)NS, g.lane);
    // (path_sweeps begins with a barrier)
    path_sweeps<T, LC, G, MAP>(g, k0, k1, fresh);
    if (IN_LDS && in.spins && g.active) copy_spins<G>(gsp, g.sp, (int)NS, g.lane);
    store_acc(g.shacc, in.acc + g.path, g.lane, g.active);
}

template <typename T, int LC, int G, int B, int MAP, bool IN_LDS>
__global__ __launch_bounds__(B) void k_resident(InstDev in, int k0, int k1, int fresh)
{
    extern __shared__ __align__(16) char smem[];
    wg_run<T, LC, G, B, MAP, IN_LDS>(in, blockIdx.x * (B / G), k0, k1, fresh != 0, smem, nullptr);
}

template <typename T, int LC, int G, int B, int MAP, bool IN_LDS>
hipError_t launch_resident(const InstDev &in, int k0, int k1, int fresh, hipStream_t s)
{
    const int L = LC ? LC : in.L;
    const size_t lds = lds_layout_bytes<T>(L, B, G, IN_LDS);
    auto kern = k_resident<T, LC, G, B, MAP, IN_LDS>;
    const int grid = (in.n_paths + (B / G) - 1) / (B / G);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(B), lds, s, in, k0, k1, fresh);
    return hipGetLastError();
}

// ------------------------------------------------------------------ persistent batch kernel
constexpr int BATCH_B = 512;

// Variant lists of the batch kernel (block BATCH_B). Index = BatchDev::variant value.
#define MMC_BATCH_VARIANTS_F32(X)                  \
    X(float, 8, 64, COLZ, true, "f32-lds-L8-g64")    \
    X(float, 12, 256, FLAT, true, "f32-lds-L12-g256") \
    X(float, 16, 512, COLZ, true, "f32-lds-L16-g512") \
    X(float, 0, 512, FLAT, true, "f32-lds-any-g512")  \
    X(float, 16, 512, COLZ, false, "f32-hbm-L16-g512") \
    X(float, 24, 512, FLAT, false, "f32-hbm-L24-g512") \
    X(float, 32, 512, COLZ, false, "f32-hbm-L32-g512") \
    X(float, 48, 512, FLAT, false, "f32-hbm-L48-g512") \
    X(float, 64, 512, COLZ, false, "f32-hbm-L64-g512") \
    X(float, 0, 512, FLAT, false, "f32-hbm-any-g512")

#define MMC_BATCH_VARIANTS_F64(X)                    \
    X(double, 8, 128, COLZ, true, "f64-lds-L8-g128")   \
    X(double, 12, 512, FLAT, true, "f64-lds-L12-g512") \
    X(double, 0, 512, FLAT, true, "f64-lds-any-g512")  \
    X(double, 16, 512, COLZ, false, "f64-hbm-L16-g512") \
    X(double, 32, 512, COLZ, false, "f64-hbm-L32-g512") \
    X(double, 0, 512, FLAT, false, "f64-hbm-any-g512")

template <typename T>
__global__ __launch_bounds__(BATCH_B) void k_batch(BatchDev bd)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int item_sh;
    T *slot = reinterpret_cast<T *>(bd.slots + (size_t)blockIdx.x * bd.slot_bytes);
    for (;;) {
        if (threadIdx.x == 0) item_sh = (int)atomicAdd(bd.head, 1u);
        __syncthreads();
        const int it = item_sh;
        __syncthreads();
        if (it >= bd.n_items) break;  // uniform: every wave leaves once the queue is empty
        const BatchItem item = bd.items[it];
        const InstDev &in = bd.inst[item.inst];
        const int total = in.n_therm + in.n_meas;
        int v = bd.variant[item.inst];
        int idx = 0;
#define MMC_BATCH_CASE(TT, LC, G, MAP, LDS, NAME) \
    if constexpr (std::is_same<T, TT>::value) {   \
        if (v == idx) wg_run<TT, LC, G, BATCH_B, MAP, LDS>(in, item.path0, 0, total, true, smem, slot); \
        ++idx;                                    \
    }
        MMC_BATCH_VARIANTS_F32(MMC_BATCH_CASE)
        MMC_BATCH_VARIANTS_F64(MMC_BATCH_CASE)
#undef MMC_BATCH_CASE
    }
}

// ------------------------------------------------------------------ plain FP64 engine
// One thread per site of one colour, spins in device memory, one launch per half-sweep;
// the sweep index lives in device memory so one captured sweep can be replayed.
__global__ __launch_bounds__(256) void k_plain_init(InstDev in)
{
    const int L = in.L, HALF = L * L * L / 2, HL = L / 2, PLANE = HL * L;
    const int h = blockIdx.x * 256 + threadIdx.x;
    const int path = blockIdx.y;
    if (blockIdx.x == 0 && threadIdx.x < 16) reinterpret_cast<double *>(in.acc + path)[threadIdx.x] = 0.0;
    if (h >= HALF) return;
    double *sp = reinterpret_cast<double *>(in.spins) + (size_t)path * 6 * HALF;
    for (int c = 0; c < 2; ++c) {
        const int col = h % PLANE;
        const Site s = make_site(L, col % HL, col / HL, h / PLANE, c);
        double x, y, z;
        if (in.init == INIT_ORDERED) {
            x = 0.0; y = 0.0; z = 1.0;
        } else {
            const Words w = philox4x32_10((uint32_t)s.id, 0u, (uint32_t)path, TAG_INIT | in.ctr3, in.key0, in.key1);
            if (in.init == INIT_ANGLES) Arith<double>::angles(w.w0, w.w1, x, y, z);
            else Arith<double>::sphere(w.w0, w.w1, x, y, z);
        }
        double *own = sp + c * 3 * HALF;
        own[s.h] = x;
        own[HALF + s.h] = y;
        own[2 * HALF + s.h] = z;
    }
}

__global__ __launch_bounds__(256) void k_plain_half(InstDev in, const int *k_dev, int c)
{
    const int L = in.L, HALF = L * L * L / 2, HL = L / 2, PLANE = HL * L;
    const int h = blockIdx.x * 256 + threadIdx.x;
    const int path = blockIdx.y;
    bool a = false;
    if (h < HALF) {
        GroupCtx<double> g;
        g.in = &in;
        g.path = path;
        g.active = true;
        g.lane = h;
        g.sp = reinterpret_cast<double *>(in.spins) + (size_t)path * 6 * HALF;
        const int col = h % PLANE;
        const Site s = make_site(L, col % HL, col / HL, h / PLANE, c);
        double pe = 0.0, px = 0.0, py = 0.0, pz = 0.0;
        a = update_site<double>(g, HALF, c, s, (uint32_t)*k_dev, in.beta, in.J, 0.0, pe, px, py, pz);
    }
    const unsigned long long cnt = (unsigned long long)__popcll(__ballot(a));
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&in.acc[path].n_accept, cnt);
}

// One workgroup per path: measures the state after the sweep, accumulates, then (thread 0)
// advances the device sweep counter.
__global__ __launch_bounds__(256) void k_plain_measure(InstDev in, int *k_dev, int k_last)
{
    __shared__ double part[4][4];
    const int L = in.L, HALF = L * L * L / 2, HL = L / 2, PLANE = HL * L;
    const int path = blockIdx.x;
    const double *sp = reinterpret_cast<const double *>(in.spins) + (size_t)path * 6 * HALF;
    const int k = *k_dev;
    const bool meas = k >= in.n_therm || k < in.trace_sweeps || k == k_last;
    if (meas) {
        double se = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        for (int h = threadIdx.x; h < HALF; h += 256) {
            const int col = h % PLANE;
            const Site s = make_site(L, col % HL, col / HL, h / PLANE, 1);
            const double *odd = sp + 3 * HALF, *even = sp;
            double hx = even[s.nb[0]], hy = even[HALF + s.nb[0]], hz = even[2 * HALF + s.nb[0]];
            for (int n = 1; n < 6; ++n) {
                hx = hx + even[s.nb[n]];
                hy = hy + even[HALF + s.nb[n]];
                hz = hz + even[2 * HALF + s.nb[n]];
            }
            const double ox = odd[h], oy = odd[HALF + h], oz = odd[2 * HALF + h];
            se = se + ((ox * hx + oy * hy) + oz * hz);
            sx += ox + even[h];
            sy += oy + even[HALF + h];
            sz += oz + even[2 * HALF + h];
        }
        se = wave_sum(se);
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        sz = wave_sum(sz);
        if ((threadIdx.x & 63) == 0) {
            part[threadIdx.x >> 6][0] = se;
            part[threadIdx.x >> 6][1] = sx;
            part[threadIdx.x >> 6][2] = sy;
            part[threadIdx.x >> 6][3] = sz;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (meas) {
            double se = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            for (int w = 0; w < 4; ++w) {
                se += part[w][0];
                sx += part[w][1];
                sy += part[w][2];
                sz += part[w][3];
            }
            const double Nd = 2.0 * HALF;
            const double e = -in.J * se / Nd, mx = sx / Nd, my = sy / Nd, mz = sz / Nd;
            PathAcc &A = in.acc[path];
            if (k >= in.n_therm) {
                const double m = sqrt(mx * mx + my * my + mz * mz);
                A.sum_e += e;
                A.sum_e2 += e * e;
                A.sum_m += m;
                A.sum_m2 += m * m;
                A.sum_m4 += (m * m) * (m * m);
            }
            if (k < in.trace_sweeps) {
                double *tr = in.trace + ((size_t)path * in.trace_sweeps + k) * 4;
                tr[0] = e;
                tr[1] = mx;
                tr[2] = my;
                tr[3] = mz;
            }
            if (k == k_last) {
                A.final_e = e;
                A.final_m[0] = mx;
                A.final_m[1] = my;
                A.final_m[2] = mz;
            }
        }
    }
    // every path's workgroup has read k; the last one to finish advances it
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned int done = atomicAdd(reinterpret_cast<unsigned int *>(k_dev + 1), 1u);
        if (done == gridDim.x - 1) {
            k_dev[1] = 0;
            __threadfence();
            atomicAdd(k_dev, 1);
        }
    }
}

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_f64(double *p, size_t n, double v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

}  // namespace

// ------------------------------------------------------------------ variant tables
#define MMC_RES(TT, LC, G, B, MAP, LDS, NAME)                                                         \
    Variant{NAME, std::is_same<TT, double>::value ? 1 : 0, LC, LDS ? 1 : 0, B, G,                      \
            (LC ? lds_layout_bytes<TT>(LC, B, G, LDS) : 0), &launch_resident<TT, LC, G, B, MAP, LDS>,           \
            (const void *)&k_resident<TT, LC, G, B, MAP, LDS>},

static const Variant k_variants[] = {
    // FP32, spins in LDS
    MMC_RES(float, 8, 64, 256, COLZ, true, "f32-lds-L8-g64-b256")
    MMC_RES(float, 8, 128, 256, COLZ, true, "f32-lds-L8-g128-b256")
    MMC_RES(float, 8, 256, 256, COLZ, true, "f32-lds-L8-g256-b256")
    MMC_RES(float, 12, 128, 256, FLAT, true, "f32-lds-L12-g128-b256")
    MMC_RES(float, 12, 256, 256, FLAT, true, "f32-lds-L12-g256-b256")
    MMC_RES(float, 16, 256, 256, COLZ, true, "f32-lds-L16-g256-b256")
    MMC_RES(float, 16, 512, 512, COLZ, true, "f32-lds-L16-g512-b512")
    MMC_RES(float, 16, 1024, 1024, COLZ, true, "f32-lds-L16-g1024-b1024")
    MMC_RES(float, 0, 256, 256, FLAT, true, "f32-lds-any-g256-b256")
    // FP32, spins in device memory
    MMC_RES(float, 24, 512, 512, FLAT, false, "f32-hbm-L24-g512-b512")
    MMC_RES(float, 32, 512, 512, COLZ, false, "f32-hbm-L32-g512-b512")
    MMC_RES(float, 32, 1024, 1024, COLZ, false, "f32-hbm-L32-g1024-b1024")
    MMC_RES(float, 48, 512, 512, FLAT, false, "f32-hbm-L48-g512-b512")
    MMC_RES(float, 64, 512, 512, COLZ, false, "f32-hbm-L64-g512-b512")
    MMC_RES(float, 64, 1024, 1024, COLZ, false, "f32-hbm-L64-g1024-b1024")
    MMC_RES(float, 0, 512, 512, FLAT, false, "f32-hbm-any-g512-b512")
    // FP64, spins in LDS
    MMC_RES(double, 8, 64, 256, COLZ, true, "f64-lds-L8-g64-b256")
    MMC_RES(double, 8, 256, 256, COLZ, true, "f64-lds-L8-g256-b256")
    MMC_RES(double, 12, 256, 256, FLAT, true, "f64-lds-L12-g256-b256")
    MMC_RES(double, 16, 512, 512, COLZ, true, "f64-lds-L16-g512-b512")
    MMC_RES(double, 0, 256, 256, FLAT, true, "f64-lds-any-g256-b256")
    // FP64, spins in device memory
    MMC_RES(double, 16, 512, 512, COLZ, false, "f64-hbm-L16-g512-b512")
    MMC_RES(double, 32, 512, 512, COLZ, false, "f64-hbm-L32-g512-b512")
    MMC_RES(double, 64, 1024, 1024, COLZ, false, "f64-hbm-L64-g1024-b1024")
    MMC_RES(double, 0, 512, 512, FLAT, false, "f64-hbm-any-g512-b512")
};
#undef MMC_RES

const Variant *variants(int *count)
{
    *count = (int)(sizeof(k_variants) / sizeof(k_variants[0]));
    return k_variants;
}

#define MMC_BV(TT, LC, G, MAP, LDS, NAME)                                                            \
    Variant{NAME, std::is_same<TT, double>::value ? 1 : 0, LC, LDS ? 1 : 0, BATCH_B, G,               \
            (LC ? lds_layout_bytes<TT>(LC, BATCH_B, G, LDS) : 0), nullptr, nullptr},
static const Variant k_batch_f32[] = {MMC_BATCH_VARIANTS_F32(MMC_BV)};
static const Variant k_batch_f64[] = {MMC_BATCH_VARIANTS_F64(MMC_BV)};
#undef MMC_BV

const Variant *batch_variants(int fp64, int *count)
{
    if (fp64) {
        *count = (int)(sizeof(k_batch_f64) / sizeof(k_batch_f64[0]));
        return k_batch_f64;
    }
    *count = (int)(sizeof(k_batch_f32) / sizeof(k_batch_f32[0]));
    return k_batch_f32;
}

int batch_block() { return BATCH_B; }

size_t variant_lds_bytes(const Variant &v, int L)
{
    return v.fp64 ? lds_layout_bytes<double>(L, v.block, v.lanes, v.lds) : lds_layout_bytes<float>(L, v.block, v.lanes, v.lds);
}

// Fixed LDS of the batch kernel: the largest footprint of its LDS variants compiled for one
// L (generic LDS variants accept any L whose footprint fits this size).
size_t batch_lds_bytes(int fp64)
{
    int n;
    const Variant *v = batch_variants(fp64, &n);
    size_t m = 0;
    for (int i = 0; i < n; ++i)
        if (v[i].lds && v[i].L) m = std::max(m, v[i].lds_bytes);
    return m;
}

int batch_paths_per_item(int fp64, int variant)
{
    int n;
    const Variant *v = batch_variants(fp64, &n);
    return v[variant].block / v[variant].lanes;
}

size_t batch_slot_bytes(int fp64, int variant, int L)
{
    int n;
    const Variant *v = batch_variants(fp64, &n);
    if (v[variant].lds) return 0;
    return (size_t)(v[variant].block / v[variant].lanes) * 3 * (size_t)L * L * L * (fp64 ? 8 : 4);
}

hipError_t launch_batch(const BatchDev &b, int fp64, int grid, hipStream_t s)
{
    const size_t lds = batch_lds_bytes(fp64);
    if (fp64) hipLaunchKernelGGL(k_batch<double>, dim3(grid), dim3(BATCH_B), lds, s, b);
    else hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(BATCH_B), lds, s, b);
    return hipGetLastError();
}

// Raises every sweep kernel's dynamic-LDS limit to what the device allows per workgroup
// minus the kernel's static LDS (once, before any launch or graph capture). HIP on gfx950
// accepts dynamic LDS up to the device limit without it, so a refusal is not an error: a
// launch that really asks for too much fails and reports itself.
static void raise_lds_limit(const void *fn, int max_lds)
{
    hipFuncAttributes a;
    int stat = 0;
    if (hipFuncGetAttributes(&a, fn) == hipSuccess) stat = (int)a.sharedSizeBytes;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds - stat);
    (void)hipGetLastError();
}

hipError_t prepare_kernels(int max_lds)
{
    static int done = 0;
    if (done) return hipSuccess;
    int n;
    const Variant *vs = variants(&n);
    for (int i = 0; i < n; ++i) raise_lds_limit(vs[i].kernel, max_lds);
    raise_lds_limit((const void *)&k_batch<float>, max_lds);
    raise_lds_limit((const void *)&k_batch<double>, max_lds);
    done = 1;
    return hipSuccess;
}

hipError_t plain_init(const InstDev &in, hipStream_t s)
{
    const int HALF = in.L * in.L * in.L / 2;
    hipLaunchKernelGGL(k_plain_init, dim3((HALF + 255) / 256, in.n_paths), dim3(256), 0, s, in);
    return hipGetLastError();
}

hipError_t plain_half(const InstDev &in, const int *k_dev, int colour, hipStream_t s)
{
    const int HALF = in.L * in.L * in.L / 2;
    hipLaunchKernelGGL(k_plain_half, dim3((HALF + 255) / 256, in.n_paths), dim3(256), 0, s, in, k_dev, colour);
    return hipGetLastError();
}

hipError_t plain_measure(const InstDev &in, int *k_dev, int k_last, hipStream_t s)
{
    hipLaunchKernelGGL(k_plain_measure, dim3(in.n_paths), dim3(256), 0, s, in, k_dev, k_last);
    return hipGetLastError();
}

hipError_t fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, reinterpret_cast<uint32_t *>(p), n, 0u);
    return hipGetLastError();
}

hipError_t fill_nan(double *p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid), dim3(256), 0, s, p, n, __builtin_nan(""));
    return hipGetLastError();
}

hipError_t set_int(int *p, int v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace mmc
