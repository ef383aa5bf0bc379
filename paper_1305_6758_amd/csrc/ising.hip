// ising.hip -- gfx950 kernels of the multipath Metropolis engine for the two-dimensional Ising
// model (arXiv:1305.6758, appendix "2D Ising model": the same multipath set-up as the
// Heisenberg model on an L x L periodic square lattice of spins s = +-1).
//
// One path per wave: its L^2 spins live in LDS as bytes, [colour][row y][j] with j = x >> 1,
// so a path of L = 60 takes 3.6 KB and a workgroup of four waves holds four paths. A wave
// sweeps its own path alone; the workgroup barrier between half-sweeps only orders each
// wave's LDS traffic (all four paths run the same number of sweeps).
//
// Random numbers: one Philox4x32-10 call serves a quad of four consecutive sites (j = 4 jq
// ... 4 jq + 3) of a row of one colour: counter (c L Q + y Q + jq, sweep, path,
// tag | instance << 8) with Q = ceil((L/2) / 4) quads per row; site j takes word j mod 4. The
// move flips s_i; with a = s_i h_i (h_i the sum of the four neighbours) it is taken iff
// (w + 1/2) 2^-32 < exp(-2 beta J a). a takes five values, so the host turns the test into an
// integer comparison w < t[a] with thresholds computed once, which is the same decision as the
// floating-point test for every word w. Energy and magnetisation are integer sums (every bond
// joins an even and an odd site: E = -J sum_odd s_i h_i), fused into the half-sweeps.
#include "engine.hpp"
#include "philox.hpp"

namespace mmc {
namespace {

constexpr int IS_B = 256;  // four waves, four paths
constexpr uint32_t TAG_ISING = 3, TAG_ISING_INIT = 4;

__device__ __forceinline__ int wave_isum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Metropolis decision for a = s h in {-4, -2, 0, 2, 4}: threshold i = (a + 4) / 2.
__device__ __forceinline__ bool ising_accept(const InstDev &in, int a, uint32_t w)
{
    const int i = (a + 4) >> 1;
    const uint32_t t = i == 0 ? in.ithr[0] : i == 1 ? in.ithr[1] : i == 2 ? in.ithr[2] : i == 3 ? in.ithr[3] : in.ithr[4];
    return ((in.iall >> i) & 1u) || w < t;
}

// Half-sweep c of sweep k over one path (sp: the path's spins in LDS). Adds the final spins to
// msum and, on the odd colour, s h to esum; accepted moves to nacc.
template <int LC>
__device__ __forceinline__ void ising_half(const InstDev &in, int8_t *sp, int L, int c, uint32_t k, uint32_t path,
                                           int lane, int &msum, int &esum, int &nacc)
{
    const int HL = L / 2, Q = (HL + 3) / 4, NQ = L * Q;
    int8_t *own = sp + c * L * HL;
    const int8_t *oth = sp + (1 - c) * L * HL;
    for (int q = lane; q < NQ; q += 64) {
        const int y = q / Q, jq = q - y * Q;
        const Words w = philox4x32_10((uint32_t)(c * NQ + q), k, path, TAG_ISING | in.ctr3, in.key0, in.key1);
        const uint32_t wu[4] = {w.w0, w.w1, w.w2, w.w3};
        const int p = (y + c) & 1;
        const int ym = y == 0 ? L - 1 : y - 1, yp = y == L - 1 ? 0 : y + 1;
        int8_t *orow = own + y * HL;
        const int8_t *r0 = oth + y * HL, *rm = oth + ym * HL, *rp = oth + yp * HL;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * jq + u;
            if ((LC != 0 && (LC / 2) % 4 == 0) || j < HL) {
                const int s = orow[j];
                const int jm = p ? j : (j == 0 ? HL - 1 : j - 1);
                const int jp = p ? (j == HL - 1 ? 0 : j + 1) : j;
                const int h = r0[jm] + r0[jp] + rm[j] + rp[j];
                const bool acc = ising_accept(in, s * h, wu[u]);
                const int f = acc ? -s : s;
                if (acc) orow[j] = (int8_t)f;
                nacc += acc;
                msum += f;
                if (c) esum += f * h;
            }
        }
    }
}

template <int LC>
__global__ __launch_bounds__(IS_B) void k_ising(InstDev in, int k0, int k1, int fresh)
{
    extern __shared__ __align__(16) char smem[];
    const int L = LC ? LC : in.L, HL = L / 2, N = L * L, Q = (HL + 3) / 4, NQ = L * Q;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pth = blockIdx.x * (IS_B / 64) + wave;
    const uint32_t path = (uint32_t)__builtin_amdgcn_readfirstlane(pth);
    const bool active = pth < in.n_paths;
    double *shacc = reinterpret_cast<double *>(smem) + 16 * wave;
    const int SPN = (N + 15) & ~15;
    int8_t *sp = reinterpret_cast<int8_t *>(smem + (IS_B / 64) * 128) + wave * SPN;
    int8_t *gsp = reinterpret_cast<int8_t *>(in.spins) + (size_t)pth * N;
    const double J = in.J, Nd = (double)N;

    if (lane < 16) shacc[lane] = (active && !fresh) ? reinterpret_cast<const double *>(in.acc + pth)[lane] : 0.0;
    if (active) {
        if (fresh) {
            // random start (counter (quad, 0, path, TAG_ISING_INIT)); ordered: all +1; mixed by path parity
            const int mode = in.init == INIT_MIXED ? ((path & 1u) ? INIT_ORDERED : INIT_SPHERE) : in.init;
            for (int q = lane; q < 2 * NQ; q += 64) {
                const int c = q >= NQ, qq = q - c * NQ, y = qq / Q, jq = qq - y * Q;
                const Words w = philox4x32_10((uint32_t)q, 0u, path, TAG_ISING_INIT | in.ctr3, in.key0, in.key1);
                const uint32_t wu[4] = {w.w0, w.w1, w.w2, w.w3};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = 4 * jq + u;
                    if (j < HL) sp[c * L * HL + y * HL + j] = (int8_t)(mode == INIT_ORDERED ? 1 : (wu[u] < 0x80000000u ? 1 : -1));
                }
            }
        } else {
            for (int i = lane; i < N; i += 64) sp[i] = gsp[i];
        }
    }
    __syncthreads();
    int nacc = 0;
    for (int k = k0; k < k1; ++k) {
        int msum = 0, esum = 0;
        if (active) ising_half<LC>(in, sp, L, 0, (uint32_t)k, path, lane, msum, esum, nacc);
        __syncthreads();
        if (active) ising_half<LC>(in, sp, L, 1, (uint32_t)k, path, lane, msum, esum, nacc);
        __syncthreads();
        const bool meas = k >= in.n_therm || k < in.trace_sweeps || k == k1 - 1;
        if (meas && active) {
            msum = wave_isum(msum);
            esum = wave_isum(esum);
            if (lane == 0) {
                const double e = -J * (double)esum / Nd, m = (double)msum / Nd;
                if (k >= in.n_therm) {
                    shacc[0] += e;
                    shacc[1] += e * e;
                    shacc[2] += fabs(m);
                    shacc[3] += m * m;
                    shacc[4] += (m * m) * (m * m);
                }
                if (k < in.trace_sweeps) {
                    double *tr = in.trace + ((size_t)path * in.trace_sweeps + k) * 4;
                    tr[0] = e;
                    tr[1] = m;
                    tr[2] = 0.0;
                    tr[3] = 0.0;
                }
                if (k == k1 - 1) {
                    shacc[5] = e;
                    shacc[6] = m;
                    shacc[7] = 0.0;
                    shacc[8] = 0.0;
                }
            }
        }
    }
    if (active) {
        nacc = wave_isum(nacc);
        if (lane == 0) reinterpret_cast<unsigned long long *>(shacc)[9] += (unsigned long long)nacc;
        for (int i = lane; i < N; i += 64) gsp[i] = sp[i];
        if (lane < 16) reinterpret_cast<double *>(in.acc + pth)[lane] = shacc[lane];
    }
}

size_t ising_lds_bytes(int L) { return (size_t)(IS_B / 64) * (128 + (((size_t)L * L + 15) & ~(size_t)15)); }

template <int LC>
hipError_t launch_ising(const InstDev &in, int k0, int k1, int fresh, hipStream_t s)
{
    const int grid = (in.n_paths + IS_B / 64 - 1) / (IS_B / 64);
    hipLaunchKernelGGL(k_ising<LC>, dim3(grid), dim3(IS_B), ising_lds_bytes(LC ? LC : in.L), s, in, k0, k1, fresh);
    return hipGetLastError();
}

}  // namespace

#define MMC_IS(LC, NAME) \
    Variant{NAME, 0, LC, 1, IS_B, 64, LC ? ising_lds_bytes(LC) : 0, &launch_ising<LC>, (const void *)&k_ising<LC>, 0},
static const Variant k_ising_variants[] = {
    MMC_IS(20, "ising2d-L20-b256")
    MMC_IS(40, "ising2d-L40-b256")
    MMC_IS(50, "ising2d-L50-b256")
    MMC_IS(60, "ising2d-L60-b256")
    MMC_IS(0, "ising2d-any-b256")
};
#undef MMC_IS

const Variant *ising_variants(int *count)
{
    *count = (int)(sizeof(k_ising_variants) / sizeof(k_ising_variants[0]));
    return k_ising_variants;
}

size_t ising_variant_lds_bytes(int L) { return ising_lds_bytes(L); }

}  // namespace mmc
