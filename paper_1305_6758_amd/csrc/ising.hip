// ising.hip -- gfx950 kernels of the multipath Metropolis engine for the two-dimensional Ising
// model (arXiv:1305.6758, appendix "2D Ising model": the same multipath set-up as the
// Heisenberg model on an L x L periodic square lattice of spins s = +-1).
//
// One path per wave: its spins live in LDS as bytes b = (s + 1) / 2, [colour][row y][j] with
// j = x >> 1, each row padded to RS = 4 ceil((L/2 + 1) / 4) bytes so that the four sites of a
// quad (j = 4 jq ... 4 jq + 3) form one aligned dword; byte L/2 of a row repeats byte 0 (the
// periodic x-neighbour of the last site), refreshed after every half-sweep. A workgroup of
// four waves holds four paths (L = 60: 3856 bytes each). A wave sweeps its own path alone: the
// LDS operations of one wave execute in order, so a wave-scope fence (no workgroup barrier)
// separates its half-sweeps and the four waves run decoupled.
//
// A quad is updated with packed byte arithmetic: the number of up neighbours n of its four
// sites is the sum of four dwords (the other colour's rows y - 1, y + 1 and the row y shifted
// by one byte either way; bytes 0..4, no carries); with a = s h = 2i - 4 the threshold index of
// a site is i = b ? n : 4 - n. Random numbers: one Philox4x32-10 call per quad, counter
// (c L Q + y Q + jq, sweep, path, tag | instance << 8), Q = ceil((L/2) / 4); site j takes word
// j mod 4. The move flips s; it is taken iff (w + 1/2) 2^-32 < exp(-2 beta J a). Downhill and
// level moves always pass; the two uphill energies (4|J| and 8|J|) have integer thresholds
// computed on the host, so the test is w < t, the same decision as the floating-point test for
// every word w. Energy and magnetisation are integer sums (every bond joins an even and an odd
// site: E = -J sum_odd s_i h_i), fused into the half-sweeps through popcounts and byte dot
// products.
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

// Orders one wave's LDS accesses before its later ones (the hardware keeps a wave's LDS
// operations in order; the fence keeps the compiler from moving accesses across).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ constexpr int ising_row_bytes(int L) { return 4 * ((L / 2 + 4) / 4); }
// One path: both colours' padded rows, and a dword of slack for the next-byte read of a row's
// last quad.
__host__ __device__ constexpr int ising_path_bytes(int L) { return (2 * L * ising_row_bytes(L) + 16 + 15) & ~15; }

// Aligned dword access to byte rows (memcpy keeps the byte and dword views of the same bytes
// well defined; it compiles to one load or store).
__device__ __forceinline__ uint32_t ld4(const uint8_t *p)
{
    uint32_t v;
    __builtin_memcpy(&v, __builtin_assume_aligned(p, 4), 4);
    return v;
}
__device__ __forceinline__ void st4(uint8_t *p, uint32_t v) { __builtin_memcpy(__builtin_assume_aligned(p, 4), &v, 4); }

// Acceptance parameters of a context, in the sign-normalised index i' = (J >= 0 ? i : 4 - i):
// i' <= 2 are downhill or level (always taken), i' = 3 and 4 are the uphill moves of 4|J| and
// 8|J| with thresholds ta and tb; all_mask bit i' set means "always" (infinite temperature).
struct IsingAcc {
    uint32_t ta, tb, all_mask, jneg;
};

__device__ __forceinline__ IsingAcc ising_acc(const InstDev &in)
{
    IsingAcc a;
    if (in.J < 0) {
        a.ta = in.ithr[1];
        a.tb = in.ithr[0];
        a.all_mask = 0;
        for (int i = 0; i < 5; ++i) a.all_mask |= ((in.iall >> i) & 1u) << (4 - i);
        a.jneg = 0x01010101u;
    } else {
        a.ta = in.ithr[3];
        a.tb = in.ithr[4];
        a.all_mask = in.iall;
        a.jneg = 0;
    }
    return a;
}

// Half-sweep c of sweep k over one path (sp: the path's bytes in LDS). Adds sum s of the
// updated sites to msum and, on the odd colour, sum s h to esum; accepted moves to nacc.
template <int LC>
__device__ __forceinline__ void ising_half(const InstDev &in, const IsingAcc &ac, uint8_t *sp, int L, int c,
                                           uint32_t k, uint32_t path, int lane, int &msum, int &esum, int &nacc)
{
    const int HL = L / 2, Q = (HL + 3) / 4, NQ = L * Q, RS = ising_row_bytes(LC ? LC : L);
    uint8_t *own = sp + c * L * RS;
    const uint8_t *oth = sp + (1 - c) * L * RS;
    for (int q = lane; q < NQ; q += 64) {
        const int y = q / Q, jq = q - y * Q, j0 = 4 * jq;
        const Words w = philox4x32_10((uint32_t)(c * NQ + q), k, path, TAG_ISING | in.ctr3, in.key0, in.key1);
        const int p = (y + c) & 1;
        const int ym = y == 0 ? L - 1 : y - 1, yp = y == L - 1 ? 0 : y + 1;
        const uint8_t *r0 = oth + y * RS;
        const uint32_t o0 = ld4(r0 + j0);
        // x-neighbours: p = 0 -> (j - 1, j), p = 1 -> (j, j + 1); the byte shifted in is the
        // other colour's site 4 jq - 1 (L/2 - 1 for the first quad) or 4 jq + 4 (the ghost copy
        // of site 0 after a row's last site)
        const uint32_t bx = r0[p ? j0 + 4 : (jq ? j0 - 1 : HL - 1)];
        const uint32_t xs = p ? ((o0 >> 8) | (bx << 24)) : ((o0 << 8) | bx);
        const uint32_t n = o0 + xs + ld4(oth + ym * RS + j0) + ld4(oth + yp * RS + j0);
        uint8_t *orow = own + y * RS + j0;
        const uint32_t b = ld4(orow);
        const uint32_t bn = b ^ ac.jneg;
        const int nv = (LC != 0 && (LC / 2) % 4 == 0) ? 4 : (HL - j0 < 4 ? HL - j0 : 4);
        const uint32_t vmask = nv == 4 ? 0x01010101u : (0x01010101u & ((1u << (8 * nv)) - 1u));
        const uint32_t wu[4] = {w.w0, w.w1, w.w2, w.w3};
        uint32_t flip = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t nu = (n >> (8 * u)) & 0xFFu, bu = (bn >> (8 * u)) & 1u;
            const uint32_t ip = bu ? nu : 4u - nu;
            const uint32_t t = ip == 4u ? ac.tb : ac.ta;
            const uint32_t acc = ((ac.all_mask >> ip) & 1u) | (uint32_t)(wu[u] < t);
            flip |= acc << (8 * u);
        }
        flip &= vmask;
        const uint32_t b2 = b ^ flip;
        st4(orow, b2);
        const uint32_t up = b2 & vmask;
        const int ups = __builtin_popcount(up);
        nacc += __builtin_popcount(flip);
        msum += 2 * ups - nv;
        if (c) {
            // sum (2b' - 1)(2n - 4) = 4 sum b'n - 8 sum b' - 2 sum n + 4 nv over the quad's sites
            const int bn_dot = (int)__builtin_amdgcn_udot4(up, n, 0u, false);
            const int n_sum = (int)__builtin_amdgcn_udot4(vmask, n, 0u, false);
            esum += 4 * bn_dot - 8 * ups - 2 * n_sum + 4 * nv;
        }
    }
    // ghost copies of this colour's first sites (after every row's last site)
    for (int y = lane; y < L; y += 64) own[y * RS + HL] = own[y * RS];
}

template <int LC>
__global__ __launch_bounds__(IS_B) void k_ising(InstDev in, int k0, int k1, int fresh)
{
    extern __shared__ __align__(16) char smem[];
    const int L = LC ? LC : in.L, HL = L / 2, N = L * L, Q = (HL + 3) / 4, NQ = L * Q;
    const int RS = ising_row_bytes(L), PB = ising_path_bytes(L);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pth = blockIdx.x * (IS_B / 64) + wave;
    const uint32_t path = (uint32_t)__builtin_amdgcn_readfirstlane(pth);
    const bool active = pth < in.n_paths;
    double *shacc = reinterpret_cast<double *>(smem) + 16 * wave;
    uint8_t *sp = reinterpret_cast<uint8_t *>(smem + (IS_B / 64) * 128) + wave * PB;
    uint8_t *gsp = reinterpret_cast<uint8_t *>(in.spins) + (size_t)pth * PB;
    const double J = in.J, Nd = (double)N;
    const IsingAcc ac = ising_acc(in);

    if (lane < 16) shacc[lane] = (active && !fresh) ? reinterpret_cast<const double *>(in.acc + pth)[lane] : 0.0;
    if (active) {
        if (fresh) {
            // random start (counter (quad, 0, path, TAG_ISING_INIT)): b = 1 iff the word < 2^31;
            // ordered: all up; mixed by path parity
            const int mode = in.init == INIT_MIXED ? ((path & 1u) ? INIT_ORDERED : INIT_SPHERE) : in.init;
            for (int i = lane; i < PB / 4; i += 64) st4(sp + 4 * i, 0u);
            for (int q = lane; q < 2 * NQ; q += 64) {
                const int c = q >= NQ, qq = q - c * NQ, y = qq / Q, jq = qq - y * Q;
                const Words w = philox4x32_10((uint32_t)q, 0u, path, TAG_ISING_INIT | in.ctr3, in.key0, in.key1);
                const uint32_t wu[4] = {w.w0, w.w1, w.w2, w.w3};
                uint32_t v = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (4 * jq + u < HL) v |= (uint32_t)(mode == INIT_ORDERED ? 1 : (wu[u] < 0x80000000u ? 1 : 0)) << (8 * u);
                st4(sp + c * L * RS + y * RS + 4 * jq, v);
            }
            for (int r = lane; r < 2 * L; r += 64) sp[r * RS + HL] = sp[r * RS];
        } else {
            for (int i = lane; i < PB / 4; i += 64) st4(sp + 4 * i, ld4(gsp + 4 * i));
        }
    }
    __syncthreads();
    int nacc = 0;
    for (int k = k0; k < k1; ++k) {
        int msum = 0, esum = 0;
        if (active) ising_half<LC>(in, ac, sp, L, 0, (uint32_t)k, path, lane, msum, esum, nacc);
        wave_sync();
        if (active) ising_half<LC>(in, ac, sp, L, 1, (uint32_t)k, path, lane, msum, esum, nacc);
        wave_sync();
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
        for (int i = lane; i < PB / 4; i += 64) st4(gsp + 4 * i, ld4(sp + 4 * i));
        if (lane < 16) reinterpret_cast<double *>(in.acc + pth)[lane] = shacc[lane];
    }
}

size_t ising_lds_bytes(int L) { return (size_t)(IS_B / 64) * (128 + (size_t)ising_path_bytes(L)); }

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

size_t ising_spin_bytes(int L) { return (size_t)ising_path_bytes(L); }
int ising_row_stride(int L) { return ising_row_bytes(L); }

}  // namespace mmc
